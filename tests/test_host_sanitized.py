"""Host validation layer under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only): the
library built with both sanitizers on its host code (device code as usual), and the C driver
tests/host_checks.c exercising every entry point's argument checks through the C ABI.  Any
out-of-bounds access, use-after-free, signed overflow or null-pointer arithmetic in the host code
makes the driver fail."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "_build", "hostsan")


def test_host_checks_under_asan_and_ubsan():
    import importlib
    B = importlib.import_module("paper_2508_06628_amd.build")
    lib = B.build_host_sanitized(OUT)
    exe = os.path.join(OUT, "host_checks")
    clang = "/opt/rocm/llvm/bin/clang"
    subprocess.run([clang, "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-g", "-O1",
                    "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "host_checks.c"), "-o", exe,
                    "-L", OUT, "-lts_mi355x_hostsan", f"-Wl,-rpath,{OUT}", "-lm"], check=True)
    # leak checking is off (the HIP runtime keeps allocations until exit); the link-order check is
    # off so that a library preloaded by the environment does not stop the sanitizer runtime
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host checks ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    assert os.path.exists(lib)
