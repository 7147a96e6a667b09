"""The differentiable-trajectory workload at its full size (Section 2's RDF-gradient use case): one
864-atom argon system (system 0 of the 16-system batch, seed 3), 500 velocity-Verlet steps at
dt = 2 fs, checkpoints every 50 steps, smeared-RDF loss against the RDF of the same simulation with
epsilon and sigma scaled by 1.05.  Loss, dL/deps, dL/dsigma and sampled rows of dL/dr_0 are compared
with the FP64 oracle's reverse pass stored in tests/golden/argon_adjoint_864_500.txt (written by the
oracle-only script beside it).  FP64 agrees to 1e-7 relative after 500 steps; FP32 pair arithmetic
to 1e-3 relative (the FP32 trajectory drifts from the FP64 one through the 500 steps)."""
import os

import numpy as np
import pytest

from workloads import argon_adjoint_batch

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FIXTURE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "argon_adjoint_864_500.txt")


def _fixture():
    vals, rows = {}, {}
    for line in open(FIXTURE):
        if line.startswith("#") or not line.strip():
            continue
        parts = line.split()
        if parts[0] == "row":
            rows[int(parts[1])] = np.array([float(x) for x in parts[2:5]])
        else:
            vals[parts[0]] = float(parts[1])
    return vals, rows


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2508_06628_amd import _native
    _native.lib()
    yield
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec,tol", [("f64", 1e-7), ("f32", 1e-3)])
def test_full_size_gradient_matches_oracle_fixture(prec, tol):
    from paper_2508_06628_amd.trajectory import RdfSpec, TrajectoryRDF
    vals, rows = _fixture()
    w = argon_adjoint_batch(16, n_steps=500).subset([0])
    n_steps = int(vals["n_steps"])
    assert w.n_atoms == int(vals["n_atoms"]) and n_steps == 500
    ex = w.extra
    eng = TrajectoryRDF(w, n_steps, int(ex["checkpoint_every"]), prec=prec,
                        rdf=RdfSpec(int(ex["rdf_bins"]), float(ex["rdf_rmax"]), float(ex["rdf_sigma"])))
    eps, sig = float(w.potential.params[0, 0, 0]), float(w.potential.params[0, 0, 1])
    pos0 = eng.batch.pos.clone()
    scale = float(ex["target_scale"])
    eng.set_target(eng.run(eps * scale, sig * scale, pos0, keep_checkpoints=False).clone())
    loss = eng.forward(eps, sig, pos0).item()
    de, ds, lr0 = eng.backward()
    eng.check_status()
    assert abs(loss - vals["loss"]) <= tol * abs(vals["loss"])
    assert abs(de - vals["dL_deps"]) <= tol * abs(vals["dL_deps"])
    assert abs(ds - vals["dL_dsigma"]) <= tol * abs(vals["dL_dsigma"])
    g = lr0.T.cpu().numpy()
    scale_r = vals["dL_dr0_max_abs"]
    assert abs(np.abs(g).max() - scale_r) <= tol * scale_r
    assert abs(np.linalg.norm(g) - vals["dL_dr0_norm"]) <= tol * vals["dL_dr0_norm"]
    for i, ref in rows.items():
        assert np.abs(g[i] - ref).max() <= tol * scale_r, (i, g[i], ref)
