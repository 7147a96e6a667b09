"""Benchmark: batched Lennard-Jones argon NVE, 64 systems x 864 atoms, on one MI355X.

One step = one velocity-Verlet step of the whole batch (device-side neighbor validity test and
rebuilds included), FP32 pair arithmetic with FP64 integration, the step loop replayed from
hipGraphs.  Prints one JSON line with atom-steps/s, the force kernel's roofline position, the
plain one-system-per-launch path on the same GPU, the adjoint (trajectory-gradient) throughput
of the 16 x 864 differentiable run, the batched FIRE relaxation of the uneven 512-system copper
batch (one persistent launch), the soft-sphere jamming batch (FIRE, then NVE), and the FP64 CPU
oracle timed on the host.

    python bench.py [--steps K] [--warmup W] [--chunk C] [--no-plain] [--no-adjoint] [--no-fire] [--no-cpu]
    python bench.py --profile-kernels --lanes L [--group G]   # short launch sequence for rocprofv3
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "atom-steps/s batched LJ NVE (64×864 atoms) + adjoint steps/s, vs plain path"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def batched_nve(api, torch, w, steps, warmup, chunk, bin_factor, lanes, group=0):
    pot = w.potential
    b = api.Batch.from_workload(w)
    nl = api.build_neighbor_list(b, pot.cutoff, w.skin, bin_factor=bin_factor, margin=1.3)
    pp = api.pair_params_from_spec(pot, w.pair_prec)
    tune = None
    if lanes == 0:
        from paper_2508_06628_amd.autotune import tune_nve
        tune = tune_nve(b, nl, pp, w.dt, w.accel)
        log(f"autotune: {tune}")
    else:
        nl.lanes_per_atom = lanes
        nl.group_atoms = group
    F = api.force_buffer(b, w.pair_prec)
    api.ts_pair_forces(b, nl, pp, F)
    chunk = max(1, min(chunk, steps))
    n_full, rest = divmod(steps, chunk)
    w_runs = max(1, -(-warmup // chunk)) if warmup > 0 else 0
    for _ in range(w_runs):
        api.ts_nve_step(b, nl, pp, w.dt, w.accel, chunk, F, use_graph=True)
    if rest:
        api.ts_nve_step(b, nl, pp, w.dt, w.accel, rest, F, use_graph=True)  # instantiate its graph
    torch.cuda.synchronize()
    nl.status.zero_()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(n_full):
        api.ts_nve_step(b, nl, pp, w.dt, w.accel, chunk, F, use_graph=True)
    if rest:
        api.ts_nve_step(b, nl, pp, w.dt, w.accel, rest, F, use_graph=True)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    st = nl.read_status()
    if st[1] or st[3] or st[4]:
        raise RuntimeError(f"neighbor list status after the timed run: {st.tolist()}")
    return dict(ms=ms, wall_s=wall, warmup_steps=w_runs * chunk + rest, rebuilds=int(st[2]),
                max_nbr=int(st[0]), capacity=nl.max_nbr, batch=b, nl=nl, pp=pp, F=F, lanes=nl.lanes_per_atom,
                group=nl.group_atoms, tune=tune)


def langevin_throughput(api, torch, w, steps, chunk, bin_factor, gamma=0.01, temp_k=85.0):
    """BAOAB Langevin on the same batch, in graph-replayed calls of `chunk` steps."""
    pot = w.potential
    b = api.Batch.from_workload(w)
    nl = api.build_neighbor_list(b, pot.cutoff, w.skin, bin_factor=bin_factor, margin=1.3)
    pp = api.pair_params_from_spec(pot, w.pair_prec)
    F = api.force_buffer(b, w.pair_prec)
    api.ts_pair_forces(b, nl, pp, F)
    k_b = 8.617333262145179e-5  # eV/K
    kT = torch.full((w.n_systems,), k_b * temp_k, dtype=torch.float64, device="cuda")
    ctr = torch.zeros(1, dtype=torch.int64, device="cuda")
    chunk = max(1, min(chunk, steps))
    n_full = max(1, steps // chunk)
    api.ts_langevin_step(b, nl, pp, w.dt, w.accel, gamma, kT, 2024, ctr, chunk, F)  # instantiate the graph
    torch.cuda.synchronize()
    nl.status.zero_()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(n_full):
        api.ts_langevin_step(b, nl, pp, w.dt, w.accel, gamma, kT, 2024, ctr, chunk, F)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    st = nl.read_status()
    if st[1] or st[3] or st[4]:
        raise RuntimeError(f"neighbor list status after the Langevin run: {st.tolist()}")
    n = n_full * chunk
    return dict(value=round(w.n_atoms * n / (ms * 1e-3), 1), unit="atom-steps/s", steps=n,
                us_per_step=round(ms * 1e3 / n, 2), gamma_per_fs=gamma, temperature_K=temp_k, rebuilds=int(st[2]))


def graph_export(api, torch, w, bin_factor, reps=50):
    """Export of the batch graph at r_graph = r_c from a valid list: mean time per export (HIP events
    on the launch stream) and its algorithmic bytes (list entries read once, positions, edges written
    with index pairs, integer shifts and vectors, the row pointer)."""
    pot = w.potential
    b = api.Batch.from_workload(w)
    nl = api.build_neighbor_list(b, pot.cutoff, w.skin, bin_factor=bin_factor, margin=1.3)
    entries = int(nl.n_nbr.sum().item())
    g = api.mlip_graph(b, nl, pot.cutoff)
    E = int(g["edge_offsets"][-1].item())
    row_ptr, offs = torch.empty_like(g["row_ptr"]), torch.empty_like(g["edge_offsets"])
    ei = torch.empty((2, E), dtype=torch.int64, device="cuda")
    sh = torch.empty((E, 3), dtype=torch.int32, device="cuda")
    vec = torch.empty((E, 3), dtype=torch.float64, device="cuda")
    api.ts_graph_export(b, nl, pot.cutoff, row_ptr, offs, ei, sh, vec)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        api.ts_graph_export(b, nl, pot.cutoff, row_ptr, offs, ei, sh, vec)
    ev1.record()
    torch.cuda.synchronize()
    us = ev0.elapsed_time(ev1) * 1e3 / reps
    alg = 4 * entries + 4 * w.n_atoms + 24 * w.n_atoms + 8 * (w.n_atoms + 1) + (16 + 12 + 24) * E
    return dict(us_per_export=round(us, 2), edges=E, list_entries=entries, edges_per_s=round(E / (us * 1e-6), 1),
                alg_bytes=alg, achieved_GBps=round(alg / (us * 1e-6) / 1e9, 1),
                frac_hbm=round(alg / (us * 1e-6) / 8e12, 4))


def measured_counter(summary: str, field: str, kernel: str):
    """A per-launch figure of ``kernel`` from a committed rocprofv3 counter summary under profiles/
    (``traffic_bytes_per_launch``: FETCH_SIZE + WRITE_SIZE scaled by a device copy of known size;
    ``valu_insts_per_launch``: SQ_INSTS_VALU), or None once the kernel sources have changed since
    those counters were taken."""
    import glob
    import hashlib
    path = os.path.join(ROOT, "profiles", summary)
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return None
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2508_06628_amd", "csrc", "*"))):
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    rec = dict(l.split(": ", 1) for l in lines if ": " in l and not l.startswith("#"))
    if rec.get("csrc_sha256") != h.hexdigest():
        return None
    v = rec.get(f"{field} {kernel}")
    return int(v) if v else None


# VALU issue peak of the chip: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-instructions per second
# (a wave64 VALU instruction occupies a 16-lane SIMD for 4 cycles; float64 FMA issues at this rate)
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9


def alu_roofline(summary: str, kernel: str, avg_us: float):
    """The kernel's VALU lane-instruction rate (committed SQ_INSTS_VALU per launch x 64 lanes ÷ the
    live average launch duration) against the chip's VALU issue peak, or None without counters."""
    n = measured_counter(summary, "valu_insts_per_launch", kernel)
    if n is None:
        return None
    achieved = n * 64 / (avg_us * 1e-6)
    return dict(bound="alu", achieved=round(achieved / 1e12, 2), peak=round(VALU_PEAK_LANE_OPS / 1e12, 2),
                unit="T lane-instructions/s", frac=round(achieved / VALU_PEAK_LANE_OPS, 4), kernel=kernel,
                valu_insts_per_launch=n)


ROOFLINE_LANES, ROOFLINE_GROUP = 2, 128


def force_kernel_roofline(api, torch, r, reps=200):
    """Average duration of the pair-force kernel alone, timed with events on the stream it is
    launched on (torch's current stream), and its algorithmic HBM bytes.  For systems that fit the
    LDS (up to 2048 atoms) the force entry point runs the step kernel in its forces-only mode: one
    workgroup per system, positions staged in LDS."""
    b, nl, pp, F = r["batch"], r["nl"], r["pp"], r["F"]
    # two lanes per atom and 128 atoms per workgroup: the autotuner's choice on this batch and the
    # configuration of the committed counter summaries (the step loop keeps the autotuner's choice)
    tuned = nl.lanes_per_atom, nl.group_atoms
    nl.lanes_per_atom, nl.group_atoms = ROOFLINE_LANES, ROOFLINE_GROUP
    stream = torch.cuda.current_stream()
    for _ in range(10):
        api.ts_pair_forces(b, nl, pp, F, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        api.ts_pair_forces(b, nl, pp, F, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    avg_ms = e0.elapsed_time(e1) / reps
    nl.lanes_per_atom, nl.group_atoms = tuned
    n, n_sys = b.n_atoms, b.n_systems
    entries = int(nl.n_nbr.sum().item())
    fbytes = 4 if F.dtype == torch.float32 else 8
    # per atom: position 24 B, list length 4 B, force 3*fbytes; per list entry 4 B;
    # per system: atom offset 8 B and cell 72 B
    alg = n * (24 + 4 + 3 * fbytes) + 4 * entries + n_sys * (8 + 72)
    achieved = alg / (avg_ms * 1e-3) / 1e9
    ftype = "float" if fbytes == 4 else "double"
    kernel = f"ts::k_step<0, {ftype}, {ROOFLINE_LANES}, 3>"
    return dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4),
                traffic=measured_counter("k_step_argon_64x864_counters.txt", "traffic_bytes_per_launch",
                                         "void " + kernel),
                kernel=kernel, avg_launch_us=round(avg_ms * 1e3, 3),
                launches_timed=reps, alg_bytes_per_launch=alg, alg_bytes_per_atom=round(alg / n, 1),
                mean_list_len=round(entries / n, 2))


def plain_path(api, torch, w, steps, bin_factor):
    """Same kernels, one system per launch sequence, no graph: systems advanced one after another."""
    pot = w.potential
    pp = api.pair_params_from_spec(pot, w.pair_prec)
    runs = []
    for s in range(w.n_systems):
        ws = w.subset([s])
        b = api.Batch.from_workload(ws)
        nl = api.build_neighbor_list(b, pot.cutoff, w.skin, bin_factor=bin_factor, margin=1.3)
        F = api.force_buffer(b, w.pair_prec)
        api.ts_pair_forces(b, nl, pp, F)
        runs.append((b, nl, F))
    for b, nl, F in runs:  # warm-up
        api.ts_nve_step(b, nl, pp, w.dt, w.accel, 2, F, use_graph=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b, nl, F in runs:
        api.ts_nve_step(b, nl, pp, w.dt, w.accel, steps, F, use_graph=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dict(value=w.n_atoms * steps / dt, steps=steps, seconds=round(dt, 4))


def adjoint_throughput(api, torch, n_systems, n_steps, checkpoint, plain=True):
    """Backward pass (segment recomputation + reverse steps) of the checkpointed trajectory gradient
    of the 16 x 864 argon batch, and the same work one system at a time without graphs (the plain
    path)."""
    from paper_2508_06628_amd.trajectory import TrajectoryRDF
    from workloads import argon_adjoint_batch
    w = argon_adjoint_batch(n_systems, n_steps=n_steps)
    eps, sig = float(w.potential.params[0, 0, 0]), float(w.potential.params[0, 0, 1])

    def one(ww, use_graph):
        eng = TrajectoryRDF(ww, n_steps, checkpoint, prec="f32", use_graph=use_graph)
        pos0 = eng.batch.pos.clone()
        g_t = eng.run(eps * 1.05, sig * 1.05, pos0).clone()
        eng.set_target(g_t)
        eng.forward(eps, sig, pos0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        eng.forward(eps, sig, pos0)
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t0
        t0 = time.perf_counter()
        de, ds, dr = eng.backward()
        torch.cuda.synchronize()
        t_bwd = time.perf_counter() - t0
        eng.check_status()
        return eng, t_fwd, t_bwd, de, ds

    eng, t_fwd, t_bwd, de, ds = one(w, True)
    out = dict(value=w.n_atoms * n_steps / t_bwd, unit="atom-steps/s (backward: recompute + reverse)",
               workload=f"argon_adjoint_{n_systems}x864_{n_steps}steps_ckpt{checkpoint}",
               steps_per_s=round(n_steps / t_bwd, 2), backward_s=round(t_bwd, 3), forward_s=round(t_fwd, 3),
               loss=float(eng.loss.item()), dL_deps=de, dL_dsigma=ds)
    if plain:
        t_plain = 0.0
        for s in range(n_systems):
            _, _, tb, _, _ = one(w.subset([s]), False)
            t_plain += tb
        out["plain_path"] = dict(value=round(w.n_atoms * n_steps / t_plain, 1), backward_s=round(t_plain, 3),
                                 unit="atom-steps/s (backward, one system at a time, no graphs)",
                                 speedup_batched_vs_plain=round(t_plain / t_bwd, 2))
    return out


def _check_list(nl, what):
    st = nl.read_status()
    if st[1] or st[3] or st[4]:
        raise RuntimeError(f"neighbor list status after {what}: {st.tolist()}")
    return st


def fire_copper(api, torch, max_iter=20000, skin=1.0):
    """Batched FIRE of positions and cell on the uneven 512-system Morse copper batch until every
    system has max |F| < fmax (and the cell force too): repeated ts_fire_step calls on the path the
    autotuner picks (one persistent launch per call, largest system first, plus a bounded tail of
    per-iteration launches; or per-iteration launches throughout) and its lanes per atom; the host
    reads the convergence flags between calls.  The list skin is a tuning parameter of the
    relaxation (forces do not depend on it): 1 A trades longer rows for fewer rebuilds under cell
    changes."""
    from paper_2508_06628_amd.autotune import tune_fire
    from workloads import copper_uneven_batch
    w = copper_uneven_batch(512, seed=2)
    pot = w.potential
    b = api.Batch.from_workload(w)
    nl = api.build_neighbor_list(b, pot.cutoff, skin, bin_factor=2, margin=1.2)
    pp = api.pair_params_from_spec(pot, w.pair_prec)
    cfgd = dict(w.extra["fire"])
    cfgd["relax_cell"] = True
    cfgd["max_iter"] = max_iter
    cfg = api.fire_config(**cfgd)
    tune = tune_fire(b, nl, pp, cfg)
    log(f"FIRE autotune: {tune}")
    fs = api.FireState(b, cfg)
    F = api.force_buffer(b, w.pair_prec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    calls = api.fire_relax(b, fs, cfg, nl, pp, F, persistent=tune["persistent"])
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    st = _check_list(nl, "copper FIRE")
    it = fs.n_iter.cpu().numpy()
    work = float((it * np.diff(b.h_offsets)).sum())
    return dict(workload=f"copper_morse_fire_cell_{w.n_systems}_uneven", n_atoms=b.n_atoms, skin_A=skin,
                seconds=round(sec, 4), calls=calls,
                converged=int(fs.converged.sum().item()), n_systems=w.n_systems, iterations_mean=round(float(it.mean()), 1),
                iterations_max=int(it.max()), value=round(work / sec, 1), unit="atom-iterations/s",
                list_rebuilds=int(st[2]), list_max_nbr=int(st[0]), list_capacity=nl.max_nbr,
                persistent=tune["persistent"], lanes_per_atom=tune["lanes_per_atom"], tune_ms=tune.get("ms"))


def copper_force_roofline(api, torch, reps=50):
    """The pair-force kernel on the uneven 512-system copper batch (72 M list entries, ~290 MB of
    list: beyond the 256 MB Infinity Cache, so its bytes come from HBM): average launch duration
    timed with events on the launch stream, and its algorithmic bytes."""
    from workloads import copper_uneven_batch
    w = copper_uneven_batch(512, seed=2)
    pot = w.potential
    b = api.Batch.from_workload(w)
    nl = api.build_neighbor_list(b, pot.cutoff, w.skin, bin_factor=2, margin=1.2)
    pp = api.pair_params_from_spec(pot, w.pair_prec)
    F = api.force_buffer(b, w.pair_prec)
    stream = torch.cuda.current_stream()
    for _ in range(5):
        api.ts_pair_forces(b, nl, pp, F, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        api.ts_pair_forces(b, nl, pp, F, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    _check_list(nl, "copper force timing")
    avg_ms = e0.elapsed_time(e1) / reps
    entries = int(nl.n_nbr.sum().item())
    n = b.n_atoms
    alg = n * (24 + 4 + 12) + 4 * entries + w.n_systems * (8 + 72)
    achieved = alg / (avg_ms * 1e-3) / 1e9
    tl = nl.lanes_per_atom if nl.lanes_per_atom > 0 else (8 if n * 4 // 64 < 2048 else 4)
    kernel = f"ts::k_step<1, float, {tl}, 3>"
    return dict(workload=f"copper_morse_forces_{w.n_systems}_uneven", kernel=kernel,
                bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4),
                traffic=measured_counter("k_step_copper_512_counters.txt", "traffic_bytes_per_launch",
                                         "void " + kernel),
                roofline_alu=alu_roofline("k_step_copper_512_counters.txt", "void " + kernel, avg_ms * 1e3),
                avg_launch_us=round(avg_ms * 1e3, 2),
                alg_bytes_per_launch=alg, list_entries=entries, mean_list_len=round(entries / n, 2), n_atoms=n)


def soft_sphere(api, torch, fire_seconds=60.0, nve_steps=2000, chunk=100):
    """Soft-sphere jamming batch (8 x 32000, binary): batched FIRE to max |F| < 1e-6 (capped by wall
    time, reported), then NVE at T = 1e-4 (reduced units) from Maxwell-Boltzmann velocities, and
    Langevin at the same temperature."""
    from workloads import maxwell_boltzmann, soft_sphere_jamming_batch
    from paper_2508_06628_amd.autotune import tune_bin_factor
    w = soft_sphere_jamming_batch(8, 32000, seed=4)
    pot = w.potential
    b = api.Batch.from_workload(w)
    nl = api.build_neighbor_list(b, pot.cutoff, w.skin, bin_factor=2, margin=1.3)
    bins = tune_bin_factor(b, nl)
    log(f"soft-sphere bin factor autotune: {bins}")
    pp = api.pair_params_from_spec(pot, w.pair_prec)
    cfg = api.fire_config(**w.extra["fire"])
    fs = api.FireState(b, cfg)
    F = api.force_buffer(b, w.pair_prec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    calls = 0
    capped = False
    while True:
        api.ts_fire_step(b, fs, cfg, nl, pp, 256, F)
        calls += 1
        if fs.converged.all().item():
            break
        if time.perf_counter() - t0 > fire_seconds:
            capped = True
            break
    torch.cuda.synchronize()
    fire_s = time.perf_counter() - t0
    _check_list(nl, "soft-sphere FIRE")
    it = fs.n_iter.cpu().numpy()
    fire_work = float((it * np.diff(b.h_offsets)).sum())
    fire = dict(seconds=round(fire_s, 3), iterations_max=int(it.max()), iterations_min=int(it.min()),
                converged=int(fs.converged.sum().item()), n_systems=w.n_systems, fmax=float(cfg.fmax),
                capped_at_seconds=fire_seconds if capped else None,
                value=round(fire_work / fire_s, 1), unit="atom-iterations/s")
    log(f"soft-sphere FIRE: {fire}")
    rng = np.random.default_rng(5)
    v = maxwell_boltzmann(rng, w.mass, w.extra["nve_temperature"], k_b=1.0, accel=1.0)
    b.vel.copy_(torch.tensor(np.ascontiguousarray(v.T), dtype=torch.float64, device=b.device))
    api.ts_pair_forces(b, nl, pp, F)
    api.ts_nve_step(b, nl, pp, w.dt, w.accel, chunk, F, use_graph=True)  # instantiate the graph
    torch.cuda.synchronize()
    nl.status.zero_()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(nve_steps // chunk):
        api.ts_nve_step(b, nl, pp, w.dt, w.accel, chunk, F, use_graph=True)
    e1.record()
    torch.cuda.synchronize()
    nve_ms = e0.elapsed_time(e1)
    st = _check_list(nl, "soft-sphere NVE")
    # Langevin at the same temperature (the per-atom loop of systems above the LDS limit)
    kT = torch.full((w.n_systems,), float(w.extra["nve_temperature"]), dtype=torch.float64, device=b.device)
    ctr = torch.zeros(1, dtype=torch.int64, device=b.device)
    api.ts_langevin_step(b, nl, pp, w.dt, w.accel, 1.0, kT, 11, ctr, chunk, F)  # instantiate the graph
    torch.cuda.synchronize()
    e0.record()
    for _ in range(nve_steps // chunk):
        api.ts_langevin_step(b, nl, pp, w.dt, w.accel, 1.0, kT, 11, ctr, chunk, F)
    e1.record()
    torch.cuda.synchronize()
    lang_ms = e0.elapsed_time(e1)
    _check_list(nl, "soft-sphere Langevin")
    return dict(workload="soft_sphere_binary_8x32000", n_atoms=b.n_atoms, bin_factor=int(nl.bin_factor),
                bin_factor_build_ms=bins["ms"], fire=fire,
                nve=dict(steps=nve_steps, ms_per_step=round(nve_ms / nve_steps, 5),
                         value=round(w.n_atoms * nve_steps / (nve_ms * 1e-3), 1), unit="atom-steps/s",
                         system_rebuilds=int(st[2]), start="FIRE end state" + (" (capped)" if capped else "")),
                langevin=dict(steps=nve_steps, gamma=1.0, ms_per_step=round(lang_ms / nve_steps, 5),
                              value=round(w.n_atoms * nve_steps / (lang_ms * 1e-3), 1), unit="atom-steps/s"))


def _oracle_nve_task(args):
    from threadpoolctl import threadpool_limits
    from oracle import integrate
    ws, steps = args
    with threadpool_limits(1):
        t0 = time.perf_counter()
        integrate.nve(ws.pos, ws.vel, ws.mass, ws.cell, ws.sys_offsets, ws.species, ws.potential, ws.dt, steps,
                      ws.accel)
        return time.perf_counter() - t0


def cpu_baseline(w, steps=2):
    """The FP64 oracle (brute-force pair sums) on the host cores: one system of the workload per
    process, as many processes as cores (at most one per system), each running ``steps`` NVE steps
    (plus the initial force evaluation); throughput = atoms x steps of all processes / wall time,
    extrapolated to the whole batch (systems are independent)."""
    import multiprocessing as mp
    cores = min(os.cpu_count() or 1, w.n_systems)
    tasks = [(w.subset([s]), steps) for s in range(cores)]
    # fresh interpreters (the parent holds a GPU context; the children only run NumPy)
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        per = pool.map(_oracle_nve_task, tasks)
    wall = time.perf_counter() - t0
    atoms = sum(t[0].n_atoms for t in tasks)
    return dict(value=round(atoms * steps / wall, 2), unit="atom-steps/s", cores=cores, kind="oracle",
                sample=f"{cores} systems x {tasks[0][0].n_atoms} atoms, one per process on {cores} cores, "
                       f"{steps} NVE steps each (+1 initial force evaluation), {wall:.1f} s wall "
                       f"(per-process {min(per):.1f}-{max(per):.1f} s), float64 NumPy, one BLAS thread per process; "
                       f"extrapolated to the {w.n_systems}-system batch")


def profile_kernels(api, torch, w, lanes, bin_factor, reps=20, copy_mib=256, group=0):
    """Fixed launch sequence for rocprofv3 runs (kernel trace and byte counters): the force
    kernel ``reps`` times, two 100-step NVE graph replays, and a plain device copy of
    ``copy_mib`` MiB whose counter readings calibrate the byte counters."""
    b = api.Batch.from_workload(w)
    pot = w.potential
    nl = api.build_neighbor_list(b, pot.cutoff, w.skin, bin_factor=bin_factor, margin=1.3)
    nl.lanes_per_atom = lanes
    nl.group_atoms = group
    pp = api.pair_params_from_spec(pot, w.pair_prec)
    F = api.force_buffer(b, w.pair_prec)
    for _ in range(reps):
        api.ts_pair_forces(b, nl, pp, F)
    for _ in range(2):
        api.ts_nve_step(b, nl, pp, w.dt, w.accel, 100, F, use_graph=True)
    n = copy_mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    return dict(mode="profile", workload=w.name, n_atoms=b.n_atoms, lanes_per_atom=lanes, force_launches=reps,
                list_entries=int(nl.n_nbr.sum().item()), copy_bytes_each_way=n * 4, copy_launches=3)


def profile_copper(api, torch, reps=20, rebuilds=10, copy_mib=256):
    """Fixed launch sequence for rocprofv3 runs on the uneven 512-system copper batch: the pair-force
    kernel ``reps`` times (its 290 MB list is beyond the Infinity Cache), ``rebuilds`` forced rebuilds
    of every row (the large-system row rebuild) and the calibration copy."""
    from workloads import copper_uneven_batch
    w = copper_uneven_batch(512, seed=2)
    b = api.Batch.from_workload(w)
    nl = api.build_neighbor_list(b, w.potential.cutoff, w.skin, bin_factor=2, margin=1.2)
    pp = api.pair_params_from_spec(w.potential, w.pair_prec)
    F = api.force_buffer(b, w.pair_prec)
    for _ in range(reps):
        api.ts_pair_forces(b, nl, pp, F)
    for _ in range(rebuilds):
        api.ts_neighbor_build(b, nl, force=True)
    n = copy_mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    entries = int(nl.n_nbr.sum().item())
    alg = b.n_atoms * (24 + 4 + 12) + 4 * entries + w.n_systems * (8 + 72)
    counts = np.diff(b.h_offsets).astype(np.float64)
    return dict(mode="profile", workload="copper_morse_forces_512_uneven", n_atoms=b.n_atoms, force_launches=reps,
                list_entries=entries, alg_bytes_per_launch=alg, rebuild_launches=rebuilds,
                rebuild_candidate_pairs=int((counts ** 2).sum()), copy_bytes_each_way=n * 4, copy_launches=3)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=15)
    ap.add_argument("--chunk", type=int, default=100)
    ap.add_argument("--bin-factor", type=int, default=2)
    ap.add_argument("--lanes", type=int, default=0, help="lanes per atom in the step kernel (0: autotune)")
    ap.add_argument("--group", type=int, default=0, help="atoms per workgroup in the step kernel (with --lanes)")
    ap.add_argument("--plain-steps", type=int, default=50)
    ap.add_argument("--adjoint-steps", type=int, default=500)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-langevin", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-export measurement")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fire", action="store_true", help="skip the copper FIRE and soft-sphere workloads")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="run a short fixed launch sequence for rocprofv3 instead of the benchmark")
    ap.add_argument("--profile-copper", action="store_true",
                    help="fixed launch sequence of the copper force kernel for rocprofv3")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (systems would shard "
              "across GPUs by bin packing; see the design notes). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2508_06628_amd import api
    from workloads import argon_batch

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    w = argon_batch(64, seed=1, n_steps=args.steps)
    log(f"workload {w.name}: {w.n_systems} systems, {w.n_atoms} atoms")
    if args.profile_copper:
        print(json.dumps(profile_copper(api, torch)), flush=True)
        return
    if args.profile_kernels:
        print(json.dumps(profile_kernels(api, torch, w, args.lanes or 4, args.bin_factor, group=args.group)), flush=True)
        return
    r = batched_nve(api, torch, w, args.steps, args.warmup, args.chunk, args.bin_factor, args.lanes, args.group)
    ms_per_step = r["ms"] / args.steps
    value = w.n_atoms * args.steps / (r["ms"] * 1e-3)
    log(f"batched NVE: {ms_per_step * 1e3:.2f} us/step, {value:.4g} atom-steps/s, rebuilds {r['rebuilds']}")
    roof = force_kernel_roofline(api, torch, r)
    log(f"force kernel: {roof['avg_launch_us']} us/launch, {roof['achieved']} GB/s algorithmic")
    # the whole step: per atom the fused step kernel reads the position, the row length, the row,
    # the velocity, the list's reference position and the mass and writes the velocity and the new
    # position; per system the offsets and the cell (rebuilds excluded: they are amortised)
    entries = int(r["nl"].n_nbr.sum().item())
    step_alg = w.n_atoms * (24 + 4 + 48 + 24 + 24 + 8) + 4 * entries + w.n_systems * (16 + 72)
    step_roof = dict(bound="hbm", alg_bytes_per_step=step_alg, achieved=round(step_alg / (ms_per_step * 1e-3) / 1e9, 1),
                     peak=HBM_PEAK_GBS, unit="GB/s",
                     frac=round(step_alg / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": r["warmup_steps"],
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair / f64 integration",
        "data": "synthetic",
        "config": {"workload": "argon_lj_nve_64x864", "n_systems": w.n_systems, "atoms_per_system": 864,
                   "n_atoms": w.n_atoms, "dt_fs": w.dt, "skin_A": w.skin, "cutoff_A": w.potential.cutoff,
                   "pair_prec": w.pair_prec, "graph_chunk_steps": args.chunk, "bin_factor": args.bin_factor,
                   "lanes_per_atom": r["lanes"], "group_atoms": r["group"],
                   "list_capacity": r["capacity"], "max_list_len": r["max_nbr"], "system_rebuilds": r["rebuilds"],
                   "wall_s": round(r["wall_s"], 4)},
        "roofline": roof,
        "roofline_alu": alu_roofline("k_step_argon_64x864_counters.txt", "void " + roof["kernel"],
                                     roof["avg_launch_us"]),
        "roofline_whole_step": step_roof,
    }
    if not args.no_plain:
        p = plain_path(api, torch, w, args.plain_steps, args.bin_factor)
        p["speedup_batched_vs_plain"] = round(value / p["value"], 2)
        out["plain_path"] = p
        log(f"plain path: {p['value']:.4g} atom-steps/s")
    if not args.no_langevin:
        out["langevin"] = langevin_throughput(api, torch, w, args.steps, args.chunk, args.bin_factor)
        log(f"langevin: {out['langevin']}")
    if not args.no_graph:
        out["graph_export"] = graph_export(api, torch, w, args.bin_factor)
        log(f"graph export: {out['graph_export']}")
    if not args.no_adjoint:
        a = adjoint_throughput(api, torch, 16, args.adjoint_steps, 50, plain=not args.no_plain)
        out["adjoint"] = a
        log(f"adjoint: {a['value']:.4g} atom-steps/s")
    if not args.no_fire:
        out["roofline_copper_forces"] = copper_force_roofline(api, torch)
        log(f"copper forces: {out['roofline_copper_forces']}")
        out["fire_copper"] = fire_copper(api, torch)
        log(f"copper FIRE: {out['fire_copper']}")
        out["soft_sphere"] = soft_sphere(api, torch)
        log(f"soft sphere: {out['soft_sphere']}")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w)
        log(f"cpu oracle: {out['cpu_baseline']['value']} atom-steps/s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
