"""Launch-shape autotuner for the batched NVE step loop and the FIRE relaxation.

The fused step kernel spreads each atom's neighbor row over ``lanes_per_atom`` lanes of a
wavefront (1, 2, 4 or 8), and a workgroup owns ``group_atoms`` atoms of one system (one or more
rounds of 256 / lanes_per_atom atoms; the system's positions are staged in LDS once per
workgroup).  The best pair depends on the row length and on how many atoms the batch has (few
atoms need more lanes per atom to fill 256 CUs; more rounds stage less).  ``tune_nve`` times a
short graph replay of the real workload for every candidate on a scratch copy of the state and
returns the fastest; results are cached on disk per (device architecture, potential, precision, size bucket)
so later runs skip the sweep.  Only timing is done here: every candidate runs the same kernels
through the C ABI and computes the same trajectory up to float64 summation order.

``tune_bin_factor`` picks the cell-list bin factor b (bins of width at least r_list / b, a stencil
of (2b + 1)^3 bins) for batches with systems above the LDS limit, the only ones the cell list
builds: it times forced rebuilds of every row; the rows themselves do not depend on b.

``tune_fire`` picks how ``ts_fire_step`` runs a relaxation: one persistent launch per call (each
system on one workgroup, converged systems freeing theirs) or the per-iteration kernels (every
open system spread over many workgroups), and the lanes per atom of the force kernel.  Batches
of many small systems favour the first, batches with large systems the second.
"""
from __future__ import annotations

import json
import math
import os
from typing import Optional

import torch

from . import api

LANE_CHOICES = (1, 2, 4, 8)
ROUND_CHOICES = (1, 2)  # atom groups per workgroup (group_atoms = rounds * 256 / lanes_per_atom)


def cache_path() -> str:
    root = os.environ.get("TS_AUTOTUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "ts_mi355x")
    return os.path.join(root, "autotune.json")


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d: dict) -> None:
    p = cache_path()
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
        tmp = p + ".tmp"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, p)
    except OSError:
        pass  # a read-only home only disables caching


def size_bucket(batch: api.Batch, nl: api.NeighborList) -> str:
    """Bucket of (atoms per batch, largest system, mean row length) on a log2 scale."""
    n = max(batch.n_atoms, 1)
    mean_row = float(nl.n_nbr.float().mean().item()) if batch.n_atoms else 0.0
    return f"n{int(math.log2(n))}_m{int(math.log2(max(batch.max_system_atoms, 1)))}_r{int(math.log2(mean_row + 1))}"


def key(batch, nl, pp) -> str:
    arch = torch.cuda.get_device_properties(batch.device).gcnArchName.split(":")[0]
    return f"{arch}/kind{pp.kind}/prec{pp.prec}/{size_bucket(batch, nl)}"


def tune_nve(batch: api.Batch, nl: api.NeighborList, pp, dt: float, accel: float, steps: int = 100,
             reps: int = 5, use_cache: bool = True, choices=LANE_CHOICES, rounds=ROUND_CHOICES) -> dict:
    """Pick lanes_per_atom and group_atoms for ``ts_nve_step`` on this workload.  Every candidate
    runs on its own scratch copy; after a warm-up replay each, the candidates are timed in ``reps``
    interleaved rounds (so that a clock ramp at the start of a process affects them alike) and each
    keeps its fastest replay of ``steps`` steps.  Returns {"lanes_per_atom": L, "group_atoms": G,
    "us_per_step": {"L/G": t, ...}, "cached": bool} and sets both on ``nl``."""
    k = key(batch, nl, pp)
    cache = _load() if use_cache else {}
    if k in cache and "group_atoms" in cache[k]:
        nl.lanes_per_atom = int(cache[k]["lanes_per_atom"])
        nl.group_atoms = int(cache[k]["group_atoms"])
        return dict(cache[k], cached=True)
    prec = "f32" if pp.prec == 0 else "f64"
    cands = [(lanes, r * 256 // lanes) for lanes in choices for r in rounds if not (lanes == 1 and r > 1)]
    trials = []
    for lanes, group in cands:
        b = batch.clone()
        trial = api.NeighborList(b, nl.cutoff, nl.skin, nl.max_nbr, nl.bin_factor, nl.half, lanes, group,
                                 nl.deferred)
        api.ts_neighbor_build(b, trial, force=True)
        F = api.force_buffer(b, prec)
        api.ts_pair_forces(b, trial, pp, F)
        api.ts_nve_step(b, trial, pp, dt, accel, steps, F, use_graph=True)  # instantiate and warm up
        trials.append(((lanes, group), b, trial, F))
    torch.cuda.synchronize()
    timings = {c: math.inf for c, _, _, _ in trials}
    for _ in range(reps):
        for c, b, trial, F in trials:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            api.ts_nve_step(b, trial, pp, dt, accel, steps, F, use_graph=True)
            e1.record()
            torch.cuda.synchronize()
            timings[c] = min(timings[c], e0.elapsed_time(e1) * 1e3 / steps)
    del trials
    api.ts_release_graphs()
    timings = {c: round(t, 3) for c, t in timings.items()}
    lanes, group = min(timings, key=timings.get)
    entry = {"lanes_per_atom": int(lanes), "group_atoms": int(group),
             "us_per_step": {f"{l2}/{g2}": v for (l2, g2), v in timings.items()}}
    if use_cache:
        cache[k] = entry
        _store(cache)
    nl.lanes_per_atom = int(lanes)
    nl.group_atoms = int(group)
    return dict(entry, cached=False)


def tuned_lanes(batch, nl, pp) -> Optional[int]:
    e = _load().get(key(batch, nl, pp))
    return None if e is None else int(e["lanes_per_atom"])


FIRE_LANE_CHOICES = (2, 4)


def tune_fire(batch: api.Batch, nl: api.NeighborList, pp, cfg, iters: int = 32, reps: int = 2,
              use_cache: bool = True, choices=FIRE_LANE_CHOICES) -> dict:
    """Pick the FIRE path (persistent launch or per-iteration kernels) and lanes_per_atom for
    ``ts_fire_step`` on this workload.  Each candidate relaxes a scratch copy of the batch from a
    fresh FIRE state: two warm-up iterations, then ``reps`` rounds of ``iters`` iterations, the
    candidates interleaved within each round; a candidate's time is the sum of its rounds (the
    relaxation advances, so every candidate covers the same iterations).  Returns
    {"persistent": P, "lanes_per_atom": L, "ms": {"P/L": t, ...}, "cached": bool} and sets the lanes
    on ``nl``."""
    k = f"fire/{key(batch, nl, pp)}/cell{int(cfg.relax_cell)}"
    cache = _load() if use_cache else {}
    if k in cache:
        nl.lanes_per_atom = int(cache[k]["lanes_per_atom"])
        return dict(cache[k], cached=True)
    prec = "f32" if pp.prec == 0 else "f64"
    trials = []
    for persistent in (True, False):
        for lanes in choices:
            b = batch.clone()
            trial = api.NeighborList(b, nl.cutoff, nl.skin, nl.max_nbr, nl.bin_factor, nl.half, lanes, nl.group_atoms)
            api.ts_neighbor_build(b, trial, force=True)
            fs = api.FireState(b, cfg)
            F = api.force_buffer(b, prec)
            api.ts_fire_step(b, fs, cfg, trial, pp, 2, F, persistent=persistent)
            trials.append(((persistent, lanes), b, trial, fs, F))
    torch.cuda.synchronize()
    timings = {c: 0.0 for c, *_ in trials}
    for _ in range(reps):
        for c, b, trial, fs, F in trials:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            api.ts_fire_step(b, fs, cfg, trial, pp, iters, F, persistent=c[0])
            e1.record()
            torch.cuda.synchronize()
            timings[c] += e0.elapsed_time(e1)
    del trials
    timings = {c: round(t, 3) for c, t in timings.items()}
    persistent, lanes = min(timings, key=timings.get)
    entry = {"persistent": bool(persistent), "lanes_per_atom": int(lanes),
             "ms": {f"{int(p2)}/{l2}": v for (p2, l2), v in timings.items()}}
    if use_cache:
        cache[k] = entry
        _store(cache)
    nl.lanes_per_atom = int(lanes)
    return dict(entry, cached=False)


BIN_FACTOR_CHOICES = (1, 2, 3, 4)
LDS_MAX_ATOMS = 2048  # systems up to this size are rebuilt by the row kernel, without bins


def tune_bin_factor(batch: api.Batch, nl: api.NeighborList, reps: int = 3, use_cache: bool = True,
                    choices=BIN_FACTOR_CHOICES) -> dict:
    """Pick the cell-list bin factor for ``nl`` on this batch by timing ``reps`` forced rebuilds of a
    scratch list per candidate.  Batches without a system above 2048 atoms are not binned: the list's
    factor is kept and nothing is timed.  Returns {"bin_factor": b, "binned": bool, "ms": {...},
    "cached": bool} and sets the factor on ``nl``."""
    if batch.max_system_atoms <= LDS_MAX_ATOMS:
        return {"bin_factor": int(nl.bin_factor), "binned": False, "ms": {}, "cached": False}
    arch = torch.cuda.get_device_properties(batch.device).gcnArchName.split(":")[0]
    k = f"{arch}/bins/r{nl.cutoff + nl.skin:.4f}/half{int(nl.half)}/{size_bucket(batch, nl)}"
    cache = _load() if use_cache else {}
    if k in cache:
        nl.bin_factor = int(cache[k]["bin_factor"])
        return dict(cache[k], cached=True)
    timings = {}
    for bf in choices:
        trial = api.NeighborList(batch, nl.cutoff, nl.skin, nl.max_nbr, bf, nl.half, nl.lanes_per_atom,
                                 nl.group_atoms)
        api.ts_neighbor_build(batch, trial, force=True)  # warm-up
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            api.ts_neighbor_build(batch, trial, force=True)
        e1.record()
        torch.cuda.synchronize()
        timings[bf] = round(e0.elapsed_time(e1) / reps, 4)
        del trial
    bf = min(timings, key=timings.get)
    entry = {"bin_factor": int(bf), "binned": True, "ms": {str(b2): v for b2, v in timings.items()}}
    if use_cache:
        cache[k] = entry
        _store(cache)
    nl.bin_factor = int(bf)
    return dict(entry, cached=False)
