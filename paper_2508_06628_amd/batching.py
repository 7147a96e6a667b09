"""AutoBatching on the device (paper Section 3): the host decisions of ``autobatch`` driving the C
ABI entry points.

* ``InFlightFire``: a stream of systems relaxed by FIRE through a batch whose total memory scaler
  stays within a capacity.  Every ``check_every`` iterations the host reads the per-system
  convergence flags; converged systems (and systems that reached max_iter) leave the batch with
  their relaxed state and waiting systems join in stream order while they fit.  Systems that
  continue keep their complete FIRE state (positions, velocities, cell, time step, mixing
  coefficient, positive-power count, iteration count, deformation and its velocity).
* ``nve_binned``: a fixed-length NVE run of many systems, packed first-fit decreasing into bins of
  at most the capacity, one batch (and one graph-replayed step loop) per bin.

The capacity comes from ``autobatch.estimate_max_scaler`` probing a ``DeviceMemoryModel`` (the exact
byte count of a batch for the classical potentials) with copies of the largest and the smallest
system, as the paper probes the model's memory.  Nothing here computes physics: every step runs
in the library's kernels.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import api
from .autobatch import DeviceMemoryModel, InFlightBatcher, bin_pack, default_probes, estimate_max_scaler, memory_scaler


def system_scalers(w, scales_with: str = "n_atoms") -> List[float]:
    counts = np.diff(w.sys_offsets)
    vols = np.abs(np.linalg.det(w.cell))
    return [memory_scaler(int(n), float(v), scales_with) for n, v in zip(counts, vols)]


def probe_capacity(w, model: DeviceMemoryModel, scalers: Sequence[float]) -> float:
    """Largest total scaler that fits the model's budget, by probing copies of the largest and the
    smallest system (capacity = min over probes of copies x scaler)."""
    counts = np.diff(w.sys_offsets)

    def fits(s, copies):
        return model.fits(int(counts[s]) * copies, copies)

    return estimate_max_scaler(fits, default_probes(scalers), scalers)


@dataclasses.dataclass
class RelaxedSystem:
    pos: np.ndarray
    cell: np.ndarray
    deform: np.ndarray  # deformation gradient D of the cell relaxation (cell = ref_cell D)
    n_iter: int
    converged: bool
    finished_at: int  # batch iteration count at which it left the batch


class InFlightFire:
    """In-flight FIRE relaxation of ``w``'s systems under ``capacity`` (memory-scaler units)."""

    def __init__(self, w, fire_kw: Dict, capacity: float, check_every: int = 64, skin: float = 0.3,
                 prec: Optional[str] = None, bin_factor: int = 2, lanes: int = 0, scales_with: str = "n_atoms",
                 device: str = "cuda"):
        if not 1 <= check_every <= 256:
            raise ValueError("check_every must be in [1, 256] (one persistent launch and its tail per check)")
        self.w, self.check_every, self.skin, self.bin_factor, self.lanes = w, check_every, skin, bin_factor, lanes
        self.prec = prec or w.pair_prec
        self.fire_kw = dict(fire_kw)
        self.cfg = api.fire_config(**self.fire_kw)
        self.pp = api.pair_params_from_spec(w.potential, self.prec)
        self.scalers = system_scalers(w, scales_with)
        self.capacity = float(capacity)
        self.batcher = InFlightBatcher(self.scalers, self.capacity)
        self.device = device
        self.results: Dict[int, RelaxedSystem] = {}
        self.schedule = []  # (batch iteration, systems in the batch)
        # per-system state of the systems on the device, for carrying over to the next batch
        self._carried: Dict[int, Dict[str, np.ndarray]] = {}

    # ---- device batch construction -------------------------------------------------------------
    def _build(self, systems: List[int]):
        w = self.w
        pos, vel, cell = [], [], []
        for s in systems:
            sl = w.system(s)
            c = self._carried.get(s)
            pos.append(c["pos"] if c else w.pos[sl])
            vel.append(c["vel"] if c else np.zeros_like(w.pos[sl]))
            cell.append(c["cell"] if c else w.cell[s])
        sub = w.subset(systems)
        b = api.Batch(np.concatenate(pos), np.concatenate(vel), sub.mass, sub.species, sub.sys_offsets, np.stack(cell),
                      self.device)
        vel_dev = b.vel.clone()
        fs = api.FireState(b, self.cfg)  # zeroes b.vel: restored below for continuing systems
        b.vel.copy_(vel_dev)
        for k, s in enumerate(systems):
            c = self._carried.get(s)
            if not c:
                continue
            fs.dt[k], fs.alpha[k] = float(c["dt"]), float(c["alpha"])
            fs.n_pos[k], fs.n_iter[k] = int(c["n_pos"]), int(c["n_iter"])
            fs.deform[k] = torch.tensor(c["deform"], dtype=torch.float64)
            fs.deform_vel[k] = torch.tensor(c["deform_vel"], dtype=torch.float64)
            fs.ref_cell[k] = torch.tensor(c["ref_cell"], dtype=torch.float64)
        nl = api.build_neighbor_list(b, w.potential.cutoff, self.skin, bin_factor=self.bin_factor, margin=1.3)
        if self.lanes:
            nl.lanes_per_atom = self.lanes
        F = api.force_buffer(b, self.prec)
        return b, fs, nl, F

    def _save(self, systems, b, fs):
        pos, vel, cell = b.positions(), b.velocities(), b.cells()
        dt, alpha, npos, nit = (fs.dt.cpu().numpy(), fs.alpha.cpu().numpy(), fs.n_pos.cpu().numpy(),
                                fs.n_iter.cpu().numpy())
        deform, dvel, rc = fs.deform.cpu().numpy(), fs.deform_vel.cpu().numpy(), fs.ref_cell.cpu().numpy()
        offs = b.h_offsets
        for k, s in enumerate(systems):
            sl = slice(int(offs[k]), int(offs[k + 1]))
            self._carried[s] = dict(pos=pos[sl], vel=vel[sl], cell=cell[k], dt=dt[k], alpha=alpha[k], n_pos=npos[k],
                                    n_iter=nit[k], deform=deform[k], deform_vel=dvel[k], ref_cell=rc[k])

    # ---- the loop --------------------------------------------------------------------------------
    def run(self, max_checks: int = 100000):
        systems = self.batcher.batch()
        step = 0
        self.schedule.append((step, tuple(systems)))
        b, fs, nl, F = self._build(systems)
        for _ in range(max_checks):
            api.ts_fire_step(b, fs, self.cfg, nl, self.pp, self.check_every, F, persistent=True)
            step += self.check_every
            st = nl.read_status()
            if st[1] or st[3] or st[4]:
                raise RuntimeError(f"neighbor list status during in-flight FIRE: {st.tolist()}")
            conv = fs.converged.cpu().numpy().astype(bool)
            nit = fs.n_iter.cpu().numpy()
            finished = conv | (nit >= int(self.cfg.max_iter))
            if finished.any():
                self._save(systems, b, fs)
                for k, s in enumerate(systems):
                    if finished[k]:
                        c = self._carried.pop(s)
                        self.results[s] = RelaxedSystem(c["pos"], c["cell"], c["deform"].reshape(3, 3), int(c["n_iter"]),
                                                        bool(conv[k]), step)
            new = self.batcher.update(list(finished))
            if self.batcher.done:
                self.schedule.append((step, ()))
                return self.results
            self.schedule.append((step, tuple(new)))
            if new != systems:  # only after departures (whose state was saved above)
                systems = new
                b, fs, nl, F = self._build(systems)
        raise RuntimeError("in-flight FIRE did not finish within max_checks")


def nve_binned(w, n_steps: int, capacity: float, prec: Optional[str] = None, lanes: int = 4, bin_factor: int = 2,
               chunk: int = 100, scales_with: str = "n_atoms", device: str = "cuda"):
    """Velocity-Verlet NVE of every system of ``w`` for ``n_steps`` steps, systems packed first-fit
    decreasing into bins of at most ``capacity``; one batch per bin, run one after another.
    Returns (positions, velocities) in the workload's atom order and the bins."""
    prec = prec or w.pair_prec
    scalers = system_scalers(w, scales_with)
    bins = bin_pack(scalers, capacity)
    pos, vel = np.empty_like(w.pos), np.empty_like(w.vel)
    pp = api.pair_params_from_spec(w.potential, prec)
    for systems in bins:
        sub = w.subset(systems)
        b = api.Batch.from_workload(sub, device)
        nl = api.build_neighbor_list(b, sub.potential.cutoff, sub.skin, bin_factor=bin_factor, margin=1.3)
        nl.lanes_per_atom = lanes
        F = api.force_buffer(b, prec)
        api.ts_pair_forces(b, nl, pp, F)
        done = 0
        while done < n_steps:
            k = min(chunk, n_steps - done)
            api.ts_nve_step(b, nl, pp, sub.dt, sub.accel, k, F, use_graph=True)
            done += k
        st = nl.read_status()
        if st[1] or st[3] or st[4]:
            raise RuntimeError(f"neighbor list status in binned NVE: {st.tolist()}")
        p, v = b.positions(), b.velocities()
        for k, s in enumerate(systems):
            sl = w.system(s)
            pos[sl] = p[int(b.h_offsets[k]):int(b.h_offsets[k + 1])]
            vel[sl] = v[int(b.h_offsets[k]):int(b.h_offsets[k + 1])]
    return pos, vel, bins
