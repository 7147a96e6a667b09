"""Python binding of the C ABI: device buffers held in torch tensors, one function per entry
point with the entry point's name.  Every function only marshals arguments; all the work runs in
the HIP library.  Arrays are on the current HIP device; calls are asynchronous on the current
torch stream unless a stream is passed.
"""
from __future__ import annotations

import ctypes
import math
from typing import Optional

import numpy as np
import torch

from . import _native as N


def _p(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# ----------------------------------------------------------------------------- batch


class Batch:
    """Batched state on the device: SoA positions/velocities [3][N] (float64), masses [N],
    species [N] (int32), system offsets [S+1] (int64, plus a host copy), system index [N],
    cells [S][3][3] (rows are lattice vectors)."""

    def __init__(self, pos, vel, mass, species, sys_offsets, cell, device="cuda"):
        pos = np.asarray(pos, dtype=np.float64)
        self.h_offsets = np.ascontiguousarray(np.asarray(sys_offsets, dtype=np.int64))
        self.n_atoms = int(pos.shape[0])
        self.n_systems = int(self.h_offsets.shape[0] - 1)
        self.device = torch.device(device)
        f64 = dict(dtype=torch.float64, device=self.device)
        self.pos = torch.tensor(np.ascontiguousarray(pos.T), **f64)
        vel = np.zeros_like(pos) if vel is None else np.asarray(vel, dtype=np.float64)
        self.vel = torch.tensor(np.ascontiguousarray(vel.T), **f64)
        self.mass = None if mass is None else torch.tensor(np.asarray(mass, dtype=np.float64), **f64)
        self.species = None if species is None else torch.tensor(np.asarray(species, dtype=np.int32),
                                                                  dtype=torch.int32, device=self.device)
        self.sys_offsets = torch.tensor(self.h_offsets, dtype=torch.int64, device=self.device)
        counts = np.diff(self.h_offsets)
        self.system_idx = torch.tensor(np.repeat(np.arange(self.n_systems, dtype=np.int32), counts),
                                       dtype=torch.int32, device=self.device)
        self.cell = torch.tensor(np.asarray(cell, dtype=np.float64).reshape(self.n_systems, 3, 3), **f64)

    @classmethod
    def from_workload(cls, w, device="cuda"):
        return cls(w.pos, w.vel, w.mass, w.species, w.sys_offsets, w.cell, device)

    @property
    def max_system_atoms(self) -> int:
        return int(np.diff(self.h_offsets).max()) if self.n_systems else 0

    def struct(self) -> N.TsBatch:
        b = N.TsBatch()
        b.n_atoms = self.n_atoms
        b.n_systems = self.n_systems
        b.stride = self.pos.shape[1]
        b.sys_offsets = self.sys_offsets.data_ptr()
        b.h_sys_offsets = self.h_offsets.ctypes.data
        b.system_idx = self.system_idx.data_ptr()
        b.pos = self.pos.data_ptr()
        b.vel = self.vel.data_ptr()
        b.mass = None if self.mass is None else self.mass.data_ptr()
        b.species = None if self.species is None else self.species.data_ptr()
        b.cell = self.cell.data_ptr()
        return b

    def positions(self) -> np.ndarray:
        return self.pos.T.cpu().numpy().copy()

    def velocities(self) -> np.ndarray:
        return self.vel.T.cpu().numpy().copy()

    def cells(self) -> np.ndarray:
        return self.cell.cpu().numpy().copy()

    def clone(self) -> "Batch":
        c = object.__new__(Batch)
        c.__dict__.update(self.__dict__)
        c.pos, c.vel, c.cell = self.pos.clone(), self.vel.clone(), self.cell.clone()
        return c


def pair_params(kind: str, params, cutoff: float, shift_energy: bool = False, prec: str = "f32") -> N.TsPairParams:
    p = np.asarray(params, dtype=np.float64)
    ns = p.shape[0]
    if ns > N.TS_MAX_SPECIES:
        raise ValueError("at most 4 species")
    pp = N.TsPairParams()
    pp.kind = N.KIND_CODES[kind]
    pp.prec = N.PREC_CODES[prec]
    pp.n_species = ns
    pp.shift_energy = 1 if shift_energy else 0
    pp.cutoff = float(cutoff)
    full = np.zeros((N.TS_MAX_SPECIES, N.TS_MAX_SPECIES, 3))
    full[:ns, :ns] = p
    for k, v in enumerate(full.reshape(-1)):
        pp.params[k] = float(v)
    return pp


def lorentz_berthelot(eps, sigma) -> np.ndarray:
    """(S, S, 3) LJ table of a mixture from per-species epsilon and sigma by the Lorentz-Berthelot
    rules, as the library's ``ts_lorentz_berthelot`` computes it; pass it as ``params``."""
    e = np.ascontiguousarray(np.asarray(eps, dtype=np.float64).reshape(-1))
    s = np.ascontiguousarray(np.asarray(sigma, dtype=np.float64).reshape(-1))
    if e.shape != s.shape:
        raise ValueError("lorentz_berthelot: one epsilon and one sigma per species")
    pp = N.TsPairParams()
    rc = N.lib().ts_lorentz_berthelot(int(e.size), e.ctypes.data, s.ctypes.data, ctypes.byref(pp))
    if rc != N.TS_OK:
        raise ValueError("lorentz_berthelot: one non-negative epsilon and one positive sigma per species, "
                         f"at most {N.TS_MAX_SPECIES} species ({N.lib().ts_strerror(rc).decode()})")
    full = np.ctypeslib.as_array(pp.params).reshape(N.TS_MAX_SPECIES, N.TS_MAX_SPECIES, 3)
    return full[:e.size, :e.size].copy()


def pair_params_from_spec(spec, prec: str = "f32") -> N.TsPairParams:
    return pair_params(spec.kind, spec.params, spec.cutoff, spec.shift_energy, prec)


# ----------------------------------------------------------------------------- neighbor list


class NeighborList:
    """Padded neighbor list of a batch (rows of packed (j, S) entries, blocks of 8 per atom)."""

    def __init__(self, batch: Batch, cutoff: float, skin: float, max_nbr: int, bin_factor: int = 1, half: bool = False,
                 lanes_per_atom: int = 0, group_atoms: int = 0, deferred: bool = False):
        self.cutoff, self.skin, self.half, self.bin_factor = float(cutoff), float(skin), bool(half), int(bin_factor)
        # second row buffer for the deferred rebuild of the fused step loops (systems up to 2048
        # atoms, full lists); other batches would never use it
        self.deferred = bool(deferred) and not self.half and 0 < batch.max_system_atoms <= 2048
        self.lanes_per_atom = int(lanes_per_atom)
        self.group_atoms = int(group_atoms)
        self.n_atoms, self.n_systems = batch.n_atoms, batch.n_systems
        self._alloc(batch, int(max_nbr))

    def _alloc(self, batch, max_nbr):
        dev = batch.device
        stride = batch.pos.shape[1]
        self.max_nbr = max_nbr
        # entry k of atom i lives at [k // 8, i, k % 8]
        self.nbr = torch.zeros(((max_nbr + 7) // 8, stride, 8), dtype=torch.int32, device=dev)
        self.n_nbr = torch.zeros(batch.n_atoms, dtype=torch.int32, device=dev)
        self.ref_pos = torch.zeros((3, stride), dtype=torch.float64, device=dev)
        self.ref_cell = torch.zeros((batch.n_systems, 9), dtype=torch.float64, device=dev)
        self.status = torch.zeros(N.TS_STATUS_WORDS, dtype=torch.int64, device=dev)
        ws = int(N.lib().ts_neighbor_workspace_bytes(batch.n_atoms, batch.n_systems))
        self.workspace = torch.zeros(ws, dtype=torch.uint8, device=dev)
        if self.deferred:
            self.nbr_alt = torch.zeros_like(self.nbr)
            self.n_nbr_alt = torch.zeros_like(self.n_nbr)
            self.ref_pos_alt = torch.zeros_like(self.ref_pos)
        else:
            self.nbr_alt = self.n_nbr_alt = self.ref_pos_alt = None

    def struct(self) -> N.TsNeighborList:
        s = N.TsNeighborList()
        s.cutoff = self.cutoff
        s.skin = self.skin
        s.half = 1 if self.half else 0
        s.max_nbr = self.max_nbr
        s.bin_factor = self.bin_factor
        s.lanes_per_atom = self.lanes_per_atom
        s.group_atoms = self.group_atoms
        s.nbr = self.nbr.data_ptr()
        s.n_nbr = self.n_nbr.data_ptr()
        s.ref_pos = self.ref_pos.data_ptr()
        s.ref_cell = self.ref_cell.data_ptr()
        s.status = self.status.data_ptr()
        s.workspace = self.workspace.data_ptr()
        s.workspace_bytes = self.workspace.numel()
        if self.deferred:
            s.nbr_alt = self.nbr_alt.data_ptr()
            s.n_nbr_alt = self.n_nbr_alt.data_ptr()
            s.ref_pos_alt = self.ref_pos_alt.data_ptr()
        return s

    def read_status(self) -> np.ndarray:
        return self.status.cpu().numpy()

    def entries(self):
        """Host copy of the list: (i, j_local, S0, S1, S2) arrays over all stored entries."""
        nbr = self.nbr.cpu().numpy().astype(np.uint32)
        n = self.n_nbr.cpu().numpy()
        rows = []
        for k in range(self.max_nbr):
            sel = np.nonzero(n > k)[0]
            if sel.size == 0:
                break
            e = nbr[k // 8, sel, k % 8]
            rows.append((sel, (e >> 15).astype(np.int64), ((e >> 10) & 31).astype(np.int64) - 16,
                         ((e >> 5) & 31).astype(np.int64) - 16, (e & 31).astype(np.int64) - 16))
        if not rows:
            z = np.zeros(0, np.int64)
            return z, z, z, z, z
        return tuple(np.concatenate([r[c] for r in rows]) for c in range(5))


def estimate_max_nbr(batch: Batch, r_list: float, margin: float = 1.3) -> int:
    counts = np.diff(batch.h_offsets)
    vols = np.abs(np.linalg.det(batch.cell.cpu().numpy()))
    rho = float((counts / np.maximum(vols, 1e-300)).max())
    return int(math.ceil(margin * 4.0 / 3.0 * math.pi * r_list ** 3 * rho)) + 16


def build_neighbor_list(batch: Batch, cutoff: float, skin: float, bin_factor: int = 1, max_nbr: Optional[int] = None,
                        margin: float = 1.25, half: bool = False, lanes_per_atom: int = 0,
                        group_atoms: int = 0, deferred: bool = False) -> NeighborList:
    """Allocate and build a list, regrowing once if the first capacity guess was too small.
    ``deferred`` gives it the second row buffer of the deferred rebuild (fused step loops)."""
    guess = max_nbr or estimate_max_nbr(batch, cutoff + skin)
    nl = NeighborList(batch, cutoff, skin, guess, bin_factor, half, lanes_per_atom, group_atoms, deferred)
    ts_neighbor_build(batch, nl, force=True)
    st = nl.read_status()
    if st[N.TS_STATUS_NONFINITE] or st[N.TS_STATUS_SHIFT]:
        raise RuntimeError(f"neighbor build status {st.tolist()}")
    if st[N.TS_STATUS_OVERFLOW] or (max_nbr is None and st[N.TS_STATUS_MAX_NBR] * margin > guess):
        need = int(math.ceil(st[N.TS_STATUS_MAX_NBR] * margin)) + 8
        nl._alloc(batch, max(need, 1))
        ts_neighbor_build(batch, nl, force=True)
        st = nl.read_status()
        if st[N.TS_STATUS_OVERFLOW]:
            raise RuntimeError("neighbor list overflow after regrowth")
    return nl


# ----------------------------------------------------------------------------- FIRE state


def fire_config(dt_start=0.1, dt_max=1.0, alpha_start=0.1, f_inc=1.1, f_dec=0.5, f_alpha=0.99, fmax=0.01,
                cell_mass=1.0, n_min=5, relax_cell=False, max_iter=100000) -> N.TsFireConfig:
    c = N.TsFireConfig()
    c.dt_start, c.dt_max, c.alpha_start = dt_start, dt_max, alpha_start
    c.f_inc, c.f_dec, c.f_alpha, c.fmax, c.cell_mass = f_inc, f_dec, f_alpha, fmax, cell_mass
    c.n_min, c.relax_cell, c.max_iter = int(n_min), 1 if relax_cell else 0, int(max_iter)
    return c


class FireState:
    def __init__(self, batch: Batch, cfg: N.TsFireConfig):
        S, dev = batch.n_systems, batch.device
        f64 = dict(dtype=torch.float64, device=dev)
        self.dt = torch.full((S,), cfg.dt_start, **f64)
        self.alpha = torch.full((S,), cfg.alpha_start, **f64)
        self.n_pos = torch.zeros(S, dtype=torch.int32, device=dev)
        self.converged = torch.zeros(S, dtype=torch.int32, device=dev)
        self.n_iter = torch.zeros(S, dtype=torch.int64, device=dev)
        self.deform = torch.eye(3, **f64).reshape(1, 9).repeat(S, 1).contiguous()
        self.deform_vel = torch.zeros((S, 9), **f64)
        self.ref_cell = batch.cell.reshape(S, 9).clone()
        self.scratch = torch.zeros((S, 32), **f64)
        batch.vel.zero_()

    def struct(self) -> N.TsFireState:
        s = N.TsFireState()
        s.dt, s.alpha, s.n_pos = self.dt.data_ptr(), self.alpha.data_ptr(), self.n_pos.data_ptr()
        s.converged, s.n_iter = self.converged.data_ptr(), self.n_iter.data_ptr()
        s.deform, s.deform_vel = self.deform.data_ptr(), self.deform_vel.data_ptr()
        s.ref_cell, s.scratch = self.ref_cell.data_ptr(), self.scratch.data_ptr()
        return s


# ----------------------------------------------------------------------------- entry points


def ts_neighbor_build(batch: Batch, nl: NeighborList, force: bool = True, stream=None):
    return N.check("ts_neighbor_build", N.lib().ts_neighbor_build(ctypes.byref(batch.struct()),
                                                                  ctypes.byref(nl.struct()), 1 if force else 0,
                                                                  _stream(stream)))


def ts_graph_export(batch, nl, r_graph, row_ptr, edge_offsets, edge_index, edge_shift=None, edge_vec=None,
                    stream=None):
    """Edges of the list within r_graph; capacity = edge_index.shape[1]."""
    cap = 0 if edge_index is None else int(edge_index.shape[1])
    return N.check("ts_graph_export", N.lib().ts_graph_export(
        ctypes.byref(batch.struct()), ctypes.byref(nl.struct()), float(r_graph), _p(row_ptr), _p(edge_offsets),
        _p(edge_index), _p(edge_shift), _p(edge_vec), cap, _stream(stream)))


def mlip_graph(batch, nl, r_graph, with_vec=True):
    """Allocate and export the batch graph: dict(row_ptr, edge_offsets, edge_index [2, E], shift [E, 3],
    vec [E, 3]).  Capacity is the list's entry count, so every edge fits (one host synchronisation)."""
    dev = batch.pos.device
    cap = int(nl.n_nbr.sum().item()) if batch.n_atoms else 0
    row_ptr = torch.empty(batch.n_atoms + 1, dtype=torch.int64, device=dev)
    offs = torch.empty(batch.n_systems + 1, dtype=torch.int64, device=dev)
    ei = torch.empty((2, cap), dtype=torch.int64, device=dev)
    sh = torch.empty((cap, 3), dtype=torch.int32, device=dev)
    vec = torch.empty((cap, 3), dtype=torch.float64, device=dev) if with_vec else None
    ts_graph_export(batch, nl, r_graph, row_ptr, offs, ei, sh, vec)
    e = int(offs[-1].item())
    return dict(row_ptr=row_ptr, edge_offsets=offs, edge_index=ei[:, :e], shift=sh[:e],
                vec=None if vec is None else vec[:e])


def ts_pair_forces(batch, nl, pp, force, energy=None, virial=None, stream=None):
    return N.check("ts_pair_forces", N.lib().ts_pair_forces(ctypes.byref(batch.struct()), ctypes.byref(nl.struct()),
                                                            ctypes.byref(pp), _p(force), _p(energy), _p(virial),
                                                            _stream(stream)))


def ts_nve_step(batch, nl, pp, dt, accel, n_steps, force, epot=None, ekin=None, virial=None, use_graph=True,
                stream=None):
    return N.check("ts_nve_step", N.lib().ts_nve_step(ctypes.byref(batch.struct()), ctypes.byref(nl.struct()),
                                                      ctypes.byref(pp), float(dt), float(accel), int(n_steps),
                                                      _p(force), _p(epot), _p(ekin), _p(virial),
                                                      1 if use_graph else 0, _stream(stream)))


def ts_langevin_step(batch, nl, pp, dt, accel, gamma, kT, seed, rng_step, n_steps, force, use_graph=True,
                     stream=None):
    """BAOAB Langevin steps; kT: device float64 [S]; rng_step: device int64 [1] step counter (advanced)."""
    return N.check("ts_langevin_step", N.lib().ts_langevin_step(
        ctypes.byref(batch.struct()), ctypes.byref(nl.struct()), ctypes.byref(pp), float(dt), float(accel),
        float(gamma), _p(kT), int(seed) & 0xFFFFFFFFFFFFFFFF, _p(rng_step), int(n_steps), _p(force),
        1 if use_graph else 0, _stream(stream)))


def ts_nve_record(batch, nl, pp, dt, accel, n_steps, force, traj, use_graph=True, stream=None):
    return N.check("ts_nve_record", N.lib().ts_nve_record(ctypes.byref(batch.struct()), ctypes.byref(nl.struct()),
                                                          ctypes.byref(pp), float(dt), float(accel), int(n_steps),
                                                          _p(force), _p(traj), 1 if use_graph else 0,
                                                          _stream(stream)))


def ts_adjoint_segment(batch, nl, pp, traj, n_steps, dt, accel, top, bottom, adj_pos, adj_vel, adj_params=None,
                       use_graph=True, stream=None):
    return N.check("ts_adjoint_segment", N.lib().ts_adjoint_segment(
        ctypes.byref(batch.struct()), ctypes.byref(nl.struct()), ctypes.byref(pp), _p(traj), int(n_steps), float(dt),
        float(accel), 1 if top else 0, 1 if bottom else 0, _p(adj_pos), _p(adj_vel), _p(adj_params),
        1 if use_graph else 0, _stream(stream)))


def ts_fire_step(batch, fs: FireState, cfg, nl, pp, n_iter, force, energy=None, virial=None, persistent=False,
                 stream=None):
    return N.check("ts_fire_step", N.lib().ts_fire_step(ctypes.byref(batch.struct()), ctypes.byref(fs.struct()),
                                                        ctypes.byref(cfg), ctypes.byref(nl.struct()),
                                                        ctypes.byref(pp), int(n_iter), _p(force), _p(energy),
                                                        _p(virial), 1 if persistent else 0, _stream(stream)))


def regrow_neighbor_list(batch: Batch, nl: NeighborList, margin: float = 1.3):
    """Reallocate the rows for the largest row length the status words recorded (times ``margin``),
    clear the status words and rebuild every system."""
    need = int(nl.read_status()[N.TS_STATUS_MAX_NBR])
    nl._alloc(batch, max(int(math.ceil(need * margin)) + 8, nl.max_nbr + 8))
    ts_neighbor_build(batch, nl, force=True)


def nve_run(batch: Batch, nl: NeighborList, pp, dt, accel, n_steps, force, chunk=100, use_graph=True, margin=1.3,
            max_replays=4):
    """``n_steps`` of ``ts_nve_step`` in calls of ``chunk`` steps with recovery from list overflow:
    after each call the host reads the status words; if a row was truncated, the state from before
    the call is restored, the list is regrown (``regrow_neighbor_list``) and rebuilt, the forces are
    re-evaluated and the call is replayed.  Non-finite positions or dropped image shifts raise.
    Returns the number of replays."""
    replays = 0
    done = 0
    nl.status.zero_()
    while done < n_steps:
        k = min(chunk, n_steps - done)
        saved = (batch.pos.clone(), batch.vel.clone(), batch.cell.clone())
        ts_nve_step(batch, nl, pp, dt, accel, k, force, use_graph=use_graph)
        st = nl.read_status()
        if st[N.TS_STATUS_NONFINITE] or st[N.TS_STATUS_SHIFT]:
            raise RuntimeError(f"nve_run: neighbor list status {st.tolist()}")
        if st[N.TS_STATUS_OVERFLOW]:
            if replays >= max_replays:
                raise RuntimeError("nve_run: list overflow persists after regrowth")
            replays += 1
            batch.pos.copy_(saved[0])
            batch.vel.copy_(saved[1])
            batch.cell.copy_(saved[2])
            regrow_neighbor_list(batch, nl, margin)
            ts_pair_forces(batch, nl, pp, force)
            nl.status.zero_()
            continue
        done += k
    return replays


def fire_relax(batch, fs: FireState, cfg, nl, pp, force, energy=None, virial=None, persistent=True,
               max_calls=100000, stream=None):
    """Repeat ``ts_fire_step(n_iter=-1)`` until every system has converged or reached max_iter: each
    call only enqueues work (its persistent launch and a bounded tail), so the host reads the
    per-system flags between calls.  Returns the number of calls."""
    n_calls = 0
    while n_calls < max_calls:
        ts_fire_step(batch, fs, cfg, nl, pp, -1, force, energy, virial, persistent, stream)
        n_calls += 1
        open_ = (fs.converged == 0) & (fs.n_iter < int(cfg.max_iter))
        if not bool(open_.any().item()):
            break
    return n_calls


def ts_pair_adjoint(batch, nl, pp, dt_drift, w_kick, accel, adj_pos, adj_vel, adj_params=None, stream=None):
    return N.check("ts_pair_adjoint", N.lib().ts_pair_adjoint(ctypes.byref(batch.struct()), ctypes.byref(nl.struct()),
                                                              ctypes.byref(pp), float(dt_drift), float(w_kick),
                                                              float(accel), _p(adj_pos), _p(adj_vel),
                                                              _p(adj_params), _stream(stream)))


def ts_pair_adjoint_noalloc(batch, nl, pp, dt_drift, w_kick, accel, adj_pos, adj_vel, adj_params=None,
                            stream=None, without_workspace=False):
    """ts_pair_adjoint with the library's static partial-sum array (no allocation; at most 4096
    systems when adj_params is given).  without_workspace passes the list with a NULL workspace."""
    st = nl.struct()
    if without_workspace:
        st.workspace = None
        st.workspace_bytes = 0
    return N.check("ts_pair_adjoint_noalloc",
                   N.lib().ts_pair_adjoint_noalloc(ctypes.byref(batch.struct()), ctypes.byref(st), ctypes.byref(pp),
                                                   float(dt_drift), float(w_kick), float(accel), _p(adj_pos),
                                                   _p(adj_vel), _p(adj_params), _stream(stream)))


def ts_rdf_smeared(batch, nl, n_bins, r_end, sigma, r_max, g, stream=None):
    return N.check("ts_rdf_smeared", N.lib().ts_rdf_smeared(ctypes.byref(batch.struct()), ctypes.byref(nl.struct()),
                                                            int(n_bins), float(r_end), float(sigma), float(r_max),
                                                            _p(g), _stream(stream)))


def ts_rdf_loss(g, g_target, loss=None, dl_dg=None, stream=None):
    S, nb = g.shape
    return N.check("ts_rdf_loss", N.lib().ts_rdf_loss(_p(g), _p(g_target), int(S), int(nb), _p(loss), _p(dl_dg),
                                                      _stream(stream)))


def ts_rdf_vjp(batch, nl, n_bins, r_end, sigma, r_max, dl_dg, grad_pos, stream=None):
    return N.check("ts_rdf_vjp", N.lib().ts_rdf_vjp(ctypes.byref(batch.struct()), ctypes.byref(nl.struct()),
                                                    int(n_bins), float(r_end), float(sigma), float(r_max), _p(dl_dg),
                                                    _p(grad_pos), _stream(stream)))


def ts_kinetic_energy(batch, accel, ekin, stream=None):
    return N.check("ts_kinetic_energy", N.lib().ts_kinetic_energy(ctypes.byref(batch.struct()), float(accel),
                                                                  _p(ekin), _stream(stream)))


def ts_release_graphs():
    N.lib().ts_release_graphs()


# ----------------------------------------------------------------------------- conveniences


def force_buffer(batch: Batch, prec: str) -> torch.Tensor:
    dt = torch.float32 if prec == "f32" else torch.float64
    return torch.zeros((3, batch.pos.shape[1]), dtype=dt, device=batch.device)


def compute_forces(batch: Batch, nl: NeighborList, pp, prec: str):
    """Forces (3, N), energies (S,), virials (S, 9) at the batch's current positions."""
    F = force_buffer(batch, prec)
    E = torch.zeros(batch.n_systems, dtype=torch.float64, device=batch.device)
    W = torch.zeros((batch.n_systems, 9), dtype=torch.float64, device=batch.device)
    ts_pair_forces(batch, nl, pp, F, E, W)
    return F, E, W
