"""FIRE structural relaxation of positions, or of positions and cell (oracle; test infrastructure only).

The paper lists structural relaxation optimizers among the batched primitives (Abstract) and
relaxation as its variable-length workload (Section 3) but names no algorithm.  This is FIRE
(Bitzek, Koskinen, Gaehler, Moseler, Gumbsch, Phys. Rev. Lett. 97, 170201 (2006)) with the
semi-implicit Euler update, applied independently per system.  Per iteration of a system:

  1. forces at the current configuration; converged systems are frozen (no update, no count);
  2. from the second iteration on, P = g . v over all the system's degrees of freedom:
       P > 0:  v <- (1 - alpha) v + alpha |v| g / |g|;  n_pos += 1;
               if n_pos > N_min: dt <- min(f_inc dt, dt_max), alpha <- f_alpha alpha
       P <= 0: v <- 0, dt <- f_dec dt, alpha <- alpha_start, n_pos <- 0
  3. v <- v + dt g / m;   x <- x + dt v.

Variable cell (deformation-gradient degrees of freedom): positions r_i = q_i D and cell
h = h0 D with D_0 = I.  The atom coordinates are q_i with generalized force g_i = F_i D^T; the cell
coordinate is Y = N_s D with generalized force G = D^-T W / N_s (from dE/dD = -D^-T W, W the
virial, stress = -W/V) and unit mass; external pressure is zero.  A system has converged when
max_i |F_i| < fmax (and max_ab |G_ab| < fmax with the cell).  Time is in units where
acceleration = F / m (Angstrom sqrt(amu/eV) for eV/Angstrom/amu).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import forces as _forces


@dataclasses.dataclass
class FireConfig:
    dt_start: float = 0.1
    dt_max: float = 1.0
    alpha_start: float = 0.1
    f_inc: float = 1.1
    f_dec: float = 0.5
    f_alpha: float = 0.99
    n_min: int = 5
    fmax: float = 0.01
    relax_cell: bool = False
    cell_mass: float = 1.0
    max_iter: int = 100000


@dataclasses.dataclass
class FireSystemState:
    pos: np.ndarray
    cell: np.ndarray
    vel: np.ndarray
    dt: float
    alpha: float
    n_pos: int = 0
    n_iter: int = 0
    converged: bool = False
    deform: np.ndarray = None  # D
    deform_vel: np.ndarray = None  # velocity of Y = N_s D
    ref_cell: np.ndarray = None  # h0


def init_state(pos, cell, cfg: FireConfig) -> FireSystemState:
    return FireSystemState(pos=np.array(pos, dtype=np.float64), cell=np.array(cell, dtype=np.float64),
                           vel=np.zeros_like(pos, dtype=np.float64), dt=cfg.dt_start, alpha=cfg.alpha_start,
                           deform=np.eye(3), deform_vel=np.zeros((3, 3)), ref_cell=np.array(cell, dtype=np.float64))


def cell_force(deform, virial, n_atoms):
    """G = D^-T W / N_s."""
    return np.linalg.inv(deform).T @ virial / n_atoms


def fire_iterate(st: FireSystemState, species, mass, potential, cfg: FireConfig, n_iter: int, log=None):
    """Advance one system by at most ``n_iter`` FIRE iterations (stops early once converged or at
    ``cfg.max_iter``).  Returns the energy, forces and virial at the final configuration."""
    n = st.pos.shape[0]
    done = 0
    while True:
        e, F, W = _forces.system_efw(st.pos, st.cell, species, potential.params, potential.kind,
                                     potential.cutoff, potential.shift_energy)
        fnorm = float(np.sqrt((F * F).sum(axis=1)).max()) if n else 0.0
        conv = fnorm < cfg.fmax
        G = None
        if cfg.relax_cell:
            G = cell_force(st.deform, W, n)
            conv = conv and float(np.abs(G).max()) < cfg.fmax
        if conv:
            st.converged = True
            return e, F, W
        if done >= n_iter or st.n_iter >= cfg.max_iter:
            return e, F, W
        g = F @ st.deform.T if cfg.relax_cell else F
        branch = 0
        if st.n_iter > 0:
            P = float((g * st.vel).sum())
            if cfg.relax_cell:
                P += float((G * st.deform_vel).sum())
            if P > 0.0:
                branch = 1
                vv = float((st.vel * st.vel).sum())
                gg = float((g * g).sum())
                if cfg.relax_cell:
                    vv += float((st.deform_vel * st.deform_vel).sum())
                    gg += float((G * G).sum())
                if gg > 0.0:
                    scale = st.alpha * np.sqrt(vv) / np.sqrt(gg)
                    st.vel = (1.0 - st.alpha) * st.vel + scale * g
                    if cfg.relax_cell:
                        st.deform_vel = (1.0 - st.alpha) * st.deform_vel + scale * G
                st.n_pos += 1
                if st.n_pos > cfg.n_min:
                    st.dt = min(st.dt * cfg.f_inc, cfg.dt_max)
                    st.alpha = st.alpha * cfg.f_alpha
            else:
                branch = -1
                st.vel = np.zeros_like(st.vel)
                st.deform_vel = np.zeros((3, 3))
                st.dt = st.dt * cfg.f_dec
                st.alpha = cfg.alpha_start
                st.n_pos = 0
        st.vel = st.vel + st.dt * g / mass[:, None]
        if cfg.relax_cell:
            st.deform_vel = st.deform_vel + st.dt * G / cfg.cell_mass
            q = st.pos @ np.linalg.inv(st.deform) + st.dt * st.vel
            st.deform = st.deform + (st.dt / n) * st.deform_vel
            st.pos = q @ st.deform
            st.cell = st.ref_cell @ st.deform
        else:
            st.pos = st.pos + st.dt * st.vel
        if log is not None:
            log.append(dict(iter=st.n_iter, branch=branch, dt=st.dt, alpha=st.alpha, fmax=fnorm))
        st.n_iter += 1
        done += 1


def relax_batch(pos, cell, sys_offsets, species, mass, potential, cfg: FireConfig, n_iter=None):
    """FIRE on every system of a batch independently.  Returns per-system states."""
    states = []
    for s in range(cell.shape[0]):
        a, b = int(sys_offsets[s]), int(sys_offsets[s + 1])
        st = init_state(pos[a:b], cell[s], cfg)
        fire_iterate(st, species[a:b], mass[a:b], potential, cfg, cfg.max_iter if n_iter is None else n_iter)
        states.append(st)
    return states
