"""Velocity-Verlet NVE and neighbor-list rebuild test (oracle; test infrastructure only).

The paper names molecular-dynamics integrators among the batched primitives (Abstract,
Section 3) without stating one; NVE here is the standard kick-drift-kick velocity Verlet with
one force evaluation per step reusing F(r_n):

    v_{n+1/2} = v_n + (dt/2) a F(r_n) / m
    r_{n+1}   = r_n + dt v_{n+1/2}
    v_{n+1}   = v_{n+1/2} + (dt/2) a F(r_{n+1}) / m

``a`` converts force/mass to length/time^2 (eV/(A amu) -> A/fs^2 for the argon workloads, 1 in
reduced units).  Kinetic energy is KE_s = (k/2) sum m v^2 with k = 1/a in those units.
"""
from __future__ import annotations

import numpy as np

from . import constants as _c
from . import forces as _forces


def kinetic_energy(vel, mass, sys_offsets, kinetic_factor):
    S = sys_offsets.shape[0] - 1
    ke = np.zeros(S)
    for s in range(S):
        a, b = int(sys_offsets[s]), int(sys_offsets[s + 1])
        ke[s] = 0.5 * kinetic_factor * float((mass[a:b, None] * vel[a:b] ** 2).sum())
    return ke


def temperature(ke, sys_offsets, k_b=_c.K_B):
    n = np.diff(sys_offsets).astype(np.float64)
    return 2.0 * ke / ((3.0 * n - 3.0) * k_b)


def nve(pos, vel, mass, cell, sys_offsets, species, potential, dt, n_steps, accel, forces0=None,
        record_every=0):
    """Run n_steps of velocity Verlet on a batch.  Returns dict(pos, vel, forces, energy, virial,
    traj) where traj holds (pos, vel, energy) every ``record_every`` steps (and step 0)."""
    pos = np.array(pos, dtype=np.float64, copy=True)
    vel = np.array(vel, dtype=np.float64, copy=True)
    inv_m = (accel / mass)[:, None]
    if forces0 is None:
        energy, F, virial = _forces.batch_efw(pos, cell, sys_offsets, species, potential)
    else:
        F = np.array(forces0, dtype=np.float64)
        energy, virial = None, None
    traj = []
    if record_every:
        traj.append((pos.copy(), vel.copy(), energy.copy() if energy is not None else None))
    for n in range(n_steps):
        vel = vel + 0.5 * dt * F * inv_m
        pos = pos + dt * vel
        energy, F, virial = _forces.batch_efw(pos, cell, sys_offsets, species, potential)
        vel = vel + 0.5 * dt * F * inv_m
        if record_every and (n + 1) % record_every == 0:
            traj.append((pos.copy(), vel.copy(), energy.copy()))
    return dict(pos=pos, vel=vel, forces=F, energy=energy, virial=virial, traj=traj)


def rebuild_needed(pos, ref_pos, cell, ref_cell, skin, r_list):
    """Whether a list built at (ref_pos, ref_cell) with radius r_list = r_c + skin may miss a pair
    now within r_c.  With M = ref_cell^-1 cell (M = I exactly when the cell is bitwise unchanged)
    a pair vector is d = d_ref M + (delta_j - delta_i), delta_i = r_i - r_i^ref M, so every pair
    within r_c is still listed while 2 max_i |delta_i| + r_list ||M - I||_F <= skin."""
    if np.array_equal(cell, ref_cell):
        delta = pos - ref_pos
        strain = 0.0
    else:
        M = np.linalg.inv(ref_cell) @ cell
        delta = pos - ref_pos @ M
        strain = float(np.linalg.norm(M - np.eye(3)))
    dmax = float(np.sqrt((delta * delta).sum(axis=1)).max()) if pos.shape[0] else 0.0
    return 2.0 * dmax + r_list * strain > skin
