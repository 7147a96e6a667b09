"""Langevin (NVT) dynamics for the batch (oracle; test infrastructure only).

The paper benchmarks batched Langevin MD (Section 4, speed benchmark) without naming a scheme.
Reading: the BAOAB splitting of Leimkuhler and Matthews (2013), one force evaluation per step,

    B: v += (dt/2) a F(r) / m
    A: r += (dt/2) v
    O: v  = c1 v + sqrt((1 - c1^2) a kT_s / m) xi,     c1 = exp(-gamma dt)
    A: r += (dt/2) v
    B: v += (dt/2) a F(r) / m          (with the force of the new positions)

with ``a`` the force/mass -> acceleration factor of the velocity-Verlet oracle (so that
(1/2) m v^2 / a is an energy and a kT_s / m the velocity variance of system s), and xi
standard normal numbers.  With gamma = 0 the O step is the identity and the scheme is
velocity Verlet.

The normals come from a counter-based generator, Philox4x32-10 (Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC 2011), keyed by the run's 64-bit seed with the
counter (atom index, step low word, step high word, 0); its four 32-bit outputs become the
uniforms u_k = (x_k + 1/2) 2^-32 and, by the Box-Muller transform, the normals
(sqrt(-2 ln u0) cos 2 pi u1, sqrt(-2 ln u0) sin 2 pi u1, sqrt(-2 ln u2) cos 2 pi u3) of the
atom's x, y, z components.  Pins: the generator's published known-answer vectors, the moments of
the normals, gamma = 0 against the velocity-Verlet oracle, and the exact variance of the O step.
"""
from __future__ import annotations

import numpy as np

from . import forces as _forces

# Philox4x32 round multipliers and key increments (the generator's published constants)
_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """Ten Philox rounds on counters ctr = (c0, c1, c2, c3) (uint32 arrays) with key (k0, k1)."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) & _MASK for x in ctr)
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    for _ in range(10):
        p0 = c0 * _M0  # < 2^64: the 32 x 32-bit product
        p1 = c2 * _M1
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ np.uint64(k0), lo1, hi0 ^ c3 ^ np.uint64(k1), lo0
        k0 = (k0 + _W0) & 0xFFFFFFFF
        k1 = (k1 + _W1) & 0xFFFFFFFF
    return tuple(x.astype(np.uint32) for x in (c0, c1, c2, c3))


def normals(seed: int, step: int, n: int) -> np.ndarray:
    """(n, 3) standard normals of atoms 0..n-1 at `step` for the 64-bit `seed`."""
    i = np.arange(n, dtype=np.uint64)
    ctr = (i, np.full(n, step & 0xFFFFFFFF), np.full(n, (step >> 32) & 0xFFFFFFFF), np.zeros(n))
    x = philox4x32_10(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))
    u = [(xk.astype(np.float64) + 0.5) * 2.0 ** -32 for xk in x]
    r0 = np.sqrt(-2.0 * np.log(u[0]))
    r2 = np.sqrt(-2.0 * np.log(u[2]))
    return np.stack([r0 * np.cos(2.0 * np.pi * u[1]), r0 * np.sin(2.0 * np.pi * u[1]),
                     r2 * np.cos(2.0 * np.pi * u[3])], axis=1)


def baoab(pos, vel, mass, cell, sys_offsets, species, potential, dt, n_steps, accel, gamma, kT, seed, step0=0,
          forces0=None):
    """n_steps of BAOAB Langevin dynamics; kT is per system.  Step k (k = 0..n_steps-1) draws the
    normals of counter step0 + k.  Returns dict(pos, vel, forces)."""
    pos = np.array(pos, dtype=np.float64, copy=True)
    vel = np.array(vel, dtype=np.float64, copy=True)
    n = pos.shape[0]
    sys_of = np.repeat(np.arange(len(sys_offsets) - 1), np.diff(sys_offsets))
    inv_m = (accel / mass)[:, None]
    sd = np.sqrt(accel * np.asarray(kT, dtype=np.float64)[sys_of] / mass)[:, None]  # sqrt(a kT / m)
    c1 = float(np.exp(-gamma * dt))
    c2 = float(np.sqrt(1.0 - c1 * c1))
    F = (_forces.batch_efw(pos, cell, sys_offsets, species, potential)[1] if forces0 is None
         else np.array(forces0, dtype=np.float64))
    for k in range(n_steps):
        vel = vel + 0.5 * dt * F * inv_m
        pos = pos + 0.5 * dt * vel
        vel = c1 * vel + c2 * sd * normals(seed, step0 + k, n)
        pos = pos + 0.5 * dt * vel
        F = _forces.batch_efw(pos, cell, sys_offsets, species, potential)[1]
        vel = vel + 0.5 * dt * F * inv_m
    return dict(pos=pos, vel=vel, forces=F)
