"""Energy, forces and virial of a batch by brute-force pair sums (oracle; test infrastructure only).

The model output schema in the paper is energy, forces and stress per system (Section 2).
With the full pair set N_full of ``pairs`` (list radius r_c), r = |d| and g = phi'(r)/r:

    E_s   = 1/2 sum_{(i,j,S) in N_full}  [phi(r) - shift]
    F_i   =     sum_{(j,S)}              g(r) d            (d = r_j - r_i + S @ cell)
    W_s   = 1/2 sum_{(i,j,S) in N_full}  -g(r) d (x) d     (virial; stress = -W / V)

Self-image pairs (i, i, S != 0) add to E and W but their force on i cancels between S and -S.
"""
from __future__ import annotations

import numpy as np

from . import pairs as _pairs
from . import potentials as _pot


def system_efw(pos, cell, species, params, kind, cutoff, shift, rows=None):
    """Energy (scalar), forces (N, 3) (only ``rows`` filled when given) and virial (3, 3) of one
    system.  With ``rows`` the energy and virial cover only pairs whose first atom is in rows."""
    n = pos.shape[0]
    p = _pairs.system_pairs(pos, cell, cutoff, rows=rows)
    sp = params[species[p["i"]], species[p["j"]]]
    m = _pot.in_range(kind, sp, p["r2"], cutoff)
    i, d, r2, sp = p["i"][m], p["d"][m], p["r2"][m], sp[m]
    r = np.sqrt(r2)
    phi, d1, _ = _pot.phi_and_derivs(kind, sp, r, cutoff)
    phi = phi - _pot.energy_shift(kind, sp, cutoff, shift)
    g = d1 / r
    f = g[:, None] * d
    forces = np.zeros((n, 3))
    np.add.at(forces, i, f)
    energy = 0.5 * phi.sum()
    virial = -0.5 * np.einsum("p,pa,pb->ab", g, d, d)
    return energy, forces, virial


def batch_efw(pos, cell, sys_offsets, species, potential):
    """Per-system energies (S,), forces (N, 3), virials (S, 3, 3) for a whole batch."""
    S = cell.shape[0]
    energy = np.zeros(S)
    forces = np.zeros_like(pos)
    virial = np.zeros((S, 3, 3))
    for s in range(S):
        a, b = int(sys_offsets[s]), int(sys_offsets[s + 1])
        e, f, w = system_efw(pos[a:b], cell[s], species[a:b], potential.params, potential.kind,
                             potential.cutoff, potential.shift_energy)
        energy[s], forces[a:b], virial[s] = e, f, w
    return energy, forces, virial


def pair_magnitude_sums(pos, cell, species, params, kind, cutoff, rows=None):
    """Per-atom A_i = sum_j |f_ij| and per-system sum |phi| and sum |r phi'|: the scales that the
    parity tolerances are relative to (a net force near zero is no scale for its own error)."""
    n = pos.shape[0]
    p = _pairs.system_pairs(pos, cell, cutoff, rows=rows)
    sp = params[species[p["i"]], species[p["j"]]]
    m = _pot.in_range(kind, sp, p["r2"], cutoff)
    i, r2, sp = p["i"][m], p["r2"][m], sp[m]
    r = np.sqrt(r2)
    phi, d1, _ = _pot.phi_and_derivs(kind, sp, r, cutoff)
    A = np.zeros(n)
    np.add.at(A, i, np.abs(d1))
    return A, 0.5 * np.abs(phi).sum(), 0.5 * np.abs(r * d1).sum()
