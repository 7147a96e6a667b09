"""Smeared-RDF loss and the reverse (adjoint) velocity-Verlet pass (oracle; test infrastructure only).

The paper motivates differentiable simulation with gradients of a radial distribution function
computed at the end of an MD trajectory with respect to model parameters (Section 2).  Readings:

RDF of system s on bins r_b = (b + 1/2) dr, b = 0..B-1, with Gaussian smearing of standard
deviation s_g, over the full periodic pair set (ordered pairs, all images) within r_max:

    g_s(r_b) = 1 / (4 pi r_b^2 rho_s N_s) sum_{(i,j,S), |d| < r_max} N(r_b - |d|; s_g),
    rho_s = N_s / V_s,  N(x; s) = exp(-x^2 / 2 s^2) / sqrt(2 pi s^2)

Loss L = 1/(S B) sum_s sum_b (g_s(r_b) - g*_s(r_b))^2.

Reverse of one velocity-Verlet step (forward: v' = v + h a F(r)/m, r_{n+1} = r + dt v',
v_{n+1} = v' + h a F(r_{n+1})/m with h = dt/2), with u(lambda) = a lambda / m and J = dF/dr
(symmetric):

    lr  <- lr + h J(r_{n+1}) u(lv);   tb += h (dF/dtheta)(r_{n+1})^T u(lv)
    lv  <- lv + dt lr
    lr  <- lr + h J(r_n) u(lv);       tb += h (dF/dtheta)(r_n)^T u(lv)

Per pair (i, j, S) with d = r_j - r_i + S cell, r = |d|, d^ = d / r and du = u_j - u_i:
    (J u)_i += phi'' (d^ . du) d^ + (phi'/r) (du - (d^ . du) d^)
    tb[s_i, s_j, k] += (dg/dtheta_k) (u_i . d)         (g = phi'/r; pair force on i is g d)
"""
from __future__ import annotations

import numpy as np

from . import pairs as _pairs
from . import potentials as _pot
from . import forces as _forces


def rdf_bins(n_bins: int, r_end: float):
    dr = r_end / n_bins
    return (np.arange(n_bins) + 0.5) * dr


def system_rdf(pos, cell, n_bins, r_end, sigma, r_max):
    rb = rdf_bins(n_bins, r_end)
    p = _pairs.system_pairs(pos, cell, r_max)
    r = np.sqrt(p["r2"])
    n = pos.shape[0]
    rho = n / abs(np.linalg.det(cell))
    gauss = np.exp(-((rb[None, :] - r[:, None]) ** 2) / (2.0 * sigma * sigma)) / np.sqrt(2.0 * np.pi * sigma * sigma)
    return gauss.sum(axis=0) / (4.0 * np.pi * rb * rb * rho * n)


def system_rdf_grad(pos, cell, n_bins, r_end, sigma, r_max, dL_dg):
    """d/dpos of sum_b dL_dg[b] g(r_b) for one system."""
    rb = rdf_bins(n_bins, r_end)
    p = _pairs.system_pairs(pos, cell, r_max)
    r = np.sqrt(p["r2"])
    n = pos.shape[0]
    rho = n / abs(np.linalg.det(cell))
    pref = dL_dg / (4.0 * np.pi * rb * rb * rho * n)
    x = rb[None, :] - r[:, None]
    gauss = np.exp(-x * x / (2.0 * sigma * sigma)) / np.sqrt(2.0 * np.pi * sigma * sigma)
    dgauss_dr = gauss * x / (sigma * sigma)  # d/dr of N(r_b - r)
    h = (dgauss_dr * pref[None, :]).sum(axis=1)  # dL/dr for each ordered pair
    dhat = p["d"] / r[:, None]
    grad = np.zeros((n, 3))
    # r depends on r_i through -dhat and on r_j through +dhat
    np.add.at(grad, p["i"], -h[:, None] * dhat)
    np.add.at(grad, p["j"], h[:, None] * dhat)
    return grad


def batch_rdf(pos, cell, sys_offsets, n_bins, r_end, sigma, r_max):
    S = cell.shape[0]
    return np.stack([system_rdf(pos[int(sys_offsets[s]):int(sys_offsets[s + 1])], cell[s], n_bins, r_end, sigma,
                                r_max) for s in range(S)])


def rdf_loss(g, g_target):
    return float(((g - g_target) ** 2).mean())


def rdf_loss_grad(pos, cell, sys_offsets, n_bins, r_end, sigma, r_max, g, g_target):
    S = cell.shape[0]
    dL_dg = 2.0 * (g - g_target) / (S * n_bins)
    grad = np.zeros_like(pos)
    for s in range(S):
        a, b = int(sys_offsets[s]), int(sys_offsets[s + 1])
        grad[a:b] = system_rdf_grad(pos[a:b], cell[s], n_bins, r_end, sigma, r_max, dL_dg[s])
    return grad


def _pair_terms(pos, cell, species, potential):
    p = _pairs.system_pairs(pos, cell, potential.cutoff)
    sp = potential.params[species[p["i"]], species[p["j"]]]
    m = _pot.in_range(potential.kind, sp, p["r2"], potential.cutoff)
    p = {k: v[m] for k, v in p.items()}
    return p, sp[m]


def system_hvp(pos, cell, species, potential, u):
    """(J u)_i with J = dF/dr of one system."""
    p, sp = _pair_terms(pos, cell, species, potential)
    r = np.sqrt(p["r2"])
    _, d1, d2 = _pot.phi_and_derivs(potential.kind, sp, r, potential.cutoff)
    dhat = p["d"] / r[:, None]
    du = u[p["j"]] - u[p["i"]]
    proj = (dhat * du).sum(axis=1)
    k = d2[:, None] * proj[:, None] * dhat + (d1 / r)[:, None] * (du - proj[:, None] * dhat)
    out = np.zeros_like(u)
    np.add.at(out, p["i"], k)
    return out


def system_param_vjp(pos, cell, species, potential, u):
    """sum_i u_i . dF_i/dtheta, accumulated per (s_i, s_j, slot)."""
    p, sp = _pair_terms(pos, cell, species, potential)
    r = np.sqrt(p["r2"])
    dg = _pot.dg_dparams(potential.kind, sp, r, potential.cutoff)
    ud = (u[p["i"]] * p["d"]).sum(axis=1)
    ns = potential.params.shape[0]
    out = np.zeros((ns, ns, 3))
    np.add.at(out, (species[p["i"]], species[p["j"]]), dg * ud[:, None])
    return out


def batch_hvp(pos, cell, sys_offsets, species, potential, u):
    out = np.zeros_like(u)
    for s in range(cell.shape[0]):
        a, b = int(sys_offsets[s]), int(sys_offsets[s + 1])
        out[a:b] = system_hvp(pos[a:b], cell[s], species[a:b], potential, u[a:b])
    return out


def batch_param_vjp(pos, cell, sys_offsets, species, potential, u):
    ns = potential.params.shape[0]
    out = np.zeros((ns, ns, 3))
    for s in range(cell.shape[0]):
        a, b = int(sys_offsets[s]), int(sys_offsets[s + 1])
        out += system_param_vjp(pos[a:b], cell[s], species[a:b], potential, u[a:b])
    return out


def reverse_nve(positions, mass, cell, sys_offsets, species, potential, dt, accel, lam_r, lam_v):
    """Reverse a velocity-Verlet trajectory whose positions r_0..r_T are ``positions`` (list).
    Starts from (lam_r, lam_v) = (dL/dr_T, dL/dv_T); returns (dL/dr_0, dL/dv_0, dL/dtheta)."""
    lam_r = np.array(lam_r, dtype=np.float64, copy=True)
    lam_v = np.array(lam_v, dtype=np.float64, copy=True)
    ns = potential.params.shape[0]
    tb = np.zeros((ns, ns, 3))
    h = 0.5 * dt
    scale = (accel / mass)[:, None]
    for n in range(len(positions) - 2, -1, -1):
        u = scale * lam_v
        lam_r = lam_r + h * batch_hvp(positions[n + 1], cell, sys_offsets, species, potential, u)
        tb += h * batch_param_vjp(positions[n + 1], cell, sys_offsets, species, potential, u)
        lam_v = lam_v + dt * lam_r
        u = scale * lam_v
        lam_r = lam_r + h * batch_hvp(positions[n], cell, sys_offsets, species, potential, u)
        tb += h * batch_param_vjp(positions[n], cell, sys_offsets, species, potential, u)
    return lam_r, lam_v, tb


def trajectory_positions(pos, vel, mass, cell, sys_offsets, species, potential, dt, n_steps, accel):
    """Forward velocity Verlet keeping every position (for the reverse pass)."""
    pos = np.array(pos, dtype=np.float64, copy=True)
    vel = np.array(vel, dtype=np.float64, copy=True)
    scale = (accel / mass)[:, None]
    _, F, _ = _forces.batch_efw(pos, cell, sys_offsets, species, potential)
    out = [pos.copy()]
    for _ in range(n_steps):
        vel = vel + 0.5 * dt * F * scale
        pos = pos + dt * vel
        _, F, _ = _forces.batch_efw(pos, cell, sys_offsets, species, potential)
        vel = vel + 0.5 * dt * F * scale
        out.append(pos.copy())
    return out, vel
