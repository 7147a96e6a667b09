"""Classical pair potentials (oracle; test infrastructure only).

The paper lists Lennard-Jones, Morse and soft-sphere among the classical potentials the engine
supports (Abstract) without writing them down; these are the textbook forms.

Per species pair the parameter triple p = params[s_i, s_j] is
    LJ           (epsilon, sigma, unused)     phi = 4 eps [(sigma/r)^12 - (sigma/r)^6]
    Morse        (D, alpha, r0)               phi = D [exp(-2 alpha (r - r0)) - 2 exp(-alpha (r - r0))]
    soft sphere  (epsilon, sigma_ij, unused)  phi = (eps / 2) (1 - r / sigma_ij)^2   for r < sigma_ij
A pair interacts when r < r_c (and, for the soft sphere, also r < sigma_ij).  With the energy
shift, phi(r) - phi(r_c) is used inside the cutoff (forces unchanged).

Shifted-force kinds ``lj_sf`` and ``morse_sf`` (the textbook smooth truncation; the paper's
differentiable-simulation use, Section 2, benefits from a force that vanishes continuously at the
cutoff): with phi the plain form,
    phi_sf(r) = phi(r) - phi(r_c) - (r - r_c) phi'(r_c)   for r < r_c,
so phi_sf(r_c) = 0 and phi_sf'(r_c) = 0; phi_sf'' = phi''.

Every function takes arrays of r and of parameter triples (one per pair) and returns float64.
"""
from __future__ import annotations

import numpy as np

KINDS = ("lj", "morse", "soft_sphere", "lj_sf", "morse_sf")


def base_kind(kind: str) -> str:
    """The plain form a shifted-force kind truncates."""
    return kind[:-3] if kind.endswith("_sf") else kind


def phi_and_derivs(kind: str, p: np.ndarray, r: np.ndarray, cutoff: float = None):
    """phi(r), phi'(r), phi''(r) for parameter rows p (P, 3) and distances r (P,).  Shifted-force
    kinds need the cutoff r_c."""
    r = np.asarray(r, dtype=np.float64)
    if kind.endswith("_sf"):
        if cutoff is None:
            raise ValueError(f"{kind} needs the cutoff")
        base = base_kind(kind)
        phi, d1, d2 = phi_and_derivs(base, p, r)
        phi_c, d1_c, _ = phi_and_derivs(base, p, np.full(r.shape[0], float(cutoff)))
        return phi - phi_c - (r - cutoff) * d1_c, d1 - d1_c, d2
    if kind == "lj":
        eps, sig = p[:, 0], p[:, 1]
        sr6 = (sig / r) ** 6
        sr12 = sr6 * sr6
        phi = 4.0 * eps * (sr12 - sr6)
        d1 = 24.0 * eps / r * (sr6 - 2.0 * sr12)
        d2 = 4.0 * eps / (r * r) * (156.0 * sr12 - 42.0 * sr6)
    elif kind == "morse":
        D, alpha, r0 = p[:, 0], p[:, 1], p[:, 2]
        x = np.exp(-alpha * (r - r0))
        phi = D * (x * x - 2.0 * x)
        d1 = 2.0 * alpha * D * (x - x * x)
        d2 = 2.0 * alpha * alpha * D * (2.0 * x * x - x)
    elif kind == "soft_sphere":
        eps, sig = p[:, 0], p[:, 1]
        u = 1.0 - r / sig
        phi = 0.5 * eps * u * u
        d1 = -eps / sig * u
        d2 = eps / (sig * sig) * np.ones_like(r)
    else:
        raise ValueError(kind)
    return phi, d1, d2


def in_range(kind: str, p: np.ndarray, r2: np.ndarray, cutoff: float) -> np.ndarray:
    kind = base_kind(kind)
    """Interaction mask, decided in float64 on squared distances: r^2 < r_c^2 (and r^2 < sigma_ij^2
    for the soft sphere)."""
    m = r2 < cutoff * cutoff
    if kind == "soft_sphere":
        m &= r2 < p[:, 1] * p[:, 1]
    return m


def energy_shift(kind: str, p: np.ndarray, cutoff: float, shift: bool) -> np.ndarray:
    """phi(r_c) per parameter row when the energy is shifted, else zeros (soft sphere and the
    shifted-force kinds, which vanish at r_c by construction: zero)."""
    if not shift or kind == "soft_sphere" or kind.endswith("_sf"):
        return np.zeros(p.shape[0])
    return phi_and_derivs(kind, p, np.full(p.shape[0], cutoff))[0]


def dg_dparams(kind: str, p: np.ndarray, r: np.ndarray, cutoff: float = None) -> np.ndarray:
    """Derivatives of g(r) = phi'(r) / r with respect to the three parameter slots, shape (P, 3).
    The pair force on i is g(r) d, so these give the pair-force parameter derivatives.  For a
    shifted-force kind g_sf(r) = g(r) - phi'(r_c) / r and phi'(r_c) = r_c g(r_c), so
    dg_sf/dtheta = dg/dtheta (r) - (r_c / r) dg/dtheta (r_c)."""
    r = np.asarray(r, dtype=np.float64)
    if kind.endswith("_sf"):
        base = base_kind(kind)
        at_c = dg_dparams(base, p, np.full(r.shape[0], float(cutoff)))
        return dg_dparams(base, p, r) - (cutoff / r)[:, None] * at_c
    out = np.zeros((r.shape[0], 3))
    if kind == "lj":
        eps, sig = p[:, 0], p[:, 1]
        sr6 = (sig / r) ** 6
        sr12 = sr6 * sr6
        g = 24.0 * eps / (r * r) * (sr6 - 2.0 * sr12)
        out[:, 0] = g / eps
        # d/dsigma of sr6 = 6 sr6 / sigma, of sr12 = 12 sr12 / sigma
        out[:, 1] = 24.0 * eps / (r * r) * (6.0 * sr6 - 24.0 * sr12) / sig
    elif kind == "morse":
        D, alpha, r0 = p[:, 0], p[:, 1], p[:, 2]
        x = np.exp(-alpha * (r - r0))
        d1 = 2.0 * alpha * D * (x - x * x)
        out[:, 0] = d1 / D / r
        dx_da = -(r - r0) * x
        out[:, 1] = (2.0 * D * (x - x * x) + 2.0 * alpha * D * (1.0 - 2.0 * x) * dx_da) / r
        dx_dr0 = alpha * x
        out[:, 2] = 2.0 * alpha * D * (1.0 - 2.0 * x) * dx_dr0 / r
    elif kind == "soft_sphere":
        eps, sig = p[:, 0], p[:, 1]
        u = 1.0 - r / sig
        out[:, 0] = -u / sig / r
        # phi' = -eps/sig + eps r / sig^2  ->  d/dsig = eps/sig^2 - 2 eps r / sig^3
        out[:, 1] = (eps / (sig * sig) - 2.0 * eps * r / sig ** 3) / r
    else:
        raise ValueError(kind)
    return out


def lorentz_berthelot(eps, sigma) -> np.ndarray:
    """LJ parameter table of a mixture from per-species (epsilon, sigma) by the Lorentz-Berthelot
    rules: epsilon_ab = sqrt(epsilon_a epsilon_b) (geometric mean), sigma_ab = (sigma_a + sigma_b) / 2
    (arithmetic mean).  Returns (S, S, 3) rows (epsilon_ab, sigma_ab, 0)."""
    eps = np.asarray(eps, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    n = eps.shape[0]
    out = np.zeros((n, n, 3))
    for a in range(n):
        for b in range(n):
            out[a, b, 0] = np.sqrt(eps[a] * eps[b])
            out[a, b, 1] = 0.5 * (sigma[a] + sigma[b])
    return out
