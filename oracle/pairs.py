"""Periodic pair sets by brute force (oracle; test infrastructure only).

Definition (the neighbor-list "graph construction" of Section 4, written out; general image
sum, so it is also right for cells narrower than twice the list radius, where one atom pair
appears under several images and an atom can be its own neighbor through a lattice vector):

    N_full = {(i, j, S) : i, j in the same system, S in Z^3, (i != j or S != 0),
              |r_j - r_i + S @ cell| < r_list}

    N_half = {(i, j, S) in N_full : i < j, or i == j and S lexicographically positive}

Positions are used as given (never wrapped), so S also absorbs whole lattice vectors by which
the caller's positions sit outside the cell.

The only shortcut is a bound that discards images which cannot be in range: for the plane
normal n_k of lattice direction k (perpendicular to the other two lattice vectors) one has
d . n_k = (s_j,k - s_i,k + S_k) w_k, with s fractional coordinates and w_k = V / |a_l x a_m| the
perpendicular width, so |d| >= |s_j,k - s_i,k + S_k| w_k.  Every image whose bound is below
r_list in all three directions is then tested exactly with the float64 predicate |d|^2 < r_list^2.
``tests/test_oracle_pairs.py`` pins this against the unbounded image loop.
"""
from __future__ import annotations

import itertools

import numpy as np


def perpendicular_widths(cell: np.ndarray) -> np.ndarray:
    """w_k = V / |a_{k+1} x a_{k+2}|: distance between neighbouring lattice planes of direction k."""
    vol = abs(np.linalg.det(cell))
    w = np.empty(3)
    for k in range(3):
        w[k] = vol / np.linalg.norm(np.cross(cell[(k + 1) % 3], cell[(k + 2) % 3]))
    return w


def system_pairs(pos: np.ndarray, cell: np.ndarray, r_list: float, rows=None, half: bool = False,
                 chunk: int = 256):
    """Pair set of one system.

    Returns a dict of arrays over pairs: ``i``, ``j`` (system-local indices), ``S`` (int64, (P, 3)),
    ``d`` ((P, 3) = r_j - r_i + S @ cell) and ``r2`` (= |d|^2).  ``rows`` restricts i to a subset
    (all j are still searched), which is how single atoms of very large systems are checked.
    """
    pos = np.asarray(pos, dtype=np.float64)
    cell = np.asarray(cell, dtype=np.float64)
    n = pos.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows, dtype=np.int64)
    frac = pos @ np.linalg.inv(cell)
    reach = r_list / perpendicular_widths(cell)
    rl2 = r_list * r_list
    out = {k: [] for k in ("i", "j", "S", "d", "r2")}
    for c0 in range(0, rows.shape[0], chunk):
        ii = rows[c0:c0 + chunk]
        ds = frac[None, :, :] - frac[ii, None, :]  # s_j - s_i, shape (c, n, 3)
        lo = np.floor((-ds - reach).min(axis=(0, 1))).astype(int)
        hi = np.ceil((-ds + reach).max(axis=(0, 1))).astype(int)
        dr = pos[None, :, :] - pos[ii, None, :]  # r_j - r_i
        for S in itertools.product(*[range(lo[k], hi[k] + 1) for k in range(3)]):
            Sv = np.asarray(S, dtype=np.float64)
            d = dr + Sv @ cell
            r2 = (d * d).sum(axis=-1)
            m = r2 < rl2
            if S == (0, 0, 0):
                m[np.arange(ii.shape[0]), ii] = False
            a, b = np.nonzero(m)
            if a.size == 0:
                continue
            out["i"].append(ii[a])
            out["j"].append(b.astype(np.int64))
            out["S"].append(np.broadcast_to(np.asarray(S, dtype=np.int64), (a.size, 3)).copy())
            out["d"].append(d[a, b])
            out["r2"].append(r2[a, b])
    if not out["i"]:
        res = dict(i=np.zeros(0, np.int64), j=np.zeros(0, np.int64), S=np.zeros((0, 3), np.int64),
                   d=np.zeros((0, 3)), r2=np.zeros(0))
    else:
        res = {k: np.concatenate(v) for k, v in out.items()}
    if half:
        keep = half_mask(res["i"], res["j"], res["S"])
        res = {k: v[keep] for k, v in res.items()}
    return res


def half_mask(i, j, S):
    """i < j, or i == j with S lexicographically positive (first non-zero component > 0)."""
    S = np.asarray(S)
    first = np.where(S[:, 0] != 0, S[:, 0], np.where(S[:, 1] != 0, S[:, 1], S[:, 2]))
    return (i < j) | ((i == j) & (first > 0))


def system_pairs_unbounded(pos, cell, r_list, image_radius: int):
    """The definition with no pruning at all: every S in [-m, m]^3.  Slow; tiny inputs only."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    res = []
    for S in itertools.product(range(-image_radius, image_radius + 1), repeat=3):
        shift = np.asarray(S, dtype=np.float64) @ cell
        for i in range(n):
            for j in range(n):
                if i == j and S == (0, 0, 0):
                    continue
                d = pos[j] - pos[i] + shift
                if float(d @ d) < r_list * r_list:
                    res.append((i, j) + tuple(S))
    return sorted(res)


def batch_pairs(pos, cell, sys_offsets, r_list, half=False):
    """Pair sets of every system of a batch, with a ``sys`` column; i, j stay system-local."""
    parts = []
    for s in range(cell.shape[0]):
        a, b = int(sys_offsets[s]), int(sys_offsets[s + 1])
        p = system_pairs(pos[a:b], cell[s], r_list, half=half)
        p["sys"] = np.full(p["i"].shape[0], s, dtype=np.int64)
        parts.append(p)
    return {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}


def pair_keys(p, r_list: float, band: float = 0.0):
    """Sorted comparison keys (sys, i, j, S0, S1, S2) after dropping every pair whose distance is
    within ``band`` of r_list (pairs that sit on the list radius up to rounding)."""
    r = np.sqrt(p["r2"])
    keep = np.abs(r - r_list) > band
    sys = p.get("sys", np.zeros(p["i"].shape[0], np.int64))
    keys = np.stack([sys, p["i"], p["j"], p["S"][:, 0], p["S"][:, 1], p["S"][:, 2]], axis=1)[keep]
    order = np.lexsort(keys.T[::-1])
    return keys[order]
