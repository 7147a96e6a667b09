"""Shared helpers of the GPU parity tests (comparison criteria and oracle calls)."""
import numpy as np

from oracle import forces as oforces
from oracle import pairs as opairs


def gpu_pair_keys(batch, nl, sys_of_atom=None):
    """Sorted (sys, i_local, j_local, S0, S1, S2) keys of a GPU list, with distances for the band."""
    i, j, s0, s1, s2 = nl.entries()
    offs = batch.h_offsets
    sys = np.searchsorted(offs, i, side="right") - 1
    il = i - offs[sys]
    pos = batch.positions()
    cell = batch.cells()
    S = np.stack([s0, s1, s2], axis=1)
    d = pos[offs[sys] + j] - pos[i] + np.einsum("pk,pkc->pc", S.astype(np.float64), cell[sys])
    p = dict(sys=sys, i=il, j=j, S=S, r2=(d * d).sum(1))
    return p


def assert_same_pairs(batch, nl, r_list, band=1e-9, half=False, systems=None, pos=None):
    """GPU list == oracle pair set (exactly, outside the band at r_list).  ``systems`` restricts the
    comparison; ``pos`` gives the positions the oracle uses (default: the batch's current ones)."""
    g = gpu_pair_keys(batch, nl)
    pos = batch.positions() if pos is None else pos
    o = opairs.batch_pairs(pos, batch.cells(), batch.h_offsets, r_list, half=half)
    if systems is not None:
        keep = np.isin(g["sys"], systems)
        g = {k: v[keep] for k, v in g.items()}
        keep = np.isin(o["sys"], systems)
        o = {k: v[keep] for k, v in o.items()}
        # distances for the band are taken at the oracle's positions on both sides
        g["r2"] = _r2_at(pos, batch, g)
    kg = opairs.pair_keys(g, r_list, band)
    ko = opairs.pair_keys(o, r_list, band)
    assert kg.shape == ko.shape, (kg.shape, ko.shape)
    assert np.array_equal(kg, ko)
    # no duplicates on the GPU side
    assert np.unique(kg, axis=0).shape[0] == kg.shape[0]
    return kg.shape[0]


def _r2_at(pos, batch, p):
    offs = batch.h_offsets
    cell = batch.cells()
    a = offs[p["sys"]]
    d = pos[a + p["j"]] - pos[a + p["i"]] + np.einsum("pk,pkc->pc", p["S"].astype(np.float64), cell[p["sys"]])
    return (d * d).sum(1)


def force_scales(pos, cell, offs, species, pot, rows=None):
    """Per-atom A_i = sum_j |phi'(r_ij)| and per-system sum|phi|, sum|r phi'| (oracle, float64)."""
    S = cell.shape[0]
    A = np.zeros(pos.shape[0])
    se = np.zeros(S)
    sw = np.zeros(S)
    for s in range(S):
        a, b = int(offs[s]), int(offs[s + 1])
        A[a:b], se[s], sw[s] = oforces.pair_magnitude_sums(pos[a:b], cell[s], species[a:b], pot.params, pot.kind,
                                                           pot.cutoff)
    return A, se, sw


def assert_forces_close(F_gpu, F_ref, A, rel):
    """|dF_i| <= rel * max(|F_i|, 0.1 A_i) (a net force near zero is no scale for its own error)."""
    err = np.linalg.norm(F_gpu - F_ref, axis=1)
    scale = np.maximum(np.linalg.norm(F_ref, axis=1), 0.1 * A)
    bad = err > rel * scale + 1e-300
    assert not bad.any(), (np.nonzero(bad)[0][:5], (err / np.maximum(scale, 1e-300)).max())
    return float((err / np.maximum(scale, 1e-300)).max())
