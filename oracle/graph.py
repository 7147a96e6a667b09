"""The neighbor list exported as a graph for learned potentials (oracle; test infrastructure only).

Learned interatomic potentials take the batch as one graph whose edges are the periodic pairs
within the model's cutoff; the paper attributes most of the speed differences between models to
the cost of building that graph (Section 4).  Written out from the pair-set definition of
``oracle.pairs``:

    E = {(i, j, S) : i, j in the same system, S in Z^3, (i != j or S != 0), |r_j - r_i + S @ cell| < r_graph}

with global atom indices.  The paper fixes no edge order; reading: edges grouped by system in
batch order, then by the center atom i, then lexicographically by (j, S0, S1, S2).  Outputs:
``row_ptr`` [N + 1] (edges of atom i are row_ptr[i] .. row_ptr[i + 1] - 1), ``edge_offsets``
[S + 1] (edges of system s), ``edge_index`` [2, E] (row 0 = i, row 1 = j), ``shift`` [E, 3]
(integer S) and ``vec`` [E, 3] (d = r_j - r_i + S @ cell).  Pins (``tests/test_oracle_graph.py``):
coordination numbers of simple cubic and face-centred cubic lattices, the pair symmetry
(i, j, S) <-> (j, i, -S), brute force over the image cube on a tiny triclinic system, and the
consistency of the offsets.
"""
from __future__ import annotations

import numpy as np

from . import pairs as _pairs


def mlip_graph(pos, cell, sys_offsets, r_graph: float):
    pos = np.asarray(pos, dtype=np.float64)
    cell = np.asarray(cell, dtype=np.float64)
    offs = np.asarray(sys_offsets, dtype=np.int64)
    n, n_sys = pos.shape[0], offs.shape[0] - 1
    ii, jj, SS, dd = [], [], [], []
    sys_edges = np.zeros(n_sys + 1, dtype=np.int64)
    for s in range(n_sys):
        a0, a1 = offs[s], offs[s + 1]
        p = _pairs.system_pairs(pos[a0:a1], cell[s], r_graph)
        order = np.lexsort((p["S"][:, 2], p["S"][:, 1], p["S"][:, 0], p["j"], p["i"]))
        ii.append(p["i"][order] + a0)
        jj.append(p["j"][order] + a0)
        SS.append(p["S"][order])
        dd.append(p["d"][order])
        sys_edges[s + 1] = sys_edges[s] + order.shape[0]
    i = np.concatenate(ii) if ii else np.zeros(0, np.int64)
    j = np.concatenate(jj) if jj else np.zeros(0, np.int64)
    S = np.concatenate(SS) if SS else np.zeros((0, 3), np.int64)
    d = np.concatenate(dd) if dd else np.zeros((0, 3))
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    row_ptr[1:] = np.cumsum(np.bincount(i, minlength=n))
    return dict(row_ptr=row_ptr, edge_offsets=sys_edges, edge_index=np.stack([i, j]).astype(np.int64),
                shift=S.astype(np.int64), vec=d)
