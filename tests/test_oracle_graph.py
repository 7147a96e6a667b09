"""Pins of the graph-export oracle: lattice coordination numbers, pair symmetry, brute force over
the image cube, and the consistency of its offsets and order."""
import itertools

import numpy as np

from oracle import graph
from tests.lattice import fcc_shells


def _cubic(m, a=1.0):
    g = np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"), -1).reshape(-1, 3)
    return g * a + 0.1, np.eye(3) * (m * a)


def test_simple_cubic_coordination():
    pos, cell = _cubic(4)
    # shells of the simple cubic lattice: 6 at a, 12 at a sqrt 2, 8 at a sqrt 3
    for r, want in ((1.05, 6), (1.5, 18), (1.8, 26)):
        g = graph.mlip_graph(pos, cell[None], [0, 64], r)
        assert np.all(np.diff(g["row_ptr"]) == want)
        assert g["edge_offsets"].tolist() == [0, 64 * want]


def test_fcc_coordination_with_shift():
    a, m = 3.6, 3
    base = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    cells = np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"), -1).reshape(-1, 3)
    pos = ((cells[:, None, :] + base[None]) * a).reshape(-1, 3) + np.array([0.3, -0.2, 0.1])
    pos[::7] += np.array([1, -1, 2]) * (m * a)  # unwrapped atoms: shifts absorb the lattice vectors
    cell = np.eye(3) * (m * a)
    r = 4.0  # between the second (a) and third (a sqrt 1.5) shells
    want = sum(c for d, c in fcc_shells(a, r).items())
    assert want == 18
    g = graph.mlip_graph(pos, cell[None], [0, pos.shape[0]], r)
    assert np.all(np.diff(g["row_ptr"]) == want)
    i, j = g["edge_index"]
    d = pos[j] - pos[i] + g["shift"] @ cell
    assert np.allclose(d, g["vec"], atol=1e-12)
    assert np.all(np.linalg.norm(g["vec"], axis=1) < r)


def test_symmetry_and_brute_force_on_tiny_triclinic_batch():
    rng = np.random.default_rng(5)
    cells = [np.array([[2.0, 0.0, 0.0], [0.7, 1.9, 0.0], [-0.4, 0.5, 2.2]]),
             np.array([[3.1, 0.2, 0.0], [0.0, 2.5, 0.3], [0.5, 0.0, 2.8]]),
             np.array([[2.4, 0.0, 0.0], [0.0, 2.4, 0.0], [0.0, 0.0, 2.4]])]
    counts = [3, 0, 1]  # an empty system and a single atom (its own images are its neighbours)
    offs = np.concatenate([[0], np.cumsum(counts)])
    pos = np.concatenate([rng.uniform(-3, 5, size=(c, 3)) for c in counts])
    r = 2.6
    g = graph.mlip_graph(pos, np.stack(cells), offs, r)
    want = []
    for s, c in enumerate(counts):
        for i, j in itertools.product(range(offs[s], offs[s + 1]), repeat=2):
            for S in itertools.product(range(-5, 6), repeat=3):
                if i == j and S == (0, 0, 0):
                    continue
                d = pos[j] - pos[i] + np.array(S, dtype=float) @ cells[s]
                if float(d @ d) < r * r:
                    want.append((i, j) + S)
    got = [tuple(int(x) for x in (i, j, *S)) for i, j, S in zip(g["edge_index"][0], g["edge_index"][1], g["shift"])]
    assert got == sorted(want)  # same set, in the order (i, j, S0, S1, S2)
    keys = set(got)
    assert all((j, i, -a, -b, -c) in keys for i, j, a, b, c in got)
    assert g["edge_offsets"][1] == g["edge_offsets"][2]  # the empty system has no edges
    assert g["row_ptr"][-1] == len(got) == g["edge_offsets"][-1]
    assert np.diff(g["row_ptr"])[offs[2]] > 0
