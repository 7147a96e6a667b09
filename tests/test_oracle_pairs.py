"""Pins of the oracle's periodic pair set against definitions that do not use it."""
import os

import numpy as np
import pytest

from oracle import pairs
from tests.lattice import fcc_shells
from workloads import random_small_batch, fcc_cell, supercell

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _keys(p):
    return sorted(zip(p["i"].tolist(), p["j"].tolist(), *[p["S"][:, k].tolist() for k in range(3)]))


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_bounded_search_equals_unbounded_image_loop(seed):
    # narrow triclinic cells (several images of one pair in range) and positions displaced by
    # whole lattice vectors: the pruned search must find exactly the unpruned definition's set
    w = random_small_batch(seed, n_systems=2, n_range=(1, 6), density=1.5, unwrap_spread=1)
    for s in range(w.n_systems):
        sl = w.system(s)
        r_list = 1.7
        got = _keys(pairs.system_pairs(w.pos[sl], w.cell[s], r_list))
        ref = pairs.system_pairs_unbounded(w.pos[sl], w.cell[s], r_list, image_radius=4)
        assert got == ref
        assert len(ref) > 0


def test_pair_set_symmetry_and_half_set():
    w = random_small_batch(7, n_systems=2, n_range=(5, 30), density=0.9, unwrap_spread=1)
    for s in range(w.n_systems):
        sl = w.system(s)
        p = pairs.system_pairs(w.pos[sl], w.cell[s], 2.2)
        full = set(_keys(p))
        mirrored = {(j, i, -a, -b, -c) for (i, j, a, b, c) in full}
        assert full == mirrored
        h = pairs.system_pairs(w.pos[sl], w.cell[s], 2.2, half=True)
        half = set(_keys(h))
        assert 2 * len(half) == len(full)
        assert half | {(j, i, -a, -b, -c) for (i, j, a, b, c) in half} == full


def _golden_shells():
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "fcc_shells.txt")) if ln.strip() and not ln.startswith("#")]
    return [(float(a), int(b)) for a, b in rows]


@pytest.mark.parametrize("reps", [(3, 3, 3), (1, 1, 1)])
def test_fcc_shell_counts(reps):
    # conventional 4-atom cell (1,1,1): width a < 2 r, so every shell comes from periodic images,
    # including each atom's own images
    a = 2.0
    basis, cell0 = fcc_cell(a)
    pos, cell = supercell(basis, cell0, reps)
    golden = _golden_shells()
    ind = fcc_shells(a, 1.8 * a)
    # the independent lattice enumeration agrees with the textbook table
    for (ra, cnt), (r, c) in zip(golden, ind.items()):
        assert abs(ra * a - r) < 1e-12 and cnt == c
    cum = 0
    for k, (ra, cnt) in enumerate(golden):
        cum += cnt
        r_list = ra * a * 1.01
        p = pairs.system_pairs(pos, cell, r_list)
        per_atom = np.bincount(p["i"], minlength=pos.shape[0])
        assert np.all(per_atom == cum), (k, per_atom[:4], cum)


def test_random_density_count():
    # Poisson points: mean neighbour count is (4/3) pi r^3 rho (N - 1) / N
    rng = np.random.default_rng(0)
    L, n, r = 8.0, 600, 1.5
    pos = rng.random((n, 3)) * L
    p = pairs.system_pairs(pos, np.eye(3) * L, r)
    mean = p["i"].shape[0] / n
    expect = 4.0 / 3.0 * np.pi * r ** 3 * (n - 1) / L ** 3
    assert abs(mean - expect) < 4.0 * np.sqrt(expect / n) + 0.05


def test_band_keys():
    p = dict(i=np.array([0, 1]), j=np.array([1, 0]), S=np.zeros((2, 3), np.int64), r2=np.array([1.0, 4.0 - 1e-12]))
    k = pairs.pair_keys(p, 2.0, band=1e-9)
    assert k.shape[0] == 1 and k[0, 1] == 0
