"""AutoBatching (paper Section 3): the oracle pinned to the paper's Figure 2 arithmetic, and the
host batcher checked against the oracle's definitions."""
import os

import numpy as np
import pytest

from oracle import autobatch as oab
from paper_2508_06628_amd import autobatch as ab

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "autobatch_fig2.txt")


def _fig2():
    rows = [ln.split() for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    probes = [(int(r[0]), int(r[1]), int(r[2])) for r in rows if r[0] != "min"]
    return probes, int([r for r in rows if r[0] == "min"][0][1])


def test_oracle_reproduces_figure_2():
    probes, expect = _fig2()
    for n, s, prod in probes:
        assert n * s == prod
    assert oab.max_memory_scaler([(n, s) for n, s, _ in probes]) == expect
    # probing by adding copies until "out of memory" with a true capacity of about 900 atoms
    fits = lambda total: total <= 900  # noqa: E731
    assert oab.copies_that_fit(fits, 400) == 2 and oab.copies_that_fit(fits, 80) == 11


def test_estimate_matches_oracle_probe():
    scalers = [400.0, 80.0, 150.0]
    cap = 900.0
    fits = lambda s, k: k * scalers[s] <= cap  # noqa: E731
    probes = ab.default_probes(scalers)
    assert probes == [0, 1]
    est = ab.estimate_max_scaler(fits, probes, scalers)
    ref = oab.max_memory_scaler([(oab.copies_that_fit(lambda t: t <= cap, scalers[p]), scalers[p]) for p in probes])
    assert est == ref == 800.0


def test_memory_scalers():
    assert ab.memory_scaler(100, 50.0, "n_atoms") == oab.memory_scaler(100, 50.0, "n_atoms") == 100.0
    assert ab.memory_scaler(100, 50.0, "n_atoms_x_density") == oab.memory_scaler(100, 50.0, "n_atoms_x_density") == 200.0
    with pytest.raises(ValueError):
        ab.memory_scaler(1, 1.0, "bogus")


@pytest.mark.parametrize("seed", range(6))
def test_bin_packing_valid_and_near_optimal(seed):
    rng = np.random.default_rng(seed)
    sizes = list(rng.integers(10, 80, size=int(rng.integers(3, 8))).astype(float))
    cap = 100.0
    bins = ab.bin_pack(sizes, cap)
    assert oab.valid_packing(bins, sizes, cap)
    opt = oab.optimal_bin_count(sizes, cap)
    # first-fit decreasing never needs more than 11/9 OPT + 6/9 bins (Dosa 2007)
    assert opt <= len(bins) <= 11 / 9 * opt + 6 / 9


def test_inflight_batcher_follows_the_schedule():
    rng = np.random.default_rng(3)
    scalers = list(rng.integers(50, 300, size=12).astype(float))
    conv = list(rng.integers(5, 60, size=12))
    cap, every = 760.0, 5
    log, done = oab.inflight_schedule(scalers, conv, cap, every)
    b = ab.InFlightBatcher(scalers, cap)
    progress = {}
    step = 0
    seen = [(0, tuple(b.batch()))]
    while not b.done:
        for _ in range(every):
            for i in b.batch():
                progress[i] = progress.get(i, 0) + 1
            step += 1
        b.update([progress[i] >= conv[i] for i in b.batch()])
        seen.append((step, tuple(b.batch())))
    assert seen == log
    assert sorted(b.completed) == list(range(12))


def test_device_memory_model_is_monotone():
    m = ab.DeviceMemoryModel(max_nbr=100, budget_bytes=10 ** 9)
    assert m.bytes(1000, 1) < m.bytes(2000, 1) < m.bytes(2000, 2)
    k = 0
    while m.fits(864 * (k + 1), k + 1):
        k += 1
    assert not m.fits(864 * (k + 1), k + 1) and m.fits(864 * k, k)
