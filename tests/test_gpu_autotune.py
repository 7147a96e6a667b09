"""Autotuners.  Step loops: lanes per atom and atoms per workgroup, timed on scratch copies.  FIRE:
the choice between the persistent launch and the per-iteration kernels (and the lanes per atom) is
made on scratch copies, leaves the caller's batch untouched, and the relaxation run with the chosen
path ends certified by the FP64 oracle (max |F_i| and max |G| below fmax).  Bin factor: rows of a
binned batch are the same for every factor, and the tuner only times batches the cell list builds."""
import numpy as np
import pytest

from oracle import fire as ofire
from oracle import forces as oforces
from workloads import copper_uneven_batch

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2508_06628_amd import _native
    _native.lib()
    yield
    torch.cuda.synchronize()


def test_tune_fire_choice_and_certified_relaxation(tmp_path, monkeypatch):
    from paper_2508_06628_amd import api
    from paper_2508_06628_amd.autotune import FIRE_LANE_CHOICES, tune_fire
    monkeypatch.setenv("TS_AUTOTUNE_CACHE", str(tmp_path))
    w = copper_uneven_batch(6, seed=93, min_sites=32, max_sites=400)
    pot = w.potential
    b = api.Batch.from_workload(w)
    nl = api.build_neighbor_list(b, pot.cutoff, 1.0, bin_factor=2, margin=1.3)
    pp = api.pair_params_from_spec(pot, "f64")
    kw = dict(w.extra["fire"])
    kw["relax_cell"] = True
    kw["max_iter"] = 5000
    cfg = api.fire_config(**kw)
    pos0, cell0 = b.positions().copy(), b.cells().copy()
    tune = tune_fire(b, nl, pp, cfg, iters=8)
    assert not tune["cached"]
    assert tune["persistent"] in (True, False) and tune["lanes_per_atom"] in FIRE_LANE_CHOICES
    assert len(tune["ms"]) == 2 * len(FIRE_LANE_CHOICES) and all(v > 0 for v in tune["ms"].values())
    assert nl.lanes_per_atom == tune["lanes_per_atom"]
    np.testing.assert_array_equal(b.positions(), pos0)
    np.testing.assert_array_equal(b.cells(), cell0)
    again = tune_fire(b, nl, pp, cfg, iters=8)
    assert again["cached"] and again["persistent"] == tune["persistent"]

    fs = api.FireState(b, cfg)
    F = api.force_buffer(b, "f64")
    api.fire_relax(b, fs, cfg, nl, pp, F, persistent=tune["persistent"])
    st = nl.read_status()
    assert st[1] == 0 and st[3] == 0 and st[4] == 0, st
    assert fs.converged.cpu().numpy().all()
    pos, cell = b.positions(), b.cells()
    deform = fs.deform.cpu().numpy().reshape(-1, 3, 3)
    fmax = w.extra["fire"]["fmax"]
    for s in range(w.n_systems):
        sl = slice(int(b.h_offsets[s]), int(b.h_offsets[s + 1]))
        _, f, Wv = oforces.system_efw(pos[sl], cell[s], w.species[sl], pot.params, pot.kind, pot.cutoff, False)
        assert np.linalg.norm(f, axis=1).max() < fmax * 1.001, s
        assert np.abs(ofire.cell_force(deform[s], Wv, f.shape[0])).max() < fmax * 1.001, s


def test_tune_bin_factor_rows_independent_of_the_factor(tmp_path, monkeypatch):
    """The cell-list bin factor is tuned by timing forced rebuilds; the rows of a binned batch do not
    depend on it (canonical order), and a batch without systems above 2048 atoms is left alone."""
    from paper_2508_06628_amd import api
    from paper_2508_06628_amd.autotune import BIN_FACTOR_CHOICES, tune_bin_factor
    from workloads import soft_sphere_jamming_batch
    monkeypatch.setenv("TS_AUTOTUNE_CACHE", str(tmp_path))
    w = soft_sphere_jamming_batch(2, 2600, seed=23)
    b = api.Batch.from_workload(w)
    lists = []
    for bf in BIN_FACTOR_CHOICES:
        nl = api.build_neighbor_list(b, w.potential.cutoff, w.skin, bin_factor=bf, margin=1.3)
        st = nl.read_status()
        assert st[1] == 0 and st[3] == 0 and st[4] == 0, st
        lists.append((nl.n_nbr.cpu().numpy(), nl.entries()))
    for n_nbr, ent in lists[1:]:
        np.testing.assert_array_equal(n_nbr, lists[0][0])
        for a, c in zip(ent, lists[0][1]):
            np.testing.assert_array_equal(a, c)
    tune = tune_bin_factor(b, nl, reps=2)
    assert tune["binned"] and tune["bin_factor"] in BIN_FACTOR_CHOICES and nl.bin_factor == tune["bin_factor"]
    assert len(tune["ms"]) == len(BIN_FACTOR_CHOICES) and not tune["cached"]
    assert tune_bin_factor(b, nl, reps=2)["cached"]
    small = copper_uneven_batch(3, seed=95, min_sites=32, max_sites=200)
    bs = api.Batch.from_workload(small)
    nls = api.build_neighbor_list(bs, small.potential.cutoff, 0.5, bin_factor=2)
    t2 = tune_bin_factor(bs, nls)
    assert not t2["binned"] and t2["bin_factor"] == 2 and nls.bin_factor == 2


def test_tune_nve_choice_cache_and_untouched_batch(tmp_path, monkeypatch):
    """The step-loop tuner times every (lanes per atom, atoms per workgroup) candidate on scratch
    copies: the caller's batch is unchanged, the choice is one of the candidates and is cached."""
    from paper_2508_06628_amd import api
    from paper_2508_06628_amd.autotune import tune_nve
    from workloads import argon_batch
    monkeypatch.setenv("TS_AUTOTUNE_CACHE", str(tmp_path))
    w = argon_batch(3, seed=41, reps=(3, 3, 3))
    b = api.Batch.from_workload(w)
    nl = api.build_neighbor_list(b, w.potential.cutoff, w.skin, bin_factor=2, margin=1.3)
    pp = api.pair_params_from_spec(w.potential, "f32")
    pos0, vel0 = b.positions().copy(), b.velocities().copy()
    t = tune_nve(b, nl, pp, w.dt, w.accel, steps=20, reps=2)
    assert not t["cached"] and len(t["us_per_step"]) == 7 and all(v > 0 for v in t["us_per_step"].values())
    assert f"{t['lanes_per_atom']}/{t['group_atoms']}" == min(t["us_per_step"], key=t["us_per_step"].get)
    assert (nl.lanes_per_atom, nl.group_atoms) == (t["lanes_per_atom"], t["group_atoms"])
    np.testing.assert_array_equal(b.positions(), pos0)
    np.testing.assert_array_equal(b.velocities(), vel0)
    assert tune_nve(b, nl, pp, w.dt, w.accel, steps=20, reps=2)["cached"]
