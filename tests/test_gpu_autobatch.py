"""AutoBatching driving the device (paper Section 3): an in-flight FIRE relaxation of a stream of
systems whose total exceeds the memory budget, and a bin-packed NVE run.

The in-flight schedule (which systems are in the batch after every check) must equal the oracle's
simulation of the in-flight batcher given each system's own iteration count at convergence, every
batch must stay within the probed capacity, and every relaxed system is certified by the FP64
oracle (max |F_i| and max |G| below fmax).  The binned NVE run must give every system exactly the
trajectory it has in one batch of all systems (systems are independent and rows are canonical)."""
import numpy as np
import pytest

from oracle import autobatch as oab
from oracle import fire as ofire
from oracle import forces as oforces
from workloads import copper_uneven_batch, maxwell_boltzmann

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2508_06628_amd import _native
    _native.lib()
    yield
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_inflight_fire_schedule_and_certified_relaxations(prec):
    from paper_2508_06628_amd.autobatch import DeviceMemoryModel
    from paper_2508_06628_amd.batching import InFlightFire, probe_capacity, system_scalers
    w = copper_uneven_batch(14, seed=81, min_sites=32, max_sites=180)
    pot = w.potential
    fire_kw = dict(w.extra["fire"])
    scalers = system_scalers(w)
    total_bytes = DeviceMemoryModel(max_nbr=160, budget_bytes=0).bytes(w.n_atoms, w.n_systems)
    model = DeviceMemoryModel(max_nbr=160, budget_bytes=total_bytes // 3)  # a third of the stream fits
    cap = probe_capacity(w, model, scalers)
    assert max(scalers) <= cap < sum(scalers)
    run = InFlightFire(w, fire_kw, cap, check_every=32, skin=1.0, prec=prec)
    res = run.run()
    assert sorted(res) == list(range(w.n_systems))
    assert all(r.converged for r in res.values()), {s: r.n_iter for s, r in res.items()}
    # the realised schedule is the in-flight batcher's, given each system's own convergence count
    log, done = oab.inflight_schedule(scalers, [res[s].n_iter for s in range(w.n_systems)], cap, 32)
    assert [(int(t), tuple(int(i) for i in b)) for t, b in run.schedule] == [(t, tuple(b)) for t, b in log]
    assert all(res[s].finished_at == done[s] for s in range(w.n_systems))
    assert all(sum(scalers[i] for i in b) <= cap for _, b in log)
    assert len({b for _, b in log}) > 2  # systems really swapped in and out
    for s in range(w.n_systems):
        sl = w.system(s)
        r = res[s]
        _, f, Wv = oforces.system_efw(r.pos, r.cell, w.species[sl], pot.params, pot.kind, pot.cutoff, False)
        assert np.linalg.norm(f, axis=1).max() < fire_kw["fmax"] * 1.001, s
        assert np.abs(ofire.cell_force(r.deform, Wv, f.shape[0])).max() < fire_kw["fmax"] * 1.001, s


def test_nve_binned_equals_one_batch():
    from paper_2508_06628_amd import api
    from paper_2508_06628_amd.batching import nve_binned, system_scalers
    w = copper_uneven_batch(9, seed=82, min_sites=32, max_sites=400)
    rng = np.random.default_rng(3)
    # Maxwell-Boltzmann velocities at 300 K in the workload's units (eV, A, amu, accel 1)
    w.vel = maxwell_boltzmann(rng, w.mass, 300.0, accel=1.0)
    w.dt = 0.05
    scalers = system_scalers(w)
    cap = sum(scalers) / 3.0
    pos_b, vel_b, bins = nve_binned(w, 60, cap, prec="f32", lanes=4)
    assert len(bins) >= 3 and oab.valid_packing(bins, scalers, cap)
    assert len(bins) >= oab.optimal_bin_count(scalers, cap)
    b = api.Batch.from_workload(w)
    nl = api.build_neighbor_list(b, w.potential.cutoff, w.skin, bin_factor=2, margin=1.3)
    nl.lanes_per_atom = 4
    pp = api.pair_params_from_spec(w.potential, "f32")
    F = api.force_buffer(b, "f32")
    api.ts_pair_forces(b, nl, pp, F)
    api.ts_nve_step(b, nl, pp, w.dt, w.accel, 60, F, use_graph=True)
    st = nl.read_status()
    assert st[1] == 0 and st[3] == 0 and st[4] == 0 and st[2] > w.n_systems  # rebuilds happened
    assert np.array_equal(b.positions(), pos_b)
    assert np.array_equal(b.velocities(), vel_b)
