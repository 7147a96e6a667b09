"""GPU parity of the shifted-force kinds (LJ and Morse truncated so that energy and force vanish
continuously at the cutoff) in every kernel family: forces, energies and virials, the fused NVE loop,
the persistent and per-iteration FIRE paths, and the pair adjoint (Hessian-vector product and
parameter derivatives)."""
import dataclasses

import numpy as np
import pytest

from oracle import adjoint as oadj
from oracle import fire as ofire
from oracle import forces as oforces
from oracle import integrate as ointeg
from tests.gpu_helpers import assert_forces_close, force_scales
from workloads import argon_batch, copper_uneven_batch, random_small_batch

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2508_06628_amd import _native
    _native.lib()
    yield
    torch.cuda.synchronize()


def _api():
    from paper_2508_06628_amd import api
    return api


def _sf_batch(kind, seed, **kw):
    w = random_small_batch(seed, kind=kind, **kw)
    w.potential = dataclasses.replace(w.potential, kind=kind + "_sf", shift_energy=False)
    return w


@pytest.mark.parametrize("kind,n_species,prec", [("lj", 1, "f64"), ("lj", 2, "f64"), ("morse", 2, "f64"),
                                                 ("lj", 2, "f32"), ("morse", 1, "f32")])
def test_shifted_force_forces(kind, n_species, prec):
    api = _api()
    w = _sf_batch(kind, 70 + n_species, n_systems=10, n_range=(1, 70), n_species=n_species, unwrap_spread=1)
    pot = w.potential
    b = api.Batch.from_workload(w)
    nl = api.build_neighbor_list(b, pot.cutoff, 0.2, bin_factor=2)
    pp = api.pair_params_from_spec(pot, prec)
    F, E, W = api.compute_forces(b, nl, pp, prec)
    E_ref, F_ref, W_ref = oforces.batch_efw(w.pos, w.cell, w.sys_offsets, w.species, pot)
    A, se, sw = force_scales(w.pos, w.cell, w.sys_offsets, w.species, pot)
    assert_forces_close(F.T.double().cpu().numpy(), F_ref, A, 1e-10 if prec == "f64" else 1e-5)
    erel = 1e-10 if prec == "f64" else 1e-6
    assert np.all(np.abs(E.cpu().numpy() - E_ref) <= erel * se + 1e-300)
    assert np.all(np.abs(W.cpu().numpy().reshape(-1, 3, 3) - W_ref).max(axis=(1, 2)) <= erel * sw + 1e-300)


@pytest.mark.parametrize("kind", ["lj", "morse"])
def test_shifted_force_nve(kind):
    # physical inputs (FCC argon at 50-300 K; strained triclinic copper from noisy sites): 25 steps
    # stay a smooth trajectory, with list rebuilds at the 0.1 skin, that the brute-force oracle
    # follows in seconds (random jittered cells hold near-overlapping pairs whose trajectories blow up)
    api = _api()
    if kind == "lj":
        w = argon_batch(3, reps=(3, 3, 3), seed=75)
        w.potential = dataclasses.replace(w.potential, kind="lj_sf", shift_energy=False)
        w.dt = 2.0
    else:
        w = copper_uneven_batch(3, seed=75, min_sites=32, max_sites=110)
        w.potential = dataclasses.replace(w.potential, kind="morse_sf")
        w.dt = 0.1
    pot = w.potential
    b = api.Batch.from_workload(w)
    nl = api.build_neighbor_list(b, pot.cutoff, 0.1)
    pp = api.pair_params_from_spec(pot, "f64")
    F, _, _ = api.compute_forces(b, nl, pp, "f64")
    E = torch.zeros(w.n_systems, dtype=torch.float64, device="cuda")
    built = int(nl.read_status()[2])
    api.ts_nve_step(b, nl, pp, w.dt, w.accel, 25, F, E)
    status = nl.read_status()
    assert status[1] == 0 and status[3] == 0 and status[4] == 0
    assert int(status[2]) > built, "the run should cross the skin and rebuild"
    ref = ointeg.nve(w.pos, w.vel, w.mass, w.cell, w.sys_offsets, w.species, pot, w.dt, 25, w.accel)
    L = np.abs(np.linalg.det(w.cell)).max() ** (1 / 3)
    assert np.abs(b.positions() - ref["pos"]).max() <= 1e-10 * L
    _, se, _ = force_scales(ref["pos"], w.cell, w.sys_offsets, w.species, pot)
    assert np.all(np.abs(E.cpu().numpy() - ref["energy"]) <= 1e-10 * se + 1e-300)


@pytest.mark.parametrize("persistent", [False, True])
def test_shifted_force_fire(persistent):
    api = _api()
    w = copper_uneven_batch(4, seed=76, min_sites=32, max_sites=110)
    w.potential = dataclasses.replace(w.potential, kind="morse_sf")
    pot = w.potential
    cfgd = dict(w.extra["fire"])
    b = api.Batch.from_workload(w)
    nl = api.build_neighbor_list(b, pot.cutoff, w.skin)
    pp = api.pair_params_from_spec(pot, "f64")
    cfg = api.fire_config(**cfgd)
    fs = api.FireState(b, cfg)
    F = api.force_buffer(b, "f64")
    api.ts_fire_step(b, fs, cfg, nl, pp, 12, F, persistent=persistent)
    ocfg = ofire.FireConfig(**cfgd)
    for s in range(w.n_systems):
        sl = w.system(s)
        st = ofire.init_state(w.pos[sl], w.cell[s], ocfg)
        ofire.fire_iterate(st, w.species[sl], w.mass[sl], pot, ocfg, 12)
        L = abs(np.linalg.det(w.cell[s])) ** (1 / 3)
        assert np.abs(b.positions()[sl] - st.pos).max() <= 1e-9 * L
        assert np.abs(b.cells()[s] - st.cell).max() <= 1e-9 * L


@pytest.mark.parametrize("kind,prec", [("lj", "f64"), ("morse", "f64"), ("lj", "f32")])
def test_shifted_force_pair_adjoint(kind, prec):
    api = _api()
    w = _sf_batch(kind, 77, n_systems=5, n_range=(5, 60), n_species=2 if kind == "lj" else 1)
    pot = w.potential
    b = api.Batch.from_workload(w)
    nl = api.build_neighbor_list(b, pot.cutoff, 0.2)
    pp = api.pair_params_from_spec(pot, prec)
    rng = np.random.default_rng(1)
    lr0, lv0 = rng.normal(size=w.pos.shape), rng.normal(size=w.pos.shape)
    lr = torch.tensor(lr0.T.copy(), device="cuda")
    lv = torch.tensor(lv0.T.copy(), device="cuda")
    tb = torch.zeros(48, dtype=torch.float64, device="cuda")
    dt, wk, accel = 0.01, 0.005, 1.0
    api.ts_pair_adjoint(b, nl, pp, dt, wk, accel, lr, lv, tb)
    u = accel * (lv0 + dt * lr0) / w.mass[:, None]
    lr_ref = lr0 + wk * oadj.batch_hvp(w.pos, w.cell, w.sys_offsets, w.species, pot, u)
    tb_ref = wk * oadj.batch_param_vjp(w.pos, w.cell, w.sys_offsets, w.species, pot, u)
    tol = 1e-8 if prec == "f64" else 1e-3
    assert np.abs(lr.T.cpu().numpy() - lr_ref).max() <= tol * np.abs(lr_ref - lr0).max()
    ns = pot.params.shape[0]
    got = tb.cpu().numpy().reshape(4, 4, 3)[:ns, :ns]
    assert np.abs(got - tb_ref).max() <= tol * np.abs(tb_ref).max()
