"""GPU parity: every entry point of the C ABI against the FP64 oracle on seeded inputs.

Sizes are small enough for the brute-force oracle but span several 256-atom blocks, ragged
system sizes, narrow triclinic cells (several images of one pair) and unwrapped positions.
"""
import numpy as np
import pytest

from oracle import adjoint as oadj
from oracle import fire as ofire
from oracle import forces as oforces
from oracle import integrate as ointeg
from oracle import pairs as opairs
from tests.gpu_helpers import assert_forces_close, assert_same_pairs, force_scales
from workloads import argon_batch, argon_single, copper_uneven_batch, random_small_batch

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


def _batch(w):
    return _api().Batch.from_workload(w)


# ----------------------------------------------------------------------------- neighbor list


@pytest.mark.parametrize("seed,bin_factor,half", [(0, 1, False), (1, 2, False), (2, 3, False), (3, 1, True),
                                                  (4, 2, True)])
def test_neighbor_pairs_exact_small(seed, bin_factor, half):
    api = _api()
    w = random_small_batch(seed, n_systems=12, n_range=(1, 60), density=0.9, unwrap_spread=2)
    b = _batch(w)
    nl = api.build_neighbor_list(b, 2.5, 0.3, bin_factor=bin_factor, half=half)
    n = assert_same_pairs(b, nl, 2.8, half=half)
    assert n > 0
    st = nl.read_status()
    assert st[1] == 0 and st[3] == 0 and st[4] == 0


def test_neighbor_pairs_exact_argon_and_copper():
    api = _api()
    w = argon_batch(2, seed=5)
    b = _batch(w)
    nl = api.build_neighbor_list(b, w.potential.cutoff, w.skin, bin_factor=2)
    assert_same_pairs(b, nl, w.potential.cutoff + w.skin)
    wc = copper_uneven_batch(6, seed=7, min_sites=32, max_sites=300)
    bc = _batch(wc)
    nlc = api.build_neighbor_list(bc, wc.potential.cutoff, wc.skin, bin_factor=1)
    assert_same_pairs(bc, nlc, wc.potential.cutoff + wc.skin)


def test_neighbor_overflow_and_nonfinite_status():
    api = _api()
    w = random_small_batch(9, n_systems=3, n_range=(20, 40), density=1.0)
    b = _batch(w)
    nl = api.NeighborList(b, 2.5, 0.0, max_nbr=4)
    api.ts_neighbor_build(b, nl, force=True)
    st = nl.read_status()
    need = max(np.bincount(opairs.system_pairs(w.pos[w.system(s)], w.cell[s], 2.5)["i"]).max() for s in range(3))
    assert st[1] == 1 and st[0] == need
    assert (nl.n_nbr.cpu().numpy() <= 4).all()
    b.pos[0, 5] = float("nan")
    nl.status.zero_()
    api.ts_neighbor_build(b, nl, force=True)
    assert nl.read_status()[3] == 1


def test_rebuild_trigger_matches_definition():
    api = _api()
    w = random_small_batch(13, n_systems=6, n_range=(20, 50), density=0.9)
    b = _batch(w)
    nl = api.build_neighbor_list(b, 2.2, 0.4)
    rng = np.random.default_rng(0)
    pos = w.pos.copy()
    moved = {1: 0.21, 3: 0.19, 4: 0.5}  # displacement of one atom per system (skin/2 = 0.2)
    for s, amt in moved.items():
        a = int(w.sys_offsets[s]) + 3
        v = rng.normal(size=3)
        pos[a] += amt * v / np.linalg.norm(v)
    b.pos.copy_(torch.tensor(pos.T.copy()))
    before = nl.read_status()[2]
    api.ts_neighbor_build(b, nl, force=False)
    rebuilt = nl.read_status()[2] - before
    expect = sum(ointeg.rebuild_needed(pos[w.system(s)], w.pos[w.system(s)], w.cell[s], w.cell[s], 0.4, 2.6)
                 for s in range(6))
    assert rebuilt == expect == 2
    # rebuilt systems hold the pair set of the new positions, the others still that of the old ones
    assert_same_pairs(b, nl, 2.6, systems=[1, 4])
    assert_same_pairs(b, nl, 2.6, systems=[0, 2, 3, 5], pos=w.pos)


# ----------------------------------------------------------------------------- forces


@pytest.mark.parametrize("kind,n_species,prec", [("lj", 1, "f64"), ("lj", 2, "f64"), ("morse", 2, "f64"),
                                                 ("soft_sphere", 2, "f64"), ("lj", 2, "f32"), ("morse", 1, "f32"),
                                                 ("soft_sphere", 3, "f32")])
def test_pair_forces_small(kind, n_species, prec):
    api = _api()
    w = random_small_batch(20 + n_species, n_systems=10, n_range=(1, 70), kind=kind, n_species=n_species,
                           unwrap_spread=1)
    pot = w.potential
    b = _batch(w)
    nl = api.build_neighbor_list(b, pot.cutoff, 0.2, bin_factor=2)
    pp = api.pair_params_from_spec(pot, prec)
    F, E, W = api.compute_forces(b, nl, pp, prec)
    Fg = F.T.double().cpu().numpy()
    E_ref, F_ref, W_ref = oforces.batch_efw(w.pos, w.cell, w.sys_offsets, w.species, pot)
    A, se, sw = force_scales(w.pos, w.cell, w.sys_offsets, w.species, pot)
    rel = 1e-10 if prec == "f64" else 1e-5
    assert_forces_close(Fg, F_ref, A, rel)
    erel = 1e-10 if prec == "f64" else 1e-6
    assert np.all(np.abs(E.cpu().numpy() - E_ref) <= erel * se + 1e-300)
    Wg = W.cpu().numpy().reshape(-1, 3, 3)
    assert np.all(np.abs(Wg - W_ref).max(axis=(1, 2)) <= erel * sw + 1e-300)


def test_pair_forces_argon_fp32_batch():
    api = _api()
    w = argon_batch(3, seed=8)
    pot = w.potential
    b = _batch(w)
    nl = api.build_neighbor_list(b, pot.cutoff, w.skin)
    pp = api.pair_params_from_spec(pot, "f32")
    F, E, W = api.compute_forces(b, nl, pp, "f32")
    E_ref, F_ref, W_ref = oforces.batch_efw(w.pos, w.cell, w.sys_offsets, w.species, pot)
    A, se, sw = force_scales(w.pos, w.cell, w.sys_offsets, w.species, pot)
    assert_forces_close(F.T.double().cpu().numpy(), F_ref, A, 1e-5)
    assert np.all(np.abs(E.cpu().numpy() - E_ref) <= 1e-6 * se)
    assert np.all(np.abs(W.cpu().numpy().reshape(-1, 3, 3) - W_ref).max(axis=(1, 2)) <= 1e-6 * sw)


# ----------------------------------------------------------------------------- NVE


def test_nve_argon_fp64_100_steps():
    api = _api()
    w = argon_single()
    pot = w.potential
    b = _batch(w)
    nl = api.build_neighbor_list(b, pot.cutoff, 0.0, bin_factor=2)
    pp = api.pair_params_from_spec(pot, "f64")
    F, _, _ = api.compute_forces(b, nl, pp, "f64")
    epot = torch.zeros(1, dtype=torch.float64, device="cuda")
    ekin = torch.zeros_like(epot)
    api.ts_nve_step(b, nl, pp, w.dt, w.accel, w.n_steps, F, epot, ekin, use_graph=True)
    ref = ointeg.nve(w.pos, w.vel, w.mass, w.cell, w.sys_offsets, w.species, pot, w.dt, w.n_steps, w.accel)
    L = abs(np.linalg.det(w.cell[0])) ** (1 / 3)
    assert np.abs(b.positions() - ref["pos"]).max() <= 1e-10 * L
    _, se, _ = force_scales(ref["pos"], w.cell, w.sys_offsets, w.species, pot)
    assert abs(epot.item() - ref["energy"][0]) <= 1e-10 * se[0]
    ke = ointeg.kinetic_energy(ref["vel"], w.mass, w.sys_offsets, w.kinetic_factor)
    assert abs(ekin.item() - ke[0]) <= 1e-10 * ke[0]
    assert nl.read_status()[2] >= 100  # rebuilt at every step (skin 0)


def test_nve_graph_equals_eager_and_batch_invariance():
    api = _api()
    w = argon_batch(3, seed=9, reps=(3, 3, 3))
    pot = w.potential
    runs = []
    for use_graph, sub in ((True, None), (False, None), (False, [1])):
        ww = w if sub is None else w.subset(sub)
        b = _batch(ww)
        nl = api.build_neighbor_list(b, pot.cutoff, w.skin)
        pp = api.pair_params_from_spec(pot, "f64")
        F, _, _ = api.compute_forces(b, nl, pp, "f64")
        api.ts_nve_step(b, nl, pp, w.dt, w.accel, 30, F, use_graph=use_graph)
        runs.append(b.positions())
    assert np.array_equal(runs[0], runs[1])
    alone = runs[2]
    inside = runs[0][w.system(1)]
    assert np.abs(alone - inside).max() <= 1e-12 * 16.0


def test_nve_argon_fp32_steps():
    api = _api()
    w = argon_batch(2, seed=10)
    pot = w.potential
    b = _batch(w)
    nl = api.build_neighbor_list(b, pot.cutoff, w.skin)
    pp = api.pair_params_from_spec(pot, "f32")
    F, _, _ = api.compute_forces(b, nl, pp, "f32")
    api.ts_nve_step(b, nl, pp, w.dt, w.accel, 1, F, use_graph=False)
    ref = ointeg.nve(w.pos, w.vel, w.mass, w.cell, w.sys_offsets, w.species, pot, w.dt, 1, w.accel)
    L = abs(np.linalg.det(w.cell[0])) ** (1 / 3)
    assert np.abs(b.positions() - ref["pos"]).max() <= 1e-10 * L
    A, _, _ = force_scales(ref["pos"], w.cell, w.sys_offsets, w.species, pot)
    assert_forces_close(F.T.double().cpu().numpy(), ref["forces"], A, 1e-5)


# ----------------------------------------------------------------------------- FIRE


def _fire_cfg_dict(**kw):
    d = dict(dt_start=0.1, dt_max=1.0, alpha_start=0.1, f_inc=1.1, f_dec=0.5, f_alpha=0.99, n_min=5, fmax=0.01,
             relax_cell=False, max_iter=100000, cell_mass=1.0)
    d.update(kw)
    return d


@pytest.mark.parametrize("relax_cell,persistent", [(False, False), (True, False), (False, True), (True, True)])
def test_fire_iterations_match_oracle(relax_cell, persistent):
    api = _api()
    w = copper_uneven_batch(4, seed=11, min_sites=32, max_sites=120)
    pot = w.potential
    cfgd = _fire_cfg_dict(relax_cell=relax_cell)
    b = _batch(w)
    nl = api.build_neighbor_list(b, pot.cutoff, w.skin)
    pp = api.pair_params_from_spec(pot, "f64")
    cfg = api.fire_config(**cfgd)
    fs = api.FireState(b, cfg)
    F = api.force_buffer(b, "f64")
    n_it = 12
    api.ts_fire_step(b, fs, cfg, nl, pp, n_it, F, persistent=persistent)
    ocfg = ofire.FireConfig(**cfgd)
    for s in range(w.n_systems):
        sl = w.system(s)
        st = ofire.init_state(w.pos[sl], w.cell[s], ocfg)
        ofire.fire_iterate(st, w.species[sl], w.mass[sl], pot, ocfg, n_it)
        L = abs(np.linalg.det(w.cell[s])) ** (1 / 3)
        assert np.abs(b.positions()[sl] - st.pos).max() <= 1e-9 * L
        if relax_cell:
            assert np.abs(b.cells()[s] - st.cell).max() <= 1e-9 * L
        assert fs.n_iter[s].item() == st.n_iter
        assert abs(fs.dt[s].item() - st.dt) <= 1e-12 * st.dt


@pytest.mark.parametrize("persistent", [False, True])
def test_fire_relaxation_certified_by_oracle(persistent):
    api = _api()
    w = copper_uneven_batch(5, seed=12, min_sites=32, max_sites=200)
    pot = w.potential
    cfgd = _fire_cfg_dict(relax_cell=True)
    b = _batch(w)
    nl = api.build_neighbor_list(b, pot.cutoff, w.skin)
    pp = api.pair_params_from_spec(pot, "f32")
    cfg = api.fire_config(**cfgd)
    fs = api.FireState(b, cfg)
    F = api.force_buffer(b, "f32")
    if persistent:
        api.ts_fire_step(b, fs, cfg, nl, pp, 4000, F, persistent=True)
    else:
        for _ in range(40):
            api.ts_fire_step(b, fs, cfg, nl, pp, 100, F)
            if fs.converged.all().item():
                break
    assert fs.converged.all().item()
    pos, cell = b.positions(), b.cells()
    for s in range(w.n_systems):
        sl = w.system(s)
        e, f, W = oforces.system_efw(pos[sl], cell[s], w.species[sl], pot.params, pot.kind, pot.cutoff, False)
        assert np.linalg.norm(f, axis=1).max() < cfgd["fmax"] * 1.001
        D = fs.deform[s].cpu().numpy().reshape(3, 3)
        G = ofire.cell_force(D, W, f.shape[0])
        assert np.abs(G).max() < cfgd["fmax"] * 1.001


# ----------------------------------------------------------------------------- adjoint and RDF


@pytest.mark.parametrize("kind,prec", [("lj", "f64"), ("morse", "f64"), ("soft_sphere", "f64"), ("lj", "f32")])
def test_pair_adjoint_one_call(kind, prec):
    api = _api()
    w = random_small_batch(30, n_systems=5, n_range=(5, 60), kind=kind, n_species=2 if kind != "morse" else 1)
    pot = w.potential
    b = _batch(w)
    nl = api.build_neighbor_list(b, pot.cutoff, 0.2)
    pp = api.pair_params_from_spec(pot, prec)
    rng = np.random.default_rng(1)
    lr0, lv0 = rng.normal(size=w.pos.shape), rng.normal(size=w.pos.shape)
    lr = torch.tensor(lr0.T.copy(), device="cuda")
    lv = torch.tensor(lv0.T.copy(), device="cuda")
    tb = torch.zeros(48, dtype=torch.float64, device="cuda")
    dt, wk, accel = 0.01, 0.005, 1.0
    api.ts_pair_adjoint(b, nl, pp, dt, wk, accel, lr, lv, tb)
    lv_ref = lv0 + dt * lr0
    u = accel * lv_ref / w.mass[:, None]
    lr_ref = lr0 + wk * oadj.batch_hvp(w.pos, w.cell, w.sys_offsets, w.species, pot, u)
    tb_ref = wk * oadj.batch_param_vjp(w.pos, w.cell, w.sys_offsets, w.species, pot, u)
    tol = 1e-8 if prec == "f64" else 1e-3
    assert np.abs(lv.T.cpu().numpy() - lv_ref).max() <= 1e-14 * np.abs(lv_ref).max()
    d = lr.T.cpu().numpy() - lr_ref
    assert np.abs(d).max() <= tol * np.abs(lr_ref - lr0).max()
    ns = pot.params.shape[0]
    got = tb.cpu().numpy().reshape(4, 4, 3)[:ns, :ns]
    assert np.abs(got - tb_ref).max() <= tol * np.abs(tb_ref).max()


def test_rdf_and_vjp():
    api = _api()
    w = argon_batch(3, seed=14, reps=(4, 4, 4))
    b = _batch(w)
    n_bins, r_end, sig, r_max = 200, 10.0, 0.05, 10.3
    nl = api.build_neighbor_list(b, r_max, 0.0)
    g = torch.zeros((w.n_systems, n_bins), dtype=torch.float64, device="cuda")
    api.ts_rdf_smeared(b, nl, n_bins, r_end, sig, r_max, g)
    g_ref = oadj.batch_rdf(w.pos, w.cell, w.sys_offsets, n_bins, r_end, sig, r_max)
    assert np.abs(g.cpu().numpy() - g_ref).max() <= 1e-10 * np.abs(g_ref).max()
    target = torch.tensor(g_ref * 1.01, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    dl = torch.zeros_like(g)
    api.ts_rdf_loss(g, target, loss, dl)
    assert abs(loss.item() - oadj.rdf_loss(g_ref, g_ref * 1.01)) <= 1e-10 * loss.item()
    grad = torch.zeros_like(b.pos)
    api.ts_rdf_vjp(b, nl, n_bins, r_end, sig, r_max, dl, grad)
    grad_ref = oadj.rdf_loss_grad(w.pos, w.cell, w.sys_offsets, n_bins, r_end, sig, r_max, g_ref, g_ref * 1.01)
    assert np.abs(grad.T.cpu().numpy() - grad_ref).max() <= 1e-9 * np.abs(grad_ref).max()


# ----------------------------------------------------------------------------- fused step loop


def _run_nve(w, prec, steps, lanes, unfused, use_graph=True, deferred=False):
    import os
    api = _api()
    os.environ["TS_NVE_UNFUSED"] = "1" if unfused else "0"
    try:
        b = _batch(w)
        nl = api.build_neighbor_list(b, w.potential.cutoff, w.skin, bin_factor=2, lanes_per_atom=lanes,
                                     deferred=deferred)
        pp = api.pair_params_from_spec(w.potential, prec)
        F, _, _ = api.compute_forces(b, nl, pp, prec)
        E = torch.zeros(w.n_systems, dtype=torch.float64, device="cuda")
        W = torch.zeros((w.n_systems, 9), dtype=torch.float64, device="cuda")
        nl.status.zero_()
        api.ts_nve_step(b, nl, pp, w.dt, w.accel, steps, F, E, None, W, use_graph=use_graph)
        torch.cuda.synchronize()
        return b, nl, F, E, W
    finally:
        os.environ.pop("TS_NVE_UNFUSED", None)


def test_fused_step_equals_multikernel_step():
    w = argon_batch(3, seed=21, reps=(4, 4, 4))
    ref = _run_nve(w, "f32", 40, 1, unfused=True)
    one = _run_nve(w, "f32", 40, 1, unfused=False, deferred=False)
    one_d = _run_nve(w, "f32", 40, 1, unfused=False, deferred=True)
    four = _run_nve(w, "f32", 40, 4, unfused=False)
    # one lane per atom sums each row in the same order: bit-identical trajectory, and with the
    # synchronous rebuild the same lists (the deferred rebuild builds some lists a step earlier:
    # other reference positions, the same trajectory)
    for run in (one, one_d):
        assert torch.equal(ref[0].pos, run[0].pos) and torch.equal(ref[0].vel, run[0].vel)
        assert torch.equal(ref[2], run[2])
    assert torch.equal(ref[1].n_nbr, one[1].n_nbr)
    assert ref[1].read_status()[2] == one[1].read_status()[2]
    # four lanes per atom change only the float64 summation order of each row
    assert (ref[0].pos - four[0].pos).abs().max().item() <= 1e-10
    assert np.allclose(ref[3].cpu().numpy(), four[3].cpu().numpy(), rtol=1e-9)
    assert np.allclose(ref[4].cpu().numpy(), four[4].cpu().numpy(), rtol=1e-8, atol=1e-12)


@pytest.mark.parametrize("lanes", [2, 8])
def test_fused_lists_match_oracle_at_reference_positions(lanes):
    # after steps with rebuilds inside the step kernel, each system's list is the oracle's pair set at the
    # positions of that system's last rebuild
    w = copper_uneven_batch(5, seed=22, min_sites=32, max_sites=400)
    w.vel[:] = np.random.default_rng(0).normal(0, 0.2, w.vel.shape)
    w.skin = 0.2
    b, nl, F, E, W = _run_nve(w, "f32", 25, lanes, unfused=False)
    assert nl.read_status()[2] > 5
    ref = nl.ref_pos.T.cpu().numpy()
    assert_same_pairs(b, nl, w.potential.cutoff + w.skin, pos=ref)
    # and the final forces, energies and virials are the oracle's at the final positions
    pos = b.positions()
    E_ref, F_ref, W_ref = oforces.batch_efw(pos, w.cell, w.sys_offsets, w.species, w.potential)
    A, se, sw = force_scales(pos, w.cell, w.sys_offsets, w.species, w.potential)
    assert_forces_close(F.T.double().cpu().numpy(), F_ref, A, 1e-5)
    assert np.all(np.abs(E.cpu().numpy() - E_ref) <= 1e-6 * se)
    assert np.all(np.abs(W.cpu().numpy().reshape(-1, 3, 3) - W_ref).max(axis=(1, 2)) <= 1e-6 * sw)


# ----------------------------------------------------------------------------- Langevin


@pytest.mark.parametrize("unfused", [False, True])
def test_langevin_matches_oracle(unfused, monkeypatch):
    # BAOAB steps with the per-atom Philox normals: same counters on both sides, so the trajectories
    # agree to float64 rounding; two calls continue the counter, eager and graph runs are identical.
    # Both step loops: the fused step kernel and the per-atom kernels around the force kernel (the
    # loop of systems too large for LDS).
    monkeypatch.setenv("TS_NVE_UNFUSED", "1" if unfused else "0")
    from oracle import langevin as olang
    api = _api()
    w = argon_batch(2, seed=17, reps=(3, 3, 3))
    pot = w.potential
    kT = np.array([0.02, 0.035])  # eV
    gamma, seed, K, t0 = 0.01, 123456789012345, 12, 5  # gamma in 1/fs
    ref = olang.baoab(w.pos, w.vel, w.mass, w.cell, w.sys_offsets, w.species, pot, w.dt, K, w.accel, gamma, kT,
                      seed, step0=t0)
    runs = []
    for use_graph in (True, False):
        b = _batch(w)
        nl = api.build_neighbor_list(b, pot.cutoff, w.skin)
        pp = api.pair_params_from_spec(pot, "f64")
        F, _, _ = api.compute_forces(b, nl, pp, "f64")
        kTd = torch.tensor(kT, device="cuda")
        ctr = torch.tensor([t0], dtype=torch.int64, device="cuda")
        api.ts_langevin_step(b, nl, pp, w.dt, w.accel, gamma, kTd, seed, ctr, K // 2, F, use_graph=use_graph)
        api.ts_langevin_step(b, nl, pp, w.dt, w.accel, gamma, kTd, seed, ctr, K - K // 2, F, use_graph=use_graph)
        torch.cuda.synchronize()
        assert int(ctr.item()) == t0 + K
        runs.append((b.positions(), b.velocities()))
        assert np.abs(runs[-1][0] - ref["pos"]).max() <= 1e-9
        assert np.abs(runs[-1][1] - ref["vel"]).max() <= 1e-9 * np.abs(ref["vel"]).max()
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])


@pytest.mark.parametrize("reps", [(3, 3, 3), (9, 8, 8)])
def test_langevin_calls_compose_and_reduce_to_nve(reps):
    # properties that hold at any size; 9 x 8 x 8 cells (2304 atoms) exceed the LDS limit of the fused
    # step and run the per-atom loop.  One call of K steps equals K calls of one step bitwise (the
    # counter continues), and without friction the steps are velocity-Verlet ones up to rounding.
    api = _api()
    w = argon_batch(1, seed=23, reps=reps)
    pot = w.potential
    kTd = torch.tensor([0.03], dtype=torch.float64, device="cuda")
    K = 6

    def setup():
        b = _batch(w)
        nl = api.build_neighbor_list(b, pot.cutoff, w.skin)
        pp = api.pair_params_from_spec(pot, "f64")
        F, _, _ = api.compute_forces(b, nl, pp, "f64")
        return b, nl, pp, F

    def langevin(calls, gamma):
        b, nl, pp, F = setup()
        ctr = torch.zeros(1, dtype=torch.int64, device="cuda")
        for k in calls:
            api.ts_langevin_step(b, nl, pp, w.dt, w.accel, gamma, kTd, 99, ctr, k, F)
        torch.cuda.synchronize()
        assert int(ctr.item()) == sum(calls)
        return b.positions(), b.velocities()

    zero = langevin([0], 0.02)  # a call of no steps changes nothing, the counter included
    assert np.array_equal(zero[0], w.pos) and np.array_equal(zero[1], w.vel)
    one, many = langevin([K], 0.02), langevin([1] * K, 0.02)
    assert np.array_equal(one[0], many[0]) and np.array_equal(one[1], many[1])
    still = langevin([K], 0.0)
    b, nl, pp, F = setup()
    api.ts_nve_step(b, nl, pp, w.dt, w.accel, K, F)
    torch.cuda.synchronize()
    L = abs(np.linalg.det(w.cell[0])) ** (1 / 3)
    assert np.abs(still[0] - b.positions()).max() <= 1e-12 * L
    assert np.abs(still[1] - b.velocities()).max() <= 1e-12 * np.abs(b.velocities()).max()
    assert np.abs(one[0] - b.positions()).max() > 1e-6  # the friction and noise did act


# ----------------------------------------------------------------------------- graph export


def _export(api, b, nl, r, cap=None, vec=True):
    n_e = int(nl.n_nbr.sum().item()) if cap is None else cap
    row_ptr = torch.full((b.n_atoms + 1,), -7, dtype=torch.int64, device="cuda")
    offs = torch.full((b.n_systems + 1,), -7, dtype=torch.int64, device="cuda")
    ei = torch.full((2, n_e), -7, dtype=torch.int64, device="cuda")
    sh = torch.full((n_e, 3), -99, dtype=torch.int32, device="cuda")
    vv = torch.full((n_e, 3), np.nan, dtype=torch.float64, device="cuda") if vec else None
    api.ts_graph_export(b, nl, r, row_ptr, offs, ei, sh, vv)
    torch.cuda.synchronize()
    return (row_ptr.cpu().numpy(), offs.cpu().numpy(), ei.cpu().numpy(), sh.cpu().numpy(),
            None if vv is None else vv.cpu().numpy())


@pytest.mark.parametrize("seed,half,r", [(40, False, 2.5), (41, False, 1.7), (42, True, 2.5)])
def test_graph_export_matches_oracle(seed, half, r):
    # every edge, its order, shifts and vectors, the CSR row pointer and the system offsets
    from oracle import graph as ograph
    from oracle.pairs import half_mask
    api = _api()
    w = random_small_batch(seed, n_systems=12, n_range=(1, 70), density=0.9, unwrap_spread=2)
    b = _batch(w)
    nl = api.build_neighbor_list(b, 2.5, 0.3, half=half)
    ref = ograph.mlip_graph(w.pos, w.cell, w.sys_offsets, r)
    if half:  # the half list keeps each pair once
        keep = half_mask(ref["edge_index"][0], ref["edge_index"][1], ref["shift"])
        sys_of = np.repeat(np.arange(w.n_systems), np.diff(w.sys_offsets))
        for k in ("shift", "vec"):
            ref[k] = ref[k][keep]
        ref["edge_index"] = ref["edge_index"][:, keep]
        ref["row_ptr"] = np.concatenate([[0], np.cumsum(np.bincount(ref["edge_index"][0], minlength=w.n_atoms))])
        ref["edge_offsets"] = np.concatenate([[0], np.cumsum(np.bincount(sys_of[ref["edge_index"][0]],
                                                                         minlength=w.n_systems))])
    # no pair within 1e-9 of r_graph, where the two float64 evaluations of |d| could disagree
    assert np.abs(np.linalg.norm(ref["vec"], axis=1) - r).min() > 1e-9
    row_ptr, offs, ei, sh, vv = _export(api, b, nl, r)
    E = int(offs[-1])
    assert E == ref["edge_index"].shape[1] > 0
    assert np.array_equal(row_ptr, ref["row_ptr"]) and np.array_equal(offs, ref["edge_offsets"])
    assert np.array_equal(ei[:, :E], ref["edge_index"])
    assert np.array_equal(sh[:E], ref["shift"])
    assert np.abs(vv[:E] - ref["vec"]).max() <= 1e-12 * max(1.0, np.abs(ref["vec"]).max())
    # capacity 0 and no edge buffers: the counts and offsets only
    rp0 = torch.empty(b.n_atoms + 1, dtype=torch.int64, device="cuda")
    of0 = torch.empty(b.n_systems + 1, dtype=torch.int64, device="cuda")
    api.ts_graph_export(b, nl, r, rp0, of0, None)
    assert np.array_equal(rp0.cpu().numpy(), row_ptr) and np.array_equal(of0.cpu().numpy(), offs)
    # a capacity below E: counts and offsets complete, the first `cap` edges written, nothing beyond
    cap = E // 3
    row_ptr2, offs2, ei2, sh2, _ = _export(api, b, nl, r, cap=cap, vec=False)
    assert np.array_equal(row_ptr2, row_ptr) and np.array_equal(offs2, offs)
    assert np.array_equal(ei2, ref["edge_index"][:, :cap]) and np.array_equal(sh2, ref["shift"][:cap])


def test_graph_export_large_system_sampled():
    # 2304 atoms (the sorted-bin list builder of large systems): the edges of sampled atoms against
    # the oracle's pairs of those rows, and the pair symmetry over the whole graph
    from oracle.pairs import system_pairs
    api = _api()
    w = argon_batch(1, seed=29, reps=(9, 8, 8))
    b = _batch(w)
    nl = api.build_neighbor_list(b, w.potential.cutoff, w.skin)
    r = w.potential.cutoff
    row_ptr, offs, ei, sh, vv = _export(api, b, nl, r)
    E = int(offs[-1])
    assert row_ptr[-1] == E and offs[0] == 0 and np.all(np.diff(row_ptr) >= 0)
    rows = np.random.default_rng(3).choice(w.n_atoms, 24, replace=False)
    p = system_pairs(w.pos, w.cell[0], r, rows=rows)
    for i in rows:
        m = p["i"] == i
        order = np.lexsort((p["S"][m, 2], p["S"][m, 1], p["S"][m, 0], p["j"][m]))
        lo, hi = row_ptr[i], row_ptr[i + 1]
        assert np.all(ei[0, lo:hi] == i)
        assert np.array_equal(ei[1, lo:hi], p["j"][m][order])
        assert np.array_equal(sh[lo:hi], p["S"][m][order])
        assert np.abs(vv[lo:hi] - p["d"][m][order]).max() <= 1e-11
    keys = set(zip(ei[0, :E].tolist(), ei[1, :E].tolist(), map(tuple, sh[:E].tolist())))
    assert all((j, i, (-a, -b_, -c)) in keys for i, j, (a, b_, c) in keys)


@pytest.mark.parametrize("unfused", [False, True])
def test_langevin_fp32_forces_short_run(unfused, monkeypatch):
    # the precision of the benchmark: float32 pair function, float64 integration.  Over three steps
    # the float32 force error (1e-5 relative) moves positions by well under 1e-8 A.
    monkeypatch.setenv("TS_NVE_UNFUSED", "1" if unfused else "0")
    from oracle import langevin as olang
    api = _api()
    w = argon_batch(3, seed=31, reps=(3, 3, 3))
    pot = w.potential
    kT = np.array([0.01, 0.02, 0.03])
    gamma, seed, K = 0.02, 2 ** 40 + 7, 3
    ref = olang.baoab(w.pos, w.vel, w.mass, w.cell, w.sys_offsets, w.species, pot, w.dt, K, w.accel, gamma, kT, seed)
    b = _batch(w)
    nl = api.build_neighbor_list(b, pot.cutoff, w.skin)
    pp = api.pair_params_from_spec(pot, "f32")
    F, _, _ = api.compute_forces(b, nl, pp, "f32")
    ctr = torch.zeros(1, dtype=torch.int64, device="cuda")
    api.ts_langevin_step(b, nl, pp, w.dt, w.accel, gamma, torch.tensor(kT, device="cuda"), seed, ctr, K, F)
    torch.cuda.synchronize()
    assert int(ctr.item()) == K
    assert np.abs(b.positions() - ref["pos"]).max() <= 1e-8
    assert np.abs(b.velocities() - ref["vel"]).max() <= 1e-7 * np.abs(ref["vel"]).max()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_lorentz_berthelot_mixture_forces(prec):
    # a three-species LJ mixture whose table comes from the mixing rules: the package's table on the
    # GPU, the oracle's own table on the CPU
    from oracle.potentials import lorentz_berthelot
    from workloads import PotentialSpec
    api = _api()
    eps, sig = [1.0, 0.6, 1.4], [1.0, 1.15, 0.9]
    w = random_small_batch(77, n_systems=6, n_range=(10, 90), kind="lj", n_species=3, unwrap_spread=1)
    gpu_pot = PotentialSpec("lj", api.lorentz_berthelot(eps, sig), 2.5, True)
    ref_pot = PotentialSpec("lj", lorentz_berthelot(eps, sig), 2.5, True)
    b = _batch(w)
    nl = api.build_neighbor_list(b, 2.5, 0.2, bin_factor=2)
    F, E, W = api.compute_forces(b, nl, api.pair_params_from_spec(gpu_pot, prec), prec)
    E_ref, F_ref, W_ref = oforces.batch_efw(w.pos, w.cell, w.sys_offsets, w.species, ref_pot)
    A, se, sw = force_scales(w.pos, w.cell, w.sys_offsets, w.species, ref_pot)
    assert_forces_close(F.T.double().cpu().numpy(), F_ref, A, 1e-10 if prec == "f64" else 1e-5)
    erel = 1e-10 if prec == "f64" else 1e-6
    assert np.all(np.abs(E.cpu().numpy() - E_ref) <= erel * se + 1e-300)
