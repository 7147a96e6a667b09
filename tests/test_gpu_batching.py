"""GPU parity of the batching paths that small tests do not reach: systems with no atoms anywhere
in a batch (fused step loops, Langevin, the reverse loop, FIRE, forces), the persistent FIRE launch
handing its tail to the per-iteration kernels (more systems than a quarter of the compute units),
and the cell-list build of systems above the LDS limit in sheared cells narrower than twice the
list radius with unwrapped positions, at every bin factor."""
import numpy as np
import pytest

from oracle import adjoint as oadj
from oracle import fire as ofire
from oracle import forces as oforces
from oracle import integrate as ointeg
from oracle import langevin as olang
from oracle import pairs as opairs
from tests.gpu_helpers import assert_forces_close, force_scales
from workloads import argon_batch, copper_uneven_batch, insert_empty_systems, narrow_triclinic_batch

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


# ----------------------------------------------------------------------------- empty systems


def _small_argon(skin=0.05):
    w = argon_batch(2, seed=31, reps=(3, 3, 3))
    w.skin = skin  # a small skin: rebuilds every few steps, so the rotating rebuild lists cycle
    return w


@pytest.mark.parametrize("empty_at", [[0], [0, 1, 2], [2]])
def test_nve_with_empty_systems(empty_at):
    api = _api()
    w = _small_argon()
    we = insert_empty_systems(w, empty_at)
    pot = w.potential
    b = api.Batch.from_workload(we)
    nl = api.build_neighbor_list(b, pot.cutoff, w.skin)
    pp = api.pair_params_from_spec(pot, "f64")
    F, _, _ = api.compute_forces(b, nl, pp, "f64")
    E = torch.zeros(we.n_systems, dtype=torch.float64, device="cuda")
    steps = 40
    api.ts_nve_step(b, nl, pp, w.dt, w.accel, steps, F, E, use_graph=True)
    torch.cuda.synchronize()
    st = nl.read_status()
    assert st[1] == 0 and st[3] == 0 and st[4] == 0
    assert st[2] >= 2 + 6  # the initial builds and several in-loop rebuilds
    ref = ointeg.nve(w.pos, w.vel, w.mass, w.cell, w.sys_offsets, w.species, pot, w.dt, steps, w.accel)
    L = abs(np.linalg.det(w.cell[0])) ** (1 / 3)
    assert np.abs(b.positions() - ref["pos"]).max() <= 1e-10 * L
    full = [s for s in range(we.n_systems) if we.sys_offsets[s + 1] > we.sys_offsets[s]]
    Eg = E.cpu().numpy()
    _, se, _ = force_scales(ref["pos"], w.cell, w.sys_offsets, w.species, pot)
    assert np.all(np.abs(Eg[full] - ref["energy"]) <= 1e-10 * se)
    empty = [s for s in range(we.n_systems) if s not in full]
    assert np.all(Eg[empty] == 0.0)


def test_langevin_with_empty_systems():
    api = _api()
    w = _small_argon()
    we = insert_empty_systems(w, [0, 1])
    pot = w.potential
    kT_full = np.array([0.02, 0.03])
    kT = np.array([0.5, 0.02, 0.7, 0.03])  # the empty systems' temperatures are never used
    gamma, seed, K = 0.01, 77, 16
    ref = olang.baoab(w.pos, w.vel, w.mass, w.cell, w.sys_offsets, w.species, pot, w.dt, K, w.accel, gamma, kT_full,
                      seed)
    b = api.Batch.from_workload(we)
    nl = api.build_neighbor_list(b, pot.cutoff, w.skin)
    pp = api.pair_params_from_spec(pot, "f64")
    F, _, _ = api.compute_forces(b, nl, pp, "f64")
    ctr = torch.zeros(1, dtype=torch.int64, device="cuda")
    api.ts_langevin_step(b, nl, pp, w.dt, w.accel, gamma, torch.tensor(kT, device="cuda"), seed, ctr, K, F)
    torch.cuda.synchronize()
    assert np.abs(b.positions() - ref["pos"]).max() <= 1e-9
    assert nl.read_status()[1] == 0


def test_adjoint_segment_with_empty_systems():
    # the recorded segment and its reverse pass on a batch with empty systems equal those of the same
    # atoms without them, and the reverse pass matches the oracle's
    api = _api()
    w = _small_argon()
    we = insert_empty_systems(w, [0, 2])
    pot = w.potential
    steps = 12
    out = []
    for ww in (w, we):
        b = api.Batch.from_workload(ww)
        nl = api.build_neighbor_list(b, pot.cutoff, w.skin)
        pp = api.pair_params_from_spec(pot, "f64")
        F, _, _ = api.compute_forces(b, nl, pp, "f64")
        traj = torch.zeros((steps + 1, 3, b.n_atoms), dtype=torch.float64, device="cuda")
        api.ts_nve_record(b, nl, pp, w.dt, w.accel, steps, F, traj)
        rng = np.random.default_rng(3)
        lr = torch.tensor(rng.normal(size=(3, b.n_atoms)), device="cuda")
        lv = torch.tensor(rng.normal(size=(3, b.n_atoms)), device="cuda")
        tb = torch.zeros(48, dtype=torch.float64, device="cuda")
        api.ts_adjoint_segment(b, nl, pp, traj, steps, w.dt, w.accel, True, True, lr, lv, tb)
        torch.cuda.synchronize()
        assert nl.read_status()[1] == 0
        out.append((traj.cpu().numpy(), lr.cpu().numpy(), lv.cpu().numpy(), tb.cpu().numpy()))
    for a, c in zip(out[0][:3], out[1][:3]):
        assert np.array_equal(a, c)
    # the parameter gradient sums per-system slots, whose summation tree shifts with the empty ones
    assert np.abs(out[0][3] - out[1][3]).max() <= 1e-13 * np.abs(out[0][3]).max()
    # the oracle's reverse pass over the same recorded positions
    rng = np.random.default_rng(3)
    lr0, lv0 = rng.normal(size=(3, w.n_atoms)).T, rng.normal(size=(3, w.n_atoms)).T
    positions = [out[0][0][k].T for k in range(steps + 1)]
    lr_ref, lv_ref, tb_ref = oadj.reverse_nve(positions, w.mass, w.cell, w.sys_offsets, w.species, pot, w.dt,
                                              w.accel, lr0, lv0)
    assert np.abs(out[1][1].T - lr_ref).max() <= 1e-8 * np.abs(lr_ref).max()
    assert np.abs(out[1][2].T - lv_ref).max() <= 1e-8 * np.abs(lv_ref).max()
    assert np.abs(out[1][3].reshape(4, 4, 3)[0, 0] - tb_ref[0, 0]).max() <= 1e-8 * np.abs(tb_ref).max()


@pytest.mark.parametrize("persistent", [False, True])
def test_fire_and_forces_with_empty_systems(persistent):
    api = _api()
    w = copper_uneven_batch(3, seed=33, min_sites=32, max_sites=90)
    we = insert_empty_systems(w, [0, 2])
    pot = w.potential
    cfgd = dict(w.extra["fire"])
    cfgd["relax_cell"] = False
    b = api.Batch.from_workload(we)
    nl = api.build_neighbor_list(b, pot.cutoff, w.skin)
    pp = api.pair_params_from_spec(pot, "f64")
    F, E, Wv = api.compute_forces(b, nl, pp, "f64")
    E_ref, F_ref, _ = oforces.batch_efw(w.pos, w.cell, w.sys_offsets, w.species, pot)
    A, _, _ = force_scales(w.pos, w.cell, w.sys_offsets, w.species, pot)
    assert_forces_close(F.T.cpu().numpy(), F_ref, A, 1e-10)
    cfg = api.fire_config(**cfgd)
    fs = api.FireState(b, cfg)
    n_it = 15
    api.ts_fire_step(b, fs, cfg, nl, pp, n_it, F, persistent=persistent)
    torch.cuda.synchronize()
    full = [s for s in range(we.n_systems) if we.sys_offsets[s + 1] > we.sys_offsets[s]]
    ocfg = ofire.FireConfig(**cfgd)
    for k, s in enumerate(full):
        sl = w.system(k)
        st = ofire.init_state(w.pos[sl], w.cell[k], ocfg)
        ofire.fire_iterate(st, w.species[sl], w.mass[sl], pot, ocfg, n_it)
        L = abs(np.linalg.det(w.cell[k])) ** (1 / 3)
        assert np.abs(b.positions()[we.system(s)] - st.pos).max() <= 1e-9 * L
        assert fs.n_iter[s].item() == st.n_iter


# ----------------------------------------------------------------------------- persistent FIRE hand-off


def _cus():
    return torch.cuda.get_device_properties(0).multi_processor_count


def _fire_handoff_batch(extra_systems):
    # more systems than a quarter of the compute units: the persistent launch hands its last
    # systems to the per-iteration kernels
    n_sys = _cus() // 4 + extra_systems
    w = copper_uneven_batch(n_sys, seed=34, min_sites=32, max_sites=72)
    return w


def test_fire_persistent_handoff_matches_oracle():
    api = _api()
    w = _fire_handoff_batch(8)
    pot = w.potential
    cfgd = dict(w.extra["fire"])  # positions and cell
    b = api.Batch.from_workload(w)
    nl = api.build_neighbor_list(b, pot.cutoff, w.skin)
    pp = api.pair_params_from_spec(pot, "f64")
    cfg = api.fire_config(**cfgd)
    fs = api.FireState(b, cfg)
    F = api.force_buffer(b, "f64")
    E = torch.zeros(w.n_systems, dtype=torch.float64, device="cuda")
    n_it = 30  # below the tail length: every system completes exactly this budget
    api.ts_fire_step(b, fs, cfg, nl, pp, n_it, F, E, persistent=True)
    torch.cuda.synchronize()
    st_nl = nl.read_status()
    assert st_nl[1] == 0 and st_nl[3] == 0 and st_nl[4] == 0
    pos, cells = b.positions(), b.cells()
    ocfg = ofire.FireConfig(**cfgd)
    it = fs.n_iter.cpu().numpy()
    conv = fs.converged.cpu().numpy()
    for s in range(w.n_systems):
        sl = w.system(s)
        st = ofire.init_state(w.pos[sl], w.cell[s], ocfg)
        e, f, _ = ofire.fire_iterate(st, w.species[sl], w.mass[sl], pot, ocfg, n_it)
        L = abs(np.linalg.det(w.cell[s])) ** (1 / 3)
        assert np.abs(pos[sl] - st.pos).max() <= 1e-9 * L, s
        assert np.abs(cells[s] - st.cell).max() <= 1e-9 * L, s
        assert it[s] == st.n_iter and bool(conv[s]) == st.converged, s
        assert abs(fs.dt[s].item() - st.dt) <= 1e-12 * st.dt, s
        assert abs(fs.alpha[s].item() - st.alpha) <= 1e-12 * st.alpha, s
        assert fs.n_pos[s].item() == st.n_pos, s
        assert abs(fs.deform_vel[s].cpu().numpy().reshape(3, 3) - st.deform_vel).max() <= 1e-9 * (
            1.0 + np.abs(st.deform_vel).max()), s
        assert abs(E[s].item() - e) <= 1e-10 * max(1.0, abs(e)), s
    assert (it == n_it).sum() >= w.n_systems - 2  # (almost) nobody converged: the budget straddled the hand-off


def test_fire_relax_handoff_certified():
    # relaxation to convergence through repeated calls (persistent launch + bounded tail), certified
    # per system by the oracle's float64 forces and cell force at the final state
    api = _api()
    w = _fire_handoff_batch(24)
    pot = w.potential
    cfgd = dict(w.extra["fire"])
    b = api.Batch.from_workload(w)
    nl = api.build_neighbor_list(b, pot.cutoff, 1.0, bin_factor=2, margin=1.2)
    pp = api.pair_params_from_spec(pot, "f32")
    cfg = api.fire_config(**cfgd)
    fs = api.FireState(b, cfg)
    F = api.force_buffer(b, "f32")
    calls = api.fire_relax(b, fs, cfg, nl, pp, F)
    torch.cuda.synchronize()
    st_nl = nl.read_status()
    assert st_nl[1] == 0 and st_nl[3] == 0 and st_nl[4] == 0
    assert fs.converged.all().item(), (calls, fs.n_iter.cpu().numpy())
    pos, cells = b.positions(), b.cells()
    rng = np.random.default_rng(5)
    for s in sorted(rng.choice(w.n_systems, size=20, replace=False)):
        sl = w.system(s)
        e, f, Wv = oforces.system_efw(pos[sl], cells[s], w.species[sl], pot.params, pot.kind, pot.cutoff, False)
        assert np.linalg.norm(f, axis=1).max() < cfgd["fmax"] * 1.001, s
        D = fs.deform[s].cpu().numpy().reshape(3, 3)
        assert np.abs(ofire.cell_force(D, Wv, f.shape[0])).max() < cfgd["fmax"] * 1.001, s


# ----------------------------------------------------------------------------- cell list of large systems


@pytest.mark.parametrize("bin_factor,half", [(1, False), (2, False), (3, True), (4, False), (4, True)])
def test_cell_list_narrow_triclinic_unwrapped(bin_factor, half):
    api = _api()
    w = narrow_triclinic_batch(40 + bin_factor, n_systems=2, empty_first=True)
    r_list = 2.8
    b = api.Batch.from_workload(w)
    nl = api.build_neighbor_list(b, 2.5, 0.3, bin_factor=bin_factor, half=half)
    st = nl.read_status()
    assert st[1] == 0 and st[3] == 0 and st[4] == 0
    i_all, j_all, s0, s1, s2 = nl.entries()
    rng = np.random.default_rng(bin_factor)
    for s in range(1, w.n_systems):
        sl = w.system(s)
        n = sl.stop - sl.start
        assert n > 2048
        rows = np.sort(rng.choice(n, size=24, replace=False))
        o = opairs.system_pairs(w.pos[sl], w.cell[s], r_list, rows=rows, half=half)
        sel = np.isin(i_all, sl.start + rows)
        g = dict(i=i_all[sel] - sl.start, j=j_all[sel], S=np.stack([s0[sel], s1[sel], s2[sel]], 1))
        d = w.pos[sl][g["j"]] - w.pos[sl][g["i"]] + g["S"] @ w.cell[s]
        g["r2"] = (d * d).sum(1)
        kg, ko = opairs.pair_keys(g, r_list, 1e-9), opairs.pair_keys(o, r_list, 1e-9)
        assert kg.shape == ko.shape and np.array_equal(kg, ko), s
        # several images of one (i, j) pair: the cells are narrower than 2 r_list
        assert np.unique(ko[:, 1:3], axis=0).shape[0] < ko.shape[0]
        # rows are stored in the canonical (j, S0, S1, S2) order
        i0 = sl.start + rows[0]
        row = np.stack([j_all[i_all == i0], s0[i_all == i0], s1[i_all == i0], s2[i_all == i0]], 1)
        assert np.array_equal(row, row[np.lexsort(row.T[::-1])])
    # an update after moving some atoms rebuilds exactly the systems over the bound
    pos = w.pos.copy()
    pos[w.system(2).start + 5] += np.array([0.2, 0.0, 0.0])  # beyond skin / 2 = 0.15
    b.pos.copy_(torch.tensor(pos.T.copy()))
    nl.status.zero_()
    api.ts_neighbor_build(b, nl, force=False)
    assert nl.read_status()[2] == 1


@pytest.mark.parametrize("narrow,half", [(4.2, False), (4.2, True), (2.5, False)])
def test_row_rebuild_large_narrow_triclinic(narrow, half):
    """Systems of 1200-2048 atoms take the row rebuild's large-system kernel (fractional coordinates
    alone in LDS); their sheared cells are narrower than 2 r_list along one direction (2.5: narrower
    than r_list itself, three images of one pair), so the slab prefilter and the multi-image exact
    pass build the rows.  Sampled rows must equal the oracle's pair sets, in canonical order."""
    api = _api()
    w = narrow_triclinic_batch(60 + int(10 * narrow) + int(half), n_systems=2, n_range=(1200, 2048), narrow=narrow,
                               empty_first=True)
    r_list = 2.8
    b = api.Batch.from_workload(w)
    assert 947 < b.max_system_atoms <= 2048
    nl = api.build_neighbor_list(b, 2.5, 0.3, bin_factor=2, half=half)
    st = nl.read_status()
    assert st[1] == 0 and st[3] == 0 and st[4] == 0
    i_all, j_all, s0, s1, s2 = nl.entries()
    rng = np.random.default_rng(int(10 * narrow))
    for s in range(1, w.n_systems):
        sl = w.system(s)
        n = sl.stop - sl.start
        rows = np.sort(rng.choice(n, size=32, replace=False))
        o = opairs.system_pairs(w.pos[sl], w.cell[s], r_list, rows=rows, half=half)
        sel = np.isin(i_all, sl.start + rows)
        g = dict(i=i_all[sel] - sl.start, j=j_all[sel], S=np.stack([s0[sel], s1[sel], s2[sel]], 1))
        d = w.pos[sl][g["j"]] - w.pos[sl][g["i"]] + g["S"] @ w.cell[s]
        g["r2"] = (d * d).sum(1)
        kg, ko = opairs.pair_keys(g, r_list, 1e-9), opairs.pair_keys(o, r_list, 1e-9)
        assert kg.shape == ko.shape and np.array_equal(kg, ko), s
        assert np.unique(ko[:, 1:3], axis=0).shape[0] < ko.shape[0]  # several images of one pair
        for r in rows[:8]:
            m = i_all == sl.start + r
            row = np.stack([j_all[m], s0[m], s1[m], s2[m]], 1)
            assert np.array_equal(row, row[np.lexsort(row.T[::-1])])


# ----------------------------------------------------------------------------- overflow recovery


def test_nve_run_recovers_from_list_overflow():
    # a list whose capacity is exactly the largest row at the start overflows once thermal motion
    # packs one more neighbor into some row; nve_run restores the state of the call's start, regrows
    # the list and replays, so the trajectory equals a run with ample capacity (float64, up to the
    # summation order of rows of different content)
    api = _api()
    w = argon_batch(2, seed=36, reps=(3, 3, 3))
    pot = w.potential
    pp = api.pair_params_from_spec(pot, "f64")
    probe = api.Batch.from_workload(w)
    nl0 = api.build_neighbor_list(probe, pot.cutoff, w.skin)
    tight = int(nl0.read_status()[0])
    runs = []
    for cap in (tight, None):
        b = api.Batch.from_workload(w)
        if cap is None:
            nl = api.build_neighbor_list(b, pot.cutoff, w.skin, margin=1.5)
        else:
            nl = api.NeighborList(b, pot.cutoff, w.skin, max_nbr=cap)
            api.ts_neighbor_build(b, nl, force=True)
            assert nl.read_status()[1] == 0
        F, _, _ = api.compute_forces(b, nl, pp, "f64")
        replays = api.nve_run(b, nl, pp, w.dt, w.accel, 300, F, chunk=50)
        runs.append((b.positions(), replays, nl.max_nbr))
    assert runs[0][1] >= 1 and runs[0][2] > tight  # the tight list overflowed and was regrown
    assert runs[1][1] == 0
    L = abs(np.linalg.det(w.cell[0])) ** (1 / 3)
    assert np.abs(runs[0][0] - runs[1][0]).max() <= 1e-9 * L
