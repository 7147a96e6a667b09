"""Pins of the oracle's integrator, rebuild test, FIRE and adjoint against closed forms and FD."""
import numpy as np
import pytest

from oracle import adjoint, fire, forces, integrate, pairs
from tests.lattice import fcc_shells
from workloads import (PotentialSpec, argon_single, fcc_cell, lj_argon_params, morse_copper_params,
                       random_small_batch, supercell)


def _chain(delta0, w, eps=1.0):
    """Two soft spheres (sigma = 1) in a 1.8-long periodic cell, touching each other and the
    other's image: for |delta| < 0.1 the relative coordinate is an exact harmonic oscillator."""
    pot = PotentialSpec("soft_sphere", np.array([[[eps, 1.0, 0.0]]]), 1.0)
    pos = np.array([[0.0, 5.0, 5.0], [0.9 + delta0, 5.0, 5.0]])
    vel = np.array([[-0.5 * w, 0.0, 0.0], [0.5 * w, 0.0, 0.0]])
    cell = np.diag([1.8, 10.0, 10.0])[None]
    return pot, pos, vel, cell


def test_velocity_verlet_harmonic_chain_closed_form():
    eps, dt, n = 1.0, 0.1, 200
    pot, pos, vel, cell = _chain(0.03, 0.1, eps)
    mass = np.ones(2)
    offs = np.array([0, 2])
    sp = np.zeros(2, np.int32)
    out = integrate.nve(pos, vel, mass, cell, offs, sp, pot, dt, n, accel=1.0, record_every=1)
    omega2 = 4.0 * eps
    theta = np.arccos(1.0 - 0.5 * omega2 * dt * dt)
    A = 0.03
    d1 = A + dt * 0.1 - 0.5 * dt * dt * omega2 * A
    B = (d1 - A * np.cos(theta)) / np.sin(theta)
    inv = []
    for k, (p, v, _) in enumerate(out["traj"]):
        delta = p[1, 0] - p[0, 0] - 0.9
        assert abs(delta - (A * np.cos(k * theta) + B * np.sin(k * theta))) < 1e-13
        vd = v[1, 0] - v[0, 0]
        inv.append(0.5 * vd * vd + 0.5 * omega2 * (1.0 - omega2 * dt * dt / 4.0) * delta * delta)
    assert np.ptp(inv) < 1e-15
    # momentum is conserved exactly by pair forces
    assert abs(out["vel"][:, 0].sum()) < 1e-15


def _argon_small():
    w = argon_single(seed=11)
    basis, cell0 = fcc_cell(5.26)
    pos, cell = supercell(basis, cell0, (3, 3, 3))
    rng = np.random.default_rng(11)
    pos = pos + rng.normal(0, 0.05, pos.shape)
    vel = w.vel[:pos.shape[0]] - w.vel[:pos.shape[0]].mean(0)
    return w, pos, vel, cell


@pytest.mark.slow
def test_nve_energy_drift_second_order():
    w, pos, vel, cell = _argon_small()
    n = pos.shape[0]
    mass = np.full(n, 39.948)
    offs = np.array([0, n])
    sp = np.zeros(n, np.int32)
    pot = lj_argon_params()
    drift = []
    for dt, steps in ((2.0, 50), (1.0, 100)):
        out = integrate.nve(pos, vel, mass, cell[None], offs, sp, pot, dt, steps, w.accel, record_every=1)
        etot = [e[0] + integrate.kinetic_energy(v, mass, offs, w.kinetic_factor)[0] for (_, v, e) in out["traj"]]
        drift.append(np.abs(np.array(etot) - etot[0]).max())
        ke0 = integrate.kinetic_energy(vel, mass, offs, w.kinetic_factor)[0]
        assert drift[-1] <= 1e-3 * ke0
    assert 2.5 < drift[0] / drift[1] < 6.5, drift


def test_rebuild_bound_keeps_every_pair():
    rng = np.random.default_rng(5)
    w = random_small_batch(21, n_systems=3, n_range=(10, 30), density=0.9)
    rc, skin = 1.6, 0.3
    r_list = rc + skin
    for s in range(w.n_systems):
        sl = w.system(s)
        ref_pos, ref_cell = w.pos[sl], w.cell[s]
        listed = set(map(tuple, pairs.pair_keys(pairs.system_pairs(ref_pos, ref_cell, r_list), r_list)))
        for trial in range(20):
            strain = rng.uniform(-1, 1, (3, 3)) * (0.02 if trial % 2 else 0.0)
            cell = ref_cell @ (np.eye(3) + strain)
            M = np.linalg.inv(ref_cell) @ cell
            delta = rng.normal(size=ref_pos.shape)
            delta /= np.linalg.norm(delta, axis=1, keepdims=True)
            budget = 0.5 * (skin - r_list * np.linalg.norm(M - np.eye(3)))
            if budget <= 0:
                continue
            delta *= rng.uniform(0, 0.999 * budget, (ref_pos.shape[0], 1))
            pos = ref_pos @ M + delta
            assert not integrate.rebuild_needed(pos, ref_pos, cell, ref_cell, skin, r_list)
            now = set(map(tuple, pairs.pair_keys(pairs.system_pairs(pos, cell, rc), rc)))
            assert now <= listed
    # and the test is not vacuous: two atoms just outside the list radius, each moved by a bit more
    # than skin/2 toward the other, come within r_c and the bound asks for a rebuild
    cell = np.eye(3) * 10.0
    ref = np.array([[1.0, 1.0, 1.0], [1.0 + r_list + 1e-3, 1.0, 1.0]])
    now = ref + np.array([[0.16, 0, 0], [-0.16, 0, 0]])
    assert integrate.rebuild_needed(now, ref, cell, cell, skin, r_list)
    assert pairs.system_pairs(ref, cell, r_list)["i"].size == 0
    assert pairs.system_pairs(now, cell, rc)["i"].size == 2


def test_fire_harmonic_chain_converges():
    pot, pos, _, cell = _chain(0.05, 0.0)
    cfg = fire.FireConfig(dt_start=0.05, dt_max=0.5, fmax=1e-8, max_iter=10000)
    st = fire.init_state(pos, cell[0], cfg)
    log = []
    fire.fire_iterate(st, np.zeros(2, np.int32), np.ones(2), pot, cfg, 10000, log=log)
    assert st.converged
    assert abs(st.pos[1, 0] - st.pos[0, 0] - 0.9) < 1e-8
    # the state machine: no power test on the first iteration, dt capped, alpha reset after P <= 0
    assert log[0]["branch"] == 0 and all(e["dt"] <= cfg.dt_max for e in log)
    for e in log:
        if e["branch"] == -1:
            assert e["alpha"] == cfg.alpha_start


def test_generalized_cell_force_is_minus_dE_dY():
    w = random_small_batch(31, n_systems=1, n_range=(6, 10), kind="lj", n_species=2)
    pot = w.potential
    h0, sp = w.cell[0], w.species
    q = w.pos @ np.linalg.inv(np.eye(3))
    D = np.eye(3) + np.array([[0.02, 0.01, -0.03], [0.0, -0.01, 0.02], [0.015, 0.0, 0.01]])
    n = q.shape[0]

    def energy(Dm):
        return forces.system_efw(q @ Dm, h0 @ Dm, sp, pot.params, pot.kind, pot.cutoff, pot.shift_energy)[0]

    _, F, W = forces.system_efw(q @ D, h0 @ D, sp, pot.params, pot.kind, pot.cutoff, pot.shift_energy)
    G = fire.cell_force(D, W, n)
    h = 1e-6
    for a in range(3):
        for b in range(3):
            Dp, Dm = D.copy(), D.copy()
            Dp[a, b] += h
            Dm[a, b] -= h
            dE_dY = (energy(Dp) - energy(Dm)) / (2 * h) / n
            assert abs(-dE_dY - G[a, b]) < 1e-6 * max(np.abs(G).max(), 1e-4)


def test_fire_cell_relaxes_fcc_morse_to_lattice_minimum():
    pot = morse_copper_params()
    shells_at = lambda a: fcc_shells(a, pot.cutoff)  # noqa: E731
    D_, al, r0 = 0.3429, 1.3588, 2.866
    phi = lambda r: D_ * (np.exp(-2 * al * (r - r0)) - 2 * np.exp(-al * (r - r0)))  # noqa: E731
    e_atom = lambda a: 0.5 * sum(c * phi(r) for r, c in shells_at(a).items())  # noqa: E731
    # golden-section search of the lattice sum (independent of the oracle's pair search)
    lo, hi = 3.2, 4.2
    g = (np.sqrt(5) - 1) / 2
    for _ in range(80):
        c, d = hi - g * (hi - lo), lo + g * (hi - lo)
        if e_atom(c) < e_atom(d):
            hi = d
        else:
            lo = c
    a_star = 0.5 * (lo + hi)
    basis, cell0 = fcc_cell(3.61)
    pos, cell = supercell(basis, cell0, (1, 1, 1))
    strain = np.array([[0.03, 0.01, 0.0], [0.01, -0.02, 0.005], [0.0, 0.005, 0.01]])
    pos, cell = pos @ (np.eye(3) + strain), cell @ (np.eye(3) + strain)
    cfg = fire.FireConfig(fmax=1e-7, relax_cell=True, max_iter=20000)
    st = fire.init_state(pos, cell, cfg)
    e, F, W = fire.fire_iterate(st, np.zeros(4, np.int32), np.full(4, 63.546), pot, cfg, cfg.max_iter)
    assert st.converged
    metric = st.cell @ st.cell.T
    np.testing.assert_allclose(metric, np.eye(3) * a_star ** 2, atol=1e-5)
    assert abs(e / 4 - e_atom(a_star)) < 1e-9


def test_pair_hvp_and_param_vjp_by_fd():
    for kind, seed in (("lj", 41), ("morse", 42), ("soft_sphere", 43)):
        w = random_small_batch(seed, n_systems=1, n_range=(8, 14), kind=kind, n_species=2, unwrap_spread=1)
        pot = w.potential
        pos, cell, sp = w.pos, w.cell[0], w.species
        rng = np.random.default_rng(seed)
        u = rng.normal(size=pos.shape)
        Ju = adjoint.system_hvp(pos, cell, sp, pot, u)
        h = 1e-6
        fp = forces.system_efw(pos + h * u, cell, sp, pot.params, pot.kind, pot.cutoff, False)[1]
        fm = forces.system_efw(pos - h * u, cell, sp, pot.params, pot.kind, pot.cutoff, False)[1]
        scale = np.abs(Ju).max()
        np.testing.assert_allclose(Ju, (fp - fm) / (2 * h), atol=1e-6 * scale)
        tb = adjoint.system_param_vjp(pos, cell, sp, pot, u)
        ns = pot.params.shape[0]
        for a in range(ns):
            for b in range(ns):
                for k in range(3 if kind == "morse" else 2):
                    # each (a, b) slot is its own parameter here (params[a,b] and params[b,a] separate)
                    P1, P2 = pot.params.copy(), pot.params.copy()
                    st = 1e-6 * pot.params[a, b, k]
                    P1[a, b, k] += st
                    P2[a, b, k] -= st
                    f1 = forces.system_efw(pos, cell, sp, P1, pot.kind, pot.cutoff, False)[1]
                    f2 = forces.system_efw(pos, cell, sp, P2, pot.kind, pot.cutoff, False)[1]
                    fd = float((u * (f1 - f2)).sum() / (2 * st))
                    assert abs(fd - tb[a, b, k]) < 1e-5 * max(abs(tb).max(), 1e-8), (kind, a, b, k)


def test_reverse_pass_matches_fd_of_trajectory():
    w = random_small_batch(51, n_systems=2, n_range=(6, 9), kind="lj", density=0.6)
    pot, dt, steps = w.potential, 0.004, 12
    rng = np.random.default_rng(0)
    cr, cv = rng.normal(size=w.pos.shape), rng.normal(size=w.pos.shape)

    def loss(pos0, params):
        p = PotentialSpec(pot.kind, params, pot.cutoff, pot.shift_energy)
        traj, vT = adjoint.trajectory_positions(pos0, w.vel, w.mass, w.cell, w.sys_offsets, w.species, p, dt,
                                                steps, 1.0)
        return float((cr * traj[-1]).sum() + (cv * vT).sum())

    traj, _ = adjoint.trajectory_positions(w.pos, w.vel, w.mass, w.cell, w.sys_offsets, w.species, pot, dt, steps,
                                           1.0)
    lr, lv, tb = adjoint.reverse_nve(traj, w.mass, w.cell, w.sys_offsets, w.species, pot, dt, 1.0, cr, cv)
    h = 1e-6
    for _ in range(4):
        dirn = rng.normal(size=w.pos.shape)
        fd = (loss(w.pos + h * dirn, pot.params) - loss(w.pos - h * dirn, pot.params)) / (2 * h)
        assert abs(fd - float((lr * dirn).sum())) < 1e-6 * max(abs(fd), 1.0)
    for k in range(2):
        P1, P2 = pot.params.copy(), pot.params.copy()
        st = 1e-6 * pot.params[0, 0, k]
        P1[0, 0, k] += st
        P2[0, 0, k] -= st
        fd = (loss(w.pos, P1) - loss(w.pos, P2)) / (2 * st)
        assert abs(fd - tb[0, 0, k]) < 1e-6 * max(abs(fd), 1.0)


def test_rdf_of_perfect_fcc_is_shell_sum():
    a, sig = 5.26, 0.05
    basis, cell0 = fcc_cell(a)
    pos, cell = supercell(basis, cell0, (3, 3, 3))
    n_bins, r_end, r_max = 200, 10.0, 10.3
    g = adjoint.system_rdf(pos, cell, n_bins, r_end, sig, r_max)
    rb = adjoint.rdf_bins(n_bins, r_end)
    rho = pos.shape[0] / abs(np.linalg.det(cell))
    ref = np.zeros(n_bins)
    for r, c in fcc_shells(a, r_max).items():
        ref += c * np.exp(-(rb - r) ** 2 / (2 * sig * sig)) / np.sqrt(2 * np.pi * sig * sig)
    ref /= 4 * np.pi * rb * rb * rho
    np.testing.assert_allclose(g, ref, rtol=1e-12, atol=1e-14)


def test_rdf_loss_gradient_by_fd():
    w = random_small_batch(61, n_systems=2, n_range=(10, 16), kind="lj", density=0.8)
    n_bins, r_end, sig, r_max = 40, 2.0, 0.1, 2.6
    rng = np.random.default_rng(2)
    g = adjoint.batch_rdf(w.pos, w.cell, w.sys_offsets, n_bins, r_end, sig, r_max)
    target = g * (1 + 0.1 * rng.normal(size=g.shape))
    grad = adjoint.rdf_loss_grad(w.pos, w.cell, w.sys_offsets, n_bins, r_end, sig, r_max, g, target)
    h = 1e-6
    for _ in range(4):
        dirn = rng.normal(size=w.pos.shape)
        lp = adjoint.rdf_loss(adjoint.batch_rdf(w.pos + h * dirn, w.cell, w.sys_offsets, n_bins, r_end, sig, r_max),
                              target)
        lm = adjoint.rdf_loss(adjoint.batch_rdf(w.pos - h * dirn, w.cell, w.sys_offsets, n_bins, r_end, sig, r_max),
                              target)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - float((grad * dirn).sum())) < 1e-6 * max(abs(fd), 1e-6)
