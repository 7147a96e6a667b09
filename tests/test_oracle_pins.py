"""Pins of oracle parts whose plausible mistakes the other oracle tests would not catch: the FIRE
step-size schedule and the order of mixing and kick, the BAOAB splitting order, the in-flight
batching schedule, and the per-atom pair-magnitude sums that scale every force tolerance."""
import numpy as np

from oracle import autobatch, fire, forces, langevin
from tests.lattice import fcc_shells
from workloads import PotentialSpec, fcc_cell, supercell

_SS = PotentialSpec("soft_sphere", np.array([[[1.0, 1.0, 0.0]]]), 1.0)


def _chain_from_rest(u0):
    """Two unit soft spheres in a 1.8-long periodic cell: atom 1 touches atom 0 and atom 0's image,
    so the relative coordinate u = x1 - x0 - 0.9 feels the exact linear force -4 u (|u| < 0.1) while
    the center of mass stays at rest."""
    pos = np.array([[0.0, 5.0, 5.0], [0.9 + u0, 5.0, 5.0]])
    cell = np.diag([1.8, 10.0, 10.0])
    return pos, cell


def test_fire_schedule_closed_form():
    """One degree of freedom from rest (Bitzek et al. 2006 with the semi-implicit Euler step): velocity
    and force stay parallel, so the mixing is the identity and the trajectory is the symplectic Euler
    map (w += -4 u dt, u += w dt) under the schedule: dt constant for the first N_min positive-power
    iterations, then dt = min(f_inc dt, dt_max) and alpha = f_alpha alpha on each later one (no power
    test on iteration 0); at the first P <= 0 (u has crossed 0) v = 0, dt = f_dec dt, alpha =
    alpha_start, n_pos = 0.  An increase one iteration early (n_pos >= N_min) or late (test before
    the increment), or a power test on iteration 0, changes dt by 10 % at some k."""
    cfg = fire.FireConfig(dt_start=0.01, dt_max=0.05, alpha_start=0.1, f_inc=1.1, f_dec=0.5, f_alpha=0.99,
                          n_min=5, fmax=1e-12, max_iter=1000)
    pos, cell = _chain_from_rest(0.05)
    st = fire.init_state(pos, cell, cfg)
    sp, m = np.zeros(2, np.int32), np.ones(2)
    # expected trajectory of (u, w) and of the per-system state
    u, w = 0.05, 0.0
    dt, alpha, n_pos = cfg.dt_start, cfg.alpha_start, 0
    reset_at, capped = None, False
    for k in range(60):
        if k > 0:
            if u * w < 0.0:  # P = g . v = -2 u w (v0 = -w/2, v1 = w/2, g = (2u, -2u))
                n_pos += 1
                if n_pos > cfg.n_min:
                    dt = min(cfg.dt_start * cfg.f_inc ** (n_pos - cfg.n_min), cfg.dt_max)
                    alpha = cfg.alpha_start * cfg.f_alpha ** (n_pos - cfg.n_min)
                    capped |= dt == cfg.dt_max
            else:
                reset_at = k
                w = 0.0
                dt, alpha, n_pos = dt * cfg.f_dec, cfg.alpha_start, 0
        w = w - 4.0 * u * dt
        u = u + w * dt
        fire.fire_iterate(st, sp, m, _SS, cfg, 1)
        got_u = st.pos[1, 0] - st.pos[0, 0] - 0.9
        got_w = st.vel[1, 0] - st.vel[0, 0]
        assert abs(st.dt - dt) <= 1e-13 * dt, (k, st.dt, dt)
        assert abs(st.alpha - alpha) <= 1e-13 * alpha, (k, st.alpha, alpha)
        assert st.n_pos == n_pos, (k, st.n_pos, n_pos)
        assert abs(got_u - u) < 1e-12 and abs(got_w - w) < 1e-12, (k, got_u, u, got_w, w)
        assert abs(st.pos[0, 0] + st.pos[1, 0] - 0.9 - 0.05) < 1e-12  # center of mass at rest
        if reset_at is not None and k >= reset_at + 2:
            break
    # the run covered the first increase (k = N_min + 1), the cap and the first reset
    assert reset_at is not None and reset_at > 20 and capped
    assert dt < cfg.dt_max


def _four_chain(disp):
    """Four unit soft spheres 0.9 apart in a 3.6-long periodic cell: nearest neighbours touch,
    next-nearest do not, so along x the force is exactly linear with two distinct non-zero normal
    frequencies (sqrt(2) and 2): a two-dimensional anisotropic quadratic well (plus translation)."""
    x = 0.9 * np.arange(4) + np.asarray(disp, dtype=np.float64)
    pos = np.stack([x, np.full(4, 5.0), np.full(4, 5.0)], axis=1)
    return pos, np.diag([3.6, 10.0, 10.0])


def test_fire_mixes_before_the_kick():
    """With alpha_start = 1 and f_alpha = 1 the mixing replaces v by |v| g^ before the kick
    v += dt g / m, so after every positive-power iteration the velocity is parallel to the current
    force with speed |v_old| + dt |g| / m (m = 1): the speed is the running sum of the impulses.  Mixing
    after the kick also leaves v parallel to g, but with speed |v_old + dt g|, which is smaller
    whenever the force has turned since the last iteration, as it does in this anisotropic well."""
    cfg = fire.FireConfig(dt_start=0.02, dt_max=0.1, alpha_start=1.0, f_alpha=1.0, fmax=1e-12, max_iter=1000)
    pos, cell = _four_chain([0.03, -0.02, 0.035, -0.01])
    st = fire.init_state(pos, cell, cfg)
    sp, m = np.zeros(4, np.int32), np.ones(4)
    checked, other_order_gap = 0, 0.0
    for k in range(40):
        v_old = st.vel.copy()
        g = forces.system_efw(st.pos, st.cell, sp, _SS.params, _SS.kind, _SS.cutoff, False)[1]
        x_old = st.pos.copy()
        fire.fire_iterate(st, sp, m, _SS, cfg, 1)
        gn, vn = np.linalg.norm(g), np.linalg.norm(st.vel)
        if k > 0 and float((g * v_old).sum()) > 0.0:
            assert abs(vn - (np.linalg.norm(v_old) + st.dt * gn)) <= 1e-12 * vn, k
            assert np.linalg.norm(st.vel - vn * g / gn) <= 1e-12 * vn, k  # parallel to the force
            other_order_gap = max(other_order_gap, (vn - np.linalg.norm(v_old + st.dt * g)) / vn)
            checked += 1
        assert np.allclose(st.pos, x_old + st.dt * st.vel, rtol=0, atol=1e-14)  # drift with the new v
    assert checked >= 10
    assert other_order_gap > 1e-6  # the other order would have failed the speed check


def test_baoab_samples_harmonic_configurations_exactly():
    """BAOAB (Leimkuhler and Matthews 2013) samples the configurations of a harmonic system exactly
    at any stable step: the mean potential energy above the minimum is (3N - 3) kT / 2.  The other
    splittings of the same parts (OBABO, velocity Verlet then O, ABOBA) sample a shadow harmonic
    system with stiffness k (1 - w^2 dt^2 / 4) per mode, i.e. +14 % to +70 % here at w_max dt = 1.5.
    A slightly compressed FCC soft-sphere crystal (12 contacts of overlap 4.5 %) at kT = 2e-4 is
    harmonic up to corrections of order 1e-4."""
    basis, cell0 = fcc_cell(1.35)
    pos0, cell = supercell(basis, cell0, (2, 2, 2))
    n = pos0.shape[0]
    offs, sp, mass = np.array([0, n]), np.zeros(n, np.int32), np.ones(n)
    e_min = forces.batch_efw(pos0, cell[None], offs, sp, _SS)[0][0]
    # the crystal's largest angular frequency is sqrt(7.8097) (fixed by the contact stiffness 1 and
    # the FCC geometry; the test below only needs a step well inside the stable range)
    dt = 1.5 / np.sqrt(7.8097)
    kT, gamma = 2e-4, 1.0
    pos, vel, F = pos0.copy(), np.zeros_like(pos0), None
    us = []
    for k in range(0, 1000, 2):
        out = langevin.baoab(pos, vel, mass, cell[None], offs, sp, _SS, dt, 2, 1.0, gamma, [kT], 2013, step0=k,
                             forces0=F)
        pos, vel, F = out["pos"], out["vel"], out["forces"]
        if k >= 200:
            us.append(forces.batch_efw(pos, cell[None], offs, sp, _SS)[0][0] - e_min)
    ratio = float(np.mean(us)) / (0.5 * (3 * n - 3) * kT)
    assert abs(ratio - 1.0) < 0.05, ratio


def test_inflight_schedule_hand_worked():
    """Six systems (memory scalers, iterations to converge) = (3, 4), (2, 2), (4, 6), (1, 3),
    (2, 5), (3, 1) streamed into a capacity of 7, converged systems removed every 2 iterations and
    the batch refilled in stream order while the next system fits (it never skips ahead):
      step 0: {0, 1} (2 would make 9)      step 2: 1 done -> {0, 2}
      step 4: 0 done -> {2, 3, 4}          step 6: none done
      step 8: 2, 3 done -> {4, 5}          step 10: 4, 5 done -> {}"""
    log, done = autobatch.inflight_schedule([3, 2, 4, 1, 2, 3], [4, 2, 6, 3, 5, 1], 7, 2)
    assert log == [(0, (0, 1)), (2, (0, 2)), (4, (2, 3, 4)), (6, (2, 3, 4)), (8, (4, 5)), (10, ())]
    assert done == {1: 2, 0: 4, 2: 8, 3: 8, 4: 10, 5: 10}


def _lj_dphi(eps, sig, r):
    """Textbook LJ derivative d/dr 4 eps ((s/r)^12 - (s/r)^6)."""
    return 4.0 * eps * (-12.0 * sig ** 12 / r ** 13 + 6.0 * sig ** 6 / r ** 7)


def _lj_phi(eps, sig, r):
    return 4.0 * eps * ((sig / r) ** 12 - (sig / r) ** 6)


def test_pair_magnitude_sums_dimer_and_fcc_shells():
    """A_i = sum_j |phi'(r_ij)| per atom, sum |phi| and sum |r phi'| over unordered pairs: for an LJ
    dimer at r = sigma (phi = 0, |phi'| = 24 eps / sigma) and at the minimum 2^(1/6) sigma (phi = -eps,
    phi' = 0); for a perfect FCC crystal with the cutoff between the second and third shells,
    A_i = 12 |phi'(a/sqrt 2)| + 6 |phi'(a)| and the per-system sums are N/2 times the shell sums
    (shell counts from direct lattice enumeration)."""
    eps, sig = 0.7, 1.3
    params = np.array([[[eps, sig, 0.0]]])
    cell = np.eye(3) * 40.0
    for r, a_exp, phi_exp in ((sig, 24.0 * eps / sig, 0.0), (2.0 ** (1 / 6) * sig, 0.0, eps)):
        pos = np.array([[1.0, 2.0, 3.0], [1.0 + r, 2.0, 3.0]])
        A, sphi, srphi = forces.pair_magnitude_sums(pos, cell, np.zeros(2, np.int32), params, "lj", 3.0 * sig)
        assert np.allclose(A, a_exp, rtol=1e-12, atol=1e-12)
        assert abs(sphi - phi_exp) <= 1e-12 and abs(srphi - r * a_exp) <= 1e-11
    a = 1.6
    basis, cell0 = fcc_cell(a)
    pos, cell = supercell(basis, cell0, (3, 3, 3))
    rc = 1.1 * a
    shells = fcc_shells(a, rc)
    assert sorted(shells.values()) == [6, 12]
    A, sphi, srphi = forces.pair_magnitude_sums(pos, cell, np.zeros(pos.shape[0], np.int32), params, "lj", rc)
    a_exp = sum(c * abs(_lj_dphi(eps, sig, r)) for r, c in shells.items())
    n = pos.shape[0]
    assert np.allclose(A, a_exp, rtol=1e-12)
    assert abs(sphi - 0.5 * n * sum(c * abs(_lj_phi(eps, sig, r)) for r, c in shells.items())) <= 1e-10 * sphi
    assert abs(srphi - 0.5 * n * sum(c * abs(r * _lj_dphi(eps, sig, r)) for r, c in shells.items())) <= 1e-10 * srphi
