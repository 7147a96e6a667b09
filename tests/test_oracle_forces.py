"""Pins of the oracle's potentials, forces and virial: closed forms, symmetry and finite differences."""
import numpy as np
import pytest
from scipy.optimize import minimize_scalar

from oracle import forces, potentials
from tests.lattice import fcc_shells
from workloads import (PotentialSpec, fcc_cell, lj_argon_params, morse_copper_params, random_small_batch,
                       soft_sphere_params, supercell)


def _dimer_energy(pot, r):
    L = 40.0
    pos = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])
    e, f, w = forces.system_efw(pos, np.eye(3) * L, np.zeros(2, np.int32), pot.params, pot.kind, pot.cutoff,
                                pot.shift_energy)
    return e, f


def test_lj_dimer_closed_form():
    pot = lj_argon_params(shift=False)
    eps, sig = 0.0104, 3.405
    res = minimize_scalar(lambda r: _dimer_energy(pot, r)[0], bounds=(3.0, 5.0), method="bounded",
                          options=dict(xatol=1e-10))
    assert abs(res.x - 2 ** (1 / 6) * sig) < 1e-6
    assert abs(res.fun + eps) < 1e-12
    # shifted at r_c = 2.5 sigma: depth -eps - phi(r_c), phi(r_c)/eps = 4 (2.5^-12 - 2.5^-6)
    pot_s = lj_argon_params(shift=True)
    e_min = _dimer_energy(pot_s, 2 ** (1 / 6) * sig)[0]
    assert abs(e_min / eps - (-0.98368311)) < 1e-8
    assert abs(4 * (2.5 ** -12 - 2.5 ** -6) - (-0.016316891)) < 1e-9
    # zero beyond the cutoff, force along +x on atom 0 is attractive at 4 A
    assert _dimer_energy(pot_s, 2.5 * sig + 1e-6)[0] == 0.0
    e, f = _dimer_energy(pot, 4.0)
    assert f[0, 0] > 0 and f[1, 0] < 0 and abs(f[0, 0] + f[1, 0]) < 1e-18


def test_morse_and_soft_sphere_dimers():
    pot = morse_copper_params(cutoff=7.0)
    res = minimize_scalar(lambda r: _dimer_energy(pot, r)[0], bounds=(2.0, 4.0), method="bounded",
                          options=dict(xatol=1e-10))
    assert abs(res.x - 2.866) < 1e-6 and abs(res.fun + 0.3429) < 1e-12
    ss = PotentialSpec("soft_sphere", np.array([[[2.0, 1.5, 0.0]]]), 1.5)
    assert abs(_dimer_energy(ss, 0.75)[0] - 0.5 * 2.0 * 0.25) < 1e-15
    assert _dimer_energy(ss, 1.5)[0] == 0.0 and _dimer_energy(ss, 1.6)[0] == 0.0


@pytest.mark.parametrize("kind", ["lj", "morse", "soft_sphere"])
def test_potential_derivatives_by_fd(kind):
    rng = np.random.default_rng(1)
    if kind == "lj":
        p = np.array([[1.3, 1.1, 0.0]] * 20)
        r = rng.uniform(0.95, 2.5, 20)
    elif kind == "morse":
        p = np.array([[0.4, 1.5, 1.2]] * 20)
        r = rng.uniform(0.8, 3.0, 20)
    else:
        p = np.array([[1.7, 1.3, 0.0]] * 20)
        r = rng.uniform(0.3, 1.25, 20)
    h = 1e-6
    phi, d1, d2 = potentials.phi_and_derivs(kind, p, r)
    pp, d1p, _ = potentials.phi_and_derivs(kind, p, r + h)
    pm, d1m, _ = potentials.phi_and_derivs(kind, p, r - h)
    np.testing.assert_allclose(d1, (pp - pm) / (2 * h), rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(d2, (d1p - d1m) / (2 * h), rtol=1e-6, atol=1e-8)
    dg = potentials.dg_dparams(kind, p, r)
    for k in range(3 if kind == "morse" else 2):
        q1, q2 = p.copy(), p.copy()
        step = 1e-6 * p[0, k]
        q1[:, k] += step
        q2[:, k] -= step
        g1 = potentials.phi_and_derivs(kind, q1, r)[1] / r
        g2 = potentials.phi_and_derivs(kind, q2, r)[1] / r
        np.testing.assert_allclose(dg[:, k], (g1 - g2) / (2 * step), rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("kind,seed", [("lj", 0), ("morse", 1), ("soft_sphere", 2), ("lj", 3)])
def test_newton_third_law_and_fd_forces(kind, seed):
    w = random_small_batch(seed, n_systems=2, n_range=(6, 14), kind=kind, n_species=2, unwrap_spread=1)
    pot = w.potential
    for s in range(w.n_systems):
        sl = w.system(s)
        pos, cell, sp = w.pos[sl], w.cell[s], w.species[sl]
        e, f, _ = forces.system_efw(pos, cell, sp, pot.params, pot.kind, pot.cutoff, pot.shift_energy)
        A, _, _ = forces.pair_magnitude_sums(pos, cell, sp, pot.params, pot.kind, pot.cutoff)
        assert np.abs(f.sum(0)).max() <= 1e-12 * max(A.sum(), 1.0)
        h = 1e-6
        for i in range(min(pos.shape[0], 5)):
            for a in range(3):
                pp, pm = pos.copy(), pos.copy()
                pp[i, a] += h
                pm[i, a] -= h
                ep = forces.system_efw(pp, cell, sp, pot.params, pot.kind, pot.cutoff, pot.shift_energy)[0]
                em = forces.system_efw(pm, cell, sp, pot.params, pot.kind, pot.cutoff, pot.shift_energy)[0]
                fd = -(ep - em) / (2 * h)
                assert abs(fd - f[i, a]) <= 1e-6 * max(abs(f[i, a]), 0.01 * A[i], 1e-6), (i, a, fd, f[i, a])


@pytest.mark.parametrize("kind,seed", [("lj", 4), ("morse", 5), ("soft_sphere", 6)])
def test_virial_is_strain_derivative(kind, seed):
    # stress = -W / V = (1/V) dE/de under r -> r (I + e), cell -> cell (I + e), e symmetric
    w = random_small_batch(seed, n_systems=1, n_range=(6, 12), kind=kind, n_species=2)
    pot = w.potential
    pos, cell, sp = w.pos, w.cell[0], w.species
    _, _, W = forces.system_efw(pos, cell, sp, pot.params, pot.kind, pot.cutoff, pot.shift_energy)
    h = 1e-6
    for a in range(3):
        for b in range(a, 3):
            e = np.zeros((3, 3))
            e[a, b] += 0.5 * h
            e[b, a] += 0.5 * h
            Ep = forces.system_efw(pos @ (np.eye(3) + e), cell @ (np.eye(3) + e), sp, pot.params, pot.kind,
                                   pot.cutoff, pot.shift_energy)[0]
            Em = forces.system_efw(pos @ (np.eye(3) - e), cell @ (np.eye(3) - e), sp, pot.params, pot.kind,
                                   pot.cutoff, pot.shift_energy)[0]
            dE = (Ep - Em) / (2 * h)
            scale = max(np.abs(W).max(), 1e-3)
            assert abs(dE - (-W[a, b])) <= 1e-6 * scale, (a, b, dE, W[a, b])


@pytest.mark.parametrize("reps,a", [((3, 3, 3), 5.26), ((1, 1, 1), 5.26), ((2, 2, 2), 5.0)])
def test_perfect_fcc_lattice_sums(reps, a):
    pot = lj_argon_params(shift=True)
    basis, cell0 = fcc_cell(a)
    pos, cell = supercell(basis, cell0, reps)
    n = pos.shape[0]
    e, f, W = forces.system_efw(pos, cell, np.zeros(n, np.int32), pot.params, pot.kind, pot.cutoff, True)
    assert np.abs(f).max() < 1e-12
    shells = fcc_shells(a, pot.cutoff)
    eps, sig = 0.0104, 3.405
    phi = lambda r: 4 * eps * ((sig / r) ** 12 - (sig / r) ** 6)  # noqa: E731
    dphi = lambda r: 24 * eps / r * ((sig / r) ** 6 - 2 * (sig / r) ** 12)  # noqa: E731
    e_atom = 0.5 * sum(c * (phi(r) - phi(pot.cutoff)) for r, c in shells.items())
    assert abs(e / n - e_atom) < 1e-12 * abs(e_atom) * 10
    # isotropic virial: W = -(1/6) sum_pairs r phi'(r) I per atom-pair sum (trace/3)
    w_iso = -0.5 * n * sum(c * r * dphi(r) for r, c in shells.items()) / 3.0
    np.testing.assert_allclose(W, np.eye(3) * w_iso, rtol=1e-11, atol=1e-13 * abs(w_iso))


def test_single_atom_self_images():
    # one atom in a small cell: only self-image pairs; zero force, E = 1/2 sum_S phi(|S cell|)
    pot = soft_sphere_params([1.0])
    cell = np.diag([0.8, 0.9, 2.0])
    e, f, _ = forces.system_efw(np.array([[0.1, 0.2, 0.3]]), cell, np.zeros(1, np.int32), pot.params, pot.kind,
                                pot.cutoff, False)
    expect = 0.5 * 2 * (0.5 * (1 - 0.8) ** 2 + 0.5 * (1 - 0.9) ** 2)
    assert abs(e - expect) < 1e-15 and np.abs(f).max() < 1e-15
