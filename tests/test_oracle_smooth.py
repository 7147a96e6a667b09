"""Pins of the oracle's shifted-force kinds (phi(r) - phi(r_c) - (r - r_c) phi'(r_c) inside r_c): the
energy and the force go to zero continuously at the cutoff (while the plain kinds jump), the force
is minus the energy gradient, the virial the strain derivative, the pair Hessian-vector product and
parameter derivatives match finite differences of the forces, and a trajectory gradient through
cutoff crossings matches central differences at a step where the plain kind's would not."""
import dataclasses

import numpy as np
import pytest

from oracle import adjoint, forces, potentials
from workloads import PotentialSpec, random_small_batch


def _sf(pot):
    return dataclasses.replace(pot, kind=pot.kind + "_sf", shift_energy=False)


def _dimer(pot, r):
    pos = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])
    e, f, _ = forces.system_efw(pos, np.eye(3) * 40.0, np.zeros(2, np.int32), pot.params, pot.kind, pot.cutoff,
                                pot.shift_energy)
    return e, f[1, 0]


@pytest.mark.parametrize("kind,params,rc", [("lj", (1.3, 1.1, 0.0), 2.5), ("morse", (0.4, 1.5, 1.2), 2.7)])
def test_energy_and_force_vanish_continuously_at_the_cutoff(kind, params, rc):
    plain = PotentialSpec(kind, np.array([[params]], dtype=np.float64), rc, True)
    sf = _sf(plain)
    # the plain (energy-shifted) kind's force jumps at r_c; its second derivative there, by central
    # differences of that force, sets the shifted-force energy's quadratic approach: E ~ phi''(r_c) d^2 / 2
    jump = _dimer(plain, rc - 1e-9)[1]
    assert abs(jump) > 1e-4
    h = 1e-4
    curv = -(_dimer(plain, rc - h)[1] - _dimer(plain, rc - 3 * h)[1]) / (2 * h)  # phi'' at rc - 2h
    for d in (1e-2, 1e-3, 1e-4):
        e, f = _dimer(sf, rc - d)
        assert abs(e - 0.5 * curv * d * d) <= 0.05 * abs(curv) * d * d, (d, e)
        assert abs(f - curv * d) <= 0.05 * abs(curv) * d, (d, f)  # force on the second atom: -phi_sf(r) = phi"(r_c) d
    assert _dimer(sf, rc + 1e-9) == (0.0, 0.0)


@pytest.mark.parametrize("kind", ["lj_sf", "morse_sf"])
def test_shifted_force_derivatives_by_fd(kind):
    rng = np.random.default_rng(2)
    p = np.array([[1.3, 1.1, 0.0]] * 20) if kind == "lj_sf" else np.array([[0.4, 1.5, 1.2]] * 20)
    r = rng.uniform(0.95, 2.4, 20)
    rc = 2.5
    h = 1e-6
    phi, d1, d2 = potentials.phi_and_derivs(kind, p, r, rc)
    pp, d1p, _ = potentials.phi_and_derivs(kind, p, r + h, rc)
    pm, d1m, _ = potentials.phi_and_derivs(kind, p, r - h, rc)
    np.testing.assert_allclose(d1, (pp - pm) / (2 * h), rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(d2, (d1p - d1m) / (2 * h), rtol=1e-6, atol=1e-8)
    dg = potentials.dg_dparams(kind, p, r, rc)
    for k in range(3 if kind == "morse_sf" else 2):
        q1, q2 = p.copy(), p.copy()
        step = 1e-6 * p[0, k]
        q1[:, k] += step
        q2[:, k] -= step
        g1 = potentials.phi_and_derivs(kind, q1, r, rc)[1] / r
        g2 = potentials.phi_and_derivs(kind, q2, r, rc)[1] / r
        np.testing.assert_allclose(dg[:, k], (g1 - g2) / (2 * step), rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("kind,seed", [("lj", 60), ("morse", 61)])
def test_shifted_force_systems_fd_forces_virial_hvp(kind, seed):
    w = random_small_batch(seed, n_systems=1, n_range=(8, 14), kind=kind, n_species=2, unwrap_spread=1)
    pot = _sf(w.potential)
    pos, cell, sp = w.pos, w.cell[0], w.species
    e, f, W = forces.system_efw(pos, cell, sp, pot.params, pot.kind, pot.cutoff, False)
    A, _, _ = forces.pair_magnitude_sums(pos, cell, sp, pot.params, pot.kind, pot.cutoff)
    assert np.abs(f.sum(0)).max() <= 1e-12 * max(A.sum(), 1.0)
    h = 1e-6
    for i in range(min(pos.shape[0], 5)):
        for a in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, a] += h
            pm[i, a] -= h
            ep = forces.system_efw(pp, cell, sp, pot.params, pot.kind, pot.cutoff, False)[0]
            em = forces.system_efw(pm, cell, sp, pot.params, pot.kind, pot.cutoff, False)[0]
            assert abs(-(ep - em) / (2 * h) - f[i, a]) <= 1e-6 * max(abs(f[i, a]), 0.01 * A[i], 1e-6)
    for a in range(3):
        for b in range(a, 3):
            e_ = np.zeros((3, 3))
            e_[a, b] += 0.5 * h
            e_[b, a] += 0.5 * h
            Ep = forces.system_efw(pos @ (np.eye(3) + e_), cell @ (np.eye(3) + e_), sp, pot.params, pot.kind,
                                   pot.cutoff, False)[0]
            Em = forces.system_efw(pos @ (np.eye(3) - e_), cell @ (np.eye(3) - e_), sp, pot.params, pot.kind,
                                   pot.cutoff, False)[0]
            assert abs((Ep - Em) / (2 * h) + W[a, b]) <= 1e-6 * max(np.abs(W).max(), 1e-3)
    rng = np.random.default_rng(seed)
    u = rng.normal(size=pos.shape)
    Ju = adjoint.system_hvp(pos, cell, sp, pot, u)
    fp = forces.system_efw(pos + h * u, cell, sp, pot.params, pot.kind, pot.cutoff, False)[1]
    fm = forces.system_efw(pos - h * u, cell, sp, pot.params, pot.kind, pot.cutoff, False)[1]
    np.testing.assert_allclose(Ju, (fp - fm) / (2 * h), atol=1e-6 * np.abs(Ju).max())
    tb = adjoint.system_param_vjp(pos, cell, sp, pot, u)
    ns = pot.params.shape[0]
    for a in range(ns):
        for b in range(ns):
            for k in range(3 if kind == "morse" else 2):
                P1, P2 = pot.params.copy(), pot.params.copy()
                st = 1e-6 * pot.params[a, b, k]
                P1[a, b, k] += st
                P2[a, b, k] -= st
                f1 = forces.system_efw(pos, cell, sp, P1, pot.kind, pot.cutoff, False)[1]
                f2 = forces.system_efw(pos, cell, sp, P2, pot.kind, pot.cutoff, False)[1]
                fd = float((u * (f1 - f2)).sum() / (2 * st))
                assert abs(fd - tb[a, b, k]) < 1e-5 * max(abs(tb).max(), 1e-8), (kind, a, b, k)


def _reverse_vs_fd(w, pot, h, n_dirs):
    """Relative differences between reverse-pass directional derivatives of a trajectory loss and
    central differences, for ``n_dirs`` random directions of the initial positions."""
    dt, steps = 0.01, 40
    rng = np.random.default_rng(4)
    vel = rng.normal(0.0, 1.0, size=w.pos.shape)
    cr = rng.normal(size=w.pos.shape)

    def loss(pos0):
        traj, _ = adjoint.trajectory_positions(pos0, vel, w.mass, w.cell, w.sys_offsets, w.species, pot, dt, steps,
                                               1.0)
        return float((cr * traj[-1]).sum())

    traj, _ = adjoint.trajectory_positions(w.pos, vel, w.mass, w.cell, w.sys_offsets, w.species, pot, dt, steps, 1.0)
    lr, _, _ = adjoint.reverse_nve(traj, w.mass, w.cell, w.sys_offsets, w.species, pot, dt, 1.0, cr,
                                   np.zeros_like(cr))
    out = []
    for _ in range(n_dirs):
        dirn = rng.normal(size=w.pos.shape)
        fd = (loss(w.pos + h * dirn) - loss(w.pos - h * dirn)) / (2 * h)
        out.append(abs(fd - float((lr * dirn).sum())) / max(abs(fd), 1.0))
    return out


def test_plain_cutoff_breaks_the_same_gradient_check():
    # the same gas with the plain (energy-shifted) kind: the force jump at r_c makes the map only
    # piecewise smooth and central differences at h = 1e-4 straddle crossings
    w = random_small_batch(62, n_systems=2, n_range=(6, 9), kind="lj", density=0.35)
    assert max(_reverse_vs_fd(w, w.potential, 1e-4, 3)) > 1e-3


def test_trajectory_gradient_through_cutoff_crossings():
    # a dilute LJ gas whose pairs cross the cutoff during the run: with the shifted-force kind the
    # trajectory map is smooth, so the reverse pass agrees with central differences at h = 1e-4
    w = random_small_batch(62, n_systems=2, n_range=(6, 9), kind="lj", density=0.35)
    pot = _sf(w.potential)
    assert max(_reverse_vs_fd(w, pot, 1e-4, 3)) < 1e-5
    dt, steps = 0.01, 40
    rng = np.random.default_rng(4)
    vel = rng.normal(0.0, 1.0, size=w.pos.shape)
    cr = rng.normal(size=w.pos.shape)

    def run(pos0, params):
        p = PotentialSpec(pot.kind, params, pot.cutoff, False)
        return adjoint.trajectory_positions(pos0, vel, w.mass, w.cell, w.sys_offsets, w.species, p, dt, steps, 1.0)

    traj, _ = run(w.pos, pot.params)
    # pairs do cross r_c along the way
    def n_in(pos):
        return sum(int((forces._pairs.system_pairs(pos[w.system(s)], w.cell[s], pot.cutoff)["r2"].size))
                   for s in range(w.n_systems))
    assert len({n_in(p) for p in traj[::4]}) > 1
    lr, _, tb = adjoint.reverse_nve(traj, w.mass, w.cell, w.sys_offsets, w.species, pot, dt, 1.0, cr,
                                   np.zeros_like(cr))
    h = 1e-4
    for _ in range(3):
        dirn = rng.normal(size=w.pos.shape)
        lp = float((cr * run(w.pos + h * dirn, pot.params)[0][-1]).sum())
        lm = float((cr * run(w.pos - h * dirn, pot.params)[0][-1]).sum())
        assert abs((lp - lm) / (2 * h) - float((lr * dirn).sum())) < 1e-5 * max(abs(lp - lm) / (2 * h), 1.0)
    for k in range(2):
        P1, P2 = pot.params.copy(), pot.params.copy()
        st = 1e-4 * pot.params[0, 0, k]
        P1[0, 0, k] += st
        P2[0, 0, k] -= st
        fd = (float((cr * run(w.pos, P1)[0][-1]).sum()) - float((cr * run(w.pos, P2)[0][-1]).sum())) / (2 * st)
        assert abs(fd - tb[0, 0, k]) < 1e-5 * max(abs(fd), 1.0), (k, fd, tb[0, 0, k])
