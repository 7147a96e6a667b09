"""Pins of the Langevin oracle: the generator's published known-answer vectors, the statistics of
its normals, the friction-free limit (velocity Verlet) and the exact variance of the O step."""
import numpy as np

from oracle import integrate, langevin
from workloads import PotentialSpec


def test_philox_known_answer_vectors():
    # Philox4x32-10 test vectors published with the generator (Salmon et al., SC 2011)
    cases = [((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
             ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
             ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
              (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1))]
    for ctr, key, want in cases:
        got = langevin.philox4x32_10([np.array([c], dtype=np.uint32) for c in ctr], key)
        assert tuple(int(x[0]) for x in got) == want


def test_normals_are_standard_and_uncorrelated():
    n = 200000
    z = langevin.normals(2024, 5, n)
    z2 = langevin.normals(2024, 6, n)
    tol = 6.0 / np.sqrt(n)
    assert np.all(np.abs(z.mean(axis=0)) < tol)
    assert np.all(np.abs(z.var(axis=0) - 1.0) < 3 * tol)
    assert abs(np.mean(z[:, 0] * z[:, 1])) < tol and abs(np.mean(z[:, 0] * z[:, 2])) < tol
    assert abs(np.mean(z[:, 0] * z2[:, 0])) < tol  # consecutive steps
    assert abs(np.mean(z[:, 0] ** 4) - 3.0) < 40 * tol  # Gaussian kurtosis
    # a different seed gives a different stream; the same seed and step the same numbers
    assert not np.array_equal(z[:10], langevin.normals(2025, 5, 10))
    assert np.array_equal(z[:10], langevin.normals(2024, 5, 10))


def test_without_friction_is_velocity_verlet():
    # two soft spheres on a periodic line (the harmonic chain of the velocity-Verlet pins)
    pot = PotentialSpec("soft_sphere", np.array([[[1.0, 1.0, 0.0]]]), 1.0)
    pos = np.array([[0.0, 5.0, 5.0], [0.93, 5.0, 5.0]])
    vel = np.array([[-0.05, 0.01, 0.0], [0.05, -0.01, 0.0]])
    cell = np.diag([1.8, 10.0, 10.0])[None]
    offs, sp, mass = np.array([0, 2]), np.zeros(2, np.int32), np.array([1.0, 2.0])
    ref = integrate.nve(pos, vel, mass, cell, offs, sp, pot, 0.1, 50, accel=1.0)
    out = langevin.baoab(pos, vel, mass, cell, offs, sp, pot, 0.1, 50, 1.0, 0.0, [0.7], seed=3)
    assert np.abs(out["pos"] - ref["pos"]).max() < 1e-13
    assert np.abs(out["vel"] - ref["vel"]).max() < 1e-13


def test_o_step_variance_of_free_atoms():
    # atoms far apart feel no force: after k steps from rest each velocity component is a sum of
    # k damped normals with variance (1 - c1^(2k)) a kT / m
    n, k, dt, gamma, kT, a = 400, 3, 0.01, 20.0, 0.5, 1.0
    grid = np.stack(np.meshgrid(np.arange(8), np.arange(8), np.arange(7), indexing="ij"), -1).reshape(-1, 3)[:n]
    pos = grid * 30.0 + 5.0
    pot = PotentialSpec("lj", np.array([[[1.0, 1.0, 0.0]]]), 2.5)
    cell = np.diag([300.0, 300.0, 300.0])[None]
    mass = np.full(n, 2.0)
    out = langevin.baoab(pos, np.zeros((n, 3)), mass, cell, np.array([0, n]), np.zeros(n, np.int32), pot, dt, k, a,
                         gamma, [kT], seed=99)
    assert np.abs(out["forces"]).max() == 0.0
    c1 = np.exp(-gamma * dt)
    want = (1.0 - c1 ** (2 * k)) * a * kT / 2.0
    got = out["vel"].var()
    assert abs(got - want) < 6.0 * want * np.sqrt(2.0 / (3 * n))
    # the positions moved by the half-step drifts of those velocities only
    assert np.abs(out["pos"] - pos).max() < 10 * dt * np.sqrt(want) * k
