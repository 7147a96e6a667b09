"""Pins of the Lorentz-Berthelot mixing table of the oracle: closed-form values, symmetry, and a
mixture of identical species that must reproduce the one-species forces."""
import numpy as np

from oracle import forces, potentials
from workloads import PotentialSpec, random_small_batch


def test_closed_form_values():
    t = potentials.lorentz_berthelot([1.0, 4.0, 0.25], [1.0, 2.0, 3.0])
    assert t.shape == (3, 3, 3)
    assert t[0, 1, 0] == 2.0 and t[1, 2, 0] == 1.0 and t[0, 2, 0] == 0.5  # geometric means
    assert t[0, 1, 1] == 1.5 and t[1, 2, 1] == 2.5 and t[0, 2, 1] == 2.0  # arithmetic means
    assert np.array_equal(t[:, :, :2], np.transpose(t, (1, 0, 2))[:, :, :2])
    for a, (e, s) in enumerate(zip([1.0, 4.0, 0.25], [1.0, 2.0, 3.0])):
        assert t[a, a, 0] == e and t[a, a, 1] == s
    assert np.all(t[:, :, 2] == 0.0)


def test_identical_species_reproduce_one_species_forces():
    w = random_small_batch(71, n_systems=2, n_range=(20, 40), kind="lj", n_species=1)
    one = PotentialSpec("lj", potentials.lorentz_berthelot([0.8], [1.1]), 2.5, True)
    two = PotentialSpec("lj", potentials.lorentz_berthelot([0.8, 0.8], [1.1, 1.1]), 2.5, True)
    species = np.random.default_rng(0).integers(0, 2, size=w.n_atoms).astype(np.int32)
    e1, f1, w1 = forces.batch_efw(w.pos, w.cell, w.sys_offsets, np.zeros(w.n_atoms, np.int32), one)
    e2, f2, w2 = forces.batch_efw(w.pos, w.cell, w.sys_offsets, species, two)
    assert np.allclose(e1, e2, rtol=1e-13, atol=0) and np.allclose(f1, f2, rtol=1e-12, atol=1e-14)
