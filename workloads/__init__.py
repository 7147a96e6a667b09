"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package only *builds inputs*: crystal supercells, random packings, random strains,
Maxwell-Boltzmann velocity draws and potential parameter tables.  It holds none of the
simulation arithmetic (no pair sums, no integrators, no optimisers), so the oracle and the
HIP path can both consume it without sharing any computation.

Every generator is deterministic given its seed: ``numpy.random.default_rng`` over a
``SeedSequence(seed)``, with one spawned child per system so that a system's draws do not
depend on how many systems are generated before it.
"""
from .generators import (  # noqa: F401
    Workload,
    PotentialSpec,
    fcc_cell,
    bcc_cell,
    supercell,
    most_cubic_supercell,
    maxwell_boltzmann,
    concat_systems,
    lj_argon_params,
    morse_copper_params,
    soft_sphere_params,
    argon_single,
    argon_batch,
    copper_uneven_batch,
    argon_adjoint_batch,
    soft_sphere_jamming_batch,
    random_small_batch,
    narrow_triclinic_batch,
    insert_empty_systems,
    ARGON_MASS,
    COPPER_MASS,
)
