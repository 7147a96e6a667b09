"""Plain FP64 CPU oracle for the batched pair-potential simulation step.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct definition that the HIP
path is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may import it.  It shares no code, constants, tables or helpers with the
HIP library or its Python binding, and it imports neither.

What it computes (the paper names these objects but defines none of them, so every definition
is the textbook one; see each module's header for its reading):

* ``pairs``      -- the full / half periodic pair set by brute force over all atom pairs and
                    every lattice image in range (neighbor-list construction, Section 4).
* ``potentials`` -- Lennard-Jones, Morse and soft-sphere pair functions and derivatives
                    (the classical potentials of the Abstract).
* ``forces``     -- per-system energy, per-atom forces and per-system virial (the model
                    output schema of energies, forces and stress, Section 2).
* ``integrate``  -- velocity-Verlet NVE, kinetic energy, the neighbor-list rebuild test
                    (molecular-dynamics integrators, Abstract).
* ``fire``       -- FIRE relaxation of positions, or of positions and cell
                    (structural relaxation optimizers, Abstract).
* ``adjoint``    -- smeared-RDF loss and the reverse (adjoint) velocity-Verlet pass for
                    gradients of a trajectory observable (differentiable simulation, Section 2).

All arithmetic is float64 NumPy.  Inputs are host arrays in the row-vector convention:
positions ``(N, 3)``, cell ``(3, 3)`` with lattice vectors as rows, Cartesian = fractional @ cell,
and pair vector d = r_j - r_i + S @ cell for the image S in Z^3.
"""
from . import constants, pairs, potentials, forces, integrate, fire, adjoint  # noqa: F401
