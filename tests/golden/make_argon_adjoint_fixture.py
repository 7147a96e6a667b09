"""Writes ``argon_adjoint_864_500.txt``: the FP64 oracle's trajectory gradient of the smeared-RDF
loss for one 864-atom argon system over 500 velocity-Verlet steps (the differentiable-simulation
use case of Section 2: the loss is the mean squared difference between the final frame's
Gaussian-smeared RDF and a target RDF made by the same simulation with epsilon and sigma scaled
by 1.05).

Only ``oracle/`` and the seeded input generators are called.  The system is system 0 of the
16 x 864 differentiable-trajectory batch (seed 3); the oracle keeps every frame, so the
checkpoint interval of the GPU engine does not enter the reference values.

    python tests/golden/make_argon_adjoint_fixture.py     # about 1.5 h on 2 host cores
"""
from __future__ import annotations

import multiprocessing as mp
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "argon_adjoint_864_500.txt")
N_STEPS = 500
SAMPLE_EVERY = 8  # rows of dL/dr0 written (every 8th atom)


def workload():
    from workloads import argon_adjoint_batch
    return argon_adjoint_batch(16, n_steps=N_STEPS).subset([0])


def _potential(w, scale):
    from workloads import PotentialSpec
    p = np.array(w.potential.params, dtype=np.float64).copy()
    p[0, 0, 0] *= scale
    p[0, 0, 1] *= scale
    return PotentialSpec(w.potential.kind, p, w.potential.cutoff, w.potential.shift_energy)


def _forward(scale):
    from oracle import adjoint as oadj
    w = workload()
    pot = _potential(w, scale)
    traj, _ = oadj.trajectory_positions(w.pos, w.vel, w.mass, w.cell, w.sys_offsets, w.species, pot, w.dt, N_STEPS,
                                        w.accel)
    print(f"forward at scale {scale} done", flush=True)
    return np.stack(traj)


def main():
    from oracle import adjoint as oadj
    w = workload()
    ex = w.extra
    n_bins, r_end, sigma = int(ex["rdf_bins"]), float(ex["rdf_rmax"]), float(ex["rdf_sigma"])
    r_max = r_end + 6 * sigma
    with mp.get_context("spawn").Pool(2) as pool:
        traj_t, traj = pool.map(_forward, [float(ex["target_scale"]), 1.0])
    g_t = oadj.batch_rdf(traj_t[-1], w.cell, w.sys_offsets, n_bins, r_end, sigma, r_max)
    g = oadj.batch_rdf(traj[-1], w.cell, w.sys_offsets, n_bins, r_end, sigma, r_max)
    loss = oadj.rdf_loss(g, g_t)
    lr_T = oadj.rdf_loss_grad(traj[-1], w.cell, w.sys_offsets, n_bins, r_end, sigma, r_max, g, g_t)
    pot = _potential(w, 1.0)
    lr0, _, tb = oadj.reverse_nve(list(traj), w.mass, w.cell, w.sys_offsets, w.species, pot, w.dt, w.accel, lr_T,
                                  np.zeros_like(lr_T))
    print("reverse pass done", flush=True)
    rows = np.arange(0, w.n_atoms, SAMPLE_EVERY)
    with open(OUT, "w") as f:
        f.write("# FP64 oracle trajectory gradient of the smeared-RDF loss (Section 2, differentiable simulation)\n")
        f.write(f"# written by tests/golden/make_argon_adjoint_fixture.py: system 0 of the 16 x 864 argon batch "
                f"(seed 3), {N_STEPS} steps, dt {w.dt} fs,\n")
        f.write(f"# RDF {n_bins} bins to {r_end} A, smearing {sigma} A, target from epsilon and sigma x "
                f"{ex['target_scale']}; oracle/ only\n")
        f.write(f"n_atoms {w.n_atoms}\nn_steps {N_STEPS}\n")
        f.write(f"loss {loss:.17e}\n")
        f.write(f"dL_deps {tb[0, 0, 0]:.17e}\ndL_dsigma {tb[0, 0, 1]:.17e}\n")
        f.write(f"dL_dr0_max_abs {np.abs(lr0).max():.17e}\ndL_dr0_norm {np.linalg.norm(lr0):.17e}\n")
        f.write(f"final_pos_checksum {traj[-1].sum():.17e}\n")
        f.write(f"# dL/dr0 of every {SAMPLE_EVERY}th atom: atom x y z\n")
        for i in rows:
            f.write(f"row {i} {lr0[i, 0]:.17e} {lr0[i, 1]:.17e} {lr0[i, 2]:.17e}\n")
    print(f"wrote {OUT}: loss {loss:.6e} dL/deps {tb[0, 0, 0]:.6e} dL/dsigma {tb[0, 0, 1]:.6e}", flush=True)


if __name__ == "__main__":
    main()
