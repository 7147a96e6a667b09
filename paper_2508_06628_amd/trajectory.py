"""Checkpointed gradient of a trajectory observable (differentiable simulation, paper Section 2:
gradients of an RDF computed at the end of an MD trajectory with respect to potential
parameters and initial positions).

Forward: velocity-Verlet NVE (``ts_nve_step``) keeping (r, v) every ``checkpoint_every`` steps,
then the smeared RDF of the final frame (``ts_rdf_smeared``) and its mean-squared distance to a
per-system target (``ts_rdf_loss``).  Backward: dL/dr_T from ``ts_rdf_vjp``; then, segment by
segment from the end, the segment is recomputed from its checkpoint keeping every position and
reversed with ``ts_pair_adjoint`` (one call per step: consecutive half kicks at the same
positions merge).  Every numerical step runs in the HIP library; this module only sequences
calls and owns the buffers.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import api


@dataclasses.dataclass
class RdfSpec:
    n_bins: int = 200
    r_end: float = 10.0
    sigma: float = 0.05

    @property
    def r_max(self) -> float:
        return self.r_end + 6.0 * self.sigma


class TrajectoryRDF:
    """Loss L(eps, sigma, r_0) of one LJ batch (kind "lj", or "lj_sf" for the shifted-force
    truncation, whose trajectory map has no force jumps at the cutoff); single-species parameters
    (eps, sigma)."""

    def __init__(self, workload, n_steps: int, checkpoint_every: int = 50, prec: str = "f32",
                 rdf: RdfSpec = RdfSpec(), skin: float = 0.3, bin_factor: int = 2, use_graph: bool = True):
        self.w = workload
        self.use_graph = bool(use_graph)
        self.n_steps = int(n_steps)
        self.K = int(checkpoint_every)
        self.prec = prec
        self.rdf = rdf
        self.skin = skin
        self.bin_factor = bin_factor
        self.batch = api.Batch.from_workload(workload)
        self.vel0 = self.batch.vel.clone()
        self.cutoff = workload.potential.cutoff
        self.nl = api.build_neighbor_list(self.batch, self.cutoff, skin, bin_factor=bin_factor, margin=1.35)
        self.nl_rdf = api.build_neighbor_list(self.batch, rdf.r_max, 0.0, bin_factor=bin_factor, margin=1.35)
        self.force = api.force_buffer(self.batch, prec)
        S = self.batch.n_systems
        dev = self.batch.device
        self.g = torch.zeros((S, rdf.n_bins), dtype=torch.float64, device=dev)
        self.target = torch.zeros_like(self.g)
        self.loss = torch.zeros(1, dtype=torch.float64, device=dev)
        self.dl_dg = torch.zeros_like(self.g)
        self.checkpoints = []
        self.params = None

    def _pp(self, eps, sigma):
        p = np.zeros((1, 1, 3))
        p[0, 0] = (eps, sigma, 0.0)
        return api.pair_params(self.w.potential.kind, p, self.cutoff, self.w.potential.shift_energy, self.prec)

    def _reset(self, pos0: torch.Tensor):
        self.batch.pos.copy_(pos0)
        self.batch.vel.copy_(self.vel0)
        api.ts_neighbor_build(self.batch, self.nl, force=True)

    def run(self, eps, sigma, pos0: torch.Tensor, keep_checkpoints=True):
        """Forward trajectory; returns the final-frame RDF (S, n_bins) tensor."""
        pp = self._pp(eps, sigma)
        self.params = (eps, sigma)
        self._reset(pos0)
        self.checkpoints = []
        done = 0
        while done < self.n_steps:
            # every segment starts from a fresh list and forces evaluated on it, so that the
            # recomputation in backward() reproduces the segment bit for bit
            api.ts_neighbor_build(self.batch, self.nl, force=True)
            api.ts_pair_forces(self.batch, self.nl, pp, self.force)
            if keep_checkpoints:
                self.checkpoints.append((self.batch.pos.clone(), self.batch.vel.clone()))
            k = min(self.K, self.n_steps - done)
            api.ts_nve_step(self.batch, self.nl, pp, self.w.dt, self.w.accel, k, self.force, use_graph=self.use_graph)
            done += k
        api.ts_neighbor_build(self.batch, self.nl_rdf, force=True)
        r = self.rdf
        api.ts_rdf_smeared(self.batch, self.nl_rdf, r.n_bins, r.r_end, r.sigma, r.r_max, self.g)
        return self.g

    def check_status(self):
        """Raise if a neighbor list overflowed, met a non-finite position or dropped an image shift
        in the calls so far (a truncated list would give wrong forces and gradients); clears them."""
        for name, nl in (("trajectory", self.nl), ("rdf", self.nl_rdf)):
            st = nl.read_status()
            if st[1] or st[3] or st[4]:
                raise RuntimeError(f"{name} neighbor list status {st.tolist()} (overflow, non-finite, shift)")
            nl.status.zero_()

    def set_target(self, g_target: torch.Tensor):
        self.target.copy_(g_target)

    def forward(self, eps, sigma, pos0: torch.Tensor) -> torch.Tensor:
        self.run(eps, sigma, pos0)
        api.ts_rdf_loss(self.g, self.target, self.loss, self.dl_dg)
        return self.loss

    def backward(self, fused: bool = True):
        """(dL/deps, dL/dsigma, dL/dr_0 (3, N)) for the last forward().  ``fused`` uses the recorded
        segment entry points (systems of at most 2048 atoms); otherwise one call per step."""
        if fused and self.batch.max_system_atoms <= 2048:
            return self._backward_segments()
        return self._backward_steps()

    def _backward_segments(self):
        eps, sigma = self.params
        pp = self._pp(eps, sigma)
        b, dt, accel = self.batch, self.w.dt, self.w.accel
        r = self.rdf
        lr = torch.zeros_like(b.pos)
        lv = torch.zeros_like(b.pos)
        tb = torch.zeros(48, dtype=torch.float64, device=b.device)
        api.ts_rdf_vjp(b, self.nl_rdf, r.n_bins, r.r_end, r.sigma, r.r_max, self.dl_dg, lr)
        n = b.n_atoms
        if getattr(self, "_traj", None) is None or self._traj.shape[0] < self.K + 1:
            self._traj = torch.empty((self.K + 1, 3, n), dtype=torch.float64, device=b.device)
        n_seg = len(self.checkpoints)
        for seg in range(n_seg - 1, -1, -1):
            p0, v0 = self.checkpoints[seg]
            k = min(self.K, self.n_steps - seg * self.K)
            b.pos.copy_(p0)
            b.vel.copy_(v0)
            api.ts_neighbor_build(b, self.nl, force=True)
            api.ts_pair_forces(b, self.nl, pp, self.force)
            api.ts_nve_record(b, self.nl, pp, dt, accel, k, self.force, self._traj, use_graph=self.use_graph)
            api.ts_adjoint_segment(b, self.nl, pp, self._traj, k, dt, accel, seg == n_seg - 1, seg == 0, lr, lv, tb,
                                   use_graph=self.use_graph)
        grads = tb.cpu().numpy()
        return float(grads[0]), float(grads[1]), lr

    def _backward_steps(self):
        eps, sigma = self.params
        pp = self._pp(eps, sigma)
        b, dt, accel = self.batch, self.w.dt, self.w.accel
        r = self.rdf
        lr = torch.zeros_like(b.pos)
        lv = torch.zeros_like(b.pos)
        tb = torch.zeros(48, dtype=torch.float64, device=b.device)
        # dL/dr_T (the batch holds r_T and nl_rdf is valid there)
        api.ts_rdf_vjp(b, self.nl_rdf, r.n_bins, r.r_end, r.sigma, r.r_max, self.dl_dg, lr)
        first = True
        seg_starts = [i * self.K for i in range(len(self.checkpoints))]
        for seg in range(len(self.checkpoints) - 1, -1, -1):
            p0, v0 = self.checkpoints[seg]
            k = min(self.K, self.n_steps - seg_starts[seg])
            # recompute the segment, keeping r_{n0} .. r_{n0+k}
            b.pos.copy_(p0)
            b.vel.copy_(v0)
            api.ts_neighbor_build(b, self.nl, force=True)
            api.ts_pair_forces(b, self.nl, pp, self.force)
            traj = [p0.clone()]
            for _ in range(k):
                api.ts_nve_step(b, self.nl, pp, dt, accel, 1, self.force, use_graph=False)
                traj.append(b.pos.clone())
            # reverse it: kick-adjoint at r_{n+1} merged with the previous step's, drift, ...
            for n in range(k, 0, -1):
                b.pos.copy_(traj[n])
                api.ts_neighbor_build(b, self.nl, force=False)
                api.ts_pair_adjoint(b, self.nl, pp, 0.0 if first else dt, 0.5 * dt if first else dt, accel, lr, lv,
                                    tb)
                first = False
            if seg == 0:
                b.pos.copy_(traj[0])
                api.ts_neighbor_build(b, self.nl, force=False)
                api.ts_pair_adjoint(b, self.nl, pp, dt, 0.5 * dt, accel, lr, lv, tb)
        grads = tb.cpu().numpy()
        return float(grads[0]), float(grads[1]), lr


class TrajectoryLoss(torch.autograd.Function):
    """L = TrajectoryLoss.apply(eps, sigma, pos0, engine): autograd entry of the checkpointed
    trajectory gradient.  eps and sigma are 0-d float64 tensors, pos0 is (3, N) float64."""

    @staticmethod
    def forward(ctx, eps, sigma, pos0, engine: TrajectoryRDF):
        ctx.engine = engine
        loss = engine.forward(float(eps), float(sigma), pos0.detach())
        return loss.clone().reshape(())

    @staticmethod
    def backward(ctx, grad_out):
        de, ds, dr = ctx.engine.backward()
        g = grad_out.to(torch.float64)
        dev = dr.device
        return (g * torch.tensor(de, dtype=torch.float64, device=dev),
                g * torch.tensor(ds, dtype=torch.float64, device=dev), g * dr, None)
