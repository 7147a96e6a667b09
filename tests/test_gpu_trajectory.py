"""GPU parity of the checkpointed trajectory gradient (RDF loss after velocity-Verlet NVE) against
the FP64 oracle's reverse pass and against central finite differences."""
import numpy as np
import pytest

from oracle import adjoint as oadj
from workloads import PotentialSpec, argon_batch

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N_STEPS, CKPT = 20, 8
RDF = dict(n_bins=200, r_end=10.0, sigma=0.05)


def _workload():
    # two 108-atom argon systems: cells narrower than twice the RDF range (several images in range)
    return argon_batch(2, reps=(3, 3, 3), seed=31, n_steps=N_STEPS)


def _oracle(w, eps, sig, target):
    pot = PotentialSpec("lj", np.array([[[eps, sig, 0.0]]]), w.potential.cutoff, w.potential.shift_energy)
    traj, _ = oadj.trajectory_positions(w.pos, w.vel, w.mass, w.cell, w.sys_offsets, w.species, pot, w.dt, N_STEPS,
                                        w.accel)
    r_max = RDF["r_end"] + 6 * RDF["sigma"]
    g = oadj.batch_rdf(traj[-1], w.cell, w.sys_offsets, RDF["n_bins"], RDF["r_end"], RDF["sigma"], r_max)
    if target is None:
        return g
    loss = oadj.rdf_loss(g, target)
    lr_T = oadj.rdf_loss_grad(traj[-1], w.cell, w.sys_offsets, RDF["n_bins"], RDF["r_end"], RDF["sigma"], r_max, g,
                              target)
    lr0, _, tb = oadj.reverse_nve(traj, w.mass, w.cell, w.sys_offsets, w.species, pot, w.dt, w.accel, lr_T,
                                  np.zeros_like(lr_T))
    return loss, lr0, tb[0, 0, 0], tb[0, 0, 1]


@pytest.fixture(scope="module")
def problem():
    assert torch.cuda.is_available()
    w = _workload()
    eps, sig = float(w.potential.params[0, 0, 0]), float(w.potential.params[0, 0, 1])
    target = _oracle(w, eps * 1.05, sig * 1.05, None)
    ref = _oracle(w, eps, sig, target)
    return w, eps, sig, target, ref


def _engine(w, prec):
    from paper_2508_06628_amd.trajectory import RdfSpec, TrajectoryRDF
    eng = TrajectoryRDF(w, N_STEPS, CKPT, prec=prec, rdf=RdfSpec(**RDF))
    return eng


@pytest.mark.parametrize("fused", [True, False])
def test_gradient_fp64_matches_oracle_reverse_pass(problem, fused):
    w, eps, sig, target, (loss_ref, lr0_ref, de_ref, ds_ref) = problem
    eng = _engine(w, "f64")
    eng.set_target(torch.tensor(target, device="cuda"))
    pos0 = eng.batch.pos.clone()
    loss = eng.forward(eps, sig, pos0).item()
    de, ds, lr0 = eng.backward(fused=fused)
    assert abs(loss - loss_ref) <= 1e-9 * abs(loss_ref)
    assert abs(de - de_ref) <= 1e-8 * abs(de_ref)
    assert abs(ds - ds_ref) <= 1e-8 * abs(ds_ref)
    g = lr0.T.cpu().numpy()
    assert np.abs(g - lr0_ref).max() <= 1e-8 * np.abs(lr0_ref).max()


def test_gradient_fp32_within_1e3_of_oracle(problem):
    w, eps, sig, target, (loss_ref, lr0_ref, de_ref, ds_ref) = problem
    eng = _engine(w, "f32")
    eng.set_target(torch.tensor(target, device="cuda"))
    pos0 = eng.batch.pos.clone()
    eng.forward(eps, sig, pos0)
    de, ds, lr0 = eng.backward()
    assert abs(de - de_ref) <= 1e-3 * abs(de_ref)
    assert abs(ds - ds_ref) <= 1e-3 * abs(ds_ref)
    assert np.abs(lr0.T.cpu().numpy() - lr0_ref).max() <= 1e-3 * np.abs(lr0_ref).max()


def test_gradient_matches_central_differences(problem):
    w, eps, sig, target, _ = problem
    eng = _engine(w, "f64")
    eng.set_target(torch.tensor(target, device="cuda"))
    pos0 = eng.batch.pos.clone()
    eng.forward(eps, sig, pos0)
    de, ds, lr0 = eng.backward()

    def L(e, s, p):
        return eng.forward(e, s, p).item()

    def central(fun, x, h):
        # central differences at h and h/2 combined by Richardson extrapolation: the O(h^2)
        # truncation error of a single central difference with h = 1e-4 relative is ~1e-5 here
        # (the 0.05 A Gaussian smearing makes the loss sharply curved in sigma)
        d1 = (fun(x + h) - fun(x - h)) / (2 * h)
        d2 = (fun(x + h / 2) - fun(x - h / 2)) / h
        return (4 * d2 - d1) / 3

    h = 1e-4
    fd_e = central(lambda e: L(e, sig, pos0), eps, h * eps)
    # sigma and positions: the discrete map has kinks within 1e-4 relative of this point (a pair
    # crosses the force cutoff, where the unshifted force jumps, at a slightly different step),
    # which no adjoint sees.  On the FP64 oracle, central differences against the reverse pass
    # give 8e-5 (sigma) and 5e-3 (positions) at h = 1e-4 sigma, but 6e-9 and 3e-8 at 1e-5 sigma:
    # step inside the smooth piece.
    fd_s = central(lambda sg: L(eps, sg, pos0), sig, 1e-5 * sig)
    assert abs(fd_e - de) <= 1e-6 * abs(de)
    assert abs(fd_s - ds) <= 1e-6 * abs(ds)
    rng = np.random.default_rng(4)
    u = rng.normal(size=pos0.shape)
    u /= np.linalg.norm(u)
    ut = torch.tensor(u, device="cuda")
    fd_p = central(lambda t: L(eps, sig, pos0 + t * ut), 0.0, 1e-5 * sig)
    assert abs(fd_p - float((lr0 * ut).sum())) <= 1e-6 * max(abs(fd_p), 1e-3 * float(lr0.abs().max()))


def test_autograd_function_routes_through_the_engine(problem):
    from paper_2508_06628_amd.trajectory import TrajectoryLoss
    w, eps, sig, target, (loss_ref, lr0_ref, de_ref, ds_ref) = problem
    eng = _engine(w, "f64")
    eng.set_target(torch.tensor(target, device="cuda"))
    e_t = torch.tensor(eps, dtype=torch.float64, device="cuda", requires_grad=True)
    s_t = torch.tensor(sig, dtype=torch.float64, device="cuda", requires_grad=True)
    p_t = eng.batch.pos.clone().requires_grad_(True)
    loss = TrajectoryLoss.apply(e_t, s_t, p_t, eng)
    loss.backward()
    assert abs(e_t.grad.item() - de_ref) <= 1e-8 * abs(de_ref)
    assert abs(s_t.grad.item() - ds_ref) <= 1e-8 * abs(ds_ref)
    assert np.abs(p_t.grad.T.cpu().numpy() - lr0_ref).max() <= 1e-8 * np.abs(lr0_ref).max()


def test_recorded_segment_equals_step_loop():
    # ts_nve_record reproduces ts_nve_step bit for bit and stores every position
    from paper_2508_06628_amd import api
    w = _workload()
    outs = []
    for record in (False, True):
        b = api.Batch.from_workload(w)
        nl = api.build_neighbor_list(b, w.potential.cutoff, 0.3)
        pp = api.pair_params_from_spec(w.potential, "f32")
        F = api.force_buffer(b, "f32")
        api.ts_pair_forces(b, nl, pp, F)
        if record:
            traj = torch.zeros((13, 3, b.n_atoms), dtype=torch.float64, device="cuda")
            api.ts_nve_record(b, nl, pp, w.dt, w.accel, 12, F, traj)
            assert torch.equal(traj[0], torch.tensor(w.pos.T.copy(), device="cuda"))
            assert torch.equal(traj[12], b.pos)
        else:
            api.ts_nve_step(b, nl, pp, w.dt, w.accel, 12, F)
        outs.append((b.pos.clone(), b.vel.clone(), F.clone()))
    for x, y in zip(*outs):
        assert torch.equal(x, y)


# ----------------------------------------------------------------------------- shifted-force LJ


def _sf_workload():
    import dataclasses
    w = _workload()
    w.potential = dataclasses.replace(w.potential, kind="lj_sf", shift_energy=False)
    return w


def _oracle_sf(w, eps, sig, target):
    pot = PotentialSpec("lj_sf", np.array([[[eps, sig, 0.0]]]), w.potential.cutoff, False)
    traj, _ = oadj.trajectory_positions(w.pos, w.vel, w.mass, w.cell, w.sys_offsets, w.species, pot, w.dt, N_STEPS,
                                        w.accel)
    r_max = RDF["r_end"] + 6 * RDF["sigma"]
    g = oadj.batch_rdf(traj[-1], w.cell, w.sys_offsets, RDF["n_bins"], RDF["r_end"], RDF["sigma"], r_max)
    if target is None:
        return g
    lr_T = oadj.rdf_loss_grad(traj[-1], w.cell, w.sys_offsets, RDF["n_bins"], RDF["r_end"], RDF["sigma"], r_max, g,
                              target)
    lr0, _, tb = oadj.reverse_nve(traj, w.mass, w.cell, w.sys_offsets, w.species, pot, w.dt, w.accel, lr_T,
                                  np.zeros_like(lr_T))
    return oadj.rdf_loss(g, target), lr0, tb[0, 0, 0], tb[0, 0, 1]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_shifted_force_gradient_matches_oracle_and_fd_at_1e4(prec):
    # with the shifted-force truncation the force has no jump at the cutoff, so central differences
    # at the 1e-4 relative step (sigma, positions as well as epsilon) agree with the adjoint
    w = _sf_workload()
    eps, sig = float(w.potential.params[0, 0, 0]), float(w.potential.params[0, 0, 1])
    target = _oracle_sf(w, eps * 1.05, sig * 1.05, None)
    loss_ref, lr0_ref, de_ref, ds_ref = _oracle_sf(w, eps, sig, target)
    eng = _engine(w, prec)
    eng.set_target(torch.tensor(target, device="cuda"))
    pos0 = eng.batch.pos.clone()
    loss = eng.forward(eps, sig, pos0).item()
    de, ds, lr0 = eng.backward()
    eng.check_status()
    tol = 1e-8 if prec == "f64" else 1e-3
    assert abs(loss - loss_ref) <= (1e-9 if prec == "f64" else 1e-4) * abs(loss_ref)
    assert abs(de - de_ref) <= tol * abs(de_ref)
    assert abs(ds - ds_ref) <= tol * abs(ds_ref)
    assert np.abs(lr0.T.cpu().numpy() - lr0_ref).max() <= tol * np.abs(lr0_ref).max()
    if prec != "f64":
        return

    def L(e, s, p):
        return eng.forward(e, s, p).item()

    def central(fun, x, h):
        d1 = (fun(x + h) - fun(x - h)) / (2 * h)
        d2 = (fun(x + h / 2) - fun(x - h / 2)) / h
        return (4 * d2 - d1) / 3

    h = 1e-4
    assert abs(central(lambda e: L(e, sig, pos0), eps, h * eps) - de) <= 1e-6 * abs(de)
    assert abs(central(lambda sg: L(eps, sg, pos0), sig, h * sig) - ds) <= 1e-6 * abs(ds)
    rng = np.random.default_rng(4)
    u = rng.normal(size=pos0.shape)
    u /= np.linalg.norm(u)
    ut = torch.tensor(u, device="cuda")
    fd_p = central(lambda t: L(eps, sig, pos0 + t * ut), 0.0, h * sig)
    assert abs(fd_p - float((lr0 * ut).sum())) <= 1e-6 * max(abs(fd_p), 1e-3 * float(lr0.abs().max()))
