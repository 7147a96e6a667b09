"""The no-allocation pair adjoint (ts_pair_adjoint_noalloc, called through the C ABI with a list that
has no workspace) against the workspace entry point ts_pair_adjoint on the same inputs: two calls
in a row on one GPU, the second on a smaller batch, so that the library's static partial-sum array
holds the first call's values when the second starts.  Per-atom adjoints are per-atom sums (no
atomics) and must agree bitwise; the parameter gradient sums workgroup partials with atomics in
float64, so it agrees to rounding.  Both are also checked against the FP64 oracle."""
import numpy as np
import pytest

from oracle import adjoint as oadj
from workloads import random_small_batch

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2508_06628_amd import _native
    _native.lib()
    yield
    torch.cuda.synchronize()


def _case(seed, n_systems, kind, prec):
    from paper_2508_06628_amd import api
    w = random_small_batch(seed, n_systems=n_systems, n_range=(5, 60), kind=kind, n_species=2 if kind == "lj" else 1)
    pot = w.potential
    b = api.Batch.from_workload(w)
    nl = api.build_neighbor_list(b, pot.cutoff, 0.2)
    pp = api.pair_params_from_spec(pot, prec)
    rng = np.random.default_rng(seed)
    lr0, lv0 = rng.normal(size=w.pos.shape), rng.normal(size=w.pos.shape)
    dt, wk, accel = 0.01, 0.005, 1.0
    outs = []
    for noalloc in (False, True):
        lr = torch.tensor(lr0.T.copy(), device="cuda")
        lv = torch.tensor(lv0.T.copy(), device="cuda")
        tb = torch.zeros(48, dtype=torch.float64, device="cuda")
        if noalloc:
            api.ts_pair_adjoint_noalloc(b, nl, pp, dt, wk, accel, lr, lv, tb, without_workspace=True)
        else:
            api.ts_pair_adjoint(b, nl, pp, dt, wk, accel, lr, lv, tb)
        torch.cuda.synchronize()
        outs.append((lr.cpu().numpy(), lv.cpu().numpy(), tb.cpu().numpy()))
    (lr_a, lv_a, tb_a), (lr_b, lv_b, tb_b) = outs
    assert np.array_equal(lr_a, lr_b)
    assert np.array_equal(lv_a, lv_b)
    assert np.abs(tb_b - tb_a).max() <= 1e-12 * np.abs(tb_a).max()
    u = accel * (lv0 + dt * lr0) / w.mass[:, None]
    lr_ref = lr0 + wk * oadj.batch_hvp(w.pos, w.cell, w.sys_offsets, w.species, pot, u)
    tb_ref = wk * oadj.batch_param_vjp(w.pos, w.cell, w.sys_offsets, w.species, pot, u)
    tol = 1e-8 if prec == "f64" else 1e-3
    assert np.abs(lr_b.T - lr_ref).max() <= tol * np.abs(lr_ref - lr0).max()
    ns = pot.params.shape[0]
    got = tb_b.reshape(4, 4, 3)[:ns, :ns]
    assert np.abs(got - tb_ref).max() <= tol * np.abs(tb_ref).max()


@pytest.mark.parametrize("kind,prec", [("lj", "f64"), ("morse", "f32")])
def test_noalloc_pair_adjoint_matches_workspace_entry_point(kind, prec):
    _case(90, 7, kind, prec)  # first call on this GPU: looks up the static array
    _case(91, 3, kind, prec)  # smaller batch: the array still holds the first call's partial sums
