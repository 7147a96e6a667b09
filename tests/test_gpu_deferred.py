"""The deferred neighbor-list rebuild of the fused step loops (a second row buffer; systems predicted
to fail the validity bound are rebuilt one step ahead by extra workgroups of the step launch) gives
bitwise the trajectory of the synchronous rebuild: forces only see pairs within the cutoff, and
both lists hold all of them in canonical order.  Checked for velocity-Verlet and Langevin, with
the default pre-flag factor and with a small one that lets lists fail before their deferred
rebuild (the synchronous fallback into either buffer), and the list left in the caller's buffer is
valid at the final positions."""
import numpy as np
import pytest

from oracle import pairs as opairs
from workloads import argon_batch

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2508_06628_amd import _native
    _native.lib()
    yield
    torch.cuda.synchronize()


def _run(w, deferred, n_steps, chunk, langevin=False, prec="f32"):
    from paper_2508_06628_amd import api
    b = api.Batch.from_workload(w)
    nl = api.build_neighbor_list(b, w.potential.cutoff, w.skin, bin_factor=2, margin=1.3, deferred=deferred)
    assert nl.deferred == deferred
    nl.lanes_per_atom = 4
    pp = api.pair_params_from_spec(w.potential, prec)
    F = api.force_buffer(b, prec)
    api.ts_pair_forces(b, nl, pp, F)
    nl.status.zero_()
    kT = torch.full((w.n_systems,), 8.617333262145179e-5 * 120.0, dtype=torch.float64, device="cuda")
    ctr = torch.zeros(1, dtype=torch.int64, device="cuda")
    done = 0
    while done < n_steps:
        k = min(chunk, n_steps - done)
        if langevin:
            api.ts_langevin_step(b, nl, pp, w.dt, w.accel, 0.01, kT, 77, ctr, k, F)
        else:
            api.ts_nve_step(b, nl, pp, w.dt, w.accel, k, F, use_graph=True)
        done += k
    torch.cuda.synchronize()
    return b, nl, F


@pytest.mark.parametrize("langevin", [False, True])
@pytest.mark.parametrize("prefactor", ["2", "0.25"])
def test_deferred_rebuild_matches_synchronous(langevin, prefactor, monkeypatch):
    monkeypatch.setenv("TS_DEFER_PREFACTOR", prefactor)
    w = argon_batch(6, reps=(3, 3, 3), seed=91)
    b0, nl0, F0 = _run(w, False, 240, 60, langevin)
    b1, nl1, F1 = _run(w, True, 240, 60, langevin)
    st0, st1 = nl0.read_status(), nl1.read_status()
    for st in (st0, st1):
        assert st[1] == 0 and st[3] == 0 and st[4] == 0
    assert st0[2] > 0 and st1[2] >= st0[2]  # rebuilds happened; deferred ones come a little earlier
    assert torch.equal(b0.pos, b1.pos)
    assert torch.equal(b0.vel, b1.vel)
    assert torch.equal(F0, F1)
    # the deferred run's list, back in the caller's buffer, holds every pair within the cutoff at
    # the final positions (with its image shift)
    pos = b1.positions()
    i_all, j_all, s0, s1, s2 = nl1.entries()
    have = set(zip(i_all.tolist(), j_all.tolist(), s0.tolist(), s1.tolist(), s2.tolist()))
    for s in range(w.n_systems):
        sl = w.system(s)
        p = opairs.system_pairs(pos[sl], w.cell[s], w.potential.cutoff - 1e-9)
        a0 = int(w.sys_offsets[s])
        for i, j, sh in zip(p["i"], p["j"], p["S"]):
            assert (a0 + int(i), int(j), int(sh[0]), int(sh[1]), int(sh[2])) in have
