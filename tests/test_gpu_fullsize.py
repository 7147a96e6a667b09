"""Parity at the workloads' full sizes, in the launch configuration the benchmark uses, on atoms
sampled from every system: the oracle computes each sampled atom's pair set and force by brute
force against its whole system."""
import numpy as np
import pytest

from oracle import forces as oforces
from oracle import pairs as opairs
from workloads import argon_batch, copper_uneven_batch, soft_sphere_jamming_batch

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _check_sampled(w, nl, b, F, prec, per_system, seed):
    rng = np.random.default_rng(seed)
    i_all, j_all, s0, s1, s2 = nl.entries()
    Fg = F.T.double().cpu().numpy()
    pot = w.potential
    r_list = nl.cutoff + nl.skin
    for s in range(w.n_systems):
        sl = w.system(s)
        n = sl.stop - sl.start
        rows = np.sort(rng.choice(n, size=min(per_system, n), replace=False))
        # pair set of the sampled rows: exact outside the 1e-9 band at r_list
        o = opairs.system_pairs(w.pos[sl], w.cell[s], r_list, rows=rows)
        sel = np.isin(i_all, sl.start + rows)
        g = dict(i=i_all[sel] - sl.start, j=j_all[sel], S=np.stack([s0[sel], s1[sel], s2[sel]], 1))
        d = w.pos[sl][g["j"]] - w.pos[sl][g["i"]] + g["S"] @ w.cell[s]
        g["r2"] = (d * d).sum(1)
        assert np.array_equal(opairs.pair_keys(g, r_list, 1e-9), opairs.pair_keys(o, r_list, 1e-9)), s
        # forces of the sampled rows
        _, F_ref, _ = oforces.system_efw(w.pos[sl], w.cell[s], w.species[sl], pot.params, pot.kind, pot.cutoff,
                                         pot.shift_energy, rows=rows)
        A, _, _ = oforces.pair_magnitude_sums(w.pos[sl], w.cell[s], w.species[sl], pot.params, pot.kind, pot.cutoff,
                                              rows=rows)
        err = np.linalg.norm(Fg[sl][rows] - F_ref[rows], axis=1)
        scale = np.maximum(np.linalg.norm(F_ref[rows], axis=1), 0.1 * A[rows])
        rel = 1e-5 if prec == "f32" else 1e-10
        assert np.all(err <= rel * scale), (s, (err / scale).max())


def _setup(w, prec, bin_factor=2):
    from paper_2508_06628_amd import api
    b = api.Batch.from_workload(w)
    nl = api.build_neighbor_list(b, w.potential.cutoff, w.skin, bin_factor=bin_factor)
    pp = api.pair_params_from_spec(w.potential, prec)
    F = api.force_buffer(b, prec)
    api.ts_pair_forces(b, nl, pp, F)
    torch.cuda.synchronize()
    st = nl.read_status()
    assert st[1] == 0 and st[3] == 0 and st[4] == 0
    return api, b, nl, pp, F


def test_argon_64x864_sampled():
    w = argon_batch(64, seed=1)
    api, b, nl, pp, F = _setup(w, "f32")
    _check_sampled(w, nl, b, F, "f32", per_system=3, seed=0)
    # one NVE step of the whole batch (the benchmark's graph path) against the oracle per sampled atom
    F0 = F.clone()
    api.ts_nve_step(b, nl, pp, w.dt, w.accel, 1, F, use_graph=True)
    torch.cuda.synchronize()
    v_half = w.vel + 0.5 * w.dt * F0.T.double().cpu().numpy() * (w.accel / w.mass)[:, None]
    pos1 = w.pos + w.dt * v_half
    L = np.abs(np.linalg.det(w.cell)).max() ** (1 / 3)
    assert np.abs(b.positions() - pos1).max() <= 1e-10 * L


def test_copper_uneven_512_sampled():
    w = copper_uneven_batch(512, seed=2)
    api, b, nl, pp, F = _setup(w, "f32", bin_factor=1)
    rng = np.random.default_rng(1)
    sub = np.sort(rng.choice(512, size=24, replace=False))
    # check a sample of systems (the smallest, narrowest cells included)
    counts = np.diff(w.sys_offsets)
    sub = np.unique(np.concatenate([sub, [int(np.argmin(counts)), int(np.argmax(counts))]]))
    Fg = F.T.double().cpu().numpy()
    ws = w.subset(sub)
    F_sub = np.concatenate([Fg[w.system(s)] for s in sub])
    i_all, j_all, s0, s1, s2 = nl.entries()
    # remap the list entries of the sampled systems onto the subset's atom numbering
    keep = np.isin(np.searchsorted(w.sys_offsets, i_all, side="right") - 1, sub)
    old_sys = np.searchsorted(w.sys_offsets, i_all[keep], side="right") - 1
    new_base = dict(zip(sub, ws.sys_offsets[:-1]))
    new_i = np.array([new_base[s] for s in old_sys]) + (i_all[keep] - w.sys_offsets[old_sys])

    class _NL:
        cutoff, skin = nl.cutoff, nl.skin

        @staticmethod
        def entries():
            return new_i, j_all[keep], s0[keep], s1[keep], s2[keep]

    _check_sampled(ws, _NL, None, torch.tensor(F_sub.T.copy()), "f32", per_system=4, seed=2)


def test_soft_sphere_8x32000_sampled():
    w = soft_sphere_jamming_batch(8, 32000, seed=4)
    api, b, nl, pp, F = _setup(w, "f32", bin_factor=1)
    _check_sampled(w, nl, b, F, "f32", per_system=6, seed=3)
