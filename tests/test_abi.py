"""The C-ABI library loads, exports every symbol the header declares, its structs match the
binding's layout, and host-side argument checks reject bad input before any launch (CPU only)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ts_api.h")


def _lib():
    from paper_2508_06628_amd import _native
    return _native


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b(ts_\w+)\s*\(", text, flags=re.M)))


def test_every_declared_symbol_is_exported_and_bound():
    N = _lib()
    L = N.lib()
    names = declared_functions()
    assert len(names) >= 13
    for name in names:
        assert hasattr(L, name), name
        assert name in N.SIGNATURES, name
    assert set(N.SIGNATURES) == set(names)
    assert L.ts_version().decode().startswith("ts-mi355x")


def test_struct_layout_matches_header(tmp_path):
    N = _lib()
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "ts_api.h"
#define P(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
  printf("ts_batch %zu\nts_pair_params %zu\nts_neighbor_list %zu\nts_fire_config %zu\nts_fire_state %zu\n",
         sizeof(ts_batch), sizeof(ts_pair_params), sizeof(ts_neighbor_list), sizeof(ts_fire_config),
         sizeof(ts_fire_state));
  P(ts_batch, cell) P(ts_batch, h_sys_offsets) P(ts_pair_params, params) P(ts_neighbor_list, workspace_bytes)
  P(ts_neighbor_list, nbr) P(ts_fire_config, max_iter) P(ts_fire_state, scratch)
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines())
    assert int(out["ts_batch"]) == ctypes.sizeof(N.TsBatch)
    assert int(out["ts_pair_params"]) == ctypes.sizeof(N.TsPairParams)
    assert int(out["ts_neighbor_list"]) == ctypes.sizeof(N.TsNeighborList)
    assert int(out["ts_fire_config"]) == ctypes.sizeof(N.TsFireConfig)
    assert int(out["ts_fire_state"]) == ctypes.sizeof(N.TsFireState)
    assert int(out["ts_batch.cell"]) == N.TsBatch.cell.offset
    assert int(out["ts_batch.h_sys_offsets"]) == N.TsBatch.h_sys_offsets.offset
    assert int(out["ts_pair_params.params"]) == N.TsPairParams.params.offset
    assert int(out["ts_neighbor_list.workspace_bytes"]) == N.TsNeighborList.workspace_bytes.offset
    assert int(out["ts_neighbor_list.nbr"]) == N.TsNeighborList.nbr.offset
    assert int(out["ts_fire_config.max_iter"]) == N.TsFireConfig.max_iter.offset
    assert int(out["ts_fire_state.scratch"]) == N.TsFireState.scratch.offset


def _fake_batch(N, offsets):
    # device pointers are never dereferenced by the host-side checks; the host offsets are
    h = np.asarray(offsets, dtype=np.int64)
    b = N.TsBatch()
    b.n_atoms = int(h[-1])
    b.n_systems = len(h) - 1
    b.stride = 0
    fake = 0x1000
    b.sys_offsets = b.system_idx = b.pos = b.vel = b.cell = fake
    b.h_sys_offsets = h.ctypes.data
    return b, h


def _pp(N, **kw):
    pp = N.TsPairParams()
    pp.kind, pp.prec, pp.n_species, pp.shift_energy, pp.cutoff = 0, 0, 1, 0, 2.5
    pp.params[0], pp.params[1] = 1.0, 1.0
    for k, v in kw.items():
        setattr(pp, k, v)
    return pp


def _nl(N, n_atoms, n_sys, **kw):
    nl = N.TsNeighborList()
    nl.cutoff, nl.skin, nl.max_nbr, nl.bin_factor = 2.5, 0.3, 64, 1
    nl.nbr = nl.n_nbr = nl.ref_pos = nl.ref_cell = nl.status = nl.workspace = 0x1000
    nl.workspace_bytes = N.lib().ts_neighbor_workspace_bytes(n_atoms, n_sys)
    for k, v in kw.items():
        setattr(nl, k, v)
    return nl


def test_host_argument_checks():
    N = _lib()
    L = N.lib()
    b, h = _fake_batch(N, [0, 10, 25])
    F = ctypes.c_void_p(0x1000)
    by = ctypes.byref
    ok_nl = _nl(N, 25, 2)
    # bad offsets: last != n_atoms
    bad, hb = _fake_batch(N, [0, 10, 25])
    bad.n_atoms = 24
    assert L.ts_pair_forces(by(bad), by(ok_nl), by(_pp(N)), F, None, None, None) == N.TS_E_INVALID
    # non-monotone offsets
    nm, hn = _fake_batch(N, [0, 12, 10, 25])
    assert L.ts_neighbor_build(by(nm), by(_nl(N, 25, 3)), 1, None) == N.TS_E_INVALID
    # unknown potential, bad prec, too many species, bad cutoff
    assert L.ts_pair_forces(by(b), by(ok_nl), by(_pp(N, kind=7)), F, None, None, None) == N.TS_E_UNSUPPORTED
    assert L.ts_pair_forces(by(b), by(ok_nl), by(_pp(N, prec=3)), F, None, None, None) == N.TS_E_UNSUPPORTED
    assert L.ts_pair_forces(by(b), by(ok_nl), by(_pp(N, n_species=5)), F, None, None, None) == N.TS_E_INVALID
    assert L.ts_pair_forces(by(b), by(ok_nl), by(_pp(N, cutoff=-1.0)), F, None, None, None) == N.TS_E_INVALID
    # list radius below the potential cutoff, half list for forces, small workspace, zero capacity
    assert L.ts_pair_forces(by(b), by(_nl(N, 25, 2, cutoff=2.0, skin=0.1)), by(_pp(N)), F, None, None,
                            None) == N.TS_E_INVALID
    assert L.ts_pair_forces(by(b), by(_nl(N, 25, 2, half=1)), by(_pp(N)), F, None, None, None) == N.TS_E_UNSUPPORTED
    assert L.ts_neighbor_build(by(b), by(_nl(N, 25, 2, workspace_bytes=16)), 1, None) == N.TS_E_INVALID
    assert L.ts_neighbor_build(by(b), by(_nl(N, 25, 2, max_nbr=0)), 1, None) == N.TS_E_INVALID
    assert L.ts_neighbor_build(by(b), by(_nl(N, 25, 2, skin=-0.1)), 1, None) == N.TS_E_INVALID
    # NVE: bad dt, missing velocities
    assert L.ts_nve_step(by(b), by(ok_nl), by(_pp(N)), -1.0, 1.0, 10, F, None, None, None, 0, None) == N.TS_E_INVALID
    nv, hv = _fake_batch(N, [0, 10, 25])
    nv.vel = None
    assert L.ts_nve_step(by(nv), by(ok_nl), by(_pp(N)), 1.0, 1.0, 10, F, None, None, None, 0, None) == N.TS_E_INVALID
    # too many atoms in one system for the 17-bit local index
    big, hbig = _fake_batch(N, [0, N.TS_MAX_SYSTEM_ATOMS + 1])
    assert L.ts_neighbor_build(by(big), by(_nl(N, N.TS_MAX_SYSTEM_ATOMS + 1, 1)), 1, None) == N.TS_E_CAPACITY
    assert L.ts_strerror(N.TS_E_CAPACITY).decode() == "size exceeds a library limit"
    # Langevin: negative or non-finite friction, missing temperature or counter, negative step count
    kT, ctr = ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000)
    pp = by(_pp(N))
    assert L.ts_langevin_step(by(b), by(ok_nl), pp, 1.0, 1.0, -0.1, kT, 1, ctr, 5, F, 0, None) == N.TS_E_INVALID
    assert L.ts_langevin_step(by(b), by(ok_nl), pp, 1.0, 1.0, float("nan"), kT, 1, ctr, 5, F, 0,
                              None) == N.TS_E_INVALID
    assert L.ts_langevin_step(by(b), by(ok_nl), pp, 1.0, 1.0, 0.1, None, 1, ctr, 5, F, 0, None) == N.TS_E_INVALID
    assert L.ts_langevin_step(by(b), by(ok_nl), pp, 1.0, 1.0, 0.1, kT, 1, None, 5, F, 0, None) == N.TS_E_INVALID
    assert L.ts_langevin_step(by(b), by(ok_nl), pp, 1.0, 1.0, 0.1, kT, 1, ctr, -1, F, 0, None) == N.TS_E_INVALID
    assert L.ts_langevin_step(by(nv), by(ok_nl), pp, 1.0, 1.0, 0.1, kT, 1, ctr, 5, F, 0, None) == N.TS_E_INVALID
    # graph export: radius beyond the list radius or not positive, missing outputs, negative capacity
    rp, eo, ei = ctypes.c_void_p(0x4000), ctypes.c_void_p(0x5000), ctypes.c_void_p(0x6000)
    r_list = ok_nl.cutoff + ok_nl.skin
    assert L.ts_graph_export(by(b), by(ok_nl), r_list * 1.01, rp, eo, ei, None, None, 10, None) == N.TS_E_INVALID
    assert L.ts_graph_export(by(b), by(ok_nl), 0.0, rp, eo, ei, None, None, 10, None) == N.TS_E_INVALID
    assert L.ts_graph_export(by(b), by(ok_nl), 1.0, None, eo, ei, None, None, 10, None) == N.TS_E_INVALID
    assert L.ts_graph_export(by(b), by(ok_nl), 1.0, rp, None, ei, None, None, 10, None) == N.TS_E_INVALID
    assert L.ts_graph_export(by(b), by(ok_nl), 1.0, rp, eo, None, None, None, 10, None) == N.TS_E_INVALID
    assert L.ts_graph_export(by(b), by(ok_nl), 1.0, rp, eo, ei, None, None, -1, None) == N.TS_E_INVALID


def test_pair_adjoint_noalloc_host_checks():
    # the no-allocation variant takes a list without workspace, rejects more systems than its static
    # array holds when the parameter gradient is wanted, and returns before any launch when there is
    # nothing to do (dt_drift = w_kick = 0), so these checks run without a GPU
    N = _lib()
    L = N.lib()
    by = ctypes.byref
    b, h = _fake_batch(N, [0, 10, 25])
    lr, lv, tb = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000)
    no_ws = _nl(N, 25, 2, workspace=None, workspace_bytes=0)
    assert L.ts_pair_adjoint_noalloc(by(b), by(no_ws), by(_pp(N)), 0.0, 0.0, 1.0, lr, lv, tb, None) == N.TS_OK
    assert L.ts_pair_adjoint(by(b), by(no_ws), by(_pp(N)), 0.0, 0.0, 1.0, lr, lv, tb, None) == N.TS_E_INVALID
    assert L.ts_pair_adjoint_noalloc(by(b), by(no_ws), by(_pp(N)), 0.0, 0.0, 1.0, None, lv, tb,
                                     None) == N.TS_E_INVALID
    many, hm = _fake_batch(N, list(range(4098)))
    nl_many = _nl(N, 4097, 4097, workspace=None, workspace_bytes=0)
    assert L.ts_pair_adjoint_noalloc(by(many), by(nl_many), by(_pp(N)), 0.0, 0.0, 1.0, lr, lv, tb,
                                     None) == N.TS_E_CAPACITY
    # without the parameter gradient there is no limit on the number of systems
    assert L.ts_pair_adjoint_noalloc(by(many), by(nl_many), by(_pp(N)), 0.0, 0.0, 1.0, lr, lv, None,
                                     None) == N.TS_OK
    at_limit, hl = _fake_batch(N, list(range(4097)))
    nl_lim = _nl(N, 4096, 4096, workspace=None, workspace_bytes=0)
    assert L.ts_pair_adjoint_noalloc(by(at_limit), by(nl_lim), by(_pp(N)), 0.0, 0.0, 1.0, lr, lv, tb,
                                     None) == N.TS_OK
