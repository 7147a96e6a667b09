"""ctypes view of the C ABI in ``include/ts_api.h`` (argument marshalling only).

The structs below mirror the header field by field; ``tests/test_abi.py`` checks their sizes
and offsets against the compiled library's expectations.  Loading fails loudly when the shared
library has not been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_size_t, c_void_p

from .build import LIB_PATH

TS_OK = 0
TS_NOT_CONVERGED = 1
TS_E_INVALID = -1
TS_E_UNSUPPORTED = -2
TS_E_CAPACITY = -3
TS_E_HIP = -4

TS_LJ, TS_MORSE, TS_SOFT_SPHERE, TS_LJ_SF, TS_MORSE_SF = 0, 1, 2, 3, 4
TS_PAIR_F32, TS_PAIR_F64 = 0, 1
TS_MAX_SPECIES = 4
TS_MAX_SYSTEM_ATOMS = 131072
TS_MAX_IMAGE_SHIFT = 15

TS_STATUS_MAX_NBR = 0
TS_STATUS_OVERFLOW = 1
TS_STATUS_REBUILDS = 2
TS_STATUS_NONFINITE = 3
TS_STATUS_SHIFT = 4
TS_STATUS_WORDS = 8
TS_FIRE_TAIL_ITERS = 256

KIND_CODES = {"lj": TS_LJ, "morse": TS_MORSE, "soft_sphere": TS_SOFT_SPHERE, "lj_sf": TS_LJ_SF,
              "morse_sf": TS_MORSE_SF}
PREC_CODES = {"f32": TS_PAIR_F32, "f64": TS_PAIR_F64}


class TsBatch(ctypes.Structure):
    _fields_ = [
        ("n_atoms", c_int64),
        ("n_systems", c_int64),
        ("stride", c_int64),
        ("sys_offsets", c_void_p),
        ("h_sys_offsets", c_void_p),
        ("system_idx", c_void_p),
        ("pos", c_void_p),
        ("vel", c_void_p),
        ("mass", c_void_p),
        ("species", c_void_p),
        ("cell", c_void_p),
    ]


class TsPairParams(ctypes.Structure):
    _fields_ = [
        ("kind", c_int32),
        ("prec", c_int32),
        ("n_species", c_int32),
        ("shift_energy", c_int32),
        ("cutoff", c_double),
        ("params", c_double * (TS_MAX_SPECIES * TS_MAX_SPECIES * 3)),
    ]


class TsNeighborList(ctypes.Structure):
    _fields_ = [
        ("cutoff", c_double),
        ("skin", c_double),
        ("half", c_int32),
        ("max_nbr", c_int32),
        ("bin_factor", c_int32),
        ("lanes_per_atom", c_int32),
        ("group_atoms", c_int32),
        ("reserved", c_int32),
        ("nbr", c_void_p),
        ("n_nbr", c_void_p),
        ("ref_pos", c_void_p),
        ("ref_cell", c_void_p),
        ("status", c_void_p),
        ("workspace", c_void_p),
        ("workspace_bytes", c_size_t),
        ("nbr_alt", c_void_p),
        ("n_nbr_alt", c_void_p),
        ("ref_pos_alt", c_void_p),
    ]


class TsFireConfig(ctypes.Structure):
    _fields_ = [
        ("dt_start", c_double),
        ("dt_max", c_double),
        ("alpha_start", c_double),
        ("f_inc", c_double),
        ("f_dec", c_double),
        ("f_alpha", c_double),
        ("fmax", c_double),
        ("cell_mass", c_double),
        ("n_min", c_int32),
        ("relax_cell", c_int32),
        ("max_iter", c_int64),
    ]


class TsFireState(ctypes.Structure):
    _fields_ = [
        ("dt", c_void_p),
        ("alpha", c_void_p),
        ("n_pos", c_void_p),
        ("converged", c_void_p),
        ("n_iter", c_void_p),
        ("deform", c_void_p),
        ("deform_vel", c_void_p),
        ("ref_cell", c_void_p),
        ("scratch", c_void_p),
    ]


# name -> (restype, argtypes): every symbol the header declares
SIGNATURES = {
    "ts_neighbor_workspace_bytes": (c_size_t, [c_int64, c_int64]),
    "ts_neighbor_build": (c_int32, [POINTER(TsBatch), POINTER(TsNeighborList), c_int32, c_void_p]),
    "ts_graph_export": (c_int32, [POINTER(TsBatch), POINTER(TsNeighborList), c_double, c_void_p, c_void_p, c_void_p,
                                  c_void_p, c_void_p, ctypes.c_int64, c_void_p]),
    "ts_lorentz_berthelot": (c_int32, [c_int32, c_void_p, c_void_p, POINTER(TsPairParams)]),
    "ts_pair_forces": (c_int32, [POINTER(TsBatch), POINTER(TsNeighborList), POINTER(TsPairParams), c_void_p,
                                 c_void_p, c_void_p, c_void_p]),
    "ts_nve_step": (c_int32, [POINTER(TsBatch), POINTER(TsNeighborList), POINTER(TsPairParams), c_double, c_double,
                              c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_void_p]),
    "ts_nve_record": (c_int32, [POINTER(TsBatch), POINTER(TsNeighborList), POINTER(TsPairParams), c_double,
                                c_double, c_int32, c_void_p, c_void_p, c_int32, c_void_p]),
    "ts_langevin_step": (c_int32, [POINTER(TsBatch), POINTER(TsNeighborList), POINTER(TsPairParams), c_double,
                                   c_double, c_double, c_void_p, ctypes.c_uint64, c_void_p, c_int32, c_void_p, c_int32,
                                   c_void_p]),
    "ts_adjoint_segment": (c_int32, [POINTER(TsBatch), POINTER(TsNeighborList), POINTER(TsPairParams), c_void_p,
                                     c_int32, c_double, c_double, c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                                     c_int32, c_void_p]),
    "ts_fire_step": (c_int32, [POINTER(TsBatch), POINTER(TsFireState), POINTER(TsFireConfig), POINTER(TsNeighborList),
                               POINTER(TsPairParams), c_int64, c_void_p, c_void_p, c_void_p, c_int32, c_void_p]),
    "ts_pair_adjoint": (c_int32, [POINTER(TsBatch), POINTER(TsNeighborList), POINTER(TsPairParams), c_double,
                                  c_double, c_double, c_void_p, c_void_p, c_void_p, c_void_p]),
    "ts_pair_adjoint_noalloc": (c_int32, [POINTER(TsBatch), POINTER(TsNeighborList), POINTER(TsPairParams), c_double,
                                          c_double, c_double, c_void_p, c_void_p, c_void_p, c_void_p]),
    "ts_rdf_smeared": (c_int32, [POINTER(TsBatch), POINTER(TsNeighborList), c_int32, c_double, c_double, c_double,
                                 c_void_p, c_void_p]),
    "ts_rdf_loss": (c_int32, [c_void_p, c_void_p, c_int64, c_int32, c_void_p, c_void_p, c_void_p]),
    "ts_rdf_vjp": (c_int32, [POINTER(TsBatch), POINTER(TsNeighborList), c_int32, c_double, c_double, c_double,
                             c_void_p, c_void_p, c_void_p]),
    "ts_kinetic_energy": (c_int32, [POINTER(TsBatch), c_double, c_void_p, c_void_p]),
    "ts_release_graphs": (None, []),
    "ts_strerror": (c_char_p, [c_int32]),
    "ts_version": (c_char_p, []),
}

_LIB = None


class TsError(RuntimeError):
    def __init__(self, name, code):
        self.code = code
        super().__init__(f"{name} failed: {code} ({lib().ts_strerror(code).decode()})")


def lib():
    """The loaded library (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2508_06628_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def check(name, code):
    if code != TS_OK and code != TS_NOT_CONVERGED:
        raise TsError(name, code)
    return code
