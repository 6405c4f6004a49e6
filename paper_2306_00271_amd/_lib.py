"""ctypes declarations of the C ABI in include/rheed.h (argument marshalling only).

The shared library is loaded from this package directory.  There is no CPU
fallback: if librheed.so is missing or cannot be loaded, importing the
binding raises.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librheed.so")

RHEED_OK, RHEED_E_INVALID, RHEED_E_HIP, RHEED_E_NOMEM, RHEED_E_UNSUPPORTED = 0, -1, -2, -3, -4
RHEED_RK4, RHEED_RK6, RHEED_SP4, RHEED_SP6, RHEED_SP4_ABA, RHEED_SP6_ABA = 0, 1, 2, 3, 4, 5
RHEED_INTENSITY_FLUX, RHEED_INTENSITY_PAPER = 0, 1
RHEED_PAIR_OK, RHEED_PAIR_SINGULAR, RHEED_PAIR_NONFINITE, RHEED_PAIR_SYNC, RHEED_PAIR_BREAKDOWN = 0, 1, 2, 3, 4
RHEED_LAYOUT_AUTO, RHEED_LAYOUT_WHOLE, RHEED_LAYOUT_SPLIT = 0, 1, 2
RHEED_STAGES_FP64, RHEED_STAGES_FP32 = 0, 1
RHEED_MAX_BEAMS = 576
RHEED_MAX_BOX = 300
RHEED_MAX_BOX_LARGE = 1024
RHEED_MAX_BOX_XL = 1536
RHEED_MAX_BOX_XXL = 4096
RHEED_NOALLOC_MAX_ATOMS = 4096


class Structure(C.Structure):
    _fields_ = [
        ("n_beams", C.c_int32),
        ("beam_hk", C.POINTER(C.c_int32)),
        ("recip", C.c_double * 4),
        ("n_slices", C.c_int32),
        ("thickness", C.c_double),
        ("wavenumber", C.c_double),
        ("n_atoms", C.c_int32),
        ("cell_area", C.c_double),
        ("scat_a", C.c_double * 4),
        ("scat_b", C.c_double * 4),
        ("kappa", C.c_double),
        ("charge", C.c_double),
        ("absorption", C.c_double),
        ("mean_inner_potential", C.c_double),
    ]


class Opts(C.Structure):
    _fields_ = [
        ("stepper", C.c_int),
        ("rhst_threshold", C.c_double),
        ("checkpoint_every", C.c_int32),
        ("convention", C.c_int),
        ("layout", C.c_int),
        ("stage_precision", C.c_int),
    ]


class PlanInfo(C.Structure):
    _fields_ = [
        ("n_struct", C.c_int32),
        ("n_pairs", C.c_int32),
        ("max_beams", C.c_int32),
        ("nodes_per_slice", C.c_int32),
        ("table_elems", C.c_int64),
        ("n_atoms_total", C.c_int64),
        ("fwd_workspace", C.c_size_t),
        ("bwd_workspace", C.c_size_t),
        ("split", C.c_int32),
        ("split_max_pairs", C.c_int32),
        ("large_pairs", C.c_int32),
        ("large_slots", C.c_int32),
        ("bulk_workspace", C.c_size_t),
        ("queue", C.c_int32),
        ("xl_pairs", C.c_int32),
        ("xl_slots", C.c_int32),
        ("xl_group", C.c_int32),
        ("xxl_pairs", C.c_int32),
        ("xxl_group", C.c_int32),
    ]


RHEED_TUNE_MAX = 8


class TuneReport(C.Structure):
    _fields_ = [
        ("n_candidates", C.c_int32),
        ("chosen", C.c_int32),
        ("split", C.c_int32 * RHEED_TUNE_MAX),
        ("large_cost_order", C.c_int32 * RHEED_TUNE_MAX),
        ("queue", C.c_int32 * RHEED_TUNE_MAX),
        ("ms", C.c_float * RHEED_TUNE_MAX),
    ]


SYMBOLS = {
    "rheed_beam_constants": ([C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)], C.c_int),
    "rheed_plan_create": ([C.POINTER(C.c_void_p), C.POINTER(Opts), C.c_int32, C.POINTER(Structure),
                           C.POINTER(C.c_int32)], C.c_int),
    "rheed_plan_destroy": ([C.c_void_p], C.c_int),
    "rheed_plan_get_info": ([C.c_void_p, C.POINTER(PlanInfo)], C.c_int),
    "rheed_plan_force_sync_failure": ([C.c_void_p, C.c_int32], C.c_int),
    "rheed_plan_table_offsets": ([C.c_void_p, C.POINTER(C.c_int64)], C.c_int),
    "rheed_plan_atom_offsets": ([C.c_void_p, C.POINTER(C.c_int64)], C.c_int),
    "rheed_potential": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "rheed_potential_backward": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "rheed_potential_backward_noalloc": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "rheed_forward": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                       C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "rheed_backward": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                        C.c_void_p], C.c_int),
    "rheed_forward_bulk": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                            C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "rheed_bulk_reflection": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int32, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "rheed_autotune": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                        C.POINTER(TuneReport)], C.c_int),
    "rheed_rfactor": ([C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "rheed_mfma_f64_peak": ([C.c_int32, C.c_int32, C.POINTER(C.c_double)], C.c_int),
    "rheed_status_string": ([C.c_int], C.c_char_p),
    "rheed_last_error": ([], C.c_char_p),
}


class RheedError(RuntimeError):
    def __init__(self, code, where, msg):
        super().__init__(f"{where}: status {code}: {msg}")
        self.code = code


def load(path: str = LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"librheed.so not found at {path}: build it with `python -m paper_2306_00271_amd.build`")
    lib = C.CDLL(path)
    for name, (argtypes, restype) in SYMBOLS.items():
        fn = getattr(lib, name)
        fn.argtypes = argtypes
        fn.restype = restype
    return lib


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        _LIB = load()
    return _LIB


def check(code: int, where: str) -> None:
    if code != RHEED_OK:
        raise RheedError(code, where, lib().rheed_last_error().decode())
