"""ctypes declarations of libfas.so (the C ABI in include/fas.h).

The library is built in place by paper_2510_11152_amd/build.py; if it is missing this
module raises instead of falling back to anything else.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfas.so")

FAS_OK = 0
FAS_NOT_CONVERGED = 1
FAS_ERR_ARG = -1
FAS_ERR_SHAPE = -2
FAS_ERR_NOMEM = -3
FAS_ERR_HIP = -4
FAS_ERR_NONFINITE = -5

FAS_BC = {"neumann": 0, "dirichlet": 1, "periodic": 2}
FAS_F64, FAS_F32 = 0, 1
FAS_FLAG_VARIABLE_KAPPA = 1
FAS_FLAG_MIXED_INNER = 2
FAS_OPT_KMAX, FAS_OPT_COARSE_SWEEPS, FAS_OPT_FUSED, FAS_OPT_PROFILE = 1, 2, 3, 4
FAS_OPT_GRAPH, FAS_OPT_AUTOTUNE, FAS_OPT_SEG_ROWS = 5, 6, 7
FAS_OPT_TILE, FAS_OPT_TILE_WAVES = 8, 9
FAS_OPT_ORDER, FAS_OPT_SYMMETRIC, FAS_OPT_ATOL, FAS_OPT_MIXED_INNER_NEXT = 10, 11, 12, 13
FAS_OPT_MARCH3_SWEEPS = 14
FAS_ORDER = {"x": 0, "u": 1, "z": 2}
FAS_K_NAMES = ("smooth", "pre", "post", "norm")
FAS_LOC = {"cell": 0, "edge_x": 1, "edge_y": 2}
FAS_NS_LAYOUT = {"memory_efficient": 0, "classical": 1}

# Every function the header declares, with (restype, argtypes).
_vp, _i, _d, _sz, _i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t, ctypes.c_int64
_pi64 = ctypes.POINTER(ctypes.c_int64)
_pd = ctypes.POINTER(ctypes.c_double)


class FasStats(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int), ("status", ctypes.c_int), ("rhs_norm", ctypes.c_double),
                ("rel_res", ctypes.c_double * 64)]


class FasKappa(ctypes.Structure):
    _fields_ = [("scalar", ctypes.c_double), ("cell", ctypes.c_void_p)]


class FasProfile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int * 4), ("ms", ctypes.c_double * 4)]


SIGNATURES = {
    "fas_workspace_size": (_sz, [_i, _pi64, _i, _i, _i]),
    "fas_grid_create": (_i, [_i, _pi64, _d, _i, _i, _i, _i, _vp, _sz, _vp, ctypes.POINTER(_vp)]),
    "fas_grid_destroy": (_i, [_vp]),
    "fas_grid_set": (_i, [_vp, _i, _d]),
    "fas_set_stream": (_i, [_vp, _vp]),
    "fas_grid_levels": (_i, [_vp]),
    "fas_level_cells": (_i64, [_vp, _i]),
    "fas_solve": (_i, [_vp, _d, _d, _vp, _vp, _vp, _d, _i, _i]),
    "fas_vcycle": (_i, [_vp, _d, _d, _vp, _vp, _vp, _i, _i, _pd]),
    "fas_vcycle_transposed": (_i, [_vp, _d, _d, _vp, _vp, _vp, _i, _i, _pd]),
    "fas_solve_transposed": (_i, [_vp, _d, _d, _vp, _vp, _vp, _d, _i, _i]),
    "fas_smooth": (_i, [_vp, _i, _d, _d, _vp, _vp, _vp, _i, _i]),
    "fas_residual": (_i, [_vp, _i, _d, _d, _vp, _vp, _vp, _vp, _pd]),
    "fas_restrict": (_i, [_vp, _i, _vp, _vp]),
    "fas_prolong_add": (_i, [_vp, _i, _vp, _vp, _vp]),
    "fas_kappa_grad": (_i, [_vp, _d, _vp, _vp, _vp, _vp]),
    "fas_solve_mixed": (_i, [_vp, _vp, _d, _d, _vp, _vp, _vp, _d, _i, _i, _i]),
    "fas_workspace_size_batched": (_sz, [_i, _pi64, _i, _i, _i, _i]),
    "fas_grid_create_batched": (_i, [_i, _pi64, _d, _i, _i, _i, _i, _i, _vp, _sz, _vp, ctypes.POINTER(_vp)]),
    "fas_solve_stacked": (_i, [_vp, _d, _d, _vp, _vp, _d, _i, _i, _vp, _vp]),
    "fas_solve_batched": (_i, [_i, _vp, _d, ctypes.POINTER(FasKappa), _vp, _vp, _d, _i, _i, _vp]),
    "fas_grain_rhs": (_i, [_vp, _i, _i, _i64, _d, _d, _d, _d, _vp, _vp]),
    "fas_solve_stacked_mixed": (_i, [_vp, _vp, _d, _d, _vp, _vp, _d, _i, _i, _i, _vp, _vp]),
    "fas_grain_argmax": (_i, [_vp, _i, _i64, _vp, _vp]),
    "fas_solve_noalloc": (_i, [_i, _pi64, _d, _i, _i, _i, _vp, _d, _d, _vp, _vp, _vp, _d, _i, _i, _i,
                               ctypes.POINTER(ctypes.c_int)]),
    "fas_stream_probe": (_i, [_vp, _i, _i64, _vp, _vp, _vp, _vp, _i, _i, _pd]),
    "fas_stag_workspace_size": (_sz, [_i, _i64, _i64, _i]),
    "fas_stag_create": (_i, [_i, _i64, _i64, _d, _i, _i, _vp, _sz, _vp, ctypes.POINTER(_vp)]),
    "fas_stag_destroy": (_i, [_vp]),
    "fas_stag_set": (_i, [_vp, _i, _d]),
    "fas_stag_levels": (_i, [_vp]),
    "fas_stag_profile": (_i, [_vp, _pd, _pd, ctypes.POINTER(ctypes.c_int)]),
    "fas_stag_solve": (_i, [_vp, _d, _d, _vp, _vp, _d, _i, _i, _i, ctypes.POINTER(ctypes.c_int), _pd]),
    "fas_stag_vcycle": (_i, [_vp, _d, _d, _vp, _vp, _i, _i]),
    "fas_stag_smooth": (_i, [_vp, _d, _d, _vp, _vp, _i]),
    "fas_stag_residual": (_i, [_vp, _d, _d, _vp, _vp, _vp, _pd]),
    "fas_ns_fields": (_i, [_i]),
    "fas_ns_workspace_size": (_sz, [_i64, _i64, _i]),
    "fas_ns_create": (_i, [_i64, _i64, _d, _d, _i, _i, _vp, _vp, _sz, _vp, ctypes.POINTER(_vp)]),
    "fas_ns_destroy": (_i, [_vp]),
    "fas_ns_set": (_i, [_vp, _i, _d]),
    "fas_ns_step": (_i, [_vp, _d, _d, _i, _vp, _vp, _vp, _d, _i, _i, _i, ctypes.POINTER(ctypes.c_int), _pd]),
    "fas_ns_memory": (_i, [_vp, ctypes.POINTER(_sz), ctypes.POINTER(_sz)]),
    "fas_get_stats": (_i, [_vp, ctypes.POINTER(FasStats)]),
    "fas_get_profile": (_i, [_vp, ctypes.POINTER(FasProfile), _i]),
    "fas_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load():
    """Load libfas.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libfas.so not found at %s: build it with paper_2510_11152_amd/build.py "
                              "(or __graft_entry__.build())" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class FasError(RuntimeError):
    def __init__(self, code, where):
        msg = load().fas_last_error().decode(errors="replace")
        super().__init__("%s failed with status %d: %s" % (where, code, msg))
        self.code = code


def check(code, where, allow_not_converged=False):
    if code == FAS_OK or (allow_not_converged and code == FAS_NOT_CONVERGED):
        return code
    raise FasError(code, where)
