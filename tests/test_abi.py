"""The C ABI library loads and exports every entry point include/fas.h declares, and
its host-side argument checks report the documented status codes without touching a
GPU."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def _declared():
    txt = "".join(open(h).read() for h in HEADERS)
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b(fas_\w+)\s*\(", txt, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2510_11152_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libfas.so is not built (run __graft_entry__.build())")
    return _lib.load()


def test_header_declares_entry_points():
    names = _declared()
    for want in ("fas_solve", "fas_vcycle", "fas_smooth", "fas_residual", "fas_restrict", "fas_prolong_add",
                 "fas_solve_mixed", "fas_kappa_grad", "fas_solve_transposed", "fas_last_error",
                 "fas_stag_solve", "fas_stag_vcycle", "fas_ns_step", "fas_ns_create"):
        assert want in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2510_11152_amd import _lib
    for name in _declared():
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, "binding lacks " + name


def _n3(*n):
    return (ctypes.c_int64 * 3)(*(list(n) + [1] * (3 - len(n))))


def test_workspace_size_shape_rules(lib):
    from paper_2510_11152_amd import _lib as F
    assert lib.fas_workspace_size(2, _n3(256, 256), F.FAS_F64, 4, 0) > 2 * 256 * 256 * 8 // 4
    assert lib.fas_workspace_size(2, _n3(250, 256), F.FAS_F64, 4, 0) == 0   # not coarsest * 2^L
    assert lib.fas_workspace_size(2, _n3(4, 4), F.FAS_F64, 4, 0) == 0       # L = 0
    assert lib.fas_workspace_size(2, _n3(64, 64), F.FAS_F64, 3, 0) == 0     # odd coarsest
    assert lib.fas_workspace_size(4, _n3(64, 64), F.FAS_F64, 4, 0) == 0     # bad dim
    big = lib.fas_workspace_size(3, _n3(64, 64, 64), F.FAS_F64, 4, F.FAS_FLAG_VARIABLE_KAPPA)
    small = lib.fas_workspace_size(3, _n3(64, 64, 64), F.FAS_F64, 4, 0)
    assert big > small
    assert lib.fas_workspace_size(2, _n3(64, 64), F.FAS_F32, 4, 0) < lib.fas_workspace_size(2, _n3(64, 64), F.FAS_F64, 4, 0)


def test_create_errors_without_gpu(lib):
    from paper_2510_11152_amd import _lib as F
    out = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: every call below fails first
    n = _n3(64, 64)
    need = lib.fas_workspace_size(2, n, F.FAS_F64, 4, 0)
    assert lib.fas_grid_create(2, _n3(60, 64), 1 / 64, 0, F.FAS_F64, 4, 0, fake, need, None, ctypes.byref(out)) == F.FAS_ERR_SHAPE
    assert lib.fas_grid_create(2, n, 1 / 64, 0, F.FAS_F64, 4, 0, fake, need - 1, None, ctypes.byref(out)) == F.FAS_ERR_NOMEM
    assert b"too small" in lib.fas_last_error()
    assert lib.fas_grid_create(2, n, 1 / 64, 7, F.FAS_F64, 4, 0, fake, need, None, ctypes.byref(out)) == F.FAS_ERR_ARG
    assert lib.fas_grid_create(2, n, -1.0, 0, F.FAS_F64, 4, 0, fake, need, None, ctypes.byref(out)) == F.FAS_ERR_ARG
    assert lib.fas_grid_create(2, n, 1 / 64, 0, F.FAS_F64, 4, 0, ctypes.c_void_p(4096 + 8), need, None,
                               ctypes.byref(out)) == F.FAS_ERR_ARG  # misaligned
    assert lib.fas_grid_create(2, _n3(6, 6), 1 / 6, 2, F.FAS_F64, 2, 0, fake, 1 << 20, None,
                               ctypes.byref(out)) == F.FAS_ERR_SHAPE  # periodic odd coarsest level


def test_solve_argument_errors_without_gpu(lib):
    """A valid plan over a fake workspace: the calls below are rejected by host checks
    before anything is enqueued."""
    from paper_2510_11152_amd import _lib as F
    out = ctypes.c_void_p()
    n = _n3(64, 64)
    need = lib.fas_workspace_size(2, n, F.FAS_F64, 4, 0)
    fake = ctypes.c_void_p(1 << 20)
    assert lib.fas_grid_create(2, n, 1 / 64, 0, F.FAS_F64, 4, 0, fake, need, None, ctypes.byref(out)) == F.FAS_OK
    g = out
    try:
        assert lib.fas_grid_levels(g) == 4
        assert lib.fas_level_cells(g, 4) == 16
        buf = ctypes.c_void_p(1 << 22)
        assert lib.fas_solve(g, 1e-3, 1.0, None, buf, buf, 1e-10, 2, 2) == F.FAS_ERR_ARG   # rhs aliases u
        assert b"alias" in lib.fas_last_error()
        assert lib.fas_solve(g, 1e-3, 1.0, None, None, buf, 1e-10, 2, 2) == F.FAS_ERR_ARG
        assert lib.fas_solve(g, -1.0, 1.0, None, ctypes.c_void_p(1 << 23), buf, 1e-10, 2, 2) == F.FAS_ERR_ARG
        assert lib.fas_solve(g, 1e-3, 1.0, ctypes.c_void_p(1 << 24), ctypes.c_void_p(1 << 23), buf, 1e-10, 2, 2) == F.FAS_ERR_ARG  # no kappa storage
        assert lib.fas_solve(g, 1e-3, 1.0, None, ctypes.c_void_p(1 << 23), buf, 1e-10, 0, 0) == F.FAS_ERR_ARG
        assert lib.fas_grid_set(g, F.FAS_OPT_KMAX, 0) == F.FAS_ERR_ARG
        assert lib.fas_grid_set(g, F.FAS_OPT_KMAX, 7) == F.FAS_OK
        assert lib.fas_grid_set(g, 99, 1) == F.FAS_ERR_ARG
        for bad in (6, 17, -2, 8.5):                     # segment height: 0 or even >= 8
            assert lib.fas_grid_set(g, F.FAS_OPT_SEG_ROWS, bad) == F.FAS_ERR_ARG
        for good in (0, 8, 120):
            assert lib.fas_grid_set(g, F.FAS_OPT_SEG_ROWS, good) == F.FAS_OK
        for bad in (4, 17, -8, 8.5):                     # waves per tile workgroup: 0 or 6..16
            assert lib.fas_grid_set(g, F.FAS_OPT_TILE_WAVES, bad) == F.FAS_ERR_ARG
        for good in (0, 6, 11, 16):
            assert lib.fas_grid_set(g, F.FAS_OPT_TILE_WAVES, good) == F.FAS_OK
        assert lib.fas_grid_set(g, F.FAS_OPT_TILE, -1) == F.FAS_ERR_ARG
        for good in (0, 4096, 1 << 20):
            assert lib.fas_grid_set(g, F.FAS_OPT_TILE, good) == F.FAS_OK
        for opt in (F.FAS_OPT_GRAPH, F.FAS_OPT_AUTOTUNE, F.FAS_OPT_PROFILE, F.FAS_OPT_FUSED):
            assert lib.fas_grid_set(g, opt, 2) == F.FAS_ERR_ARG
            assert lib.fas_grid_set(g, opt, 0) == F.FAS_OK
        for bad in (-1, 3, 1.5):                         # set order: X, U or Z
            assert lib.fas_grid_set(g, F.FAS_OPT_ORDER, bad) == F.FAS_ERR_ARG
        for good in (F.FAS_ORDER["u"], F.FAS_ORDER["z"], F.FAS_ORDER["x"]):
            assert lib.fas_grid_set(g, F.FAS_OPT_ORDER, good) == F.FAS_OK
        assert lib.fas_grid_set(g, F.FAS_OPT_SYMMETRIC, 2) == F.FAS_ERR_ARG
        assert lib.fas_grid_set(g, F.FAS_OPT_SYMMETRIC, 1) == F.FAS_OK
        assert lib.fas_grid_set(g, F.FAS_OPT_SYMMETRIC, 0) == F.FAS_OK
        for bad in (-1e-9, float("nan"), float("inf")):   # absolute tolerance: finite, >= 0
            assert lib.fas_grid_set(g, F.FAS_OPT_ATOL, bad) == F.FAS_ERR_ARG
        for good in (0.0, 1.5e-9, 3.0):
            assert lib.fas_grid_set(g, F.FAS_OPT_ATOL, good) == F.FAS_OK
        assert lib.fas_restrict(g, 4, buf, ctypes.c_void_p(1 << 23)) == F.FAS_ERR_ARG     # no coarser level
        assert lib.fas_kappa_grad(g, 1e-3, None, buf, buf, buf) == F.FAS_ERR_ARG
    finally:
        assert lib.fas_grid_destroy(g) == F.FAS_OK


def test_staggered_workspace_size_shape_rules(lib):
    for loc in (0, 1, 2):
        assert lib.fas_stag_workspace_size(loc, 64, 64, 4) > 0
        assert lib.fas_stag_workspace_size(loc, 64, 16, 4) > 0
        assert lib.fas_stag_workspace_size(loc, 48, 48, 4) > 0      # 48 = 6 * 2^3
        assert lib.fas_stag_workspace_size(loc, 4, 4, 4) == 0       # one level only
        assert lib.fas_stag_workspace_size(loc, 64, 64, 1) == 0     # coarsest < 2
    assert lib.fas_stag_workspace_size(3, 64, 64, 4) == 0           # unknown location
    assert lib.fas_ns_workspace_size(64, 64, 4) >= lib.fas_stag_workspace_size(0, 64, 64, 4) + 64 * 64 * 8
    assert lib.fas_ns_fields(0) == 6 and lib.fas_ns_fields(1) == 9 and lib.fas_ns_fields(2) == 0


def test_staggered_create_errors_without_gpu(lib):
    from paper_2510_11152_amd import _lib
    out = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 40)   # never dereferenced by create
    size = lib.fas_stag_workspace_size(1, 64, 64, 4)
    assert lib.fas_stag_create(1, 64, 64, 1 / 64, 1, 4, fake, size - 1, None, ctypes.byref(out)) == _lib.FAS_ERR_NOMEM
    assert lib.fas_stag_create(1, 64, 64, 1 / 64, 0, 4, fake, size, None, ctypes.byref(out)) == _lib.FAS_ERR_ARG
    assert lib.fas_stag_create(1, 64, 64, -1.0, 1, 4, fake, size, None, ctypes.byref(out)) == _lib.FAS_ERR_ARG
    assert lib.fas_stag_create(1, 4, 4, 0.25, 1, 4, fake, size, None, ctypes.byref(out)) == _lib.FAS_ERR_SHAPE
    assert lib.fas_stag_create(1, 64, 64, 1 / 64, 1, 4, fake, size, None, ctypes.byref(out)) == _lib.FAS_OK
    s = out
    assert lib.fas_stag_levels(s) == 5                               # 64 .. 4
    assert lib.fas_stag_set(s, _lib.FAS_OPT_COARSE_SWEEPS, 0.0) == _lib.FAS_ERR_ARG
    assert lib.fas_stag_set(s, _lib.FAS_OPT_KMAX, 10.0) == _lib.FAS_ERR_ARG
    assert lib.fas_stag_set(s, _lib.FAS_OPT_COARSE_SWEEPS, 8.0) == _lib.FAS_OK
    assert lib.fas_stag_set(s, _lib.FAS_OPT_FUSED, 0.0) == _lib.FAS_OK
    assert lib.fas_stag_set(s, _lib.FAS_OPT_FUSED, 2.0) == _lib.FAS_ERR_ARG
    assert lib.fas_stag_set(s, _lib.FAS_OPT_PROFILE, 2.0) == _lib.FAS_ERR_ARG
    assert lib.fas_stag_profile(s, None, None, None) == _lib.FAS_ERR_ARG   # profiling off
    buf = ctypes.c_void_p(1 << 41)
    assert lib.fas_stag_solve(s, 1.0, 0.1, buf, buf, 1e-9, 2, 2, 20, None, None) == _lib.FAS_ERR_ARG   # aliased
    assert lib.fas_stag_vcycle(s, 1.0, 0.1, None, buf, 2, 2) == _lib.FAS_ERR_ARG
    assert lib.fas_stag_destroy(s) == _lib.FAS_OK
    # projection step
    ws = lib.fas_ns_workspace_size(64, 64, 4)
    fields = (ctypes.c_void_p * 6)(*[(i + 2) << 40 for i in range(6)])
    assert lib.fas_ns_create(64, 64, 1 / 64, 10.0, 0, 4, fields, fake, ws - 1, None, ctypes.byref(out)) == _lib.FAS_ERR_NOMEM
    dup = (ctypes.c_void_p * 6)(*[(2 << 40)] * 6)
    assert lib.fas_ns_create(64, 64, 1 / 64, 10.0, 0, 4, dup, fake, ws, None, ctypes.byref(out)) == _lib.FAS_ERR_ARG
    assert lib.fas_ns_create(64, 64, 1 / 64, 10.0, 5, 4, fields, fake, ws, None, ctypes.byref(out)) == _lib.FAS_ERR_ARG
    assert lib.fas_ns_create(64, 64, 1 / 64, 10.0, 0, 4, fields, fake, ws, None, ctypes.byref(out)) == _lib.FAS_OK
    ns = out
    fb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.fas_ns_memory(ns, ctypes.byref(fb), ctypes.byref(wb)) == _lib.FAS_OK
    assert fb.value == 2 * (63 * 64 * 2 + 64 * 64) * 8 and wb.value == ws
    assert lib.fas_ns_step(ns, -1.0, 0.0, 0, None, None, None, 1e-9, 2, 2, 20, None, None) == _lib.FAS_ERR_ARG
    assert lib.fas_ns_step(ns, 0.1, 0.0, 5, None, None, None, 1e-9, 2, 2, 20, None, None) == _lib.FAS_ERR_ARG
    assert lib.fas_ns_destroy(ns) == _lib.FAS_OK
