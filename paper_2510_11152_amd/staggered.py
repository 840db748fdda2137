"""Python binding of the staggered-grid solver and the projection step (include/fas_stag.h):
argument marshalling only.  Every step runs in the HIP kernels of libfas.so; torch provides
the device memory (fields and workspace) and the stream.

Array shapes (float64, contiguous, x fastest) on an nx x ny cell grid:
  'cell'   (ny, nx)        pressure
  'edge_x' (ny, nx - 1)    u at the interior east-west edges
  'edge_y' (ny - 1, nx)    v at the interior north-south edges
"""
import ctypes

import torch

from . import _lib
from ._lib import check, load


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _check_array(t, shape, device, name):
    if t.dtype != torch.float64 or not t.is_contiguous() or tuple(t.shape) != tuple(shape) or t.device != device:
        raise ValueError("%s must be a contiguous float64 tensor of shape %s on %s" % (name, tuple(shape), device))


def _device(device):
    d = torch.device(device)
    if d.type == "cuda" and d.index is None:
        d = torch.device("cuda", torch.cuda.current_device())
    return d


def shape_of(loc, nx, ny):
    return {"cell": (ny, nx), "edge_x": (ny, nx - 1), "edge_y": (ny - 1, nx)}[loc]


class StaggeredSolver:
    """a w - c Lap_h w = f for one staggered variable (Section 4.1): loc 'cell' (bc
    'neumann' or 'dirichlet'), 'edge_x' or 'edge_y' (Dirichlet walls)."""

    def __init__(self, loc, nx, ny, h, bc="dirichlet", coarsest=4, device="cuda", stream=None):
        L = load()
        self.loc, self.nx, self.ny, self.h = loc, int(nx), int(ny), float(h)
        self.device = _device(device)
        self.shape = shape_of(loc, self.nx, self.ny)
        code = _lib.FAS_LOC[loc]
        size = L.fas_stag_workspace_size(code, self.nx, self.ny, coarsest)
        if size == 0:
            raise ValueError("invalid staggered grid: %d x %d, coarsest %d" % (self.nx, self.ny, coarsest))
        self.workspace = torch.empty(size, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        out = ctypes.c_void_p()
        check(L.fas_stag_create(code, self.nx, self.ny, self.h, 0 if bc == "neumann" else 1, coarsest,
                                _ptr(self.workspace), size, ctypes.c_void_p(self.stream.cuda_stream),
                                ctypes.byref(out)), "fas_stag_create")
        self.handle = out
        self.levels = L.fas_stag_levels(out)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None and getattr(_lib, "load", None) is not None:
            try:
                _lib.load().fas_stag_destroy(h)
            except Exception:
                pass
            self.handle = None

    def set(self, coarse_sweeps=None, fused=None, profile=None):
        """coarse_sweeps: sweeps on the coarsest level; fused: 1 (default) persistent tail
        and fused transfers, 0 one kernel per step and level (identical results); profile:
        time the finest level's fused pre- and post-smoothing launches with HIP events."""
        if coarse_sweeps is not None:
            check(load().fas_stag_set(self.handle, _lib.FAS_OPT_COARSE_SWEEPS, float(coarse_sweeps)), "fas_stag_set")
        if fused is not None:
            check(load().fas_stag_set(self.handle, _lib.FAS_OPT_FUSED, float(int(fused))), "fas_stag_set")
        if profile is not None:
            check(load().fas_stag_set(self.handle, _lib.FAS_OPT_PROFILE, float(int(profile))), "fas_stag_set")

    def profile(self):
        """(pre-smoothing us, post-smoothing us, cycles timed) of the finest level."""
        pre, post, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
        check(load().fas_stag_profile(self.handle, ctypes.byref(pre), ctypes.byref(post), ctypes.byref(n)),
              "fas_stag_profile")
        return pre.value, post.value, n.value

    def _args(self, f, w):
        _check_array(f, self.shape, self.device, "f")
        _check_array(w, self.shape, self.device, "w")

    def solve(self, a, c, f, w, tol, nu1=2, nu2=2, kmax=20):
        """Returns (status, cycles, res)."""
        self._args(f, w)
        cyc = ctypes.c_int()
        res = ctypes.c_double()
        st = check(load().fas_stag_solve(self.handle, float(a), float(c), _ptr(f), _ptr(w), float(tol), nu1, nu2,
                                         kmax, ctypes.byref(cyc), ctypes.byref(res)),
                   "fas_stag_solve", allow_not_converged=True)
        return st, cyc.value, res.value

    def vcycle(self, a, c, f, w, nu1=2, nu2=2):
        self._args(f, w)
        check(load().fas_stag_vcycle(self.handle, float(a), float(c), _ptr(f), _ptr(w), nu1, nu2), "fas_stag_vcycle")

    def smooth(self, a, c, f, w, nu):
        self._args(f, w)
        check(load().fas_stag_smooth(self.handle, float(a), float(c), _ptr(f), _ptr(w), nu), "fas_stag_smooth")

    def residual(self, a, c, f, w, r=None):
        """Returns h ||f - L w||_2 (and fills r if given)."""
        self._args(f, w)
        if r is not None:
            _check_array(r, self.shape, self.device, "r")
        res = ctypes.c_double()
        check(load().fas_stag_residual(self.handle, float(a), float(c), _ptr(f), _ptr(w),
                                       None if r is None else _ptr(r), ctypes.byref(res)), "fas_stag_residual")
        return res.value


class NavierStokes2D:
    """Scheme 1 (first-order projection, Section 4.2) on an nx x ny grid of spacing h.

    layout 'memory_efficient' keeps 6 fields (U_old, U_new, V_old, V_new, P_old, P_new) and
    writes u^{n+1} over u^n; 'classical' keeps 9 (U_new, U_old, U~, ...) and copies new ->
    old every step.  The state u^n, v^n, p^n is self.u, self.v, self.p (views of U_old,
    V_old, P_old)."""

    def __init__(self, nx, ny, h, re, layout="memory_efficient", coarsest=4, device="cuda", stream=None):
        L = load()
        self.nx, self.ny, self.h, self.re = int(nx), int(ny), float(h), float(re)
        self.layout = layout
        self.device = _device(device)
        code = _lib.FAS_NS_LAYOUT[layout]
        nf = L.fas_ns_fields(code)
        su, sv, sp = shape_of("edge_x", nx, ny), shape_of("edge_y", nx, ny), shape_of("cell", nx, ny)
        shapes = [su, su, sv, sv, sp, sp] if nf == 6 else [su, su, su, sv, sv, sv, sp, sp, sp]
        self.fields = [torch.zeros(s, dtype=torch.float64, device=self.device) for s in shapes]
        size = L.fas_ns_workspace_size(self.nx, self.ny, coarsest)
        if size == 0:
            raise ValueError("invalid grid: %d x %d, coarsest %d" % (self.nx, self.ny, coarsest))
        self.workspace = torch.empty(size, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ptrs = (ctypes.c_void_p * nf)(*[f.data_ptr() for f in self.fields])
        out = ctypes.c_void_p()
        check(L.fas_ns_create(self.nx, self.ny, self.h, self.re, code, coarsest, ptrs, _ptr(self.workspace), size,
                              ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(out)), "fas_ns_create")
        self.handle = out
        if nf == 6:
            self.u, self.ut, self.v, self.vt, self.p, self.pt = self.fields
        else:
            _, self.u, self.ut, _, self.v, self.vt, _, self.p, self.pt = self.fields

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None and getattr(_lib, "load", None) is not None:
            try:
                _lib.load().fas_ns_destroy(h)
            except Exception:
                pass
            self.handle = None

    def set(self, coarse_sweeps=None, fused=None):
        if coarse_sweeps is not None:
            check(load().fas_ns_set(self.handle, _lib.FAS_OPT_COARSE_SWEEPS, float(coarse_sweeps)), "fas_ns_set")
        if fused is not None:
            check(load().fas_ns_set(self.handle, _lib.FAS_OPT_FUSED, float(int(fused))), "fas_ns_set")

    def step(self, dt, lid=0.0, force_u=(), force_v=(), coef=(), tol=1e-9, nu1=2, nu2=2, kmax=20):
        """One step; force_u / force_v: up to 4 source fields each (device tensors of the u
        and v shapes), coef their coefficients.  Returns (status, cycles[3], res[3])."""
        nf = len(coef)
        if len(force_u) != nf or len(force_v) != nf:
            raise ValueError("force_u, force_v and coef must have the same length")
        for t in force_u:
            _check_array(t, self.u.shape, self.device, "force_u")
        for t in force_v:
            _check_array(t, self.v.shape, self.device, "force_v")
        fu = (ctypes.c_void_p * max(nf, 1))(*[t.data_ptr() for t in force_u])
        fv = (ctypes.c_void_p * max(nf, 1))(*[t.data_ptr() for t in force_v])
        cf = (ctypes.c_double * max(nf, 1))(*[float(c) for c in coef])
        cyc = (ctypes.c_int * 3)()
        res = (ctypes.c_double * 3)()
        st = check(load().fas_ns_step(self.handle, float(dt), float(lid), nf, fu if nf else None, fv if nf else None,
                                      cf if nf else None, float(tol), nu1, nu2, kmax, cyc, res),
                   "fas_ns_step", allow_not_converged=True)
        return st, list(cyc), list(res)

    def memory(self):
        """(field bytes, workspace bytes)."""
        fb, wb = ctypes.c_size_t(), ctypes.c_size_t()
        check(load().fas_ns_memory(self.handle, ctypes.byref(fb), ctypes.byref(wb)), "fas_ns_memory")
        return fb.value, wb.value
