"""Python binding of libfas: argument marshalling only.

Device memory and streams come from PyTorch; every step of the solver runs in the HIP
kernels of libfas.so.  Tensors are contiguous, shaped (ny, nx) in 2D or (nz, ny, nx)
in 3D (x fastest), on the grid's device, in the grid's dtype.
"""
import ctypes

import torch

from . import _lib
from ._lib import check, load

_DT = {torch.float64: _lib.FAS_F64, torch.float32: _lib.FAS_F32}


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Grid:
    """Grid plan + caller-owned workspace (a torch uint8 tensor).

    n: cells per axis (nx, ny) or (nx, ny, nz); h: finest spacing; bc: 'neumann',
    'dirichlet' or 'periodic'; coarsest: cells along the shortest axis of the coarsest
    level; variable_kappa: reserve storage for a cell coefficient hierarchy;
    mixed_inner: FP32 grid used as the inner solver of solve_mixed."""

    def __init__(self, n, h, bc="neumann", dtype=torch.float64, coarsest=4, variable_kappa=False,
                 mixed_inner=False, device="cuda", stream=None, batch=1):
        L = load()
        self.batch = int(batch)
        self.n = tuple(int(x) for x in n)
        self.dim = len(self.n)
        self.h = float(h)
        self.bc = bc
        self.dtype = dtype
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        flags = (_lib.FAS_FLAG_VARIABLE_KAPPA if variable_kappa else 0) | (_lib.FAS_FLAG_MIXED_INNER if mixed_inner else 0)
        n3 = (ctypes.c_int64 * 3)(*(list(self.n) + [1] * (3 - self.dim)))
        size = L.fas_workspace_size_batched(self.dim, n3, _DT[dtype], coarsest, flags, self.batch)
        if size == 0:
            raise ValueError("invalid grid: n=%s coarsest=%d" % (self.n, coarsest))
        self.workspace = torch.empty(size, dtype=torch.uint8, device=self.device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h_out = ctypes.c_void_p()
        check(L.fas_grid_create_batched(self.dim, n3, self.h, _lib.FAS_BC[bc], _DT[dtype], coarsest, flags,
                                        self.batch, _ptr(self.workspace), size, ctypes.c_void_p(stream.cuda_stream),
                                        ctypes.byref(h_out)), "fas_grid_create_batched")
        self.handle = h_out
        self.levels = L.fas_grid_levels(self.handle)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None and getattr(_lib, "load", None) is not None:
            try:
                _lib.load().fas_grid_destroy(h)
            except Exception:  # interpreter shutdown: module globals already cleared
                pass
            self.handle = None

    def shape(self, level=0):
        return tuple(m >> level for m in reversed(self.n))

    def set(self, kmax=None, coarse_sweeps=None, fused=None, profile=None, graph=None, autotune=None,
            seg_rows=None, tile=None, tile_waves=None, order=None, symmetric=None, atol=None, march3_sweeps=None):
        """Solver options (fas_grid_set).  order: smoother set order 'x' (default), 'u' or
        'z'; symmetric: every second sweep in reverse set order (1234-4321); atol: a solve
        also stops once ||rhs - A u||_2 <= atol (0: none); march3_sweeps: most sweeps per
        3D plane-march pass (1 or 2, the default; identical results)."""
        L = load()
        if kmax is not None:
            check(L.fas_grid_set(self.handle, _lib.FAS_OPT_KMAX, float(kmax)), "fas_grid_set")
        if coarse_sweeps is not None:
            check(L.fas_grid_set(self.handle, _lib.FAS_OPT_COARSE_SWEEPS, float(coarse_sweeps)), "fas_grid_set")
        if fused is not None:
            check(L.fas_grid_set(self.handle, _lib.FAS_OPT_FUSED, float(int(fused))), "fas_grid_set")
        if profile is not None:
            check(L.fas_grid_set(self.handle, _lib.FAS_OPT_PROFILE, float(int(profile))), "fas_grid_set")
        if graph is not None:
            check(L.fas_grid_set(self.handle, _lib.FAS_OPT_GRAPH, float(int(graph))), "fas_grid_set")
        if autotune is not None:
            check(L.fas_grid_set(self.handle, _lib.FAS_OPT_AUTOTUNE, float(int(autotune))), "fas_grid_set")
        if seg_rows is not None:
            check(L.fas_grid_set(self.handle, _lib.FAS_OPT_SEG_ROWS, float(seg_rows)), "fas_grid_set")
        if tile is not None:
            check(L.fas_grid_set(self.handle, _lib.FAS_OPT_TILE, float(tile)), "fas_grid_set")
        if tile_waves is not None:
            check(L.fas_grid_set(self.handle, _lib.FAS_OPT_TILE_WAVES, float(tile_waves)), "fas_grid_set")
        if order is not None:
            check(L.fas_grid_set(self.handle, _lib.FAS_OPT_ORDER, float(_lib.FAS_ORDER[order])), "fas_grid_set")
        if symmetric is not None:
            check(L.fas_grid_set(self.handle, _lib.FAS_OPT_SYMMETRIC, float(int(symmetric))), "fas_grid_set")
        if atol is not None:
            check(L.fas_grid_set(self.handle, _lib.FAS_OPT_ATOL, float(atol)), "fas_grid_set")
        if march3_sweeps is not None:
            check(L.fas_grid_set(self.handle, _lib.FAS_OPT_MARCH3_SWEEPS, float(march3_sweeps)), "fas_grid_set")
        return self

    def profile(self, reset=True):
        """{kernel class: (launches, total ms)} of finest-level launches (profile=True)."""
        p = _lib.FasProfile()
        check(load().fas_get_profile(self.handle, ctypes.byref(p), int(reset)), "fas_get_profile")
        return {name: (p.launches[i], p.ms[i]) for i, name in enumerate(_lib.FAS_K_NAMES)}

    def _arr(self, t, level=0, name="array", dtype=None):
        if t is None:
            return None
        want = dtype or self.dtype
        if t.dtype != want or t.device != self.device or not t.is_contiguous() or tuple(t.shape) != self.shape(level):
            raise ValueError("%s must be a contiguous %s tensor of shape %s on %s (got %s %s %s)" % (
                name, want, self.shape(level), self.device, t.dtype, tuple(t.shape), t.device))
        return t

    # ---------------------------------------------------------------- solves
    def solve(self, rhs, u, dt, kappa=1.0, kappa_cell=None, tol=1e-10, nu1=2, nu2=2, transposed=False):
        """Solve A u = rhs in place (u: initial guess in, solution out).  Returns the
        status (0 converged, 1 kmax reached)."""
        self._arr(rhs, name="rhs"), self._arr(u, name="u"), self._arr(kappa_cell, name="kappa_cell")
        fn = load().fas_solve_transposed if transposed else load().fas_solve
        return check(fn(self.handle, dt, kappa, _ptr(kappa_cell), _ptr(rhs), _ptr(u), tol, nu1, nu2),
                     "fas_solve", allow_not_converged=True)

    def vcycle(self, rhs, u, dt, kappa=1.0, kappa_cell=None, nu1=2, nu2=2, transposed=False, with_residual=False):
        self._arr(rhs, name="rhs"), self._arr(u, name="u"), self._arr(kappa_cell, name="kappa_cell")
        rr = ctypes.c_double(0.0)
        fn = load().fas_vcycle_transposed if transposed else load().fas_vcycle
        check(fn(self.handle, dt, kappa, _ptr(kappa_cell), _ptr(rhs), _ptr(u), nu1, nu2,
                 ctypes.byref(rr) if with_residual else None), "fas_vcycle")
        return rr.value if with_residual else None

    # ---------------------------------------------------------------- building blocks
    def smooth(self, level, rhs, u, dt, kappa=1.0, kappa_cell=None, sweeps=1, reverse=False):
        self._arr(rhs, level, "rhs"), self._arr(u, level, "u"), self._arr(kappa_cell, level, "kappa_cell")
        check(load().fas_smooth(self.handle, level, dt, kappa, _ptr(kappa_cell), _ptr(rhs), _ptr(u), sweeps,
                                int(reverse)), "fas_smooth")

    def residual(self, level, rhs, u, dt, kappa=1.0, kappa_cell=None, out=None, with_norm=False):
        self._arr(rhs, level, "rhs"), self._arr(u, level, "u"), self._arr(kappa_cell, level, "kappa_cell")
        r = torch.empty_like(u) if out is None else self._arr(out, level, "out")
        nrm = ctypes.c_double(0.0)
        check(load().fas_residual(self.handle, level, dt, kappa, _ptr(kappa_cell), _ptr(rhs), _ptr(u), _ptr(r),
                                  ctypes.byref(nrm) if with_norm else None), "fas_residual")
        return (r, nrm.value) if with_norm else r

    def restrict(self, level, fine, out=None):
        self._arr(fine, level, "fine")
        c = torch.empty(self.shape(level + 1), dtype=self.dtype, device=self.device) if out is None else out
        self._arr(c, level + 1, "out")
        check(load().fas_restrict(self.handle, level, _ptr(fine), _ptr(c)), "fas_restrict")
        return c

    def prolong_add(self, level, c_new, c_old, fine):
        self._arr(c_new, level + 1, "c_new"), self._arr(c_old, level + 1, "c_old"), self._arr(fine, level, "fine")
        check(load().fas_prolong_add(self.handle, level, _ptr(c_new), _ptr(c_old), _ptr(fine)), "fas_prolong_add")

    def kappa_grad(self, dt, kappa_cell, mu, u, gkappa):
        for t, nm in ((kappa_cell, "kappa_cell"), (mu, "mu"), (u, "u"), (gkappa, "gkappa")):
            self._arr(t, 0, nm)
        check(load().fas_kappa_grad(self.handle, dt, _ptr(kappa_cell), _ptr(mu), _ptr(u), _ptr(gkappa)),
              "fas_kappa_grad")

    def solve_stacked(self, rhs, u, dt, kappa=1.0, tol=1e-10, nu1=2, nu2=2):
        """All `batch` problems of a stacked grid at once; rhs, u shaped (batch, *shape).
        Returns (status per problem, V-cycles per problem) as lists."""
        want = (self.batch,) + self.shape()
        for t, nm in ((rhs, "rhs"), (u, "u")):
            if t.dtype != self.dtype or t.device != self.device or not t.is_contiguous() or tuple(t.shape) != want:
                raise ValueError("%s must be a contiguous %s tensor of shape %s on %s" % (nm, self.dtype, want, self.device))
        st = (ctypes.c_int * self.batch)()
        cy = (ctypes.c_int * self.batch)()
        code = load().fas_solve_stacked(self.handle, dt, kappa, _ptr(rhs), _ptr(u), tol, nu1, nu2, st, cy)
        if code not in (_lib.FAS_OK, _lib.FAS_NOT_CONVERGED):
            check(code, "fas_solve_stacked")
        return list(st), list(cy)

    def stats(self):
        s = _lib.FasStats()
        check(load().fas_get_stats(self.handle, ctypes.byref(s)), "fas_get_stats")
        c = s.cycles
        return {"cycles": c, "status": s.status, "rhs_norm": s.rhs_norm,
                "rel_res": [s.rel_res[i] for i in range(min(c + 1, 64))]}


def solve_mixed(g64, g32, rhs, u, dt, kappa=1.0, kappa_cell=None, tol=1e-10, nu1=2, nu2=2, inner=2, inner_next=0):
    """FP64 defect correction around FP32 V-cycles (g32 built with mixed_inner=True):
    `inner` FP32 cycles in the first correction, `inner_next` (if > 0) in the later ones."""
    g64._arr(rhs, name="rhs"), g64._arr(u, name="u"), g64._arr(kappa_cell, name="kappa_cell")
    check(load().fas_grid_set(g64.handle, _lib.FAS_OPT_MIXED_INNER_NEXT, float(inner_next)), "fas_grid_set")
    return check(load().fas_solve_mixed(g64.handle, g32.handle, dt, kappa, _ptr(kappa_cell), _ptr(rhs), _ptr(u),
                                        tol, nu1, nu2, inner), "fas_solve_mixed", allow_not_converged=True)


def solve_stacked_mixed(g64, g32, rhs, u, dt, kappa=1.0, tol=1e-10, nu1=2, nu2=2, inner=2, inner_next=0):
    """FP64 defect correction around FP32 V-cycles for every problem of stacked grids
    (g64 FP64, g32 FP32 with mixed_inner=True, the same batch); rhs, u shaped (batch,
    *shape); `inner_next` as in solve_mixed.  Returns (status per problem, outer
    corrections per problem)."""
    check(load().fas_grid_set(g64.handle, _lib.FAS_OPT_MIXED_INNER_NEXT, float(inner_next)), "fas_grid_set")
    want = (g64.batch,) + g64.shape()
    for t, nm in ((rhs, "rhs"), (u, "u")):
        if t.dtype != torch.float64 or t.device != g64.device or not t.is_contiguous() or tuple(t.shape) != want:
            raise ValueError("%s must be a contiguous float64 tensor of shape %s on %s" % (nm, want, g64.device))
    st = (ctypes.c_int * g64.batch)()
    cy = (ctypes.c_int * g64.batch)()
    code = load().fas_solve_stacked_mixed(g64.handle, g32.handle, dt, kappa, _ptr(rhs), _ptr(u), tol, nu1, nu2,
                                          inner, st, cy)
    if code not in (_lib.FAS_OK, _lib.FAS_NOT_CONVERGED):
        check(code, "fas_solve_stacked_mixed")
    return list(st), list(cy)


def heat(grid, u0, steps, dt, kappa=1.0, kappa_cell=None, tol=1e-10, nu1=2, nu2=2, keep=False):
    """Backward-Euler heat steps: rhs = u^n, warm start u = u^n, solve.  Returns u^T
    (and the list of states when keep=True)."""
    u = u0.clone()
    rhs = torch.empty_like(u)
    states = [u.clone()] if keep else None
    for _ in range(steps):
        rhs.copy_(u)
        st = grid.solve(rhs, u, dt, kappa, kappa_cell, tol, nu1, nu2)
        if st != _lib.FAS_OK:
            raise RuntimeError("heat step did not converge")
        if keep:
            states.append(u.clone())
    return (u, states) if keep else u


def solve_batched(grids, rhs_list, u_list, dt, kappa=1.0, kappa_cells=None, tol=1e-10, nu1=2, nu2=2):
    """Problem p solves A_p u_list[p] = rhs_list[p] on grids[p], all advanced together by
    fas_solve_batched (one launch per pass over every problem).  kappa: one constant or
    one per problem; kappa_cells: None or one cell field per problem.  u_list entries
    are updated in place.  Returns the per-problem status list (fas_get_stats of each
    grid gives its cycles)."""
    m = len(grids)
    if len(rhs_list) != m or len(u_list) != m:
        raise ValueError("expected %d right-hand sides and iterates" % m)
    kap = list(kappa) if isinstance(kappa, (list, tuple)) else [kappa] * m
    cells = list(kappa_cells) if kappa_cells is not None else [None] * m
    if len(kap) != m or len(cells) != m:
        raise ValueError("expected one kappa per problem")
    for g, r, u, c in zip(grids, rhs_list, u_list, cells):
        g._arr(r, name="rhs"), g._arr(u, name="u"), g._arr(c, name="kappa_cell")
    K = (_lib.FasKappa * m)(*[_lib.FasKappa(float(k), _ptr(c)) for k, c in zip(kap, cells)])
    G = (ctypes.c_void_p * m)(*[g.handle for g in grids])
    R = (ctypes.c_void_p * m)(*[r.data_ptr() for r in rhs_list])
    U = (ctypes.c_void_p * m)(*[u.data_ptr() for u in u_list])
    st = (ctypes.c_int * m)()
    code = load().fas_solve_batched(m, G, dt, K, R, U, tol, nu1, nu2, st)
    if code not in (_lib.FAS_OK, _lib.FAS_NOT_CONVERGED):
        check(code, "fas_solve_batched")
    return list(st)


class UnevenBatch:
    """Problems of different sizes on the unit square (h = 1/n), one grid each, solved
    together by one fas_solve_batched call.  The grids are planned once, so repeated
    solves reuse their workspaces and launch descriptors."""

    def __init__(self, shapes, dtype=torch.float64, coarsest=4, bc="neumann", device="cuda"):
        self.shapes = [tuple(s) for s in shapes]
        self.grids = [Grid(tuple(reversed(s)), 1.0 / s[-1], bc=bc, dtype=dtype, coarsest=coarsest, device=device)
                      for s in self.shapes]

    def solve(self, rhs_list, u_list, dt, kappa=1.0, tol=1e-10, nu1=2, nu2=2):
        """u_list entries are updated in place; returns per-problem (status, V-cycles)
        lists in input order."""
        status = solve_batched(self.grids, rhs_list, u_list, dt, kappa, None, tol, nu1, nu2)
        return status, [g.stats()["cycles"] for g in self.grids]


def solve_uneven(rhs_list, u_list, dt, kappa=1.0, tol=1e-10, nu1=2, nu2=2, coarsest=4, bc="neumann"):
    """Problems of different sizes on the unit square (h = 1/n), solved together (a
    one-shot UnevenBatch).  u_list entries are updated in place.  Returns per-problem
    (status, V-cycles) lists in input order."""
    for i, (r, u) in enumerate(zip(rhs_list, u_list)):
        if r.shape != u.shape or r.dtype != u.dtype:
            raise ValueError("rhs and u of problem %d differ in shape or dtype" % i)
    dtypes = {r.dtype for r in rhs_list}
    devices = {r.device for r in rhs_list}
    if len(dtypes) > 1 or len(devices) > 1:
        raise ValueError("all problems must share one dtype and device")
    batch = UnevenBatch([tuple(r.shape) for r in rhs_list], dtype=rhs_list[0].dtype, coarsest=coarsest, bc=bc,
                        device=rhs_list[0].device)
    return batch.solve(rhs_list, u_list, dt, kappa, tol, nu1, nu2)
