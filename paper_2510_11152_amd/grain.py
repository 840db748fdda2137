"""Multi-order-parameter grain growth (Section 3.3.1) as a batched workload.

One semi-implicit step of the Allen-Cahn system for q order parameters eta_i on a
periodic grid (L = alpha = beta = gamma = 1):

    (I - dt*kappa*Lap) eta_i^{n+1} = eta_i^n - dt * ((eta_i^3 - eta_i) + 3 eta_i (S - eta_i^2)),
    S = sum_j (eta_j^n)^2,

i.e. one right-hand-side kernel (fas_grain_rhs) and one batched solve of the q
independent Helmholtz problems (fas_solve_stacked, one stacked grid), warm-started from eta^n.
"""
import ctypes

import torch

from . import _lib
from .api import Grid, solve_stacked_mixed


_DT = {torch.float32: _lib.FAS_F32, torch.float64: _lib.FAS_F64}


def grain_rhs(eta, dt, out=None, alpha=1.0, beta=1.0, gamma=1.5):
    """f_i for every field; eta: (q, ...) float32 or float64 (2D or 3D fields), contiguous,
    on the device (the right-hand side is computed in eta's precision).  alpha, beta,
    gamma: the free energy's coefficients (the paper: 1, 1, 1; the grain workload: 1, 1,
    1.5)."""
    if eta.dtype not in _DT or not eta.is_contiguous() or eta.dim() < 3:
        raise ValueError("eta must be a contiguous float32 or float64 (q, ...) tensor of 2D or 3D fields")
    out = torch.empty_like(eta) if out is None else out
    if out.shape != eta.shape or out.dtype != eta.dtype or not out.is_contiguous():
        raise ValueError("out must match eta")
    stream = torch.cuda.current_stream(eta.device).cuda_stream
    q = eta.shape[0]
    _lib.check(_lib.load().fas_grain_rhs(ctypes.c_void_p(stream), _DT[eta.dtype], q, eta.numel() // q, dt, alpha,
                                         beta, gamma, ctypes.c_void_p(eta.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr())),
               "fas_grain_rhs")
    return out


def grain_map(eta, out=None):
    """Per cell, the index of the dominant order parameter (fas_grain_argmax); eta: (q, ...)
    float32 on the device (2D or 3D fields).  Returns an int32 tensor of the field shape."""
    if eta.dtype != torch.float32 or not eta.is_contiguous() or eta.dim() < 3:
        raise ValueError("eta must be a contiguous float32 (q, ...) tensor of 2D or 3D fields")
    q = eta.shape[0]
    cells = eta.numel() // q
    out = torch.empty(eta.shape[1:], dtype=torch.int32, device=eta.device) if out is None else out
    if out.dtype != torch.int32 or not out.is_contiguous() or out.numel() != cells:
        raise ValueError("out must be a contiguous int32 tensor of the field shape")
    stream = torch.cuda.current_stream(eta.device).cuda_stream
    _lib.check(_lib.load().fas_grain_argmax(ctypes.c_void_p(stream), q, cells, ctypes.c_void_p(eta.data_ptr()),
                                            ctypes.c_void_p(out.data_ptr())), "fas_grain_argmax")
    return out


def count_grains(label):
    """Grains of a periodic grain map (numpy int array, 2D or 3D): connected regions (face
    neighbours, wrapped at the edges) of one dominant index.  Returns (grains, mean size in
    cells).  Host-side labelling by repeated minimum propagation over equal neighbours."""
    import numpy as np
    lab = np.asarray(label)
    comp = np.arange(lab.size, dtype=np.int64).reshape(lab.shape)
    shifts = tuple((a, s) for a in range(lab.ndim) for s in (1, -1))
    same = [(lab == np.roll(lab, s, axis=a)) for a, s in shifts]
    while True:
        new = comp
        for (a, s), eq in zip(shifts, same):
            new = np.where(eq, np.minimum(new, np.roll(comp, s, axis=a)), new)
        # pointer jumping: each cell takes its root's current label
        new = new.reshape(-1)[new.reshape(-1)].reshape(lab.shape)
        if np.array_equal(new, comp):
            break
        comp = new
    grains = int(np.unique(comp).size)
    return grains, lab.size / grains


class GrainGrowth:
    """q fields on an n^dim periodic grid, spacing h, time step dt, gradient coefficient
    kappa, solved to relative residual tol per field (or absolute residual atol: a field
    whose grains have vanished decays towards zero, where a relative test is out of reach
    in FP32).  precision: 'fp32' (FP32 state and
    solves, one stacked grid), 'fp64' (FP64 state and solves) or 'mixed' (FP64 state,
    right-hand side and defect correction around `inner` FP32 V-cycles, two stacked
    grids)."""

    def __init__(self, q, n, h=1.0, dt=0.1, kappa=1.0, tol=1e-6, coarsest=4, nu1=2, nu2=2, device="cuda",
                 graph=False, autotune=False, precision="fp32", inner=2, dim=2, atol=0.0, alpha=1.0, beta=1.0,
                 gamma=1.5):
        if precision not in ("fp32", "fp64", "mixed"):
            raise ValueError("precision must be 'fp32', 'fp64' or 'mixed'")
        self.q, self.n, self.h, self.dt, self.kappa, self.tol = q, n, h, dt, kappa, tol
        self.nu1, self.nu2, self.precision, self.inner = nu1, nu2, precision, inner
        self.alpha, self.beta, self.gamma = alpha, beta, gamma
        dtype = torch.float32 if precision == "fp32" else torch.float64
        self.grid = Grid((n,) * dim, h, bc="periodic", dtype=dtype, coarsest=coarsest, device=device, batch=q)
        self.grid.set(graph=graph, autotune=autotune, atol=atol)
        self.inner_grid = None
        if precision == "mixed":
            self.inner_grid = Grid((n,) * dim, h, bc="periodic", dtype=torch.float32, coarsest=coarsest,
                                   device=device, batch=q, mixed_inner=True).set(autotune=autotune)
        self.rhs = None

    def step(self, eta):
        """Advance eta (q, n, n[, n]) in place by one step; returns per-field cycle counts (outer
        corrections in the mixed form)."""
        self.rhs = grain_rhs(eta, self.dt, self.rhs, self.alpha, self.beta, self.gamma)
        if self.inner_grid is not None:
            st, cy = solve_stacked_mixed(self.grid, self.inner_grid, self.rhs, eta, self.dt, self.kappa, self.tol,
                                         self.nu1, self.nu2, self.inner)
        else:
            st, cy = self.grid.solve_stacked(self.rhs, eta, self.dt, self.kappa, self.tol, self.nu1, self.nu2)
        if any(s != 0 for s in st):
            raise RuntimeError("grain-growth solve did not converge for %d fields" % sum(s != 0 for s in st))
        return cy
