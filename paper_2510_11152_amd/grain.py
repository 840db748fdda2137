"""Multi-order-parameter grain growth (Section 3.3.1) as a batched workload.

One semi-implicit step of the Allen-Cahn system for q order parameters eta_i on a
periodic grid (L = alpha = beta = gamma = 1):

    (I - dt*kappa*Lap) eta_i^{n+1} = eta_i^n - dt * ((eta_i^3 - eta_i) + 3 eta_i (S - eta_i^2)),
    S = sum_j (eta_j^n)^2,

i.e. one right-hand-side kernel (fas_grain_rhs) and one batched solve of the q
independent Helmholtz problems (fas_solve_batched), warm-started from eta^n.
"""
import ctypes

import torch

from . import _lib
from .api import Grid


def grain_rhs(eta, dt, out=None):
    """f_i for every field; eta: (q, ny, nx) float32 contiguous on the device."""
    if eta.dtype != torch.float32 or not eta.is_contiguous() or eta.dim() != 3:
        raise ValueError("eta must be a contiguous float32 (q, ny, nx) tensor")
    out = torch.empty_like(eta) if out is None else out
    stream = torch.cuda.current_stream(eta.device).cuda_stream
    q, ny, nx = eta.shape
    _lib.check(_lib.load().fas_grain_rhs(ctypes.c_void_p(stream), q, ny * nx, dt, ctypes.c_void_p(eta.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr())), "fas_grain_rhs")
    return out


class GrainGrowth:
    """q fields on an n x n periodic grid, spacing h, time step dt, gradient coefficient
    kappa; FP32 storage and solves (relative residual tol per field)."""

    def __init__(self, q, n, h=1.0, dt=0.1, kappa=1.0, tol=1e-6, coarsest=4, nu1=2, nu2=2, device="cuda",
                 graph=False, autotune=False):
        self.q, self.n, self.h, self.dt, self.kappa, self.tol = q, n, h, dt, kappa, tol
        self.nu1, self.nu2 = nu1, nu2
        self.grid = Grid((n, n), h, bc="periodic", dtype=torch.float32, coarsest=coarsest, device=device, batch=q)
        self.grid.set(graph=graph, autotune=autotune)
        self.rhs = None

    def step(self, eta):
        """Advance eta (q, n, n) in place by one step; returns per-field cycle counts."""
        self.rhs = grain_rhs(eta, self.dt, self.rhs)
        st, cy = self.grid.solve_batched(self.rhs, eta, self.dt, self.kappa, self.tol, self.nu1, self.nu2)
        if any(s != 0 for s in st):
            raise RuntimeError("grain-growth solve did not converge for %d fields" % sum(s != 0 for s in st))
        return cy
