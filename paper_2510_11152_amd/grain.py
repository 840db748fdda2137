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


def grain_map(eta, out=None):
    """Per cell, the index of the dominant order parameter (fas_grain_argmax); eta: (q, ny,
    nx) float32 on the device.  Returns an int32 (ny, nx) tensor."""
    if eta.dtype != torch.float32 or not eta.is_contiguous() or eta.dim() != 3:
        raise ValueError("eta must be a contiguous float32 (q, ny, nx) tensor")
    q, ny, nx = eta.shape
    out = torch.empty((ny, nx), dtype=torch.int32, device=eta.device) if out is None else out
    stream = torch.cuda.current_stream(eta.device).cuda_stream
    _lib.check(_lib.load().fas_grain_argmax(ctypes.c_void_p(stream), q, ny * nx, ctypes.c_void_p(eta.data_ptr()),
                                            ctypes.c_void_p(out.data_ptr())), "fas_grain_argmax")
    return out


def count_grains(label):
    """Grains of a periodic grain map (numpy int array, ny x nx): connected regions (4-
    neighbour, wrapped at the edges) of one dominant index.  Returns (grains, mean area in
    cells).  Host-side labelling by repeated minimum propagation over equal neighbours."""
    import numpy as np
    lab = np.asarray(label)
    comp = np.arange(lab.size, dtype=np.int64).reshape(lab.shape)
    same = [(lab == np.roll(lab, s, axis=a)) for a, s in ((0, 1), (0, -1), (1, 1), (1, -1))]
    shifts = ((0, 1), (0, -1), (1, 1), (1, -1))
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
        st, cy = self.grid.solve_stacked(self.rhs, eta, self.dt, self.kappa, self.tol, self.nu1, self.nu2)
        if any(s != 0 for s in st):
            raise RuntimeError("grain-growth solve did not converge for %d fields" % sum(s != 0 for s in st))
        return cy
