"""CPU oracle for the matrix-free FAS V-cycle (arXiv 2510.11152, Section 2, App. A-C).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's CPU
baseline may use this package; the GPU library never imports it and shares no code
with it.  Everything runs single-threaded on the host in the precision of the arrays
passed in (float64, or float32 for the inner cycle of the mixed-precision form).

Arrays are numpy, C-contiguous, shaped (ny, nx) in 2D and (nz, ny, nx) in 3D, so x is
the fastest axis (the paper's p(i, j) with i along x).

Parity unpinned: none of the functions here; each is pinned by tests/test_oracle_*.py
(dense direct solves, DCT/DST/FFT closed forms, the paper's Tables 2-3, mass
conservation, contraction factors, literal X-MCGS set order, adjoint identities).
"""
import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

from . import build as _build

BC = {"neumann": 0, "dirichlet": 1, "periodic": 2}


class _OgProblem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("bc", ctypes.c_int),
        ("n", ctypes.c_long * 3),
        ("h", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("kappa", ctypes.c_double),
        ("coarsest", ctypes.c_int),
        ("nuc", ctypes.c_int),
        ("order", ctypes.c_int),
        ("symmetric", ctypes.c_int),
        ("atol", ctypes.c_double),
    ]


ORDERS = {"x": 0, "u": 1, "z": 2}


_lib = None


def lib():
    """Load liboracle.so, building it first when it is missing or stale."""
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        P = ctypes.POINTER(_OgProblem)
        vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        L.og_levels.argtypes = [P]
        L.og_levels.restype = i
        L.og_level_cells.argtypes = [P, i]
        L.og_level_cells.restype = ctypes.c_long
        for s in ("d", "s"):
            getattr(L, "og_smooth_" + s).argtypes = [P, i, vp, vp, vp, i, i]
            getattr(L, "og_apply_" + s).argtypes = [P, i, vp, vp, vp]
            getattr(L, "og_residual_" + s).argtypes = [P, i, vp, vp, vp, vp]
            getattr(L, "og_restrict_" + s).argtypes = [P, i, vp, vp]
            getattr(L, "og_prolong_add_" + s).argtypes = [P, i, vp, vp, vp]
            getattr(L, "og_vcycle_" + s).argtypes = [P, vp, vp, vp, i, i, i]
            getattr(L, "og_vcycle_" + s).restype = i
            getattr(L, "og_solve_" + s).argtypes = [P, vp, vp, vp, d, i, i, i, i, vp, vp]
            getattr(L, "og_solve_" + s).restype = i
        L.og_solve_mixed.argtypes = [P, vp, vp, vp, d, i, i, i, i, i, vp, vp]
        L.og_solve_mixed.restype = i
        L.og_kappa_grad_d.argtypes = [P, vp, vp, vp, vp]
        _lib = L
    return _lib


@dataclass
class Problem:
    """One backward-Euler step u - dt*div(kappa grad u) = f on a cell-centred grid.

    n is (nx, ny) or (nx, ny, nz); h equal on every axis (Section 2.1).  kappa is the
    constant coefficient; a cell field is passed separately as `kap`.
    """

    n: tuple
    h: float
    dt: float = 1.0
    kappa: float = 1.0
    bc: str = "neumann"
    coarsest: int = 4
    nuc: int = 2
    order: str = "x"          # multi-colour set order of a sweep: "x", "u" or "z" (Section 2.3)
    symmetric: bool = False   # every second sweep in reverse set order (1234-4321)
    atol: float = 0.0         # a solve also stops once ||f - A u||_2 <= atol (Algorithm 1's absolute test)
    _c: _OgProblem = field(default=None, repr=False, compare=False)

    @property
    def dim(self):
        return len(self.n)

    def c(self):
        p = _OgProblem()
        p.dim = self.dim
        p.bc = BC[self.bc]
        for a in range(3):
            p.n[a] = self.n[a] if a < self.dim else 1
        p.h, p.dt, p.kappa = float(self.h), float(self.dt), float(self.kappa)
        p.coarsest, p.nuc = int(self.coarsest), int(self.nuc)
        p.order, p.symmetric = ORDERS[self.order], int(bool(self.symmetric))
        p.atol = float(self.atol)
        return p

    def shape(self, lev=0):
        """numpy shape of level `lev` (x last)."""
        return tuple(int(m) >> lev for m in reversed(self.n))

    def levels(self):
        return lib().og_levels(ctypes.byref(self.c()))


def _sfx(a):
    if a.dtype == np.float64:
        return "d"
    if a.dtype == np.float32:
        return "s"
    raise TypeError("oracle arrays must be float64 or float32, got %s" % a.dtype)


def _ptr(a):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(P, lev, *arrays):
    shp = P.shape(lev)
    dt = None
    for a in arrays:
        if a is None:
            continue
        if tuple(a.shape) != shp:
            raise ValueError("array shape %s != level shape %s" % (a.shape, shp))
        if dt is None:
            dt = a.dtype
        elif a.dtype != dt:
            raise TypeError("mixed dtypes")


def smooth(P, lev, f, u, sweeps, reverse=False, kap=None):
    """In-place X-MCGS (= red-black, odd index sum first) sweeps on level `lev`."""
    _check(P, lev, f, u, kap)
    getattr(lib(), "og_smooth_" + _sfx(u))(ctypes.byref(P.c()), lev, _ptr(kap), _ptr(f), _ptr(u), sweeps, int(reverse))


def apply(P, lev, u, kap=None):
    _check(P, lev, u, kap)
    out = np.empty_like(u)
    getattr(lib(), "og_apply_" + _sfx(u))(ctypes.byref(P.c()), lev, _ptr(kap), _ptr(u), _ptr(out))
    return out


def residual(P, lev, f, u, kap=None):
    _check(P, lev, f, u, kap)
    out = np.empty_like(u)
    getattr(lib(), "og_residual_" + _sfx(u))(ctypes.byref(P.c()), lev, _ptr(kap), _ptr(f), _ptr(u), _ptr(out))
    return out


def restrict(P, lev, fine):
    _check(P, lev, fine)
    out = np.empty(P.shape(lev + 1), dtype=fine.dtype)
    getattr(lib(), "og_restrict_" + _sfx(fine))(ctypes.byref(P.c()), lev, _ptr(fine), _ptr(out))
    return out


def prolong_add(P, lev, cnew, cold, fine):
    _check(P, lev, fine)
    _check(P, lev + 1, cnew, cold)
    getattr(lib(), "og_prolong_add_" + _sfx(fine))(ctypes.byref(P.c()), lev, _ptr(cnew), _ptr(cold), _ptr(fine))


def vcycle(P, f, u, nu1=2, nu2=2, transposed=False, kap=None):
    """One FAS V-cycle on the finest level, u updated in place."""
    _check(P, 0, f, u, kap)
    rc = getattr(lib(), "og_vcycle_" + _sfx(u))(
        ctypes.byref(P.c()), _ptr(kap), _ptr(f), _ptr(u), nu1, nu2, int(transposed))
    if rc:
        raise ValueError("invalid grid hierarchy for %r" % (P,))


def solve(P, f, u, tol=1e-10, nu1=2, nu2=2, kmax=100, transposed=False, kap=None):
    """V-cycles until ||f - A u|| <= tol*||f|| (or <= P.atol).  Returns (status, cycles, rel_hist)."""
    _check(P, 0, f, u, kap)
    hist = np.zeros(kmax, dtype=np.float64)
    cyc = ctypes.c_int(0)
    st = getattr(lib(), "og_solve_" + _sfx(u))(
        ctypes.byref(P.c()), _ptr(kap), _ptr(f), _ptr(u), float(tol), nu1, nu2, kmax, int(transposed),
        ctypes.byref(cyc), _ptr(hist))
    if st < 0:
        raise ValueError("invalid grid hierarchy for %r" % (P,))
    return st, cyc.value, hist[: cyc.value]


def solve_mixed(P, f, u, tol=1e-10, nu1=2, nu2=2, inner=2, kmax=50, kap=None, inner_next=0):
    """FP64 defect correction around FP32 V-cycles: `inner` FP32 cycles in the first
    correction, `inner_next` (if > 0, else `inner`) in the later ones.  Returns (status,
    outer, rel_hist)."""
    _check(P, 0, f, u, kap)
    assert u.dtype == np.float64
    hist = np.zeros(kmax + 1, dtype=np.float64)
    outer = ctypes.c_int(0)
    st = lib().og_solve_mixed(ctypes.byref(P.c()), _ptr(kap), _ptr(f), _ptr(u), float(tol), nu1, nu2, inner,
                              inner_next, kmax, ctypes.byref(outer), _ptr(hist))
    if st < 0:
        raise ValueError("invalid grid hierarchy for %r" % (P,))
    return st, outer.value, hist[: outer.value + 1]


def kappa_grad(P, kap, mu, u, g):
    """g -= mu^T (dA/dkappa) u  (finest level, float64)."""
    _check(P, 0, kap, mu, u, g)
    lib().og_kappa_grad_d(ctypes.byref(P.c()), _ptr(kap), _ptr(mu), _ptr(u), _ptr(g))


def heat(P, u0, steps, tol=1e-10, nu1=2, nu2=2, kap=None, kmax=100, keep=False):
    """Backward-Euler steps: f = u^n, warm start u = u^n, solve.  Returns u^T (and the
    list of states when keep=True) and the cycle counts."""
    u = u0.copy()
    states = [u.copy()] if keep else None
    cycles = []
    for _ in range(steps):
        f = u.copy()
        st, c, _h = solve(P, f, u, tol, nu1, nu2, kmax, kap=kap)
        if st != 0:
            raise RuntimeError("oracle solve did not converge")
        cycles.append(c)
        if keep:
            states.append(u.copy())
    return (u, states, cycles) if keep else (u, cycles)


def heat_adjoint(P, u0, kap, steps, u_tgt, tol=1e-10, nu1=2, nu2=2, kmax=100):
    """Loss ||u_T - u_tgt||^2 of `steps` backward-Euler steps and its gradients with
    respect to u0 and the cell coefficient kap.

    Adjoint recursion: lambda_T = 2 (u_T - u_tgt); for n = T..1: mu = A^{-T} lambda_n
    (transposed V-cycles), g_kappa -= mu^T (dA/dkappa) u_n, lambda_{n-1} = mu.
    Returns (loss, grad_u0, grad_kappa)."""
    uT, states, _ = heat(P, u0, steps, tol, nu1, nu2, kap=kap, kmax=kmax, keep=True)
    diff = uT - u_tgt
    loss = float(np.sum(diff * diff))
    lam = 2.0 * diff
    g = np.zeros_like(u0)
    for n in range(steps, 0, -1):
        mu = np.zeros_like(lam)
        st, _c, _h = solve(P, lam, mu, tol, nu1, nu2, kmax, transposed=True, kap=kap)
        if st != 0:
            raise RuntimeError("oracle adjoint solve did not converge")
        if kap is not None:
            kappa_grad(P, kap, mu, states[n], g)
        lam = mu
    return loss, lam, g
