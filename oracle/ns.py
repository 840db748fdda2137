"""Oracle of the 2D incompressible Navier-Stokes projection step (test infrastructure only).

Only tests, the smoke check and the bench's CPU baseline use this module; the library never
imports it.

Section 4.2, Scheme 1 (first-order projection) on the staggered grid of Section 2.1:
u at EW edges (shape ny x (nx-1)), v at NS edges ((ny-1) x nx), p at cell centres (ny x nx),
all walls no-slip except an optional constant tangential speed `lid` of u on the top wall.
One step, as the classical implementation orders it (the table of the classical first-order
scheme, steps 1-11; steps 12-15 are the copies new -> old):

  f_u = u^n + dt ((F_u - conv_u) - (p^n_{i+1} - p^n_i) / h)
  (1 - (dt/Re) Lap) u~ = f_u                 (staggered FAS solve, EDGE_X)
  f_v, v~ likewise                           (EDGE_Y)
  -dt Lap p~ = -div(u~, v~)                  (CELL, homogeneous Neumann, a = 0)
  u^{n+1} = u~ - dt (p~_{i+1} - p~_i) / h,   v^{n+1} likewise,   p^{n+1} = p^n + p~

F is a separable forcing sum_k c_k Phi_k (fields and coefficients from the caller; the
manufactured solution of Section 4.4.3 is a sum of three such terms).

Convection conv = a_x d_x(phi) + a_y d_y(phi) with third-order WENO derivatives (the
Hamilton-Jacobi WENO3 of Jiang and Peng with Jiang-Shu smoothness weights): with the forward
differences d0 = phi_{i-1} - phi_{i-2}, d1 = phi_i - phi_{i-1}, d2 = phi_{i+1} - phi_i,

  phi_x^- = ((d1 + d2) - w (d0 - 2 d1 + d2)) / (2h),
  w = 1 / (1 + 2 r^2),  r = (eps + (d1 - d0)^2) / (eps + (d2 - d1)^2),  eps = 1e-6,

and phi_x^+ the mirror image; the upwind choice is branch-free,
a d(phi) = max(a, 0) phi^- + min(a, 0) phi^+ (the paper replaces the WENO branches by array
operations).  The advecting velocity across is the mean of the four nearest values of the
other component.  Two ghost layers beyond each wall extend the stencils by odd reflection
about the wall value g (ghost = 2 g - mirror value).
"""
import numpy as np

from . import staggered as st

WENO_EPS = 1e-6


def _weno_pair(pm2, pm1, p0, pp1, pp2, ih):
    """(phi^-, phi^+) at the centre of the five values along one axis; ih = 1/h."""
    d0 = pm1 - pm2
    d1 = p0 - pm1
    d2 = pp1 - p0
    rm = (WENO_EPS + (d1 - d0) * (d1 - d0)) / (WENO_EPS + (d2 - d1) * (d2 - d1))
    wm = 1.0 / (1.0 + 2.0 * (rm * rm))
    minus = ((d1 + d2) - wm * ((d0 - 2.0 * d1) + d2)) * (0.5 * ih)
    e0 = pp2 - pp1
    e1 = pp1 - p0
    e2 = p0 - pm1
    rp = (WENO_EPS + (e1 - e0) * (e1 - e0)) / (WENO_EPS + (e2 - e1) * (e2 - e1))
    wp = 1.0 / (1.0 + 2.0 * (rp * rp))
    plus = ((e1 + e2) - wp * ((e0 - 2.0 * e1) + e2)) * (0.5 * ih)
    return minus, plus


def _weno_along_x(e, ih):
    r = slice(2, -2)
    return _weno_pair(e[r, 0:-4], e[r, 1:-3], e[r, 2:-2], e[r, 3:-1], e[r, 4:], ih)


def _weno_along_y(e, ih):
    c = slice(2, -2)
    return _weno_pair(e[0:-4, c], e[1:-3, c], e[2:-2, c], e[3:-1, c], e[4:, c], ih)


def _upwind(a, minus, plus):
    return np.maximum(a, 0.0) * minus + np.minimum(a, 0.0) * plus


def _ext_u(u, lid):
    """u with two ghost layers on every side: the wall points x = 0, 1 (value 0) and their
    odd reflections along x; cell-type ghosts (2g - mirror value) along y with g = 0 below
    and g = lid above.  Interior u sits at [2:-2, 2:-2]."""
    ny, m = u.shape
    e = np.zeros((ny + 4, m + 4))
    e[2:-2, 2:-2] = u
    e[2:-2, 1] = 0.0
    e[2:-2, -2] = 0.0
    e[2:-2, 0] = 2.0 * 0.0 - u[:, 0]
    e[2:-2, -1] = 2.0 * 0.0 - u[:, -1]
    e[1, 2:-2] = 2.0 * 0.0 - e[2, 2:-2]
    e[0, 2:-2] = 2.0 * 0.0 - e[3, 2:-2]
    e[-2, 2:-2] = 2.0 * lid - e[-3, 2:-2]
    e[-1, 2:-2] = 2.0 * lid - e[-4, 2:-2]
    return e


def _ext_v(v):
    """v with two ghost layers: the wall points y = 0, 1 (value 0) and their odd reflections
    along y; cell-type ghosts (2 * 0 - mirror value) along x.  Interior v at [2:-2, 2:-2]."""
    m, nx = v.shape
    e = np.zeros((m + 4, nx + 4))
    e[2:-2, 2:-2] = v
    e[1, 2:-2] = 0.0
    e[-2, 2:-2] = 0.0
    e[0, 2:-2] = 2.0 * 0.0 - v[0, :]
    e[-1, 2:-2] = 2.0 * 0.0 - v[-1, :]
    e[2:-2, 1] = 2.0 * 0.0 - e[2:-2, 2]
    e[2:-2, 0] = 2.0 * 0.0 - e[2:-2, 3]
    e[2:-2, -2] = 2.0 * 0.0 - e[2:-2, -3]
    e[2:-2, -1] = 2.0 * 0.0 - e[2:-2, -4]
    return e


def _vbar_at_u(v):
    """Mean of the four v around each u point: ((vS_W + vS_E) + (vN_W + vN_E)) * 0.25 with
    the wall values 0 below the first and above the last row."""
    m, nx = v.shape
    vp = np.zeros((m + 2, nx))
    vp[1:-1] = v
    south, north = vp[:-1], vp[1:]            # (ny, nx)
    return ((south[:, :-1] + south[:, 1:]) + (north[:, :-1] + north[:, 1:])) * 0.25


def _ubar_at_v(u):
    """Mean of the four u around each v point: ((uS_W + uS_E) + (uN_W + uN_E)) * 0.25 with
    the wall values 0 left of the first and right of the last column."""
    ny, m = u.shape
    up = np.zeros((ny, m + 2))
    up[:, 1:-1] = u
    west, east = up[:, :-1], up[:, 1:]        # (ny, nx)
    return ((west[:-1] + east[:-1]) + (west[1:] + east[1:])) * 0.25


def conv_u(u, v, h, lid=0.0):
    """u d_x u + vbar d_y u at every interior EW edge."""
    ih = 1.0 / h
    e = _ext_u(u, lid)
    xm, xp = _weno_along_x(e, ih)
    ym, yp = _weno_along_y(e, ih)
    return _upwind(u, xm, xp) + _upwind(_vbar_at_u(v), ym, yp)


def conv_v(u, v, h):
    """ubar d_x v + v d_y v at every interior NS edge."""
    ih = 1.0 / h
    e = _ext_v(v)
    xm, xp = _weno_along_x(e, ih)
    ym, yp = _weno_along_y(e, ih)
    return _upwind(_ubar_at_v(u), xm, xp) + _upwind(v, ym, yp)


def forcing(fields, coef, shape):
    """sum_k coef[k] * fields[k], summed left to right (0 when there are none)."""
    F = np.zeros(shape)
    for k, (phi, ck) in enumerate(zip(fields, coef)):
        F = ck * phi if k == 0 else F + ck * phi
    return F


def momentum_rhs_u(u, v, p, h, dt, Fu, lid=0.0):
    ih = 1.0 / h
    gp = (p[:, 1:] - p[:, :-1]) * ih
    return u + dt * ((Fu - conv_u(u, v, h, lid)) - gp)


def momentum_rhs_v(u, v, p, h, dt, Fv):
    ih = 1.0 / h
    gp = (p[1:, :] - p[:-1, :]) * ih
    return v + dt * ((Fv - conv_v(u, v, h)) - gp)


def lift_lid(fu, h, c, lid):
    """The top wall's tangential speed moved into the u right-hand side: the ghost row
    2 lid - u enters the last row's Laplacian as 2 c lid / h^2."""
    ih2 = 1.0 / (h * h)
    fu = fu.copy()
    fu[-1, :] = fu[-1, :] + (2.0 * c * lid) * ih2
    return fu


def divergence(u, v, h):
    """(u_E - u_W + v_N - v_S) / h per cell, wall values 0."""
    ny, nx = u.shape[0], v.shape[1]
    up = np.zeros((ny, nx + 1))
    up[:, 1:-1] = u
    vp = np.zeros((ny + 1, nx))
    vp[1:-1, :] = v
    return ((up[:, 1:] - up[:, :-1]) + (vp[1:, :] - vp[:-1, :])) * (1.0 / h)


def project(ut, vt, pt, p, h, dt):
    """u^{n+1} = u~ - dt d_x p~, v^{n+1} = v~ - dt d_y p~, p^{n+1} = p^n + p~."""
    ih = 1.0 / h
    un = ut - dt * ((pt[:, 1:] - pt[:, :-1]) * ih)
    vn = vt - dt * ((pt[1:, :] - pt[:-1, :]) * ih)
    return un, vn, p + pt


class Projection:
    """Scheme 1 in the classical arrangement: the nine fields u^n, u~, u^{n+1}, v^n, v~,
    v^{n+1}, p^n, p~, p^{n+1} (the 2D subset of the twelve of the classical table), with
    u~, v~ and p~ kept from step to step as the next solves' initial guesses."""

    def __init__(self, nx, ny, h, re, coarsest=4, nuc=16, lid=0.0):
        self.h, self.re, self.lid = float(h), float(re), float(lid)
        self.Pu = st.StagProblem(st.EDGE_X, nx, ny, h, coarsest=coarsest, nuc=nuc)
        self.Pv = st.StagProblem(st.EDGE_Y, nx, ny, h, coarsest=coarsest, nuc=nuc)
        self.Pp = st.StagProblem(st.CELL, nx, ny, h, cell_bc="neumann", coarsest=coarsest, nuc=nuc)
        self.u = np.zeros(self.Pu.shape())
        self.v = np.zeros(self.Pv.shape())
        self.p = np.zeros(self.Pp.shape())
        self.ut, self.vt, self.pt = self.u.copy(), self.v.copy(), self.p.copy()

    def step(self, dt, Fu_fields=(), Fv_fields=(), coef=(), tol=1e-9, nu1=2, nu2=2, kmax=20):
        """One step; returns the three solves' (status, cycles, res)."""
        h, c = self.h, dt / self.re
        Fu = forcing(Fu_fields, coef, self.u.shape)
        Fv = forcing(Fv_fields, coef, self.v.shape)
        fu = lift_lid(momentum_rhs_u(self.u, self.v, self.p, h, dt, Fu, self.lid), h, c, self.lid)
        fv = momentum_rhs_v(self.u, self.v, self.p, h, dt, Fv)
        su = st.solve(self.Pu, 1.0, c, fu, self.ut, tol, nu1, nu2, kmax)
        sv = st.solve(self.Pv, 1.0, c, fv, self.vt, tol, nu1, nu2, kmax)
        fp = -divergence(self.ut, self.vt, h)
        sp = st.solve(self.Pp, 0.0, dt, fp, self.pt, tol, nu1, nu2, kmax)
        un, vn, pn = project(self.ut, self.vt, self.pt, self.p, h, dt)
        self.u, self.v, self.p = un, vn, pn
        return su, sv, sp


# ---- Section 4.4.3's manufactured solution ------------------------------------------------
def grid_points(nx, ny, h):
    """Coordinates of the u, v and p points: (xu, yu), (xv, yv), (xp, yp) as 2D arrays."""
    xc = (np.arange(nx) + 0.5) * h
    yc = (np.arange(ny) + 0.5) * h
    xe = np.arange(1, nx) * h
    ye = np.arange(1, ny) * h
    return np.meshgrid(xe, yc), np.meshgrid(xc, ye), np.meshgrid(xc, yc)


def exact(nx, ny, h, t):
    """u = sin t sin^2(pi x) sin(2 pi y), v = -sin t sin(2 pi x) sin^2(pi y),
    p = sin t (sin(pi y) - 2/pi) at the staggered points."""
    (xu, yu), (xv, yv), (xp, yp) = grid_points(nx, ny, h)
    pi = np.pi
    s = np.sin(t)
    u = s * np.sin(pi * xu) ** 2 * np.sin(2 * pi * yu)
    v = -s * np.sin(2 * pi * xv) * np.sin(pi * yv) ** 2
    p = s * (np.sin(pi * yp) - 2.0 / pi)
    return u, v, p


def manufactured_fields(nx, ny, h, re):
    """Phi fields with F(t) = cos t Phi_0 + sin t Phi_1 + sin^2 t Phi_2 for u and for v:
    the source that makes the exact solution satisfy the momentum equation (eq. Ns_1)."""
    (xu, yu), (xv, yv), _ = grid_points(nx, ny, h)
    pi = np.pi
    S, C = np.sin, np.cos
    # u = s a(x, y):  a = sin^2(pi x) sin(2 pi y)
    a = S(pi * xu) ** 2 * S(2 * pi * yu)
    a_x = pi * S(2 * pi * xu) * S(2 * pi * yu)
    a_y = 2 * pi * S(pi * xu) ** 2 * C(2 * pi * yu)
    a_xx = 2 * pi ** 2 * C(2 * pi * xu) * S(2 * pi * yu)
    a_yy = -4 * pi ** 2 * S(pi * xu) ** 2 * S(2 * pi * yu)
    b_at_u = -S(2 * pi * xu) * S(pi * yu) ** 2          # v / sin t at the u points
    u0 = a
    u1 = -(a_xx + a_yy) / re                             # p_x = 0
    u2 = a * a_x + b_at_u * a_y
    # v = s b(x, y):  b = -sin(2 pi x) sin^2(pi y)
    b = -S(2 * pi * xv) * S(pi * yv) ** 2
    b_x = -2 * pi * C(2 * pi * xv) * S(pi * yv) ** 2
    b_y = -pi * S(2 * pi * xv) * S(2 * pi * yv)
    b_xx = 4 * pi ** 2 * S(2 * pi * xv) * S(pi * yv) ** 2
    b_yy = -2 * pi ** 2 * S(2 * pi * xv) * C(2 * pi * yv)
    a_at_v = S(pi * xv) ** 2 * S(2 * pi * yv)
    v0 = b
    v1 = -(b_xx + b_yy) / re + pi * C(pi * yv)           # p_y / sin t
    v2 = a_at_v * b_x + b * b_y
    return (u0, u1, u2), (v0, v1, v2)


def manufactured_coef(t):
    return (np.cos(t), np.sin(t), np.sin(t) ** 2)


def l2(e, h):
    return h * float(np.sqrt(np.sum(e * e)))


def convergence_run(n, dt, re=10.0, t_end=1.0, tol=1e-9, nu1=2, nu2=2, kmax=20, force_at="new"):
    """Section 4.4.3: Scheme 1 from the exact state at t = 0 to t_end; returns the L2 errors
    (u, v, p) at t_end (p compared after removing both means: the Neumann pressure is
    defined up to a constant) and the solve counts."""
    h = 1.0 / n
    nsteps = int(round(t_end / dt))
    S = Projection(n, n, h, re)
    S.u, S.v, S.p = exact(n, n, h, 0.0)
    Fu, Fv = manufactured_fields(n, n, h, re)
    cycles = []
    for k in range(nsteps):
        tf = (k + 1) * dt if force_at == "new" else k * dt
        out = S.step(dt, Fu, Fv, manufactured_coef(tf), tol, nu1, nu2, kmax)
        cycles.append([o[1] for o in out])
    ue, ve, pe = exact(n, n, h, nsteps * dt)
    dp = (S.p - S.p.mean()) - (pe - pe.mean())
    return (l2(S.u - ue, h), l2(S.v - ve, h), l2(dp, h)), cycles
