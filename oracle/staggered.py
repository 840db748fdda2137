"""Oracle of the 2D staggered-grid FAS multigrid solver (test infrastructure only).

Only tests, the smoke check and the bench's CPU baseline use this module; the library never
imports it.

Section 4.1 extends the cell-centred matrix-free FAS solver (Section 2.2, Algorithm 1) to the
variables of a staggered grid (Section 2.1): pressure at cell centres, the x velocity u at the
east-west (EW) edge centres x_{i+1/2} = i h (i = 1 .. M-1 interior, i = 0 and M on the
boundary), the y velocity v at the north-south (NS) edge centres.  Every variable solves

    a w - c Lap_h w = f                 (5-point Laplacian, spacing h on both axes)

on its own interior index set, with homogeneous boundary data (the caller moves non-zero
boundary values into f).  Per axis, a location is one of three kinds:

  'cn'  cell-centred, homogeneous Neumann (ghost = adjacent value), eq. boundry1-2 style;
  'cd'  cell-centred, homogeneous Dirichlet (ghost = - adjacent value);
  'v'   edge-centred along that axis (the boundary points x_{1/2}, x_{M+1/2} hold 0).

  location   x kind   y kind   unknowns (rows x columns)
  CELL       cn / cd  cn / cd  ny x nx
  EDGE_X     v        cd       ny x (nx - 1)      (u, EW edges)
  EDGE_Y     cd       v        (ny - 1) x nx      (v, NS edges)

Arrays are numpy float64 of shape (rows, columns) with x along the last axis.

Point formulas (one fixed evaluation order each; W, E, S, N are the four neighbours, or 0.0
where a neighbour is a ghost or a boundary point):
  s  = (W + E) + (S + N)
  D  = a h^2 + c k,   k = 4 + (#'cd' ghosts) - (#'cn' ghosts)
  smoother (Gauss-Seidel update):   w = (c s + h^2 f) / D
  operator:                         L w = (D w - c s) / h^2   (as (D w - c s) * (1 / h^2))
  residual:                         r = f - L w

Smoother (Section 2.3, eqs. FCGS-1..4; Section 4.1 for edges): the four parity sets of the
X-shape partition are updated in the order 1, 2, 3, 4; sets 1 and 2 are the points whose two
indices have different parities, sets 3 and 4 those with equal parities.  For the 5-point
operator no point of a set neighbours another point of the first two sets or of the last two,
so one X-MCGS sweep is a red-black Gauss-Seidel sweep that first updates the points with
(ix + iy) odd (0-based indices: the 1-based interior numbering shifts both indices by one),
then those with (ix + iy) even.

Restriction (Appendix C for cells, Appendix D for edges).  Coarse index K covers fine cells
2K, 2K+1 along a cell-centred axis; along an edge axis the coarse unknown K coincides with the
fine unknown 2K + 1 and its neighbours are 2K and 2K + 2.
  CELL:    ((w[2J,2K] + w[2J,2K+1]) + (w[2J+1,2K] + w[2J+1,2K+1])) * 0.25
  EDGE_X:  (g(2J) + g(2J+1)) * 0.125,  g(y) = (w[y,2K] + 2 w[y,2K+1]) + w[y,2K+2]
  EDGE_Y:  the same with the axes exchanged (groups of three along y, summed along x).
Appendix D prints the EW restriction with the (1, 2, 1) weights across three rows and two
columns placed half a fine cell off the coarse edge it defines; taken here with the two index
roles exchanged: (1, 2, 1)/4 along the edge-normal axis over the coincident fine edge and its
two neighbours, times the average of the two fine cells along the other axis (the standard
six-point restriction, centred on the coarse edge, exact for linear functions).

Prolongation of a correction e (FAS, Algorithm 1: e = w_c - R w_f):
  CELL:    injection (Appendix C).
  EDGE_X:  Appendix D: first along y at the coincident fine columns,
           fine row 2J: (3 e[J] + e[J-1]) * 0.25,  fine row 2J+1: (3 e[J] + e[J+1]) * 0.25
           (ghost e[-1] = -e[0], e[Jc] = -e[Jc-1]: homogeneous Dirichlet), then along x:
           fine column 2K+1 (coincident): that value; fine column 2K: (left + right) * 0.5,
           with 0 at the boundary edges.
  EDGE_Y:  the same with the axes exchanged.

V-cycle and solve: Algorithm 1 with ghost-free FAS coarse right-hand side
f_c = R r + L_c(R w), the coarsest level smoothed nu_c times (Remark 1), stopping on the
absolute residual res = h ||r||_2 <= tol (eq. residual) or after kmax cycles.
"""
import numpy as np

CELL, EDGE_X, EDGE_Y = 0, 1, 2


class StagProblem:
    """A staggered variable on an nx x ny cell grid of spacing h.

    loc: CELL, EDGE_X or EDGE_Y; cell_bc: 'neumann' or 'dirichlet' for CELL (edge
    locations are always Dirichlet); coarsest: the smallest number of cells per axis of the
    coarsest level (levels halve both axes while both stay even and >= coarsest);
    nuc: sweeps on the coarsest level."""

    def __init__(self, loc, nx, ny, h, cell_bc="neumann", coarsest=4, nuc=16):
        assert loc in (CELL, EDGE_X, EDGE_Y)
        self.loc, self.nx, self.ny, self.h = loc, int(nx), int(ny), float(h)
        self.cell_bc, self.coarsest, self.nuc = cell_bc, int(coarsest), int(nuc)
        ck = "cn" if cell_bc == "neumann" else "cd"
        self.kinds = {CELL: (ck, ck), EDGE_X: ("v", "cd"), EDGE_Y: ("cd", "v")}[loc]  # (x, y)
        dims = [(self.nx, self.ny)]
        while True:
            mx, my = dims[-1]
            if mx % 2 or my % 2 or mx // 2 < self.coarsest or my // 2 < self.coarsest:
                break
            dims.append((mx // 2, my // 2))
        self.cells = dims

    @property
    def levels(self):
        return len(self.cells)

    def shape(self, l=0):
        mx, my = self.cells[l]
        kx, ky = self.kinds
        return (my - 1 if ky == "v" else my, mx - 1 if kx == "v" else mx)

    def spacing(self, l=0):
        return self.h * float(1 << l)

    def kcount(self, l=0):
        """k = 4 + (#'cd' ghosts) - (#'cn' ghosts) at every unknown of level l."""
        ny, nx = self.shape(l)
        k = np.full((ny, nx), 4.0)
        kx, ky = self.kinds
        d = {"cn": -1.0, "cd": 1.0, "v": 0.0}
        k[:, 0] += d[kx]
        k[:, -1] += d[kx]
        k[0, :] += d[ky]
        k[-1, :] += d[ky]
        return k


def _nbsum(w):
    """s = (W + E) + (S + N), 0.0 for neighbours outside the unknown set."""
    p = np.zeros((w.shape[0] + 2, w.shape[1] + 2))
    p[1:-1, 1:-1] = w
    return (p[1:-1, :-2] + p[1:-1, 2:]) + (p[:-2, 1:-1] + p[2:, 1:-1])


def _consts(P, l, a, c):
    h = P.spacing(l)
    h2 = h * h
    D = a * h2 + c * P.kcount(l)
    return h2, 1.0 / h2, D


def apply(P, l, a, c, w):
    """L w on level l."""
    h2, ih2, D = _consts(P, l, a, c)
    return (D * w - c * _nbsum(w)) * ih2


def residual(P, l, a, c, f, w):
    return f - apply(P, l, a, c, w)


def res_norm(P, a, c, f, w):
    """Section 2.2, eq. residual: h (sum r^2)^(1/2) on the finest level."""
    r = residual(P, 0, a, c, f, w)
    return P.h * float(np.sqrt(np.sum(r * r)))


def smooth(P, l, a, c, f, w, nu):
    """nu X-MCGS sweeps in place (sets 1-2, then 3-4: red-black with (ix+iy) odd first)."""
    h2, _, D = _consts(P, l, a, c)
    ny, nx = w.shape
    par = (np.arange(ny)[:, None] + np.arange(nx)[None, :]) & 1
    hf = h2 * f
    for _ in range(nu):
        for colour in (1, 0):
            new = (c * _nbsum(w) + hf) / D
            m = par == colour
            w[m] = new[m]
    return w


def restrict(P, l, w):
    """R from level l to l + 1 (Appendix C for cells, Appendix D for edges)."""
    if P.loc == CELL:
        return ((w[0::2, 0::2] + w[0::2, 1::2]) + (w[1::2, 0::2] + w[1::2, 1::2])) * 0.25
    if P.loc == EDGE_X:
        g = (w[:, 0:-2:2] + 2.0 * w[:, 1::2]) + w[:, 2::2]
        return (g[0::2, :] + g[1::2, :]) * 0.125
    g = (w[0:-2:2, :] + 2.0 * w[1::2, :]) + w[2::2, :]
    return (g[:, 0::2] + g[:, 1::2]) * 0.125


def _lin_cell(e, n_fine, axis):
    """Appendix D along a Dirichlet cell-centred axis: fine 2J from (3 e[J] + e[J-1]) / 4,
    fine 2J+1 from (3 e[J] + e[J+1]) / 4, ghosts -e[0] and -e[last]."""
    e = np.moveaxis(e, axis, 0)
    lo = np.concatenate([-e[:1], e[:-1]], axis=0)
    hi = np.concatenate([e[1:], -e[-1:]], axis=0)
    out = np.empty((n_fine,) + e.shape[1:])
    out[0::2] = (3.0 * e + lo) * 0.25
    out[1::2] = (3.0 * e + hi) * 0.25
    return np.moveaxis(out, 0, axis)


def _lin_vertex(e, n_fine, axis):
    """Appendix D along an edge axis: coincident fine unknowns 2K+1 take e[K], the others
    the mean of their two coarse neighbours (0 at the boundary points)."""
    e = np.moveaxis(e, axis, 0)
    z = np.zeros((1,) + e.shape[1:])
    left = np.concatenate([z, e], axis=0)
    right = np.concatenate([e, z], axis=0)
    out = np.empty((n_fine,) + e.shape[1:])
    out[1::2] = e
    out[0::2] = (left + right) * 0.5
    return np.moveaxis(out, 0, axis)


def prolong(P, l, e):
    """P from level l + 1 to level l of a correction e."""
    ny, nx = P.shape(l)
    if P.loc == CELL:
        return np.repeat(np.repeat(e, 2, axis=0), 2, axis=1)
    if P.loc == EDGE_X:
        return _lin_vertex(_lin_cell(e, ny, 0), nx, 1)
    return _lin_vertex(_lin_cell(e, nx, 1), ny, 0)


def vcycle(P, a, c, f, w, nu1=2, nu2=2, l=0):
    """One FAS V-cycle (Algorithm 1) from level l, w updated in place."""
    if l == P.levels - 1:
        return smooth(P, l, a, c, f, w, P.nuc)
    smooth(P, l, a, c, f, w, nu1)
    wc = restrict(P, l, w)
    wc0 = wc.copy()
    rc = restrict(P, l, residual(P, l, a, c, f, w))
    fc = rc + apply(P, l + 1, a, c, wc)
    vcycle(P, a, c, fc, wc, nu1, nu2, l + 1)
    w += prolong(P, l, wc - wc0)
    return smooth(P, l, a, c, f, w, nu2)


def solve(P, a, c, f, w, tol, nu1=2, nu2=2, kmax=20):
    """Algorithm 1's outer loop: V-cycles until h ||r||_2 <= tol or kmax cycles.
    Returns (status, cycles, res) with status 0 converged, 1 not converged."""
    res = res_norm(P, a, c, f, w)
    k = 0
    while res > tol and k < kmax:
        vcycle(P, a, c, f, w, nu1, nu2)
        k += 1
        res = res_norm(P, a, c, f, w)
    return (0 if res <= tol else 1), k, res
