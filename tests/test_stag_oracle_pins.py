"""Pins of the staggered-grid and Navier-Stokes oracles (oracle/staggered.py, oracle/ns.py)
against closed forms, brute force and the values Section 4.4.3 prints."""
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla
from scipy import sparse

from oracle import ns
from oracle import staggered as st

LOCS = [(st.CELL, "neumann"), (st.CELL, "dirichlet"), (st.EDGE_X, None), (st.EDGE_Y, None)]
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table6_first_order.txt")


def _prob(loc, bc, n, m=None, **kw):
    return st.StagProblem(loc, n, m or n, 1.0 / n, cell_bc=bc or "dirichlet", **kw)


def _points(P):
    """Coordinates of the unknowns along x and y (edge axes at i h, cell axes at (i+1/2) h)."""
    ny, nx = P.shape()
    kx, ky = P.kinds
    x = (np.arange(nx) + (1.0 if kx == "v" else 0.5)) * P.h
    y = (np.arange(ny) + (1.0 if ky == "v" else 0.5)) * P.h
    return np.meshgrid(x, y)


def _mode(P, kx_, ky_):
    """A discrete eigenvector of the operator on the Lx x Ly domain: sin(k pi x / Lx) along a
    Dirichlet axis (zero at the wall points, odd about the wall for cell-centred ghosts),
    cos(k pi x / Lx) along a Neumann one; eigenvalue of -Lap_h:
    (4/h^2)(sin^2(k pi h / (2 Lx)) + sin^2(m pi h / (2 Ly)))."""
    X, Y = _points(P)
    Lx, Ly = P.nx * P.h, P.ny * P.h
    fx = np.cos if P.kinds[0] == "cn" else np.sin
    fy = np.cos if P.kinds[1] == "cn" else np.sin
    w = fx(kx_ * np.pi * X / Lx) * fy(ky_ * np.pi * Y / Ly)
    lam = 4.0 / P.h ** 2 * (np.sin(kx_ * np.pi * P.h / (2 * Lx)) ** 2 + np.sin(ky_ * np.pi * P.h / (2 * Ly)) ** 2)
    return w, lam


@pytest.mark.parametrize("loc,bc", LOCS)
@pytest.mark.parametrize("a,c", [(1.0, 0.01), (0.0, 1.0), (2.0, 0.5)])
def test_apply_on_eigenvectors(loc, bc, a, c):
    P = _prob(loc, bc, 32, 16)
    for kx_, ky_ in [(1, 1), (3, 2), (7, 5)]:
        w, lam = _mode(P, kx_, ky_)
        got = st.apply(P, 0, a, c, w)
        assert np.allclose(got, (a + c * lam) * w, rtol=0, atol=1e-9 * (a + c * lam))


def _dense(P, l, a, c):
    ny, nx = P.shape(l)
    N = nx * ny
    A = np.zeros((N, N))
    for k in range(N):
        e = np.zeros(N)
        e[k] = 1.0
        A[:, k] = st.apply(P, l, a, c, e.reshape(ny, nx)).ravel()
    return A


@pytest.mark.parametrize("loc,bc", LOCS)
def test_sweep_is_gauss_seidel_in_set_order(loc, bc):
    """One sweep equals point Gauss-Seidel on the assembled matrix, visiting the points of
    sets 1-2 ((ix + iy) odd) and then those of sets 3-4, one at a time."""
    P = _prob(loc, bc, 8, 16)
    a, c = (0.0, 1.0) if bc == "neumann" else (1.0, 0.05)
    rng = np.random.default_rng(3)
    ny, nx = P.shape()
    f = rng.standard_normal((ny, nx))
    w0 = rng.standard_normal((ny, nx))
    A = _dense(P, 0, a, c)
    x = w0.ravel().copy()
    order = [(iy, ix) for par in (1, 0) for iy in range(ny) for ix in range(nx) if (ix + iy) % 2 == par]
    for iy, ix in order:
        k = iy * nx + ix
        x[k] += (f.ravel()[k] - A[k] @ x) / A[k, k]
    got = st.smooth(P, 0, a, c, f, w0.copy(), 1)
    assert np.allclose(got.ravel(), x, rtol=0, atol=1e-12 * np.abs(x).max())


@pytest.mark.parametrize("loc,bc", LOCS)
def test_restriction_is_exact_for_linear_functions(loc, bc):
    """R of alpha + beta x + gamma y is the same function at the coarse points."""
    P = _prob(loc, bc, 32, 16)
    X, Y = _points(P)
    w = 0.3 + 1.7 * X - 0.9 * Y
    wc = st.restrict(P, 0, w)
    Pc = _prob(loc, bc, 16, 8)
    Xc, Yc = _points(Pc)
    assert wc.shape == Pc.shape()
    assert np.allclose(wc, 0.3 + 1.7 * Xc - 0.9 * Yc, rtol=0, atol=1e-13)


@pytest.mark.parametrize("loc", [st.EDGE_X, st.EDGE_Y])
def test_prolongation_is_linear_interpolation(loc):
    """Away from the walls P reproduces linear functions; at the walls it uses the
    homogeneous boundary values (0 at wall points, odd ghosts across cell-centred walls)."""
    P = _prob(loc, None, 32, 32)
    Pc = _prob(loc, None, 16, 16)
    Xc, Yc = _points(Pc)
    X, Y = _points(P)
    e = 0.25 + 0.5 * Xc + 0.75 * Yc
    got = st.prolong(P, 0, e)
    want = 0.25 + 0.5 * X + 0.75 * Y
    inner = (slice(2, -2), slice(2, -2))
    assert np.allclose(got[inner], want[inner], rtol=0, atol=1e-13)
    # tent(x) tent(y), tent(s) = min(s, 1 - s), vanishes on every wall; its kink lies on a
    # coarse point along the edge axis, so P reproduces it at every point whose cell-axis
    # stencil stays on one side of the middle: the two rows (columns) next to each wall,
    # where the odd ghost across the wall enters
    tent = lambda s: np.minimum(s, 1.0 - s)  # noqa: E731
    got = st.prolong(P, 0, tent(Xc) * tent(Yc))
    want = tent(X) * tent(Y)
    axis = 0 if loc == st.EDGE_X else 1
    assert np.allclose(np.take(got, [0, 1, -2, -1], axis=axis), np.take(want, [0, 1, -2, -1], axis=axis),
                       rtol=0, atol=1e-13)


def test_cell_transfer_is_appendix_c():
    P = _prob(st.CELL, "neumann", 8, 8)
    rng = np.random.default_rng(0)
    w = rng.standard_normal(P.shape())
    assert np.allclose(st.restrict(P, 0, w), w.reshape(4, 2, 4, 2).mean(axis=(1, 3)), rtol=0, atol=1e-15)
    e = rng.standard_normal((4, 4))
    assert np.array_equal(st.prolong(P, 0, e), np.kron(e, np.ones((2, 2))))


@pytest.mark.parametrize("loc,bc", LOCS)
def test_converged_solve_matches_direct_solve(loc, bc):
    P = _prob(loc, bc, 32, 16)
    a, c = (0.0, 1.0) if bc == "neumann" else (1.0, 0.01)
    rng = np.random.default_rng(7)
    ny, nx = P.shape()
    f = rng.standard_normal((ny, nx))
    if a == 0.0:
        f -= f.mean()                      # compatible right-hand side of the singular problem
    w = np.zeros((ny, nx))
    status, cycles, res = st.solve(P, a, c, f, w, 1e-11, kmax=60)
    assert status == 0 and cycles < 30
    A = sparse.csr_matrix(_dense(P, 0, a, c))
    if a == 0.0:
        x = np.linalg.lstsq(A.toarray(), f.ravel(), rcond=None)[0]
        assert np.allclose(w.ravel() - w.mean(), x - x.mean(), rtol=0, atol=1e-9)
    else:
        x = spla.spsolve(A, f.ravel())
        assert np.allclose(w.ravel(), x, rtol=0, atol=1e-10 * np.abs(x).max())


@pytest.mark.parametrize("loc,bc", LOCS)
def test_vcycle_contracts_independently_of_the_grid(loc, bc):
    a, c = (0.0, 1.0) if bc == "neumann" else (1.0, 1.0)
    rates = []
    for n in (64, 128):
        P = _prob(loc, bc, n)
        rng = np.random.default_rng(n)
        f = rng.standard_normal(P.shape())
        if a == 0.0:
            f -= f.mean()
        w = np.zeros(P.shape())
        r0 = st.res_norm(P, a, c, f, w)
        for _ in range(4):
            st.vcycle(P, a, c, f, w)
        rates.append((st.res_norm(P, a, c, f, w) / r0) ** 0.25)
    assert max(rates) < 0.2
    assert abs(rates[0] - rates[1]) < 0.1


@pytest.mark.parametrize("loc,bc", [(st.CELL, "dirichlet"), (st.EDGE_X, None), (st.EDGE_Y, None)])
def test_second_order_accuracy(loc, bc):
    """w - Lap w = f with the exact solution sin(pi x) sin(pi y) (zero on every wall):
    the discrete error falls by about 4 per halving of h."""
    errs = []
    for n in (32, 64, 128):
        P = _prob(loc, bc, n)
        X, Y = _points(P)
        ex = np.sin(np.pi * X) * np.sin(np.pi * Y)
        f = (1.0 + 2 * np.pi ** 2) * ex
        w = np.zeros(P.shape())
        st.solve(P, 1.0, 1.0, f, w, 1e-12, kmax=40)
        errs.append(np.abs(w - ex).max())
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


# ---- WENO3 ---------------------------------------------------------------------------------
def test_weno_is_exact_for_linear_data_and_reduces_to_the_linear_scheme():
    h = 0.1
    x = np.arange(5) * h
    phi = 2.0 + 3.0 * x
    m, p = ns._weno_pair(*phi, 1.0 / h)
    assert abs(m - 3.0) < 1e-12 and abs(p - 3.0) < 1e-12
    # quadratic data: equal second differences on both sides, so r = 1, w = 1/3 and the
    # left-biased derivative is the linear third-order upwind formula
    phi = 1.0 + x - 2.0 * x ** 2
    m, p = ns._weno_pair(*phi, 1.0 / h)
    lin_m = (phi[0] - 6 * phi[1] + 3 * phi[2] + 2 * phi[3]) / (6 * h)
    lin_p = (-phi[4] + 6 * phi[3] - 3 * phi[2] - 2 * phi[1]) / (6 * h)
    assert abs(m - lin_m) < 1e-12 and abs(p - lin_p) < 1e-12
    assert abs(m - (1.0 - 4.0 * x[2])) < 1e-12          # exact for quadratics


def test_weno_picks_the_smooth_side_at_a_jump():
    """Left of a jump the left-biased derivative ignores it (weight -> 1: the one-sided
    second-order formula); the mirrored one leans on it."""
    h = 1.0
    phi = np.array([0.0, 1.0, 2.0, 10.0, 11.0])
    m, _ = ns._weno_pair(*phi, 1.0 / h)
    assert abs(m - (3 * phi[2] - 4 * phi[1] + phi[0]) / (2 * h)) < 1e-3


def test_weno_derivative_converges():
    errs = []
    for n in (32, 64, 128):
        h = 1.0 / n
        x = np.arange(-2, n + 3) * h
        phi = np.sin(2 * np.pi * x)
        m, p = ns._weno_pair(phi[:-4], phi[1:-3], phi[2:-2], phi[3:-1], phi[4:], 1.0 / h)
        d = 2 * np.pi * np.cos(2 * np.pi * x[2:-2])
        errs.append(max(np.abs(m - d).max(), np.abs(p - d).max()))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


def test_convection_converges_to_the_advective_derivative():
    """conv_u -> u u_x + v u_y and conv_v -> u v_x + v v_y for the divergence-free field of
    the manufactured solution (which vanishes on the walls)."""
    errs = []
    for n in (32, 64, 128):
        h = 1.0 / n
        u, v, _ = ns.exact(n, n, h, np.pi / 2)
        (Fu, Fv) = ns.manufactured_fields(n, n, h, 10.0)
        errs.append(max(np.abs(ns.conv_u(u, v, h) - Fu[2]).max(), np.abs(ns.conv_v(u, v, h) - Fv[2]).max()))
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0


def test_manufactured_forcing_satisfies_the_momentum_equation():
    """F = u_t + u.grad u - Lap u / Re + grad p, checked by central differences of the exact
    solution in t and in space at a few points."""
    re, t, d = 10.0, 0.7, 1e-4
    rng = np.random.default_rng(1)
    pi = np.pi
    S, C = np.sin, np.cos

    def U(x, y, t):
        return S(t) * S(pi * x) ** 2 * S(2 * pi * y)

    def V(x, y, t):
        return -S(t) * S(2 * pi * x) * S(pi * y) ** 2

    def Pr(x, y, t):
        return S(t) * (S(pi * y) - 2 / pi)

    def lap(F, x, y):
        return (F(x + d, y, t) + F(x - d, y, t) + F(x, y + d, t) + F(x, y - d, t) - 4 * F(x, y, t)) / d ** 2

    def dx(F, x, y):
        return (F(x + d, y, t) - F(x - d, y, t)) / (2 * d)

    def dy(F, x, y):
        return (F(x, y + d, t) - F(x, y - d, t)) / (2 * d)

    n = 16
    h = 1.0 / n
    (Fu, Fv) = ns.manufactured_fields(n, n, h, re)
    co = ns.manufactured_coef(t)
    fu = sum(c * f for c, f in zip(co, Fu))
    fv = sum(c * f for c, f in zip(co, Fv))
    (xu, yu), (xv, yv), _ = ns.grid_points(n, n, h)
    for _ in range(5):
        i, j = rng.integers(1, n - 2, 2)
        x, y = xu[j, i], yu[j, i]
        want = ((U(x, y, t + d) - U(x, y, t - d)) / (2 * d) + U(x, y, t) * dx(U, x, y) + V(x, y, t) * dy(U, x, y)
                - lap(U, x, y) / re + dx(Pr, x, y))
        assert abs(fu[j, i] - want) < 1e-4 * (1 + abs(want))
        x, y = xv[j, i], yv[j, i]
        want = ((V(x, y, t + d) - V(x, y, t - d)) / (2 * d) + U(x, y, t) * dx(V, x, y) + V(x, y, t) * dy(V, x, y)
                - lap(V, x, y) / re + dy(Pr, x, y))
        assert abs(fv[j, i] - want) < 1e-4 * (1 + abs(want))


def test_manufactured_velocity_is_divergence_free():
    n = 64
    u, v, _ = ns.exact(n, n, 1.0 / n, 0.8)
    assert np.abs(ns.divergence(u, v, 1.0 / n)).max() < 1e-10


def test_projection_leaves_a_divergence_free_velocity():
    """After a step, div u^{n+1} = -(pressure residual) / dt, so it vanishes with the
    pressure solve's residual."""
    n = 64
    h = 1.0 / n
    S = ns.Projection(n, n, h, 100.0, lid=1.0)
    for _ in range(3):
        (su, sv, sp) = S.step(0.01, tol=1e-11, kmax=40)
        assert su[0] == 0 and sv[0] == 0 and sp[0] == 0
    div = ns.divergence(S.u, S.v, h)
    assert h * np.sqrt(np.sum(div ** 2)) < 2e-11 / 0.01


def _golden():
    rows = [list(map(float, ln.split())) for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    return {r[0]: r[1:] for r in rows}


def test_first_order_scheme_reproduces_the_printed_errors():
    """Section 4.4.3: on 256^2 the errors at t = 1 of Scheme 1 with the forcing taken at
    t^{n+1} are within 4% of the values printed for 4096^2 (the gap is the spatial error of
    the coarser grid, which shrinks towards the printed values as the grid is refined)."""
    gold = _golden()
    for dt in (0.1, 0.05):
        errs, cycles = ns.convergence_run(256, dt)
        for got, want in zip(errs, gold[dt]):
            assert abs(got / want - 1.0) < 0.04, (dt, errs, gold[dt])
        assert max(max(c) for c in cycles) <= 8


def test_first_order_scheme_converges_at_first_order():
    gold = _golden()
    prev = None
    for dt in (0.1, 0.05, 0.025):
        errs, _ = ns.convergence_run(128, dt)
        if prev is not None:
            rates = np.log2(np.array(prev) / np.array(errs))
            printed = np.log2(np.array(gold[dt * 2]) / np.array(gold[dt]))
            assert np.all(rates > 0.9) and np.all(rates < 1.5), rates
            assert np.all(np.abs(rates - printed) < 0.15), (rates, printed)
        prev = errs
