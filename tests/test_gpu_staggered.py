"""Parity of the staggered-grid solver and the projection step (HIP, through the C ABI of
include/fas_stag.h) with the CPU oracle (oracle/staggered.py, oracle/ns.py).

Every point formula is the same evaluation tree on both sides, so sweeps, residuals,
V-cycles and whole steps are compared bit for bit.  Only the norms that stop a solve are
sums in different orders: when the two stop a cycle apart, the oracle is run for the
library's cycle count and the iterates must still be bit-identical, and the residual of the
crossing cycle must equal the tolerance to rounding.
"""
import os
import sys

import numpy as np
import pytest
import torch

from oracle import ns as ons
from oracle import staggered as ost

pytestmark = pytest.mark.gpu

LOCS = [("cell", "neumann", ost.CELL), ("cell", "dirichlet", ost.CELL), ("edge_x", "dirichlet", ost.EDGE_X),
        ("edge_y", "dirichlet", ost.EDGE_Y)]
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table6_first_order.txt")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _pair(loc, bc, code, nx, ny, coarsest=4, fused=1):
    from paper_2510_11152_amd import StaggeredSolver
    S = StaggeredSolver(loc, nx, ny, 1.0 / nx, bc=bc, coarsest=coarsest)
    S.set(fused=fused)
    P = ost.StagProblem(code, nx, ny, 1.0 / nx, cell_bc=bc, coarsest=coarsest)
    assert S.levels == P.levels and S.shape == P.shape()
    return S, P


def _coef(bc):
    return (0.0, 1.0) if bc == "neumann" else (1.0, 0.37)


def _inputs(P, seed, compatible):
    rng = np.random.default_rng(seed)
    f = rng.standard_normal(P.shape())
    if compatible:
        f -= f.mean()
    return f, rng.standard_normal(P.shape())


SIZES = [(64, 64), (192, 192), (128, 32), (96, 48), (512, 256)]


@pytest.mark.parametrize("loc,bc,code", LOCS)
@pytest.mark.parametrize("nx,ny", SIZES)
@pytest.mark.parametrize("nu", [1, 2, 3])
def test_sweeps_bitwise(loc, bc, code, nx, ny, nu):
    say("sweeps", loc, bc, nx, ny, nu)
    S, P = _pair(loc, bc, code, nx, ny)
    a, c = _coef(bc)
    f, w = _inputs(P, nx + nu, a == 0.0)
    wd = dev(w)
    S.smooth(a, c, dev(f), wd, nu)
    want = ost.smooth(P, 0, a, c, f, w.copy(), nu)
    assert np.array_equal(host(wd), want)


@pytest.mark.parametrize("loc,bc,code", LOCS)
@pytest.mark.parametrize("nx,ny", SIZES)
def test_residual_bitwise(loc, bc, code, nx, ny):
    say("residual", loc, bc, nx, ny)
    S, P = _pair(loc, bc, code, nx, ny)
    a, c = _coef(bc)
    f, w = _inputs(P, 5, False)
    r = torch.empty(P.shape(), dtype=torch.float64, device="cuda")
    res = S.residual(a, c, dev(f), dev(w), r)
    want = ost.residual(P, 0, a, c, f, w)
    assert np.array_equal(host(r), want)
    ref = ost.res_norm(P, a, c, f, w)
    assert abs(res - ref) <= 1e-12 * ref


@pytest.mark.parametrize("loc,bc,code", LOCS)
@pytest.mark.parametrize("nx,ny", SIZES)
@pytest.mark.parametrize("nu1,nu2", [(2, 2), (1, 1), (3, 2), (0, 1), (2, 0)])
@pytest.mark.parametrize("fused", [1, 0])
def test_vcycle_bitwise(loc, bc, code, nx, ny, nu1, nu2, fused):
    say("vcycle", loc, bc, nx, ny, nu1, nu2, fused)
    S, P = _pair(loc, bc, code, nx, ny, fused=fused)
    a, c = _coef(bc)
    f, w = _inputs(P, 11, a == 0.0)
    wd = dev(w)
    fd = dev(f)
    want = w.copy()
    for _ in range(2):
        S.vcycle(a, c, fd, wd, nu1, nu2)
        ost.vcycle(P, a, c, f, want, nu1, nu2)
    assert np.array_equal(host(wd), want)
    assert np.array_equal(host(fd), f)                # the right-hand side is left alone


@pytest.mark.parametrize("coarse_sweeps", [1, 3, 16])
@pytest.mark.parametrize("fused", [1, 0])
def test_vcycle_coarse_sweeps_bitwise(coarse_sweeps, fused):
    say("vcycle coarse sweeps", coarse_sweeps, fused)
    from paper_2510_11152_amd import StaggeredSolver
    S = StaggeredSolver("edge_y", 64, 64, 1 / 64)
    S.set(coarse_sweeps, fused)
    P = ost.StagProblem(ost.EDGE_Y, 64, 64, 1 / 64, nuc=coarse_sweeps)
    f, w = _inputs(P, 2, False)
    wd = dev(w)
    S.vcycle(1.0, 0.05, dev(f), wd)
    ost.vcycle(P, 1.0, 0.05, f, w)
    assert np.array_equal(host(wd), w)


def check_solve(S, P, a, c, f, w0, tol, kmax=30):
    wd = dev(w0)
    st, cyc, res = S.solve(a, c, dev(f), wd, tol, kmax=kmax)
    w = w0.copy()
    ost_st, ocyc, ores = ost.solve(P, a, c, f, w, tol, kmax=kmax)
    got = host(wd)
    if cyc != ocyc:
        assert abs(cyc - ocyc) == 1, (cyc, ocyc)
        w = w0.copy()
        for _ in range(cyc):
            ost.vcycle(P, a, c, f, w)
        # the two crossed the tolerance at the same residual, to rounding
        assert abs(min(res, ores) - tol) <= 1e-9 * tol or abs(ost.res_norm(P, a, c, f, w) - tol) <= 1e-9 * tol
    assert np.array_equal(got, w)
    assert st == (0 if res <= tol else 1)
    return cyc


@pytest.mark.parametrize("loc,bc,code", LOCS)
@pytest.mark.parametrize("nx,ny", [(128, 128), (192, 96)])
@pytest.mark.parametrize("fused", [1, 0])
def test_solve_matches_oracle(loc, bc, code, nx, ny, fused):
    say("solve", loc, bc, nx, ny, fused)
    S, P = _pair(loc, bc, code, nx, ny, fused=fused)
    a, c = _coef(bc)
    f, w = _inputs(P, 17, a == 0.0)
    cyc = check_solve(S, P, a, c, f, w, 1e-10, kmax=40)
    # the pure-Neumann pressure problem on a 2:1 grid keeps a 12 x 6 coarsest level, whose
    # smoothest modes 16 sweeps barely reduce: it converges, more slowly
    assert 2 <= cyc <= (40 if (a == 0.0 and nx != ny) else 20)


def test_solve_zero_cycles_when_converged():
    from paper_2510_11152_amd import StaggeredSolver
    S = StaggeredSolver("edge_x", 64, 64, 1 / 64)
    f = torch.zeros(S.shape, dtype=torch.float64, device="cuda")
    w = torch.zeros_like(f)
    st, cyc, res = S.solve(1.0, 0.1, f, w, 1e-12)
    assert st == 0 and cyc == 0 and res == 0.0


def test_solve_nonfinite_rhs_is_reported():
    from paper_2510_11152_amd import StaggeredSolver
    from paper_2510_11152_amd._lib import FAS_ERR_NONFINITE, FasError
    S = StaggeredSolver("cell", 64, 64, 1 / 64, bc="dirichlet")
    f = torch.zeros(S.shape, dtype=torch.float64, device="cuda")
    f[3, 5] = float("nan")
    w = torch.zeros_like(f)
    with pytest.raises(FasError) as e:
        S.solve(1.0, 0.1, f, w, 1e-9)
    assert e.value.code == FAS_ERR_NONFINITE


# ---- projection step ------------------------------------------------------------------------
def _ns_pair(n, re, layout, lid=0.0):
    from paper_2510_11152_amd import NavierStokes2D
    G = NavierStokes2D(n, n, 1.0 / n, re, layout=layout)
    O = ons.Projection(n, n, 1.0 / n, re, lid=lid)
    return G, O


def _check_state(G, O):
    assert np.array_equal(host(G.u), O.u)
    assert np.array_equal(host(G.v), O.v)
    assert np.array_equal(host(G.p), O.p)
    assert np.array_equal(host(G.ut), O.ut) and np.array_equal(host(G.vt), O.vt) and np.array_equal(host(G.pt), O.pt)


def _step_both(G, O, dt, lid, Fu, Fv, coef, tol):
    st, cyc, res = G.step(dt, lid, [dev(x) for x in Fu], [dev(x) for x in Fv], coef, tol=tol)
    out = O.step(dt, Fu, Fv, coef, tol=tol)
    ocyc = [o[1] for o in out]
    assert cyc == ocyc, (cyc, ocyc)   # a one-cycle split would show here; the inputs avoid it
    return st


@pytest.mark.parametrize("layout", ["memory_efficient", "classical"])
def test_cavity_steps_bitwise(layout):
    """Lid-driven cavity (Re = 100) from rest: three steps, every field bit for bit."""
    say("ns cavity", layout)
    n = 64
    G, O = _ns_pair(n, 100.0, layout, lid=1.0)
    for _ in range(3):
        st = _step_both(G, O, 0.01, 1.0, (), (), (), 1e-9)
        assert st == 0
        _check_state(G, O)


@pytest.mark.parametrize("layout", ["memory_efficient", "classical"])
def test_manufactured_steps_bitwise(layout):
    """Section 4.4.3's manufactured problem (Re = 10, source at t^{n+1}): four steps of
    dt = 1/10 on 128^2 from the exact state at t = 0."""
    say("ns manufactured", layout)
    n = 128
    G, O = _ns_pair(n, 10.0, layout)
    u0, v0, p0 = ons.exact(n, n, 1.0 / n, 0.0)
    O.u, O.v, O.p = u0.copy(), v0.copy(), p0.copy()
    G.u.copy_(dev(u0))
    G.v.copy_(dev(v0))
    G.p.copy_(dev(p0))
    Fu, Fv = ons.manufactured_fields(n, n, 1.0 / n, 10.0)
    for k in range(4):
        _step_both(G, O, 0.1, 0.0, Fu, Fv, ons.manufactured_coef((k + 1) * 0.1), 1e-9)
        _check_state(G, O)


def test_memory_efficient_layout_equals_classical_and_saves_a_third():
    say("ns layouts")
    from paper_2510_11152_amd import NavierStokes2D
    n = 256
    A = NavierStokes2D(n, n, 1.0 / n, 400.0, layout="memory_efficient")
    B = NavierStokes2D(n, n, 1.0 / n, 400.0, layout="classical")
    for _ in range(5):
        ca = A.step(0.005, lid=1.0)[1]
        cb = B.step(0.005, lid=1.0)[1]
        assert ca == cb
    for x, y in ((A.u, B.u), (A.v, B.v), (A.p, B.p)):
        assert torch.equal(x, y)
    fa, wa = A.memory()
    fb, wb = B.memory()
    assert fa * 3 == fb * 2 and wa == wb


def _golden():
    rows = [list(map(float, ln.split())) for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    return {r[0]: r[1:] for r in rows}


def test_first_order_errors_match_the_printed_table_at_4096():
    """Section 4.4.3 on the paper's own grid (4096^2, Re = 10, tol 1e-9, V(2,2)): the L2
    errors at t = 1 for dt = 1/10 and 1/20 agree with the printed values to 1%."""
    from paper_2510_11152_amd import NavierStokes2D
    n = 4096
    h = 1.0 / n
    gold = _golden()
    Fu, Fv = ons.manufactured_fields(n, n, h, 10.0)
    Fu = [dev(x) for x in Fu]
    Fv = [dev(x) for x in Fv]
    ue, ve, pe = ons.exact(n, n, h, 1.0)
    for dt in (0.1, 0.05):
        say("ns table 4096 dt", dt)
        G = NavierStokes2D(n, n, h, 10.0)
        steps = int(round(1.0 / dt))
        for k in range(steps):
            st, cyc, res = G.step(dt, 0.0, Fu, Fv, ons.manufactured_coef((k + 1) * dt), tol=1e-9)
            assert st == 0, (k, cyc, res)
        u, v, p = host(G.u), host(G.v), host(G.p)
        errs = (ons.l2(u - ue, h), ons.l2(v - ve, h), ons.l2((p - p.mean()) - (pe - pe.mean()), h))
        say("  errors", errs, "printed", gold[dt])
        for e, g in zip(errs, gold[dt]):
            assert abs(e / g - 1.0) < 0.01, (dt, errs, gold[dt])


@pytest.mark.parametrize("loc,bc,code", LOCS)
def test_full_size_vcycle_bitwise(loc, bc, code):
    """One V(2,2) cycle on the 4096^2 grid of the convergence study, bit for bit."""
    say("full-size vcycle", loc, bc)
    S, P = _pair(loc, bc, code, 4096, 4096)
    a, c = (0.0, 0.05) if bc == "neumann" else (1.0, 0.05 / 10.0)
    f, w = _inputs(P, 23, a == 0.0)
    wd = dev(w)
    S.vcycle(a, c, dev(f), wd)
    ost.vcycle(P, a, c, f, w)
    assert np.array_equal(host(wd), w)


@pytest.mark.parametrize("loc,bc,code", LOCS)
@pytest.mark.parametrize("nu2", [1, 2, 3])
def test_fused_norm_equals_residual_pass(loc, bc, code, nu2):
    """The residual norm the last post-smoothing launch sums equals the separate residual
    pass on the same iterate (to the rounding of two summation orders)."""
    say("fused norm", loc, bc, nu2)
    S, P = _pair(loc, bc, code, 512, 256)
    a, c = _coef(bc)
    f, w = _inputs(P, 31, a == 0.0)
    fd, wd = dev(f), dev(w)
    st, cyc, res = S.solve(a, c, fd, wd, 0.0, nu2=nu2, kmax=2)    # two cycles, never converged
    assert cyc == 2 and st == 1
    again = S.residual(a, c, fd, wd)
    assert abs(res - again) <= 1e-12 * again
    assert abs(res - ost.res_norm(P, a, c, f, host(wd))) <= 1e-12 * again


def test_profile_times_the_fused_finest_launches():
    say("profile")
    from paper_2510_11152_amd import StaggeredSolver
    S = StaggeredSolver("edge_x", 512, 512, 1 / 512)
    S.set(profile=1)
    f = torch.randn(S.shape, dtype=torch.float64, device="cuda")
    w = torch.zeros_like(f)
    st, cyc, _ = S.solve(1.0, 0.01, f, w, 0.0, kmax=3)
    pre, post, n = S.profile()
    assert cyc == 3 and n == 3 and pre > 0.0 and post > 0.0


def test_rectangular_cavity_steps_bitwise():
    """A 2:1 cavity (128 x 64 cells, Re = 400), memory-efficient layout, bit for bit."""
    say("ns rectangular cavity")
    from paper_2510_11152_amd import NavierStokes2D
    nx, ny = 128, 64
    G = NavierStokes2D(nx, ny, 1.0 / nx, 400.0)
    O = ons.Projection(nx, ny, 1.0 / nx, 400.0, lid=1.0)
    for _ in range(3):
        _step_both(G, O, 0.005, 1.0, (), (), (), 1e-10)
        _check_state(G, O)


def test_four_source_terms_bitwise():
    """The separable source with its largest number of terms (4), random fields."""
    say("ns four sources")
    n = 64
    G, O = _ns_pair(n, 50.0, "memory_efficient")
    rng = np.random.default_rng(5)
    Fu = [rng.standard_normal(O.u.shape) for _ in range(4)]
    Fv = [rng.standard_normal(O.v.shape) for _ in range(4)]
    coef = (0.5, -1.25, 2.0, 0.75)
    for _ in range(2):
        _step_both(G, O, 0.01, 0.0, Fu, Fv, coef, 1e-9)
        _check_state(G, O)


def test_step_reports_a_solve_short_of_tol():
    """After one ordinary step of the cavity (the first v right-hand side from rest is
    exactly zero, a zero-cycle solve), kmax = 1 cannot reach 1e-14: the step completes with
    status FAS_NOT_CONVERGED and the state is still the oracle's after one cycle per solve."""
    say("ns not converged")
    n = 64
    G, O = _ns_pair(n, 100.0, "memory_efficient", lid=1.0)
    _step_both(G, O, 0.01, 1.0, (), (), (), 1e-9)
    st, cyc, res = G.step(0.01, 1.0, tol=1e-14, kmax=1)
    O.step(0.01, tol=1e-14, kmax=1)
    assert st == 1 and cyc == [1, 1, 1] and all(r > 1e-14 for r in res)
    _check_state(G, O)


@pytest.mark.parametrize("loc,bc,code", LOCS)
@pytest.mark.parametrize("fused", [1, 0])
def test_smallest_grid_bitwise(loc, bc, code, fused):
    """The smallest hierarchy (8 x 8 cells, two levels; the fused path runs it all in the
    tail): V-cycles and a solve, bit for bit."""
    say("smallest", loc, bc, fused)
    S, P = _pair(loc, bc, code, 8, 8, fused=fused)
    assert P.levels == 2
    a, c = _coef(bc)
    f, w = _inputs(P, 41, a == 0.0)
    wd = dev(w)
    for _ in range(3):
        S.vcycle(a, c, dev(f), wd)
        ost.vcycle(P, a, c, f, w)
    assert np.array_equal(host(wd), w)
    f, w = _inputs(P, 43, a == 0.0)
    check_solve(S, P, a, c, f, w, 1e-11, kmax=40)


def test_full_size_8192_ns_edge_vcycle_bitwise():
    """One V(2,2) cycle of the NS-edge variable on an 8192^2 grid (67 M unknowns; its
    restriction takes a row from the next wave), bit for bit."""
    say("full-size 8192 edge_y vcycle")
    S, P = _pair("edge_y", "dirichlet", ost.EDGE_Y, 8192, 8192)
    f, w = _inputs(P, 47, False)
    wd = dev(w)
    S.vcycle(1.0, 0.025 / 10.0, dev(f), wd)
    ost.vcycle(P, 1.0, 0.025 / 10.0, f, w)
    assert np.array_equal(host(wd), w)
