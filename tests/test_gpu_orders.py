"""GPU parity of the smoother's set orders (Section 2.3: X, U and Z partitions, the
1234-1234 and 1234-4321 sequences; Appendix B's eight sets in 3D) against the CPU oracle.
Orders other than X run one launch per index-parity set; every update is the same point
formula as the oracle's, so sweeps, V-cycles and solves are bit-identical."""
import numpy as np
import pytest
import torch

import fas_inputs as I
import oracle as O
from parity_util import check_solve

pytestmark = pytest.mark.gpu

DEV = "cuda"
TD = {np.float64: torch.float64, np.float32: torch.float32}
ORDERS = [("u", False), ("z", False), ("x", True), ("u", True), ("z", True)]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def grid_for(P, dtype, variable=False):
    from paper_2510_11152_amd import Grid
    return Grid(P.n, P.h, bc=P.bc, dtype=TD[dtype], coarsest=P.coarsest, variable_kappa=variable).set(
        coarse_sweeps=P.nuc, order=P.order, symmetric=P.symmetric)


def _problem(n, bc, order, symmetric, coarsest=4, dt=0.37, kappa=1.3, nuc=2):
    return O.Problem(n=n, h=1.0 / n[0], dt=dt, kappa=kappa, bc=bc, coarsest=coarsest, nuc=nuc, order=order,
                     symmetric=symmetric)


@pytest.mark.parametrize("order,symmetric", ORDERS)
@pytest.mark.parametrize("n,coarsest,bc", [((64, 48), 6, "neumann"), ((96, 64), 4, "dirichlet"), ((32, 32), 4, "periodic"),
                                           ((24, 16, 8), 2, "neumann"), ((16, 16, 16), 4, "dirichlet"),
                                           ((24, 16, 16), 4, "periodic")])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("variable", [False, True])
def test_set_order_sweeps_bitwise(order, symmetric, n, coarsest, bc, dtype, variable):
    P = _problem(n, bc, order, symmetric, coarsest=coarsest)
    g = grid_for(P, dtype, variable)
    kap = np.exp(0.5 * I.random_field(P.shape(), 3)).astype(dtype) if variable else None
    f = I.random_field(P.shape(), 10).astype(dtype)
    u = I.random_field(P.shape(), 20).astype(dtype)
    for reverse in (False, True):
        uo = u.copy()
        O.smooth(P, 0, f, uo, 3, reverse=reverse, kap=kap)
        ug = dev(u)
        g.smooth(0, dev(f), ug, P.dt, P.kappa, None if kap is None else dev(kap), sweeps=3, reverse=reverse)
        assert np.array_equal(host(ug), uo), reverse
    if order != "x" or symmetric:
        # a different order changes the iterate (the orders are not all the same sweep)
        Px = _problem(n, bc, "x", False, coarsest=coarsest)
        ux = u.copy()
        O.smooth(Px, 0, f, ux, 3, kap=kap)
        assert not np.array_equal(ux, uo)


@pytest.mark.parametrize("order,symmetric", ORDERS)
@pytest.mark.parametrize("n,bc", [((128, 128), "neumann"), ((96, 64), "dirichlet"), ((64, 64), "periodic"),
                                  ((16, 16, 16), "neumann"), ((32, 16, 16), "dirichlet")])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("transposed", [False, True])
def test_set_order_vcycles_bitwise(order, symmetric, n, bc, dtype, transposed):
    P = _problem(n, bc, order, symmetric, dt=0.05, kappa=0.9, nuc=3)
    g = grid_for(P, dtype)
    f = I.random_field(P.shape(), 5).astype(dtype)
    u = I.random_field(P.shape(), 6).astype(dtype)
    ug, fg = dev(u), dev(f)
    for it in range(3):
        O.vcycle(P, f, u, 2, 2, transposed=transposed)
        g.vcycle(fg, ug, P.dt, P.kappa, nu1=2, nu2=2, transposed=transposed)
        assert np.array_equal(host(ug), u), it


@pytest.mark.parametrize("order,symmetric", [("x", False)] + ORDERS)
def test_set_order_solve_matches_oracle_paper_setting(order, symmetric):
    """The ordering study's setting (Section 2.3): p - Lap p = f with Dirichlet boundaries,
    coarsest 2^2, two sweeps, from a zero guess; the library's solve is the oracle's."""
    n = 128
    P = O.Problem(n=(n, n), h=1.0 / n, dt=1.0, kappa=1.0, bc="dirichlet", coarsest=2, nuc=2, order=order,
                  symmetric=symmetric)
    f = I.random_field(P.shape(), 31)
    u0 = np.zeros_like(f)
    g = grid_for(P, np.float64)
    ug = dev(u0)
    st = g.solve(dev(f), ug, P.dt, P.kappa, tol=1e-9)
    assert st == 0
    s = g.stats()
    check_solve(P, f, u0, host(ug), s["cycles"], 1e-9, gpu_hist=s["rel_res"])


def test_order_option_drops_fused_passes_and_restores_them():
    """Switching to U and back to X gives the fused two-colour result again (bit for bit)."""
    n = 256
    P = _problem((n, n), "neumann", "x", False, dt=1e-3, kappa=1.0)
    f = I.random_field(P.shape(), 7)
    g = grid_for(P, np.float64)
    ref = dev(f)
    g.vcycle(dev(f), ref, P.dt, P.kappa)
    g.set(order="u")
    uu = dev(f)
    g.vcycle(dev(f), uu, P.dt, P.kappa)
    g.set(order="x")
    ux = dev(f)
    g.vcycle(dev(f), ux, P.dt, P.kappa)
    assert torch.equal(ux, ref)
    assert not torch.equal(uu, ref)
    uo = f.copy()
    O.vcycle(P, f, uo, 2, 2)
    assert np.array_equal(host(ref), uo)
