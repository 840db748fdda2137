"""Adjoint of the multi-step heat solve (torch.autograd over the C ABI): gradients with
respect to u0 and a cell kappa against the CPU oracle's adjoint, against central finite
differences, and torch.autograd.gradcheck; checkpoint recomputation is bit-exact."""
import numpy as np
import pytest
import torch

import fas_inputs as I
import oracle as O

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _adjoint_case(n, seed=3):
    kap = I.kappa_field(n, seed)
    u0 = I.heat_2d_small(n, seed + 1)
    tgt = I.heat_2d_small(n, seed + 2)
    return kap, u0, tgt


def test_adjoint_matches_oracle_64():
    """64^2 instance of the differentiable workload: kappa = exp(0.5 g), 20 steps,
    dt = 1e-4, checkpoint every 4; gradients against the oracle's adjoint."""
    from paper_2510_11152_amd import heat_loss_and_grads
    n, T, dt = 64, 20, 1e-4
    kap, u0, tgt = _adjoint_case(n)
    P = O.Problem(n=(n, n), h=1 / n, dt=dt, bc="neumann", coarsest=4, nuc=2)
    lo, gu_o, gk_o = O.heat_adjoint(P, u0, kap, T, tgt, tol=1e-12)
    t = lambda a: torch.from_numpy(a).to(DEV)
    lg, gu, gk = heat_loss_and_grads(t(u0), t(kap), t(tgt), T, dt, ckpt=4, tol=1e-12)
    assert abs(lg - lo) <= 1e-9 * lo
    gu, gk = gu.cpu().numpy(), gk.cpu().numpy()
    assert np.abs(gu - gu_o).max() <= 1e-8 * np.abs(gu_o).max()
    assert np.abs(gk - gk_o).max() <= 1e-8 * np.abs(gk_o).max()


def test_adjoint_matches_finite_differences_64():
    """Directional derivatives along random directions against central differences:
    the loss is quadratic in u0 (exact FD), and smooth in kappa (FD step 1e-5)."""
    from paper_2510_11152_amd import HeatSolveFn, Grid
    n, T, dt, tol = 64, 20, 1e-4, 1e-13
    kap, u0, tgt = _adjoint_case(n)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    g = Grid((n, n), 1 / n, dtype=torch.float64, coarsest=4, variable_kappa=True)

    def loss(u, k):
        uT = HeatSolveFn.apply(t(u), t(k), g, T, dt, 4, tol, 2, 2)
        return float(((uT - t(tgt)) ** 2).sum().item())

    a = t(u0).requires_grad_(True)
    k = t(kap).requires_grad_(True)
    uT = HeatSolveFn.apply(a, k, g, T, dt, 4, tol, 2, 2)
    ((uT - t(tgt)) ** 2).sum().backward()
    rng = np.random.default_rng(11)
    du = rng.standard_normal(u0.shape)
    dk = rng.standard_normal(kap.shape) * kap
    for eps_u in (1e-3,):
        fd = (loss(u0 + eps_u * du, kap) - loss(u0 - eps_u * du, kap)) / (2 * eps_u)
        an = float((a.grad.cpu().numpy() * du).sum())
        assert abs(fd - an) <= 1e-6 * abs(an)
    eps_k = 1e-4
    fd = (loss(u0, kap + eps_k * dk) - loss(u0, kap - eps_k * dk)) / (2 * eps_k)
    an = float((k.grad.cpu().numpy() * dk).sum())
    assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-30)


def test_gradcheck_small():
    from paper_2510_11152_amd import HeatSolveFn, Grid
    n = 8
    g = Grid((n, n), 1 / n, dtype=torch.float64, coarsest=2, variable_kappa=True).set(coarse_sweeps=20)
    gen = torch.Generator().manual_seed(0)
    u0 = torch.rand((n, n), generator=gen, dtype=torch.float64).to(DEV).requires_grad_(True)
    k = (0.5 + torch.rand((n, n), generator=gen, dtype=torch.float64)).to(DEV).requires_grad_(True)
    f = lambda u, kk: HeatSolveFn.apply(u, kk, g, 3, 0.02, 2, 1e-14, 2, 2)
    assert torch.autograd.gradcheck(f, (u0, k), eps=1e-6, atol=1e-7, rtol=1e-5)


def test_checkpoint_recompute_is_bitwise():
    from paper_2510_11152_amd import Grid, heat
    from paper_2510_11152_amd.autograd import recompute_segment
    n = 128
    kap, u0, _ = _adjoint_case(n)
    g = Grid((n, n), 1 / n, dtype=torch.float64, coarsest=4, variable_kappa=True)
    k = torch.from_numpy(kap).to(DEV)
    uT, states = heat(g, torch.from_numpy(u0).to(DEV), 8, 1e-4, kappa_cell=k, keep=True)
    seg = recompute_segment(g, states[4], 4, 1e-4, k, 1e-10, 2, 2)
    for a, b in zip(seg, states[4:]):
        assert torch.equal(a, b)
