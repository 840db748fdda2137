"""Batched solves: every member of a batch equals the single-problem solve of the same
precision and parameters (the same kernels, partial sums and stopping decisions: equal
cycle counts and bits) and the oracle's solve of that member; the grain-growth
right-hand side equals the oracle's, and a grain step matches the oracle's FP32 solves."""
import numpy as np
import pytest
import torch

import fas_inputs as I
import oracle as O
from oracle import grain as OG
from parity_util import check_solve

pytestmark = pytest.mark.gpu
DEV = "cuda"
TD = {np.float64: torch.float64, np.float32: torch.float32}


@pytest.mark.parametrize("n,bc,dtype,coarsest", [((256, 256), "neumann", np.float64, 4), ((128, 128), "periodic", np.float32, 4),
                                                 ((512, 256), "dirichlet", np.float64, 4), ((64, 64), "neumann", np.float32, 4),
                                                 ((16, 16, 16), "neumann", np.float64, 4)])
def test_batch_members_equal_single_solves(n, bc, dtype, coarsest):
    from paper_2510_11152_amd import Grid
    B, dt, tol = 5, 2e-3, 1e-10 if dtype == np.float64 else 1e-5
    P = O.Problem(n=n, h=1.0 / n[0], dt=dt, bc=bc, coarsest=coarsest)
    shape = P.shape()
    rhs = np.stack([I.random_field(shape, 100 + b) * (b + 1) for b in range(B)]).astype(dtype)
    u0 = np.stack([I.random_field(shape, 200 + b) for b in range(B)]).astype(dtype)
    # member 2 starts from its converged solution: it stops after one cycle and sits out
    gs = Grid(n, P.h, bc=bc, dtype=TD[dtype], coarsest=coarsest)
    pre = torch.from_numpy(u0[2].copy()).to(DEV)
    assert gs.solve(torch.from_numpy(rhs[2].copy()).to(DEV), pre, dt, tol=tol) == 0
    u0[2] = pre.cpu().numpy()
    gb = Grid(n, P.h, bc=bc, dtype=TD[dtype], coarsest=coarsest, batch=B)
    ub = torch.from_numpy(u0).to(DEV)
    st, cy = gb.solve_batched(torch.from_numpy(rhs).to(DEV), ub, dt, tol=tol)
    assert all(s == 0 for s in st), st
    assert cy[2] == 1 and max(cy) > 1, cy
    got = ub.cpu().numpy()
    for b in range(B):
        us = torch.from_numpy(u0[b].copy()).to(DEV)
        assert gs.solve(torch.from_numpy(rhs[b].copy()).to(DEV), us, dt, tol=tol) == 0
        c = gs.stats()["cycles"]
        assert c == cy[b], (b, c, cy[b])
        assert torch.equal(us, ub[b]), b
        check_solve(P, rhs[b], u0[b], got[b], cy[b], tol)


def test_grain_rhs_matches_oracle_bitwise():
    from paper_2510_11152_amd import grain_rhs
    eta = I.grain_init(q=37, n=64, seed=6)
    eta[:, :8, :8] = np.random.default_rng(1).uniform(-1, 1, (37, 8, 8)).astype(np.float32)
    f = grain_rhs(torch.from_numpy(eta).to(DEV), 0.1)
    torch.cuda.synchronize()
    assert np.array_equal(f.cpu().numpy(), OG.grain_rhs(eta, 0.1))


def test_grain_step_matches_oracle():
    """One step of the 2D grain-growth model (periodic, h = 1, dt = 0.1, kappa = 1,
    FP32) on 12 fields of 128^2: each field's solve against the oracle's FP32 solve."""
    from paper_2510_11152_amd import GrainGrowth
    q, n, dt = 12, 128, 0.1
    eta0 = I.grain_init(q=q, n=n, seed=6)
    eta0 += np.float32(0.3) * np.sin(np.arange(n, dtype=np.float32) / 7.0)[None, None, :] * (np.arange(q) % 3 == 0)[:, None, None]
    model = GrainGrowth(q, n, h=1.0, dt=dt, kappa=1.0, tol=1e-6)
    eta = torch.from_numpy(eta0).to(DEV)
    cy = model.step(eta)
    got = eta.cpu().numpy()
    f = OG.grain_rhs(eta0, dt)
    P = O.Problem(n=(n, n), h=1.0, dt=dt, kappa=1.0, bc="periodic", coarsest=4, nuc=2)
    for i in range(q):
        check_solve(P, f[i], eta0[i], got[i], cy[i], 1e-6)


def test_grain_full_size_sampled_fields_match_oracle():
    """The grain-growth workload at full size (1189 fields on 512^2, periodic, h = 1,
    dt = 0.1, FP32, tol 1e-6): one step in one batched launch sequence; four sampled
    fields (first, last and two between) against the oracle's right-hand side and its
    FP32 solves, bit for bit at equal cycle counts."""
    from paper_2510_11152_amd import GrainGrowth
    q, n, dt = 1189, 512, 0.1
    eta0 = I.grain_init(q=q, n=n, seed=6)
    model = GrainGrowth(q, n, h=1.0, dt=dt, kappa=1.0, tol=1e-6)
    eta = torch.from_numpy(eta0).to(DEV)
    cy = model.step(eta)
    f_gpu = model.rhs
    P = O.Problem(n=(n, n), h=1.0, dt=dt, kappa=1.0, bc="periodic", coarsest=4, nuc=2)
    f = OG.grain_rhs(eta0, dt)
    for i in (0, 417, 888, q - 1):
        assert np.array_equal(f_gpu[i].cpu().numpy(), f[i]), i
        check_solve(P, f[i], eta0[i], eta[i].cpu().numpy(), cy[i], 1e-6)
    del eta, model, f_gpu
    torch.cuda.empty_cache()


def test_uneven_batch_groups_equal_single_solves():
    """Problems of several sizes: one batched solve per size group, each member equal to
    its single solve."""
    from paper_2510_11152_amd import solve_uneven, Grid
    sizes = [64, 128, 64, 256, 128, 64]
    fields = [I.cosine_modes(m, 2, 16, np.random.default_rng(50 + b)) for b, m in enumerate(sizes)]
    us = [torch.from_numpy(f.copy()).to(DEV) for f in fields]
    rhs = [torch.from_numpy(f.copy()).to(DEV) for f in fields]
    st, cy = solve_uneven(rhs, us, dt=1e-4, tol=1e-10)
    assert all(s == 0 for s in st)
    for b, m in enumerate(sizes):
        g = Grid((m, m), 1.0 / m, coarsest=4)
        u = rhs[b].clone()
        assert g.solve(rhs[b], u, 1e-4, tol=1e-10) == 0
        assert g.stats()["cycles"] == cy[b], b
        assert torch.equal(u, us[b]), b
        P = O.Problem(n=(m, m), h=1.0 / m, dt=1e-4, bc="neumann", coarsest=4, nuc=2)
        check_solve(P, fields[b], fields[b], us[b].cpu().numpy(), cy[b], 1e-10)


def test_uneven_batch_reuse_with_graph_and_autotune():
    """A planned UnevenBatch solved twice (the second solve replays the captured cycles and
    the tuned segment heights) gives the one-shot solve's bits both times."""
    from paper_2510_11152_amd import UnevenBatch, solve_uneven
    sizes = [128, 64, 256, 128, 64]
    fields = [I.cosine_modes(m, 2, 16, np.random.default_rng(70 + b)) for b, m in enumerate(sizes)]
    rhs = [torch.from_numpy(f.copy()).to(DEV) for f in fields]
    ref = [r.clone() for r in rhs]
    st0, cy0 = solve_uneven(rhs, ref, dt=1e-4, tol=1e-10)
    ub = UnevenBatch([tuple(r.shape) for r in rhs], device=DEV, graph=True, autotune=True)
    for rep in range(2):
        us = [r.clone() for r in rhs]
        st, cy = ub.solve(rhs, us, 1e-4, tol=1e-10)
        assert st == st0 and all(s == 0 for s in st)
        assert cy == cy0, rep
        for b in range(len(sizes)):
            assert torch.equal(us[b], ref[b]), (rep, b)


def test_batched_graph_replay_equals_launches():
    from paper_2510_11152_amd import Grid
    B, n = 6, (256, 256)
    P = O.Problem(n=n, h=1 / 256, dt=1e-3, bc="neumann", coarsest=4)
    rhs = torch.from_numpy(np.stack([I.random_field(P.shape(), 300 + b) for b in range(B)])).to(DEV)
    ua, ub = rhs.clone(), rhs.clone()
    sa = Grid(n, P.h, batch=B).solve_batched(rhs, ua, P.dt, tol=1e-10)
    sb = Grid(n, P.h, batch=B).set(graph=True).solve_batched(rhs, ub, P.dt, tol=1e-10)
    assert sa == sb
    assert torch.equal(ua, ub)
    got, r = ua.cpu().numpy(), rhs.cpu().numpy()
    for b in range(B):
        check_solve(P, r[b], r[b], got[b], sa[1][b], 1e-10)


@pytest.mark.parametrize("graph", [False, True])
def test_batched_solve_after_a_longer_solve_is_unchanged(graph):
    """After a batched solve that took c cycles, the next one runs its first c - 2 cycles
    without a host check; problems that converge inside that window must stay as they
    are. A loose-tolerance batched solve after a tight one (and one from converged
    iterates) equals the same solve on a fresh grid: statuses, cycles and bits."""
    from paper_2510_11152_amd import Grid
    B, n = 4, (256, 128)
    P = O.Problem(n=n, h=1 / 256, dt=1e-3, bc="dirichlet", coarsest=4)
    rhs = torch.from_numpy(np.stack([I.random_field(P.shape(), 400 + b) * (b + 1) for b in range(B)])).to(DEV)
    g = Grid(n, P.h, bc="dirichlet", batch=B).set(graph=graph)
    u = rhs.clone()
    st, cy = g.solve_batched(rhs, u, P.dt, tol=1e-10)
    assert all(s == 0 for s in st) and max(cy) > 3
    for tol, u0 in ((1e-3, rhs), (1e-3, u.clone()), (1e-10, rhs)):
        ua, ub = u0.clone(), u0.clone()
        sa = g.solve_batched(rhs, ua, P.dt, tol=tol)
        sb = Grid(n, P.h, bc="dirichlet", batch=B).set(graph=graph).solve_batched(rhs, ub, P.dt, tol=tol)
        assert sa == sb, (tol, sa, sb)
        assert torch.equal(ua, ub), tol
