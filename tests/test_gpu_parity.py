"""GPU parity: the HIP library (through the C ABI) against the CPU oracle on the same
seeded inputs.  Integer-exact structure and identical per-point evaluation trees make
every iterate bit-identical; only reductions (norms) may differ in the last bits, so a
solve may stop one cycle away from the oracle's, and is then compared with the oracle
at its own cycle count (parity_util.check_solve)."""
import numpy as np
import pytest
import torch

import fas_inputs as I
import oracle as O
from parity_util import check_mixed, check_solve

pytestmark = pytest.mark.gpu

DEV = "cuda"
TD = {np.float64: torch.float64, np.float32: torch.float32}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def grid_for(P, dtype, variable=False, mixed=False):
    from paper_2510_11152_amd import Grid
    return Grid(P.n, P.h, bc=P.bc, dtype=TD[dtype], coarsest=P.coarsest, variable_kappa=variable,
                mixed_inner=mixed).set(coarse_sweeps=P.nuc)


# (n, coarsest): square, rectangular, several tiles with a ragged remainder, 3D
SHAPES = [((64, 64), 4), ((96, 64), 4), ((72, 48), 6), ((256, 256), 4), ((16, 16, 16), 4), ((32, 24, 16), 4)]
BCS = ["neumann", "dirichlet", "periodic"]


def _problem(n, coarsest, bc, dt=0.37, kappa=1.3, nuc=2):
    return O.Problem(n=n, h=1.0 / n[0], dt=dt, kappa=kappa, bc=bc, coarsest=coarsest, nuc=nuc)


def _kap_levels(P, kap, dtype, upto):
    ks = [kap.astype(dtype)]
    for l in range(upto):
        ks.append(O.restrict(P, l, ks[-1]))
    return ks


def _two_colourable(n, coarsest, bc):
    """Periodic grids need even sizes on every level (the library rejects the rest)."""
    if bc != "periodic":
        return True
    L = (min(n) // coarsest).bit_length() - 1
    return all((m >> L) % 2 == 0 for m in n)


SMOOTH_CASES = [(n, c, bc) for n, c in SHAPES for bc in BCS if _two_colourable(n, c, bc)]


@pytest.mark.parametrize("n,coarsest,bc", SMOOTH_CASES)
@pytest.mark.parametrize("variable", [False, True])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_smooth_residual_bitwise(n, coarsest, bc, variable, dtype):
    P = _problem(n, coarsest, bc)
    g = grid_for(P, dtype, variable)
    kap = np.exp(0.5 * I.random_field(P.shape(), 3)) if variable else None
    ks = _kap_levels(P, kap, dtype, 1) if variable else [None, None]
    for lev in (0, 1):
        f = I.random_field(P.shape(lev), 10 + lev).astype(dtype)
        u = I.random_field(P.shape(lev), 20 + lev).astype(dtype)
        for reverse in (False, True):
            uo = u.copy()
            O.smooth(P, lev, f, uo, 2, reverse=reverse, kap=ks[lev])
            ug = dev(u)
            g.smooth(lev, dev(f), ug, P.dt, P.kappa, None if ks[lev] is None else dev(ks[lev]), sweeps=2,
                     reverse=reverse)
            assert np.array_equal(host(ug), uo), (lev, reverse)
        ro = O.residual(P, lev, f, u, kap=ks[lev])
        rg = g.residual(lev, dev(f), dev(u), P.dt, P.kappa, None if ks[lev] is None else dev(ks[lev]))
        assert np.array_equal(host(rg), ro)


@pytest.mark.parametrize("n,coarsest", SHAPES)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_restrict_prolong_bitwise(n, coarsest, dtype):
    P = _problem(n, coarsest, "neumann")
    g = grid_for(P, dtype)
    x = I.random_field(P.shape(0), 1).astype(dtype)
    c_new = I.random_field(P.shape(1), 2).astype(dtype)
    c_old = I.random_field(P.shape(1), 3).astype(dtype)
    assert np.array_equal(host(g.restrict(0, dev(x))), O.restrict(P, 0, x))
    fo = x.copy()
    O.prolong_add(P, 0, c_new, c_old, fo)
    fg = dev(x)
    g.prolong_add(0, dev(c_new), dev(c_old), fg)
    assert np.array_equal(host(fg), fo)


VC_CASES = [((64, 64), 4, "neumann"), ((96, 64), 4, "dirichlet"), ((72, 48), 6, "neumann"), ((96, 64), 4, "periodic"),
            ((256, 256), 4, "neumann"), ((16, 16, 16), 4, "neumann"), ((32, 24, 16), 4, "dirichlet"),
            ((16, 16, 16), 2, "periodic")]


@pytest.mark.parametrize("n,coarsest,bc", VC_CASES)
@pytest.mark.parametrize("variable", [False, True])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("transposed", [False, True])
def test_vcycle_iterates_bitwise(n, coarsest, bc, variable, dtype, transposed):
    P = _problem(n, coarsest, bc, dt=0.05, kappa=0.9, nuc=3)
    g = grid_for(P, dtype, variable)
    kap = np.exp(0.5 * I.random_field(P.shape(), 4)).astype(dtype) if variable else None
    f = I.random_field(P.shape(), 5).astype(dtype)
    u = I.random_field(P.shape(), 6).astype(dtype)
    ug = dev(u)
    fg = dev(f)
    kg = None if kap is None else dev(kap)
    for it in range(3):
        O.vcycle(P, f, u, 2, 1, transposed=transposed, kap=kap)
        g.vcycle(fg, ug, P.dt, P.kappa, kg, nu1=2, nu2=1, transposed=transposed)
        assert np.array_equal(host(ug), u), it


# fused 2D passes: row marches only, block tiles on every fused level (16- and 8-wave tiles)
FUSED_PATHS = {"march": {"tile": 0}, "tile16": {"tile": 1 << 30, "tile_waves": 16},
               "tile8": {"tile": 1 << 30, "tile_waves": 8}}


@pytest.mark.parametrize("n,bc", [((1024, 512), "neumann"), ((512, 1024), "dirichlet"), ((1024, 512), "periodic"),
                                  ((4096, 128), "neumann"), ((4096, 128), "dirichlet"), ((4096, 128), "periodic")])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("nu", [(2, 2), (1, 3), (3, 0)])
@pytest.mark.parametrize("path", sorted(FUSED_PATHS))
def test_vcycle_many_tiles_bitwise(n, bc, dtype, nu, path):
    """Grids of many fused tiles (interior and boundary tiles, every nu variant, wide
    grids with a ragged last strip), through row marches or block tiles: V-cycles equal
    the oracle's bits, and equal the library's own one-phase-per-launch path."""
    P = _problem(n, 4, bc, dt=2e-4, kappa=1.0, nuc=2)
    g = grid_for(P, dtype).set(**FUSED_PATHS[path])
    f = I.random_field(P.shape(), 8).astype(dtype)
    u = I.random_field(P.shape(), 9).astype(dtype)
    ug, ub, fg = dev(u), dev(u), dev(f)
    gb = grid_for(P, dtype).set(fused=False)
    for it in range(2):
        O.vcycle(P, f, u, nu[0], nu[1])
        rel = g.vcycle(fg, ug, P.dt, nu1=nu[0], nu2=nu[1], with_residual=True)
        gb.vcycle(fg, ub, P.dt, nu1=nu[0], nu2=nu[1])
        assert np.array_equal(host(ug), u), it
        assert torch.equal(ug, ub)
        ro = np.linalg.norm(O.residual(P, 0, f, u).astype(np.float64)) / np.linalg.norm(f.astype(np.float64))
        assert abs(rel - ro) <= 1e-10 * ro


@pytest.mark.parametrize("n,bc", [((1024, 512), "neumann"), ((512, 1024), "dirichlet"), ((1024, 512), "periodic")])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("nu", [(2, 2), (1, 3), (3, 0)])
@pytest.mark.parametrize("transposed", [False, True])
@pytest.mark.parametrize("path", ["march", "tile8"])
def test_vcycle_many_tiles_cell_kappa_bitwise(n, bc, dtype, nu, transposed, path):
    """Cell kappa on grids of many tiles or march strips: face weights formed inside the
    pass (harmonic means, boundary faces) give the oracle's bits, plain and transposed."""
    P = _problem(n, 4, bc, dt=2e-4, kappa=1.0, nuc=2)
    g = grid_for(P, dtype, variable=True).set(**FUSED_PATHS[path])
    kap = np.exp(0.5 * I.random_field(P.shape(), 10)).astype(dtype)
    f = I.random_field(P.shape(), 11).astype(dtype)
    u = I.random_field(P.shape(), 12).astype(dtype)
    ug, fg, kg = dev(u), dev(f), dev(kap)
    for it in range(2):
        O.vcycle(P, f, u, nu[0], nu[1], transposed=transposed, kap=kap)
        g.vcycle(fg, ug, P.dt, P.kappa, kg, nu1=nu[0], nu2=nu[1], transposed=transposed)
        assert np.array_equal(host(ug), u), it


def test_heat_256_steps_match_oracle():
    """2D heat backward Euler, three steps, 256^2, h = 1/256, dt = 1e-3, Neumann, FP64,
    16 cosine modes, V(2,2) to 1e-10: same cycle counts, the same bits, the same residual
    history and ||f|| (which the first tile pass sums; later steps also run their first
    cycles without a host check)."""
    u0 = I.heat_2d_small()
    P = O.Problem(n=(256, 256), h=1 / 256, dt=1e-3, bc="neumann", coarsest=4, nuc=2)
    g = grid_for(P, np.float64)
    rhs = u0.copy()
    for step in range(3):
        ug = dev(rhs)
        assert g.solve(dev(rhs), ug, P.dt, tol=1e-10) == 0
        s = g.stats()
        got = host(ug)
        check_solve(P, rhs, rhs, got, s["cycles"], 1e-10, gpu_hist=s["rel_res"][: s["cycles"]])
        nf = float(np.sqrt(np.dot(rhs.ravel(), rhs.ravel())))
        assert abs(s["rhs_norm"] - nf) <= 1e-12 * nf, step
        rhs = got


@pytest.mark.parametrize("n,dtype", [((512, 512), np.float64), ((256, 128), np.float32), ((32, 32, 32), np.float64)])
@pytest.mark.parametrize("transposed", [False, True])
def test_solve_after_a_longer_solve_is_unchanged(n, dtype, transposed):
    """A solve enqueues the first cycles without a host check when the previous solve on
    the grid took more cycles; cycles enqueued after its convergence must do nothing. A
    loose-tolerance solve after a tight one (and a tight one after it, and a solve that
    converges at once) equals the same solve on a fresh grid: bits, cycles, residuals."""
    P = _problem(n, 4, "neumann", dt=1e-3, kappa=1.0, nuc=2)
    tight, loose = (1e-10, 1e-3) if dtype == np.float64 else (1e-5, 1e-2)
    f = dev(I.random_field(P.shape(), 81).astype(dtype))
    g = grid_for(P, dtype)
    u = f.clone()
    assert g.solve(f, u, P.dt, tol=tight, transposed=transposed) == 0
    long_cycles = g.stats()["cycles"]
    for tol, u0 in ((loose, f), (tight, f), (loose, u.clone())):
        ua, ub = u0.clone(), u0.clone()
        assert g.solve(f, ua, P.dt, tol=tol, transposed=transposed) == 0
        sa = g.stats()
        fresh = grid_for(P, dtype)
        assert fresh.solve(f, ub, P.dt, tol=tol, transposed=transposed) == 0
        sb = fresh.stats()
        assert sa["cycles"] == sb["cycles"], (tol, sa["cycles"], sb["cycles"])
        assert torch.equal(ua, ub), tol
        assert sa["rel_res"][: sa["cycles"]] == sb["rel_res"][: sb["cycles"]]
        assert sa["rhs_norm"] == sb["rhs_norm"]
    assert long_cycles > 3


@pytest.mark.parametrize("n,coarsest,bc", [((128, 128), 4, "neumann"), ((32, 32, 32), 4, "neumann"),
                                           ((128, 64), 4, "dirichlet"), ((512, 384), 6, "periodic"),
                                           ((1024, 512), 4, "neumann"), ((64, 64, 64), 4, "dirichlet"),
                                           ((32, 32), 4, "neumann"), ((96, 64, 32), 4, "periodic"),
                                           ((128, 64, 32), 4, "dirichlet")])
@pytest.mark.parametrize("variable", [False, True])
@pytest.mark.parametrize("inner", [1, 3])
def test_mixed_precision_matches_oracle(n, coarsest, bc, variable, inner):
    """FP32 inner cycles inside FP64 defect correction (tile passes that start from zero
    and add into the FP64 iterate, 3D plane marches and the 3D residual march of the outer
    step, a grid held entirely by the coarse tail): the corrections equal the oracle's mixed
    solve bit for bit at equal correction counts, with its residual history, and the result
    is within 1e-9 of the FP64 solution."""
    P = _problem(n, coarsest, bc, dt=1e-3, kappa=1.0)
    kap = np.exp(0.5 * I.random_field(P.shape(), 7)) if variable else None
    f = I.cosine_modes(max(n), len(n), 16, np.random.default_rng(1))[tuple(slice(0, m) for m in P.shape())]
    f = np.ascontiguousarray(f) + 0.01 * I.random_field(P.shape(), 8)
    g64 = grid_for(P, np.float64, variable)
    g32 = grid_for(P, np.float32, variable, mixed=True)
    from paper_2510_11152_amd import solve_mixed
    kg = None if kap is None else dev(kap)
    for rep in range(2):  # the second solve runs its first evaluations without a host check
        ug = dev(f)
        assert solve_mixed(g64, g32, dev(f), ug, P.dt, P.kappa, kg, tol=1e-10, inner=inner) == 0
        s = g64.stats()
        got = host(ug)
        check_mixed(P, f, f, got, s["cycles"], 1e-10, inner=inner, kap=kap, gpu_hist=s["rel_res"][: s["cycles"] + 1])
    ref = f.copy()
    O.solve(P, f, ref, 1e-13, kap=kap)
    assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max()


@pytest.mark.parametrize("n,coarsest,bc,inner,inner_next", [((128, 128), 4, "neumann", 4, 2), ((256, 128), 4, "dirichlet", 3, 1),
                                                           ((32, 32, 32), 4, "neumann", 4, 3)])
def test_mixed_inner_schedule_matches_oracle(n, coarsest, bc, inner, inner_next):
    """A smaller number of inner cycles after the first correction (FAS_OPT_MIXED_INNER_NEXT):
    bit for bit the oracle's defect correction with the same schedule."""
    P = _problem(n, coarsest, bc, dt=1e-3, kappa=1.0)
    f = I.cosine_modes(max(n), len(n), 16, np.random.default_rng(2))[tuple(slice(0, m) for m in P.shape())]
    f = np.ascontiguousarray(f) + 0.01 * I.random_field(P.shape(), 9)
    g64 = grid_for(P, np.float64, False)
    g32 = grid_for(P, np.float32, False, mixed=True)
    from paper_2510_11152_amd import solve_mixed
    for rep in range(2):
        ug = dev(f)
        assert solve_mixed(g64, g32, dev(f), ug, P.dt, P.kappa, None, tol=1e-10, inner=inner,
                           inner_next=inner_next) == 0
        s = g64.stats()
        check_mixed(P, f, f, host(ug), s["cycles"], 1e-10, inner=inner, gpu_hist=s["rel_res"][: s["cycles"] + 1],
                    inner_next=inner_next)


@pytest.mark.parametrize("n,bc", [((64, 64), "neumann"), ((32, 64), "dirichlet"), ((16, 16, 16), "periodic")])
def test_kappa_grad_bitwise(n, bc):
    P = _problem(n, 4, bc)
    g = grid_for(P, np.float64, True)
    kap = np.exp(0.5 * I.random_field(P.shape(), 1))
    mu = I.random_field(P.shape(), 2)
    u = I.random_field(P.shape(), 3)
    g0 = I.random_field(P.shape(), 4)
    go = g0.copy()
    O.kappa_grad(P, kap, mu, u, go)
    gg = dev(g0)
    g.kappa_grad(P.dt, dev(kap), dev(mu), dev(u), gg)
    assert np.array_equal(host(gg), go)


def test_solve_reports_not_converged_and_is_deterministic():
    P = _problem((128, 128), 4, "neumann", dt=1e-3, kappa=1.0)
    g = grid_for(P, np.float64)
    g.set(kmax=1)
    f = dev(I.heat_2d_small(128))
    u1 = f.clone()
    assert g.solve(f, u1, P.dt, tol=1e-12) == 1
    g.set(kmax=100)
    a, b = f.clone(), f.clone()
    g.solve(f, a, P.dt, tol=1e-12)
    g.solve(f, b, P.dt, tol=1e-12)
    assert torch.equal(a, b)


@pytest.mark.parametrize("n,bc", [((64, 64, 64), "neumann"), ((128, 64, 32), "dirichlet"), ((64, 64, 64), "periodic"),
                                  ((96, 64, 32), "neumann")])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("nu", [(2, 2), (1, 1), (2, 1), (1, 3), (3, 2), (4, 4)])
@pytest.mark.parametrize("sweeps", [2, 1])
def test_vcycle_3d_plane_march_bitwise(n, bc, dtype, nu, sweeps):
    """3D grids large enough for the plane-march kernels (tiles with interior and
    boundary tiles, ragged tiles, an odd number of passes, one or two sweeps per pass):
    V-cycles equal the oracle's bits and the library's own one-phase-per-launch path."""
    P = _problem(n, 4, bc, dt=2e-4, kappa=1.0, nuc=2)
    g = grid_for(P, dtype).set(march3_sweeps=sweeps)
    gb = grid_for(P, dtype).set(fused=False)
    f = I.random_field(P.shape(), 18).astype(dtype)
    u = I.random_field(P.shape(), 19).astype(dtype)
    ug, ub, fg = dev(u), dev(u), dev(f)
    for it in range(2):
        O.vcycle(P, f, u, nu[0], nu[1])
        rel = g.vcycle(fg, ug, P.dt, nu1=nu[0], nu2=nu[1], with_residual=True)
        gb.vcycle(fg, ub, P.dt, nu1=nu[0], nu2=nu[1])
        assert np.array_equal(host(ug), u), it
        assert torch.equal(ug, ub)
        ro = np.linalg.norm(O.residual(P, 0, f, u).astype(np.float64)) / np.linalg.norm(f.astype(np.float64))
        assert abs(rel - ro) <= 1e-10 * ro


@pytest.mark.parametrize("n,dtype", [((1024, 512), np.float64), ((64, 64, 64), np.float32), ((256, 256), np.float32),
                                     ((128, 64, 32), np.float64)])
def test_graph_and_autotune_give_the_same_bits(n, dtype):
    """A solve with the V-cycle captured in a HIP graph, and with autotuned march segment
    heights, gives the same iterate as the plain launches (128 x 64 x 32: a coarse plane-march
    level whose passes start in its second buffer, which the autotuner must not overwrite)."""
    P = _problem(n, 4, "neumann", dt=1e-3, kappa=1.0)
    f = dev(I.random_field(P.shape(), 31).astype(dtype))
    tol = 1e-9 if dtype == np.float64 else 1e-5
    ref = f.clone()
    g0 = grid_for(P, dtype)
    assert g0.solve(f, ref, P.dt, tol=tol) == 0
    c0 = g0.stats()["cycles"]
    check_solve(P, host(f), host(f), host(ref), c0, tol)
    for opts in ({"graph": True}, {"autotune": True}, {"graph": True, "autotune": True}):
        g = grid_for(P, dtype).set(**opts)
        for rep in range(2):  # second solve replays the cached graph
            u = f.clone()
            assert g.solve(f, u, P.dt, tol=tol) == 0
            # the same kernels and partial sums: the same stopping decisions and bits
            assert g.stats()["cycles"] == c0, (opts, rep)
            assert torch.equal(u, ref), (opts, rep)


@pytest.mark.parametrize("n", [(256, 256), (32, 32, 32)])
def test_graph_replay_follows_option_changes(n):
    """A captured cycle is dropped when an option that its launches depend on changes:
    after set(coarse_sweeps=...) (or a change of the tile shape) a graph-replayed solve
    equals a fresh grid's solve with the new options, bits and cycles."""
    P = _problem(n, 4, "neumann", dt=1.0, kappa=1.0)
    f = dev(I.random_field(P.shape(), 32))
    g = grid_for(P, np.float64).set(graph=True, kmax=6)
    u = f.clone()
    g.solve(f, u, P.dt, tol=1e-9)
    current = {"graph": True, "kmax": 6, "coarse_sweeps": P.nuc}
    for opts in ({"coarse_sweeps": 7}, {"coarse_sweeps": 1}, {"tile_waves": 16} if len(n) == 2 else {"fused": False}):
        g.set(**opts)
        current.update(opts)
        fresh = grid_for(P, np.float64).set(**current)
        ua, ub = f.clone(), f.clone()
        sa = g.solve(f, ua, P.dt, tol=1e-9)
        sb = fresh.solve(f, ub, P.dt, tol=1e-9)
        assert sa == sb and g.stats()["cycles"] == fresh.stats()["cycles"], opts
        assert torch.equal(ua, ub), opts
        # and both are the oracle's iterate after that many cycles
        Pn = _problem(n, 4, "neumann", dt=1.0, kappa=1.0, nuc=current["coarse_sweeps"])
        ref = host(f)
        for _ in range(g.stats()["cycles"]):
            O.vcycle(Pn, host(f), ref, 2, 2)
        assert np.array_equal(host(ua), ref), opts


@pytest.mark.parametrize("n,bc,dtype", [((1024, 512), "neumann", np.float64), ((1024, 512), "periodic", np.float32),
                                        ((512, 1024), "dirichlet", np.float64), ((64, 64, 64), "neumann", np.float64),
                                        ((96, 64, 32), "periodic", np.float32), ((4096, 128), "dirichlet", np.float64),
                                        ((4096, 128), "periodic", np.float32)])
@pytest.mark.parametrize("rows", [8, 30, 118, 256])
def test_forced_segment_heights_give_the_same_bits(n, bc, dtype, rows):
    """The march segmentation (rows or planes per segment, including heights that leave a
    ragged last segment) changes only the schedule: V-cycle iterates equal the oracle's."""
    P = _problem(n, 4, bc, dt=2e-4, kappa=1.0, nuc=2)
    g = grid_for(P, dtype).set(seg_rows=rows, tile=0)
    f = I.random_field(P.shape(), 41).astype(dtype)
    u = I.random_field(P.shape(), 42).astype(dtype)
    ug, fg = dev(u), dev(f)
    for it in range(2):
        O.vcycle(P, f, u, 2, 2)
        g.vcycle(fg, ug, P.dt, nu1=2, nu2=2)
        assert np.array_equal(host(ug), u), it


@pytest.mark.parametrize("n,coarsest,bc", [((128, 64), 4, "neumann"), ((352, 96), 6, "dirichlet"),
                                           ((352, 96), 6, "periodic"), ((1024, 1024), 4, "periodic"),
                                           ((2048, 256), 4, "neumann")])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("nu", [(3, 1), (2, 2)])
@pytest.mark.parametrize("waves", [6, 8, 12, 16])
@pytest.mark.parametrize("transposed", [False, True])
@pytest.mark.parametrize("variable", [False, True])
def test_tile_passes_bitwise(n, coarsest, bc, dtype, nu, waves, transposed, variable):
    """Block tiles on every fused level (a level one window wide and a row of tiles high,
    ragged last tiles across x and y, every boundary kind, both colour orders, constant
    and cell kappa; cell-kappa tiles take at most 8 waves): V-cycle iterates equal the
    oracle's bits, and the residual norm from the per-tile partial sums agrees with the
    oracle's to 1e-10."""
    P = _problem(n, coarsest, bc, dt=2e-4, kappa=1.0, nuc=2)
    g = grid_for(P, dtype, variable).set(tile=1 << 30, tile_waves=waves)
    f = I.random_field(P.shape(), 71).astype(dtype)
    u = I.random_field(P.shape(), 72).astype(dtype)
    kap = np.exp(0.5 * I.random_field(P.shape(), 73)).astype(dtype) if variable else None
    ug, fg = dev(u), dev(f)
    kg = None if kap is None else dev(kap)
    for it in range(2):
        O.vcycle(P, f, u, nu[0], nu[1], transposed=transposed, kap=kap)
        rel = g.vcycle(fg, ug, P.dt, P.kappa, kg, nu1=nu[0], nu2=nu[1], transposed=transposed, with_residual=True)
        assert np.array_equal(host(ug), u), it
        ro = np.linalg.norm(O.residual(P, 0, f, u, kap=kap).astype(np.float64)) / np.linalg.norm(f.astype(np.float64))
        assert abs(rel - ro) <= 1e-10 * ro


def test_tile_options_are_checked():
    from paper_2510_11152_amd import Grid
    from paper_2510_11152_amd._lib import FasError
    g = Grid((128, 128), 1 / 128)
    for bad in (4, 17, -8):
        with pytest.raises(FasError):
            g.set(tile_waves=bad)
    with pytest.raises(FasError):
        g.set(tile=-1)
    g.set(tile=0, tile_waves=0)


def test_march3_sweeps_option_is_checked():
    from paper_2510_11152_amd import Grid
    from paper_2510_11152_amd._lib import FasError
    g = Grid((64, 64, 64), 1 / 64)
    for bad in (0, 3, -1, 1.5):
        with pytest.raises(FasError):
            g.set(march3_sweeps=bad)
    g.set(march3_sweeps=1).set(march3_sweeps=2)


def test_segment_height_option_is_checked():
    from paper_2510_11152_amd import Grid
    from paper_2510_11152_amd._lib import FasError
    g = Grid((128, 128), 1 / 128)
    for bad in (6, 17, -2):
        with pytest.raises(FasError):
            g.set(seg_rows=bad)
    g.set(seg_rows=0)


# ---- full sizes, against the oracle --------------------------------------------------------
# One oracle V-cycle costs about 5 s at 8192^2 and 11 s at 512^3 on one host core, so the
# benchmark's own sizes are compared with the oracle directly, in the launch shapes the
# benchmark times (default options).

def _free(*ts):
    del ts
    torch.cuda.empty_cache()


@pytest.mark.parametrize("bc", ["neumann", "periodic"])
def test_full_size_8192_vcycle_matches_oracle(bc):
    """8192^2 FP64 (the 2D heat benchmark's grid, dt = 1e-4): one V(2,2) cycle through the
    default block tiles, and through the row marches, equals the oracle's cycle bit for
    bit on every cell; the cycle's residual norm (per-tile partial sums) agrees to 1e-12."""
    n = 8192
    P = _problem((n, n), 4, bc, dt=1e-4, kappa=1.0, nuc=2)
    f = I.heat_2d_large(n)
    uo = f.copy()
    O.vcycle(P, f, uo, 2, 2)
    fg = dev(f)
    for opts in ({}, {"tile": 0}):
        ug = fg.clone()
        rel = grid_for(P, np.float64).set(**opts).vcycle(fg, ug, P.dt, nu1=2, nu2=2, with_residual=True)
        assert np.array_equal(host(ug), uo), opts
        del ug
        torch.cuda.empty_cache()
    ro = np.linalg.norm(O.residual(P, 0, f, uo)) / np.linalg.norm(f)
    assert abs(rel - ro) <= 1e-12 * ro


def test_full_size_8192_heat_step_matches_oracle():
    """The first step of the 8192^2 heat benchmark (FP64, dt = 1e-4, Neumann, V(2,2) to
    1e-10 relative residual): the library's plain solve is the oracle's solve (bit for
    bit at equal cycle counts, residual history to 1e-12); the mixed-precision solve (3
    FP32 cycles per correction) is the oracle's mixed solve bit for bit and within 1e-9 of
    its FP64 solution (max-norm error relative to max|u|)."""
    from paper_2510_11152_amd import solve_mixed
    n = 8192
    P = _problem((n, n), 4, "neumann", dt=1e-4, kappa=1.0, nuc=2)
    f = I.heat_2d_large(n)
    uo = f.copy()
    st, cyc, hist = O.solve(P, f, uo, 1e-10)
    assert st == 0
    fg = dev(f)
    g = grid_for(P, np.float64)
    ug = fg.clone()
    assert g.solve(fg, ug, P.dt, tol=1e-10) == 0
    s = g.stats()
    check_solve(P, f, f, host(ug), s["cycles"], 1e-10, gpu_hist=s["rel_res"][: s["cycles"]],
                oracle_result=(cyc, hist, uo))
    del ug
    g32 = grid_for(P, np.float32, mixed=True)
    um = fg.clone()
    assert solve_mixed(g, g32, fg, um, P.dt, tol=1e-10, inner=3) == 0
    got = host(um)
    s = g.stats()
    check_mixed(P, f, f, got, s["cycles"], 1e-10, inner=3, gpu_hist=s["rel_res"][: s["cycles"] + 1])
    err = np.abs(got - uo).max() / np.abs(uo).max()
    print("8192^2 mixed vs FP64 oracle: max rel error %.3e, %d corrections" % (err, s["cycles"]))
    assert err <= 1e-9
    del um, fg, g, g32
    torch.cuda.empty_cache()


def test_full_size_512cube_vcycle_matches_oracle():
    """512^3 FP64 (the 3D heat benchmark, plane-march launch shapes): one V(2,2) cycle
    equals the oracle's cycle bit for bit on every cell."""
    n = 512
    P = _problem((n, n, n), 4, "neumann", dt=1e-4, kappa=1.0, nuc=2)
    f = I.heat_3d(n)
    uo = f.copy()
    O.vcycle(P, f, uo, 2, 2)
    fg = dev(f)
    ug = fg.clone()
    rel = grid_for(P, np.float64).vcycle(fg, ug, P.dt, nu1=2, nu2=2, with_residual=True)
    assert np.array_equal(host(ug), uo)
    ug.copy_(fg)  # the same cycle with one sweep per plane-march pass
    grid_for(P, np.float64).set(march3_sweeps=1).vcycle(fg, ug, P.dt, nu1=2, nu2=2)
    assert np.array_equal(host(ug), uo)
    del ug, fg
    torch.cuda.empty_cache()
    ro = np.linalg.norm(O.residual(P, 0, f, uo)) / np.linalg.norm(f)
    assert abs(rel - ro) <= 1e-12 * ro


def test_full_size_8192_residual_matches_oracle():
    """The residual at 8192^2 (FP64, Neumann) equals the oracle's cell by cell, and its
    2-norm agrees to 1e-12 (a reduction: the order of the sum differs)."""
    n = 8192
    P = _problem((n, n), 4, "neumann", dt=1e-4, kappa=1.0, nuc=2)
    f = I.heat_2d_large(n)
    u = I.random_field(P.shape(), 51)
    g = grid_for(P, np.float64)
    r, nrm = g.residual(0, dev(f), dev(u), P.dt, with_norm=True)
    ro = O.residual(P, 0, f, u)
    assert np.array_equal(host(r), ro)
    rn = float(np.sqrt(np.dot(ro.ravel(), ro.ravel())))
    assert abs(nrm - rn) <= 1e-12 * rn


@pytest.mark.parametrize("transposed", [False, True])
def test_full_size_2048_cell_kappa_vcycle_matches_oracle(transposed):
    """The differentiable workload's size (2048^2 FP64, kappa = exp(g/2) of a smooth
    cosine field, harmonic-mean faces): two plain or transposed V(2,2) cycles through the
    cell-kappa tiles (as timed) and through the marches equal the oracle's bit for bit;
    a transposed solve to 1e-10 is the oracle's transposed solve."""
    n = 2048
    P = _problem((n, n), 4, "neumann", dt=1e-4, kappa=1.0, nuc=2)
    kap = I.kappa_field(n)
    f = I.random_field(P.shape(), 61)
    uo = f.copy()
    for _ in range(2):
        O.vcycle(P, f, uo, 2, 2, transposed=transposed, kap=kap)
    fg, kg = dev(f), dev(kap)
    for opts in ({}, {"tile": 0}):
        ug = fg.clone()
        ga = grid_for(P, np.float64, variable=True).set(**opts)
        for _ in range(2):
            ga.vcycle(fg, ug, P.dt, 1.0, kg, nu1=2, nu2=2, transposed=transposed)
        assert np.array_equal(host(ug), uo), opts
    ug = fg.clone()
    ga = grid_for(P, np.float64, variable=True)
    assert ga.solve(fg, ug, P.dt, 1.0, kg, tol=1e-10, transposed=transposed) == 0
    s = ga.stats()
    check_solve(P, f, f, host(ug), s["cycles"], 1e-10, transposed=transposed, kap=kap,
                gpu_hist=s["rel_res"][: s["cycles"]])


@pytest.mark.parametrize("where", ["rhs", "u"])
@pytest.mark.parametrize("form", ["plain", "mixed", "stacked", "array", "stacked_mixed"])
def test_non_finite_input_is_reported(where, form):
    """A NaN in the right-hand side or the initial guess makes the residual norm NaN; the
    solve stops with FAS_ERR_NONFINITE (raised as FasError) instead of iterating to kmax."""
    from paper_2510_11152_amd import Grid, solve_mixed
    from paper_2510_11152_amd._lib import FAS_ERR_NONFINITE, FasError
    n = 128
    P = _problem((n, n), 4, "neumann", dt=1e-3, kappa=1.0)
    f = I.random_field(P.shape(), 90)
    u = f.copy()
    (f if where == "rhs" else u)[17, 33] = np.nan
    with pytest.raises(FasError) as e:
        if form == "plain":
            grid_for(P, np.float64).solve(dev(f), dev(u), P.dt, tol=1e-10)
        elif form == "mixed":
            solve_mixed(grid_for(P, np.float64), grid_for(P, np.float32, mixed=True), dev(f), dev(u), P.dt, tol=1e-10)
        elif form == "stacked_mixed":
            from paper_2510_11152_amd import solve_stacked_mixed
            g64, g32 = Grid((n, n), P.h, batch=3), Grid((n, n), P.h, dtype=torch.float32, batch=3, mixed_inner=True)
            F = dev(np.stack([I.random_field(P.shape(), 91), f, I.random_field(P.shape(), 92)]))
            U = dev(np.stack([I.random_field(P.shape(), 93), u, I.random_field(P.shape(), 94)]))
            solve_stacked_mixed(g64, g32, F, U, P.dt, tol=1e-10)
        elif form == "stacked":
            gb = Grid((n, n), P.h, batch=3)
            F = dev(np.stack([I.random_field(P.shape(), 91), f, I.random_field(P.shape(), 92)]))
            U = dev(np.stack([I.random_field(P.shape(), 93), u, I.random_field(P.shape(), 94)]))
            gb.solve_stacked(F, U, P.dt, tol=1e-10)
        else:
            from paper_2510_11152_amd import solve_batched
            gs = [Grid((n, n), P.h), Grid((2 * n, 2 * n), P.h / 2)]
            F = [dev(f), dev(I.random_field((2 * n, 2 * n), 95))]
            U = [dev(u), dev(I.random_field((2 * n, 2 * n), 96))]
            solve_batched(gs, F, U, P.dt, tol=1e-10)
    assert e.value.code == FAS_ERR_NONFINITE


@pytest.mark.parametrize("form", ["plain", "mixed", "stacked", "array"])
def test_absolute_tolerance_matches_oracle(form):
    """FAS_OPT_ATOL (Algorithm 1's absolute test): with the relative test off, a solve stops
    at the oracle's cycle, the first whose ||f - A u||_2 <= atol; a stacked or array-form
    member whose right-hand side is tiny stops after its first cycle."""
    from paper_2510_11152_amd import Grid, solve_batched, solve_mixed, solve_stacked_mixed
    n = 256
    P0 = _problem((n, n), 4, "periodic", dt=2e-3, kappa=1.0)
    f = I.random_field(P0.shape(), 120)
    u0 = np.zeros_like(f)
    st, cyc, hist = O.solve(P0, f, u0.copy(), 1e-12)
    nf = np.sqrt(np.sum(f * f))
    k = max(2, cyc // 2)
    atol = 0.5 * (hist[k - 2] + hist[k - 1]) * nf  # between cycle k-1's and cycle k's residual
    P = _problem((n, n), 4, "periodic", dt=2e-3, kappa=1.0)
    P.atol = atol
    if form == "plain":
        g = grid_for(P, np.float64).set(atol=atol)
        ug = dev(u0)
        assert g.solve(dev(f), ug, P.dt, tol=0.0) == 0
        check_solve(P, f, u0, host(ug), g.stats()["cycles"], 0.0)
        assert g.stats()["cycles"] == k
    elif form == "mixed":
        g64, g32 = grid_for(P, np.float64).set(atol=atol), grid_for(P, np.float32, mixed=True)
        ug = dev(u0)
        assert solve_mixed(g64, g32, dev(f), ug, P.dt, tol=0.0) == 0
        check_mixed(P, f, u0, host(ug), g64.stats()["cycles"], 0.0)
    else:
        tiny = f * 1e-30
        if form == "stacked":
            gb = Grid((n, n), P.h, bc="periodic", batch=2).set(atol=atol)
            U = dev(np.stack([u0, u0]))
            st, cy = gb.solve_stacked(dev(np.stack([f, tiny])), U, P.dt, tol=0.0)
        else:
            gs = [Grid((n, n), P.h, bc="periodic").set(atol=atol), Grid((n, n), P.h, bc="periodic").set(atol=atol)]
            U = [dev(u0), dev(u0)]
            st = solve_batched(gs, [dev(f), dev(tiny)], U, P.dt, tol=0.0)
            cy = [g.stats()["cycles"] for g in gs]
        assert st == [0, 0] and cy == [k, 1], (st, cy)
        uo = u0.copy()
        for _ in range(k):
            O.vcycle(P, f, uo, 2, 2)
        assert np.array_equal(host(U[0]), uo)
