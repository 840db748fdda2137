"""Solve-level comparison of the HIP library with the CPU oracle (imported by the GPU tests).

Iterates of the two are bit-identical cycle by cycle: every point formula is the same
evaluation tree on both sides.  Only the residual norms that decide when a solve stops
are reductions in different orders (the oracle sums sequentially, the library per tile
and then in a fixed tree), so the two may stop one cycle apart when a residual falls
within rounding of the tolerance.  Then the comparison is made at equal cycle counts:
the oracle runs exactly as many cycles as the library did and the iterates must be
bit-identical, and the residual of the crossing cycle must equal the tolerance to
rounding.  No case passes without comparing the iterate.
"""
import numpy as np

import oracle as O

# relative agreement of a residual norm computed in two summation orders: each of the two
# sums of N non-negative squares is within (N - 1) u of the exact sum (u = 2^-53), so the
# two norms agree to about N u; 1e-12 below 9000 cells
NORM_RTOL = 1e-12


def norm_rtol(ncells):
    return max(NORM_RTOL, float(ncells) * 2.0 ** -53)


def oracle_cycles(P, f, u0, cycles, nu1=2, nu2=2, transposed=False, kap=None):
    """u0 after exactly `cycles` oracle V-cycles (u0 is not modified)."""
    u = u0.copy()
    for _ in range(cycles):
        O.vcycle(P, f, u, nu1, nu2, transposed=transposed, kap=kap)
    return u


def check_solve(P, f, u0, got, gpu_cycles, tol, nu1=2, nu2=2, transposed=False, kap=None, kmax=100,
                gpu_hist=None, oracle_result=None):
    """Assert that a library solve of A u = f from u0 that ran `gpu_cycles` cycles and
    returned `got` is the oracle's solve (bit for bit at equal cycle counts).
    gpu_hist: the library's relative residual after each cycle (optional).
    oracle_result: (cycles, hist, u) of an oracle solve already run on the same input.
    Returns the oracle's cycle count."""
    if oracle_result is None:
        uo = u0.copy()
        st, cyc, hist = O.solve(P, f, uo, tol, nu1, nu2, kmax, transposed=transposed, kap=kap)
        assert st == 0, "oracle did not converge"
    else:
        cyc, hist, uo = oracle_result
    rtol = norm_rtol(np.asarray(f).size)
    assert abs(gpu_cycles - cyc) <= 1, (gpu_cycles, cyc)
    if gpu_cycles == cyc:
        assert np.array_equal(got, uo), "iterates differ at equal cycle counts"
    else:
        # one side stopped a cycle earlier: the residual after the earlier stop sits on
        # the tolerance up to the rounding of the two sums, and the iterates still agree
        # bit for bit at the library's cycle count
        k = min(gpu_cycles, cyc)
        assert abs(hist[k - 1] - tol) <= rtol * tol, (k, hist[k - 1], tol)
        ref = oracle_cycles(P, f, u0, gpu_cycles, nu1, nu2, transposed, kap)
        assert np.array_equal(got, ref), "iterates differ at the library's cycle count"
    if gpu_hist is not None:
        k = min(gpu_cycles, cyc, len(gpu_hist))
        np.testing.assert_allclose(np.asarray(gpu_hist[:k]), hist[:k], rtol=rtol, atol=0)
    return cyc


def check_mixed(P, f, u0, got, gpu_corrections, tol, nu1=2, nu2=2, inner=2, kap=None, gpu_hist=None, inner_next=0):
    """The same comparison for the mixed-precision defect correction: its iterates are the
    oracle's bit for bit (FP64 residual and update, FP32 inner cycles, an unscaled cast),
    and only the outer stopping test is a reduction.  Returns the oracle's corrections."""
    rtol = norm_rtol(np.asarray(f).size)
    uo = u0.copy()
    st, outer, hist = O.solve_mixed(P, f, uo, tol, nu1, nu2, inner, kap=kap, inner_next=inner_next)
    assert st == 0, "oracle mixed solve did not converge"
    assert abs(gpu_corrections - outer) <= 1, (gpu_corrections, outer)
    if gpu_corrections == outer:
        assert np.array_equal(got, uo), "iterates differ at equal correction counts"
    else:
        k = min(gpu_corrections, outer)
        assert abs(hist[k] - tol) <= rtol * tol, (k, hist[k], tol)
        ref = u0.copy()
        O.solve_mixed(P, f, ref, 0.0, nu1, nu2, inner, kmax=gpu_corrections, kap=kap, inner_next=inner_next)
        assert np.array_equal(got, ref), "iterates differ at the library's correction count"
    if gpu_hist is not None:
        k = min(gpu_corrections, outer) + 1
        np.testing.assert_allclose(np.asarray(gpu_hist[:k]), hist[:k], rtol=rtol, atol=0)
    return outer
