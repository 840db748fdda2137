// Kernels of the staggered-grid FAS solver (Section 4.1, Appendices C-D) and of the
// first-order projection step (Section 4.2, Scheme 1).
//
// Point formulas (one fixed evaluation tree each; the library is built with
// -ffp-contract=off so every kernel rounds them identically):
//   s = (W + E) + (S + N)             neighbours, 0.0 for ghosts and wall points
//   k = 4 + (#odd ghosts) - (#even ghosts),   D = a h^2 + c k
//   sweep update   w = (c s + h^2 f) / D
//   operator       L w = (D w - c s) * (1 / h^2),    residual r = f - L w
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>

#include "fas_device.h"
#include "fas_internal.h"
#include "stag_internal.h"

namespace fas {
namespace stag {

namespace {

__device__ __forceinline__ double kshift(int kind) { return kind == K_CN ? -1.0 : (kind == K_CD ? 1.0 : 0.0); }

// k of the point (x, y) of level L.
__device__ __forceinline__ double kcount(const Lev& L, int x, int y)
{
    double k = 4.0;
    if (x == 0) k += kshift(L.kx);
    if (x == L.nx - 1) k += kshift(L.kx);
    if (y == 0) k += kshift(L.ky);
    if (y == L.ny - 1) k += kshift(L.ky);
    return k;
}

__device__ __forceinline__ double diag(const Lev& L, int x, int y) { return L.a * L.h2 + L.c * kcount(L, x, y); }

__device__ __forceinline__ double nbsum(const Lev& L, const double* u, int x, int y)
{
    const size_t i = (size_t)y * L.nx + x;
    const double W = x > 0 ? u[i - 1] : 0.0;
    const double E = x < L.nx - 1 ? u[i + 1] : 0.0;
    const double S = y > 0 ? u[i - L.nx] : 0.0;
    const double N = y < L.ny - 1 ? u[i + L.nx] : 0.0;
    return (W + E) + (S + N);
}

__device__ __forceinline__ double resid_at(const Lev& L, const double* f, const double* u, int x, int y)
{
    const size_t i = (size_t)y * L.nx + x;
    return f[i] - (diag(L, x, y) * u[i] - L.c * nbsum(L, u, x, y)) * L.ih2;
}

// ---- transfers ------------------------------------------------------------------------------
// Restriction (Appendix C for cells; Appendix D's six-point form for edges) of the iterate
// and of the residual (computed at the fine taps on the fly) at coarse point (K, J).
template <int LOC>
__device__ __forceinline__ void restrict_point(const Lev& Lf, const double* f, const double* u, int K, int J,
                                               double& ru, double& rr)
{
    if (LOC == LOC_CELL) {
        const int x = 2 * K, y = 2 * J;
        const size_t i = (size_t)y * Lf.nx + x;
        ru = ((u[i] + u[i + 1]) + (u[i + Lf.nx] + u[i + Lf.nx + 1])) * 0.25;
        rr = ((resid_at(Lf, f, u, x, y) + resid_at(Lf, f, u, x + 1, y)) +
              (resid_at(Lf, f, u, x, y + 1) + resid_at(Lf, f, u, x + 1, y + 1))) * 0.25;
    } else if (LOC == LOC_EDGE_X) {
        double gu[2], gr[2];
        for (int q = 0; q < 2; ++q) {
            const int y = 2 * J + q, x = 2 * K;
            const size_t i = (size_t)y * Lf.nx + x;
            gu[q] = (u[i] + 2.0 * u[i + 1]) + u[i + 2];
            gr[q] = (resid_at(Lf, f, u, x, y) + 2.0 * resid_at(Lf, f, u, x + 1, y)) + resid_at(Lf, f, u, x + 2, y);
        }
        ru = (gu[0] + gu[1]) * 0.125;
        rr = (gr[0] + gr[1]) * 0.125;
    } else {
        double gu[2], gr[2];
        for (int q = 0; q < 2; ++q) {
            const int x = 2 * K + q, y = 2 * J;
            const size_t i = (size_t)y * Lf.nx + x;
            gu[q] = (u[i] + 2.0 * u[i + Lf.nx]) + u[i + 2 * (size_t)Lf.nx];
            gr[q] = (resid_at(Lf, f, u, x, y) + 2.0 * resid_at(Lf, f, u, x, y + 1)) + resid_at(Lf, f, u, x, y + 2);
        }
        ru = (gu[0] + gu[1]) * 0.125;
        rr = (gr[0] + gr[1]) * 0.125;
    }
}

// Prolongation of the correction e = uc - uc0 (Appendix C: injection; Appendix D: linear
// along the cell-centred axis with odd ghosts first, then midpoint means along the edge axis
// with 0 at the wall points).  Coarse (stag_internal.h) gives e(K, J).
// Linear interpolation along a cell-centred axis from the coarse value of the cell and that
// of its neighbour on the side of the fine point (odd ghost beyond the last cell).
__device__ __forceinline__ double lin_cell(double e0, double enb) { return (3.0 * e0 + enb) * 0.25; }

// P e at fine point (x, y).
template <int LOC>
__device__ __forceinline__ double prolong_point(const Coarse& C, int x, int y)
{
    if (LOC == LOC_CELL) return C.e(x >> 1, y >> 1);
    if (LOC == LOC_EDGE_X) {
        const int J = y >> 1;
        auto col = [&](int K) {
            const double e0 = C.e(K, J);
            const double nb = (y & 1) ? (J < C.ncy - 1 ? C.e(K, J + 1) : -e0) : (J > 0 ? C.e(K, J - 1) : -e0);
            return lin_cell(e0, nb);
        };
        const int K = x >> 1;
        if (x & 1) return col(K);
        const double left = K >= 1 ? col(K - 1) : 0.0;
        const double right = K <= C.ncx - 1 ? col(K) : 0.0;
        return (left + right) * 0.5;
    }
    const int K = x >> 1;
    auto row = [&](int J) {
        const double e0 = C.e(K, J);
        const double nb = (x & 1) ? (K < C.ncx - 1 ? C.e(K + 1, J) : -e0) : (K > 0 ? C.e(K - 1, J) : -e0);
        return lin_cell(e0, nb);
    };
    const int J = y >> 1;
    if (y & 1) return row(J);
    const double below = J >= 1 ? row(J - 1) : 0.0;
    const double above = J <= C.ncy - 1 ? row(J) : 0.0;
    return (below + above) * 0.5;
}

template <int LOC>
__global__ __launch_bounds__(256) void k_restrict(Lev Lf, const double* __restrict__ f, const double* __restrict__ u,
                                                  int ncx, int ncy, double* __restrict__ uc,
                                                  double* __restrict__ uc0, double* __restrict__ rc)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)ncx * ncy) return;
    double ru, rr;
    restrict_point<LOC>(Lf, f, u, (int)(t % ncx), (int)(t / ncx), ru, rr);
    uc[t] = ru;
    uc0[t] = ru;
    rc[t] = rr;
}

__global__ __launch_bounds__(256) void k_form_rhs(Lev L, const double* __restrict__ r, const double* __restrict__ u,
                                                  double* __restrict__ f)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)L.nx * L.ny) return;
    const int x = (int)(t % L.nx), y = (int)(t / L.nx);
    f[t] = r[t] + (diag(L, x, y) * u[t] - L.c * nbsum(L, u, x, y)) * L.ih2;
}

__global__ __launch_bounds__(256) void k_coarse_rhs(Lev L, double* __restrict__ f, const double* __restrict__ u)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)L.nx * L.ny) return;
    const int x = (int)(t % L.nx), y = (int)(t / L.nx);
    f[t] = f[t] + (diag(L, x, y) * u[t] - L.c * nbsum(L, u, x, y)) * L.ih2;
}

template <int LOC>
__global__ __launch_bounds__(256) void k_correct(Lev Lf, Coarse C, const double* usrc, double* udst)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)Lf.nx * Lf.ny) return;
    udst[t] = usrc[t] + prolong_point<LOC>(C, (int)(t % Lf.nx), (int)(t / Lf.nx));
}

// Coarse corrections a lane's window columns need, loaded at once: e(K', J') for K' in
// {K} (cells), {K-1, K} (EW edges) or {K-1, K, K+1} (NS edges), K = x0 / 2, and the RPW/2 + 3
// coarse rows around the lane's rows.  pe<PAR, I, S>() evaluates prolong_point at
// (x0 + S, yw + I) from the table with the same operations (yw of parity PAR), so the result
// is the same bit for bit; entries outside the coarse grid are never used.
template <int LOC, int RPW>
struct CorrTable {
    static constexpr int NK = LOC == LOC_CELL ? 1 : (LOC == LOC_EDGE_X ? 2 : 3);
    static constexpr int NJ = RPW / 2 + 3;
    double E[NK][NJ];
    int K, Jb;
    __device__ __forceinline__ void load(const Coarse& C, int x0, int yw)
    {
        K = x0 >> 1;
        Jb = (yw >> 1) - 1;
        const int Kb = K - (LOC == LOC_CELL ? 0 : 1);
#pragma unroll
        for (int kk = 0; kk < NK; ++kk)
#pragma unroll
            for (int jj = 0; jj < NJ; ++jj) {
                const int Kq = Kb + kk, Jq = Jb + jj;
                E[kk][jj] = (Kq >= 0 && Kq < C.ncx && Jq >= 0 && Jq < C.ncy) ? C.e(Kq, Jq) : 0.0;
            }
    }
    template <int PAR, int I, int S>
    __device__ __forceinline__ double pe(const Coarse& C) const
    {
        constexpr int jj = ((PAR + I) >> 1) + 1;  // J - Jb
        constexpr bool yodd = ((PAR + I) & 1) != 0;
        const int J = Jb + jj;
        if constexpr (LOC == LOC_CELL) {
            return E[0][jj];
        } else if constexpr (LOC == LOC_EDGE_X) {
            auto col = [&](int kk) {
                const double e0 = E[kk][jj];
                const double nb = yodd ? (J < C.ncy - 1 ? E[kk][jj + 1] : -e0) : (J > 0 ? E[kk][jj - 1] : -e0);
                return lin_cell(e0, nb);
            };
            if constexpr (S == 1) {
                return col(1);
            } else {
                const double left = K >= 1 ? col(0) : 0.0;
                const double right = K <= C.ncx - 1 ? col(1) : 0.0;
                return (left + right) * 0.5;
            }
        } else {
            auto row = [&](int j) {
                const double e0 = E[1][j];
                const double nb = S == 1 ? (K < C.ncx - 1 ? E[2][j] : -e0) : (K > 0 ? E[0][j] : -e0);
                return lin_cell(e0, nb);
            };
            if constexpr (yodd) {
                return row(jj);
            } else {
                const double below = J >= 1 ? row(jj - 1) : 0.0;
                const double above = J <= C.ncy - 1 ? row(jj) : 0.0;
                return (below + above) * 0.5;
            }
        }
    }
};

template <int LOC, int RPW, int PAR, int I>
__device__ __forceinline__ void corr_row(const CorrTable<LOC, RPW>& T, const Coarse& C, int yw, int ny, bool in0,
                                         bool in1, double (&u0)[RPW], double (&u1)[RPW])
{
    const int gy = yw + I;
    if (gy < 0 || gy >= ny) return;
    if (in0) u0[I] = u0[I] + T.template pe<PAR, I, 0>(C);
    if (in1) u1[I] = u1[I] + T.template pe<PAR, I, 1>(C);
}

template <int LOC, int RPW, int PAR, int... I>
__device__ __forceinline__ void corr_rows(const CorrTable<LOC, RPW>& T, const Coarse& C, int yw, int ny, bool in0,
                                          bool in1, double (&u0)[RPW], double (&u1)[RPW],
                                          std::integer_sequence<int, I...>)
{
    (corr_row<LOC, RPW, PAR, I>(T, C, yw, ny, in0, in1, u0, u1), ...);
}

// ---- red-black sweeps on an LDS window ------------------------------------------------------
// A 512-thread block (8 waves) loads a 128-column window of the iterate into LDS: lane l of a
// wave owns the column pair (2l, 2l + 1) of the window and each wave WY/8 rows, whose
// right-hand side values stay in registers.  The block runs nu red-black sweeps on the window
// and writes its interior.  Half-sweep k updates values at distance >= k from the window's
// edge correctly, so after 2 nu half-sweeps the values at distance >= 2 nu are exactly what
// nu sweeps over the whole grid give.  Values outside the grid stay 0 in LDS (the 0.0
// neighbours of the point formula).  Within a half-sweep the updated points read only
// points of the other colour, so the update runs in place.  Window geometry (rows, margins of
// the written region): sweep_geom().  Windows are 32 rows: 54 to 105 VGPRs and 32 KiB of
// LDS, so two to four blocks share a compute unit (64-row windows, with half the halo share,
// measured slower in every variant).
//
// The window origin is even (the margins and the interior width are even along x), so in a
// row of one colour exactly one column of every pair is updated, the same one for the whole
// wave: every lane updates one point per row.  Even and odd columns sit in separate LDS
// arrays, which makes every LDS access of a wave 64 consecutive doubles.
//
// Variants (each a fixed set of point formulas of the per-level kernels, so the results are
// the same bit for bit):
//   CORR  the FAS correction is applied as the window is loaded (u = uin + P e, as k_correct);
//   NORM  one more ring of margin; each block writes the sum of the squared residuals of the
//         values it wrote to io.partials (one value per block), replacing a residual pass;
//   RHS   f holds the restricted residual r of the finer level: the FAS right-hand side
//         f = r + L u is formed from the loaded window before the sweeps (as k_coarse_rhs)
//         and written to io.fout;
//   RES   after the sweeps, the residual is formed in registers and the block restricts its
//         written region into the coarse level (as k_restrict): io.uc = io.uc0 = R u,
//         io.rc = R r.  Along an edge axis the third tap of a coarse point lies one column
//         (lane shuffle) or one row (exchanged through LDS across waves) past the region.
template <int NU, int LOC, bool CORR, bool NORM, bool RHS, bool RES>
__global__ __launch_bounds__(512) void k_sweep(Lev L, const double* __restrict__ f, const double* __restrict__ uin,
                                               double* __restrict__ uout, int tiles_x, SweepIO io)
{
    constexpr SweepGeom G = sweep_geom(NU, NORM, RES);
    constexpr int WY = G.wy, HX = G.hx, HY = G.hy, OX = G.ox, OY = G.oy, RPW = WY / 8;
    static_assert(HX % 2 == 0 && OY % 2 == 0 && RPW % 2 == 0, "window geometry");
    __shared__ double se[WY][kTile];  // even columns of the window
    __shared__ double so[WY][kTile];  // odd columns
    const unsigned b = xcd_block(blockIdx.x, gridDim.x);
    const int tx = (int)(b % (unsigned)tiles_x), ty = (int)(b / (unsigned)tiles_x);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int x0 = tx * OX - HX + 2 * lane;  // grid column of the lane's even column
    const int yw = ty * OY - HY + w * RPW;   // grid row of the wave's first row
    const bool in0 = x0 >= 0 && x0 < L.nx, in1 = x0 + 1 >= 0 && x0 + 1 < L.nx;
    double u0[RPW], u1[RPW], f0[RPW], f1[RPW];
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
        const int gy = yw + i;
        const bool row = gy >= 0 && gy < L.ny;
        const size_t idx = row ? (size_t)gy * L.nx + (size_t)(in0 ? x0 : 0) : 0;
        u0[i] = row && in0 ? uin[idx] : 0.0;
        f0[i] = row && in0 ? f[idx] : 0.0;
        u1[i] = row && in1 ? uin[(size_t)gy * L.nx + x0 + 1] : 0.0;
        f1[i] = row && in1 ? f[(size_t)gy * L.nx + x0 + 1] : 0.0;
    }
    if (CORR) {
        // the coarse values are loaded with the window, then P e is added row by row
        CorrTable<LOC, RPW> T;
        T.load(io.C, x0, yw);
        if (yw & 1)
            corr_rows<LOC, RPW, 1>(T, io.C, yw, L.ny, in0, in1, u0, u1, std::make_integer_sequence<int, RPW>{});
        else
            corr_rows<LOC, RPW, 0>(T, io.C, yw, L.ny, in0, in1, u0, u1, std::make_integer_sequence<int, RPW>{});
    }
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
        se[w * RPW + i][lane] = u0[i];
        so[w * RPW + i][lane] = u1[i];
    }
    // k along x of the two columns
    double kx0 = 4.0, kx1 = 4.0;
    if (x0 == 0) kx0 += kshift(L.kx);
    if (x0 == L.nx - 1) kx0 += kshift(L.kx);
    if (x0 + 1 == 0) kx1 += kshift(L.kx);
    if (x0 + 1 == L.nx - 1) kx1 += kshift(L.kx);
    auto kyof = [&](int gy) {
        double ky = 0.0;
        if (gy == 0) ky += kshift(L.ky);
        if (gy == L.ny - 1) ky += kshift(L.ky);
        return ky;
    };
    // L u at the even / odd point of window row r from the values in LDS
    auto Lu_even = [&](int r, double ky) {
        const double D = L.a * L.h2 + L.c * (kx0 + ky);
        const double s = (so[r][lane - 1] + so[r][lane]) + (se[r - 1][lane] + se[r + 1][lane]);
        return (D * se[r][lane] - L.c * s) * L.ih2;
    };
    auto Lu_odd = [&](int r, double ky) {
        const double D = L.a * L.h2 + L.c * (kx1 + ky);
        const double s = (se[r][lane] + se[r][lane + 1]) + (so[r - 1][lane] + so[r + 1][lane]);
        return (D * so[r][lane] - L.c * s) * L.ih2;
    };
    __syncthreads();
    if (RHS) {
        // f = r + L u from the values as loaded, at every point with its four neighbours in
        // the window (the sweeps update no other)
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int r = w * RPW + i, gy = yw + i;
            if (r < 1 || r > WY - 2 || gy < 0 || gy >= L.ny) continue;
            const double ky = kyof(gy);
            if (in0 && lane >= 1) f0[i] = f0[i] + Lu_even(r, ky);
            if (in1 && lane <= 62) f1[i] = f1[i] + Lu_odd(r, ky);
        }
        __syncthreads();
    }
#pragma unroll
    for (int hs = 0; hs < 2 * NU; ++hs) {
        const int colour = (hs & 1) ^ 1;  // sets 1-2 (odd index sum) first
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int r = w * RPW + i, gy = yw + i;
            if (r < 1 || r > WY - 2 || gy < 0 || gy >= L.ny) continue;
            const int odd = (colour + gy) & 1;  // the pair's column with this colour (wave-uniform)
            double k = odd ? kx1 : kx0;
            if (gy == 0) k += kshift(L.ky);
            if (gy == L.ny - 1) k += kshift(L.ky);
            const double D = L.a * L.h2 + L.c * k;
            if (odd) {
                if (lane == 63 || !in1) continue;
                const double s = (se[r][lane] + se[r][lane + 1]) + (so[r - 1][lane] + so[r + 1][lane]);
                so[r][lane] = (L.c * s + L.h2 * f1[i]) / D;
            } else {
                if (lane == 0 || !in0) continue;
                const double s = (so[r][lane - 1] + so[r][lane]) + (se[r - 1][lane] + se[r + 1][lane]);
                se[r][lane] = (L.c * s + L.h2 * f0[i]) / D;
            }
        }
        __syncthreads();
    }
    const bool colw = 2 * lane >= HX && 2 * lane < HX + OX;  // the lane's pair is written
    double acc = 0.0;
    if (colw) {
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int r = w * RPW + i, gy = yw + i;
            if (r < HY || r >= HY + OY || gy < 0 || gy >= L.ny) continue;
            if (in0) uout[(size_t)gy * L.nx + x0] = se[r][lane];
            if (in1) uout[(size_t)gy * L.nx + x0 + 1] = so[r][lane];
            if (RHS) {
                if (in0) io.fout[(size_t)gy * L.nx + x0] = f0[i];
                if (in1) io.fout[(size_t)gy * L.nx + x0 + 1] = f1[i];
            }
            if (NORM) {
                const double ky = kyof(gy);
                if (in0) {
                    const double rv = f0[i] - Lu_even(r, ky);
                    acc = acc + rv * rv;
                }
                if (in1) {
                    const double rv = f1[i] - Lu_odd(r, ky);
                    acc = acc + rv * rv;
                }
            }
        }
    }
    if (NORM) {
        // fixed-order reduction: butterfly within each wave, then the 8 wave sums in order
        for (int o = 32; o > 0; o >>= 1) acc = acc + __shfl_xor(acc, o, 64);
        __shared__ double red[8];
        if (lane == 0) red[w] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = red[0];
            for (int k = 1; k < 8; ++k) t = t + red[k];
            io.partials[blockIdx.x] = t;
        }
    }
    if (RES) {
        // residuals f - L u in place of f, wherever every neighbour is final (distance
        // >= 2 nu + 1 from the window edge; the written region and one ring around it)
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int r = w * RPW + i, gy = yw + i;
            if (r < 2 * NU + 1 || r > WY - 2 * NU - 2 || gy < 0 || gy >= L.ny) continue;
            const double ky = kyof(gy);
            if (in0 && 2 * lane >= 2 * NU + 1) f0[i] = f0[i] - Lu_even(r, ky);
            if (in1 && 2 * lane + 1 <= 2 * kTile - 2 * NU - 2) f1[i] = f1[i] - Lu_odd(r, ky);
        }
        // the third tap of an edge axis: the next lane's even column (EDGE_X), the next
        // wave's first row (EDGE_Y)
        double nx0[RPW];
        if (LOC == LOC_EDGE_X) {
#pragma unroll
            for (int i = 0; i < RPW; ++i) nx0[i] = __shfl_down(f0[i], 1, 64);
        }
        __shared__ double xre[LOC == LOC_EDGE_Y ? 8 : 1][kTile], xro[LOC == LOC_EDGE_Y ? 8 : 1][kTile];
        if (LOC == LOC_EDGE_Y) {
            xre[w][lane] = f0[0];
            xro[w][lane] = f1[0];
            __syncthreads();
        }
        if (colw) {
            const int K = x0 >> 1;  // x0 >= 0 here
#pragma unroll
            for (int p = 0; p < RPW / 2; ++p) {
                const int r = w * RPW + 2 * p, gy = yw + 2 * p;  // gy even
                if (r < HY || r >= HY + OY || gy < 0) continue;
                const int J = gy >> 1;
                if (J >= io.ncy || K >= io.ncx) continue;
                double ru, rr;
                if (LOC == LOC_CELL) {
                    ru = ((se[r][lane] + so[r][lane]) + (se[r + 1][lane] + so[r + 1][lane])) * 0.25;
                    rr = ((f0[2 * p] + f1[2 * p]) + (f0[2 * p + 1] + f1[2 * p + 1])) * 0.25;
                } else if (LOC == LOC_EDGE_X) {
                    const double gu0 = (se[r][lane] + 2.0 * so[r][lane]) + se[r][lane + 1];
                    const double gu1 = (se[r + 1][lane] + 2.0 * so[r + 1][lane]) + se[r + 1][lane + 1];
                    const double gr0 = (f0[2 * p] + 2.0 * f1[2 * p]) + nx0[2 * p];
                    const double gr1 = (f0[2 * p + 1] + 2.0 * f1[2 * p + 1]) + nx0[2 * p + 1];
                    ru = (gu0 + gu1) * 0.125;
                    rr = (gr0 + gr1) * 0.125;
                } else {
                    const double e2 = 2 * p + 2 < RPW ? f0[(2 * p + 2) % RPW] : xre[(w + 1) & 7][lane];
                    const double o2 = 2 * p + 2 < RPW ? f1[(2 * p + 2) % RPW] : xro[(w + 1) & 7][lane];
                    const double gu0 = (se[r][lane] + 2.0 * se[r + 1][lane]) + se[r + 2][lane];
                    const double gu1 = (so[r][lane] + 2.0 * so[r + 1][lane]) + so[r + 2][lane];
                    const double gr0 = (f0[2 * p] + 2.0 * f0[2 * p + 1]) + e2;
                    const double gr1 = (f1[2 * p] + 2.0 * f1[2 * p + 1]) + o2;
                    ru = (gu0 + gu1) * 0.125;
                    rr = (gr0 + gr1) * 0.125;
                }
                const size_t c = (size_t)J * io.ncx + K;
                io.uc[c] = ru;
                io.uc0[c] = ru;
                io.rc[c] = rr;
            }
        }
    }
}

// ---- persistent coarse tail ------------------------------------------------------------------
// One 1024-thread workgroup runs the V-cycle of the coarsest levels (top .. coarsest) with
// every array in LDS: the top level's iterate and right-hand side are loaded once and the
// iterate is written back at the end, instead of five launches per level.  Each step uses
// the point formulas of the per-level kernels, so the result is the same bit for bit.
// The workgroup as 32 x 32 threads: (tx, ty) walks columns and rows with stride 32, so no
// point index is divided by a row length.
__device__ __forceinline__ int ttx() { return threadIdx.x & 31; }
__device__ __forceinline__ int tty() { return threadIdx.x >> 5; }

__device__ void tail_smooth(const Lev& L, const double* f, double* u, int nu)
{
    for (int sw = 0; sw < nu; ++sw) {
        for (int colour = 1; colour >= 0; --colour) {  // sets 1-2 (odd index sum) first
            for (int y = tty(); y < L.ny; y += 32) {
                const int x0 = (colour + y) & 1;  // first column of this colour in row y
                for (int x = x0 + 2 * ttx(); x < L.nx; x += 64) {
                    const int t = y * L.nx + x;
                    u[t] = (L.c * nbsum(L, u, x, y) + L.h2 * f[t]) / diag(L, x, y);
                }
            }
            __syncthreads();
        }
    }
}

template <int LOC>
__global__ __launch_bounds__(1024) void k_tail(TailArgs A)
{
    __shared__ double lds[kTailDoubles];
    const int n0 = A.op[0].nx * A.op[0].ny;
    for (int t = threadIdx.x; t < n0; t += blockDim.x) {
        lds[A.ou[0] + t] = A.u[t];
        lds[A.of[0] + t] = A.r ? A.r[t] : A.f[t];
    }
    __syncthreads();
    if (A.r) {
        // f = r + L u from the loaded iterate (as k_coarse_rhs)
        const Lev& L = A.op[0];
        double* u = lds + A.ou[0];
        double* f = lds + A.of[0];
        // f at a point depends on r only at that point: formed in place
        for (int y = tty(); y < L.ny; y += 32)
            for (int x = ttx(); x < L.nx; x += 32) {
                const int t = y * L.nx + x;
                f[t] = f[t] + (diag(L, x, y) * u[t] - L.c * nbsum(L, u, x, y)) * L.ih2;
            }
        __syncthreads();
    }
    for (int l = 0; l + 1 < A.nlev; ++l) {
        const Lev& L = A.op[l];
        const Lev& Lc = A.op[l + 1];
        double* u = lds + A.ou[l];
        const double* f = lds + A.of[l];
        tail_smooth(L, f, u, A.nu1);
        double* uc = lds + A.ou[l + 1];
        double* uc0 = lds + A.ou0[l + 1];
        double* fc = lds + A.of[l + 1];
        for (int J = tty(); J < Lc.ny; J += 32)
            for (int K = ttx(); K < Lc.nx; K += 32) {
                double ru, rr;
                restrict_point<LOC>(L, f, u, K, J, ru, rr);
                const int t = J * Lc.nx + K;
                uc[t] = ru;
                uc0[t] = ru;
                fc[t] = rr;
            }
        __syncthreads();
        for (int y = tty(); y < Lc.ny; y += 32)
            for (int x = ttx(); x < Lc.nx; x += 32) {
                const int t = y * Lc.nx + x;
                fc[t] = fc[t] + (diag(Lc, x, y) * uc[t] - Lc.c * nbsum(Lc, uc, x, y)) * Lc.ih2;
            }
        __syncthreads();
    }
    const int lc = A.nlev - 1;
    tail_smooth(A.op[lc], lds + A.of[lc], lds + A.ou[lc], A.nuc);  // Remark 1
    for (int l = A.nlev - 2; l >= 0; --l) {
        const Lev& L = A.op[l];
        const Coarse C{lds + A.ou[l + 1], lds + A.ou0[l + 1], A.op[l + 1].nx, A.op[l + 1].ny};
        double* u = lds + A.ou[l];
        for (int y = tty(); y < L.ny; y += 32)
            for (int x = ttx(); x < L.nx; x += 32) {
                const int t = y * L.nx + x;
                u[t] = u[t] + prolong_point<LOC>(C, x, y);
            }
        __syncthreads();
        tail_smooth(L, lds + A.of[l], u, A.nu2);
    }
    for (int t = threadIdx.x; t < n0; t += blockDim.x) A.u[t] = lds[A.ou[0] + t];
}

// ---- residual norm -------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v, double* sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + o];
        __syncthreads();
    }
    return sh[0];
}

__global__ __launch_bounds__(256) void k_resnorm(Lev L, const double* __restrict__ f, const double* __restrict__ u,
                                                 double* __restrict__ r, double* __restrict__ partials)
{
    __shared__ double sh[256];
    const int64_t n = (int64_t)L.nx * L.ny;
    double acc = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)gridDim.x * 256) {
        const int x = (int)(t % L.nx), y = (int)(t / L.nx);
        const double rv = resid_at(L, f, u, x, y);
        if (r) r[t] = rv;
        acc = acc + rv * rv;
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_sum(const double* __restrict__ partials, int n, double* __restrict__ out)
{
    __shared__ double sh[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) acc = acc + partials[i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) out[0] = s;
}

__global__ __launch_bounds__(256) void k_copy(const double* __restrict__ src, double* __restrict__ dst, int64_t n)
{
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)gridDim.x * 256) dst[t] = src[t];
}

// ---- projection step ------------------------------------------------------------------------
constexpr double kWenoEps = 1e-6;

// Third-order WENO derivatives (Hamilton-Jacobi form, Jiang-Shu smoothness ratio) at the
// centre of five values along one axis: the left-biased phi^- and the right-biased phi^+.
__device__ __forceinline__ void weno_pair(double pm2, double pm1, double p0, double pp1, double pp2, double ih,
                                          double& minus, double& plus)
{
    const double d0 = pm1 - pm2, d1 = p0 - pm1, d2 = pp1 - p0;
    const double rm = (kWenoEps + (d1 - d0) * (d1 - d0)) / (kWenoEps + (d2 - d1) * (d2 - d1));
    const double wm = 1.0 / (1.0 + 2.0 * (rm * rm));
    minus = ((d1 + d2) - wm * ((d0 - 2.0 * d1) + d2)) * (0.5 * ih);
    const double e0 = pp2 - pp1, e1 = pp1 - p0, e2 = p0 - pm1;
    const double rp = (kWenoEps + (e1 - e0) * (e1 - e0)) / (kWenoEps + (e2 - e1) * (e2 - e1));
    const double wp = 1.0 / (1.0 + 2.0 * (rp * rp));
    plus = ((e1 + e2) - wp * ((e0 - 2.0 * e1) + e2)) * (0.5 * ih);
}

// Branch-free upwinding: max(a, 0) phi^- + min(a, 0) phi^+.
__device__ __forceinline__ double upwind(double a, double minus, double plus)
{
    return (a > 0.0 ? a : 0.0) * minus + (a < 0.0 ? a : 0.0) * plus;
}

__device__ __forceinline__ double forcing(const NsArgs& A, const double* const* F, size_t i)
{
    double s = 0.0;
    for (int k = 0; k < A.nforce; ++k) s = k == 0 ? A.coef[0] * F[0][i] : s + A.coef[k] * F[k][i];
    return s;
}

// u extended by two layers beyond each wall: wall points x = 0, 1 hold 0, their odd
// reflections beyond; along y cell-type ghosts 2 g - mirror (g = 0 below, lid above).
__device__ __forceinline__ double u_ext(const double* u, int m, int ny, int a, int b, double lid)
{
    if (b >= 0 && b < ny) {
        if (a >= 0 && a < m) return u[(size_t)b * m + a];
        if (a == -1 || a == m) return 0.0;
        if (a == -2) return 2.0 * 0.0 - u[(size_t)b * m];
        return 2.0 * 0.0 - u[(size_t)b * m + m - 1];  // a == m + 1
    }
    if (b == -1) return 2.0 * 0.0 - u[a];
    if (b == -2) return 2.0 * 0.0 - u[(size_t)m + a];
    if (b == ny) return 2.0 * lid - u[(size_t)(ny - 1) * m + a];
    return 2.0 * lid - u[(size_t)(ny - 2) * m + a];  // b == ny + 1
}

// v extended likewise: wall points y = 0, 1 hold 0 with odd reflections beyond; along x
// cell-type ghosts 2 * 0 - mirror.
__device__ __forceinline__ double v_ext(const double* v, int nx, int m, int ii, int jj)
{
    if (ii >= 0 && ii < nx) {
        if (jj >= 0 && jj < m) return v[(size_t)jj * nx + ii];
        if (jj == -1 || jj == m) return 0.0;
        if (jj == -2) return 2.0 * 0.0 - v[ii];
        return 2.0 * 0.0 - v[(size_t)(m - 1) * nx + ii];  // jj == m + 1
    }
    if (ii == -1) return 2.0 * 0.0 - v[(size_t)jj * nx];
    if (ii == -2) return 2.0 * 0.0 - v[(size_t)jj * nx + 1];
    if (ii == nx) return 2.0 * 0.0 - v[(size_t)jj * nx + nx - 1];
    return 2.0 * 0.0 - v[(size_t)jj * nx + nx - 2];  // ii == nx + 1
}

__global__ __launch_bounds__(256) void k_rhs_u(NsArgs A, const double* __restrict__ u, const double* __restrict__ v,
                                               const double* __restrict__ p, double* __restrict__ fu)
{
    const int m = A.nx - 1, ny = A.ny;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)m * ny) return;
    const int a = (int)(t % m), b = (int)(t / m);
    const double u0 = u[t];
    double xm, xp, ym, yp;
    weno_pair(u_ext(u, m, ny, a - 2, b, A.lid), u_ext(u, m, ny, a - 1, b, A.lid), u0,
              u_ext(u, m, ny, a + 1, b, A.lid), u_ext(u, m, ny, a + 2, b, A.lid), A.ih, xm, xp);
    weno_pair(u_ext(u, m, ny, a, b - 2, A.lid), u_ext(u, m, ny, a, b - 1, A.lid), u0,
              u_ext(u, m, ny, a, b + 1, A.lid), u_ext(u, m, ny, a, b + 2, A.lid), A.ih, ym, yp);
    // mean of the four v around the point (wall values 0 below the first, above the last row)
    const int nx = A.nx;
    const double sW = b > 0 ? v[(size_t)(b - 1) * nx + a] : 0.0;
    const double sE = b > 0 ? v[(size_t)(b - 1) * nx + a + 1] : 0.0;
    const double nW = b < ny - 1 ? v[(size_t)b * nx + a] : 0.0;
    const double nE = b < ny - 1 ? v[(size_t)b * nx + a + 1] : 0.0;
    const double vbar = ((sW + sE) + (nW + nE)) * 0.25;
    const double conv = upwind(u0, xm, xp) + upwind(vbar, ym, yp);
    const double gp = (p[(size_t)b * nx + a + 1] - p[(size_t)b * nx + a]) * A.ih;
    const double F = forcing(A, A.fu, (size_t)t);
    double r = u0 + A.dt * ((F - conv) - gp);
    if (b == ny - 1) r = r + A.lift;
    fu[t] = r;
}

__global__ __launch_bounds__(256) void k_rhs_v(NsArgs A, const double* __restrict__ u, const double* __restrict__ v,
                                               const double* __restrict__ p, double* __restrict__ fv)
{
    const int nx = A.nx, m = A.ny - 1;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)m * nx) return;
    const int ii = (int)(t % nx), jj = (int)(t / nx);
    const double v0 = v[t];
    double xm, xp, ym, yp;
    weno_pair(v_ext(v, nx, m, ii - 2, jj), v_ext(v, nx, m, ii - 1, jj), v0, v_ext(v, nx, m, ii + 1, jj),
              v_ext(v, nx, m, ii + 2, jj), A.ih, xm, xp);
    weno_pair(v_ext(v, nx, m, ii, jj - 2), v_ext(v, nx, m, ii, jj - 1), v0, v_ext(v, nx, m, ii, jj + 1),
              v_ext(v, nx, m, ii, jj + 2), A.ih, ym, yp);
    // mean of the four u around the point (wall values 0 left of the first, right of the
    // last column)
    const int mu = nx - 1;
    const double sW = ii > 0 ? u[(size_t)jj * mu + ii - 1] : 0.0;
    const double sE = ii < nx - 1 ? u[(size_t)jj * mu + ii] : 0.0;
    const double nW = ii > 0 ? u[(size_t)(jj + 1) * mu + ii - 1] : 0.0;
    const double nE = ii < nx - 1 ? u[(size_t)(jj + 1) * mu + ii] : 0.0;
    const double ubar = ((sW + sE) + (nW + nE)) * 0.25;
    const double conv = upwind(ubar, xm, xp) + upwind(v0, ym, yp);
    const double gp = (p[(size_t)(jj + 1) * nx + ii] - p[(size_t)jj * nx + ii]) * A.ih;
    const double F = forcing(A, A.fv, (size_t)t);
    fv[t] = v0 + A.dt * ((F - conv) - gp);
}

__global__ __launch_bounds__(256) void k_neg_div(NsArgs A, const double* __restrict__ ut, const double* __restrict__ vt,
                                                 double* __restrict__ fp)
{
    const int nx = A.nx, ny = A.ny;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nx * ny) return;
    const int i = (int)(t % nx), j = (int)(t / nx);
    const int mu = nx - 1;
    const double uW = i > 0 ? ut[(size_t)j * mu + i - 1] : 0.0;
    const double uE = i < nx - 1 ? ut[(size_t)j * mu + i] : 0.0;
    const double vS = j > 0 ? vt[(size_t)(j - 1) * nx + i] : 0.0;
    const double vN = j < ny - 1 ? vt[(size_t)j * nx + i] : 0.0;
    fp[t] = -(((uE - uW) + (vN - vS)) * A.ih);
}

__global__ __launch_bounds__(256) void k_project(NsArgs A, const double* __restrict__ ut, const double* __restrict__ vt,
                                                 const double* __restrict__ pt, const double* p_in,
                                                 double* __restrict__ u_out, double* __restrict__ v_out,
                                                 double* p_out)
{
    const int nx = A.nx, ny = A.ny;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nx * ny) return;
    const int i = (int)(t % nx), j = (int)(t / nx);
    const double pc = pt[t];
    if (i < nx - 1) {
        const size_t k = (size_t)j * (nx - 1) + i;
        u_out[k] = ut[k] - A.dt * ((pt[t + 1] - pc) * A.ih);
    }
    if (j < ny - 1) v_out[t] = vt[t] - A.dt * ((pt[t + nx] - pc) * A.ih);
    p_out[t] = p_in[t] + pc;
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

template <int NU, int LOC, bool CORR, bool NORM, bool RHS, bool RES>
void sweep_go(hipStream_t s, dim3 grid, const Lev& L, const double* f, const double* uin, double* uout, int tx,
              const SweepIO& io)
{
    hipLaunchKernelGGL((k_sweep<NU, LOC, CORR, NORM, RHS, RES>), grid, dim3(512), 0, s, L, f, uin, uout, tx, io);
}

template <int NU, int LOC>
void sweep_flags(hipStream_t s, dim3 grid, const Lev& L, const double* f, const double* uin, double* uout, int tx,
                 const SweepIO& io, unsigned flags)
{
    switch (flags) {
    case 0: sweep_go<NU, LOC_CELL, false, false, false, false>(s, grid, L, f, uin, uout, tx, io); break;
    case SW_CORR: sweep_go<NU, LOC, true, false, false, false>(s, grid, L, f, uin, uout, tx, io); break;
    case SW_CORR | SW_NORM: sweep_go<NU, LOC, true, true, false, false>(s, grid, L, f, uin, uout, tx, io); break;
    case SW_RHS: sweep_go<NU, LOC_CELL, false, false, true, false>(s, grid, L, f, uin, uout, tx, io); break;
    case SW_RES: sweep_go<NU, LOC, false, false, false, true>(s, grid, L, f, uin, uout, tx, io); break;
    case SW_RHS | SW_RES: sweep_go<NU, LOC, false, false, true, true>(s, grid, L, f, uin, uout, tx, io); break;
    default: throw Error(FAS_ERR_ARG, "internal: unsupported sweep variant");
    }
}

int sweep_blocks(const Lev& L, int nu, unsigned flags, int* tiles_x)
{
    const SweepGeom g = sweep_geom(nu, (flags & SW_NORM) != 0, (flags & SW_RES) != 0);
    const int tx = (L.nx + g.ox - 1) / g.ox, ty = (L.ny + g.oy - 1) / g.oy;
    if (tiles_x) *tiles_x = tx;
    return tx * ty;
}

int launch_sweep(hipStream_t s, int loc, const Lev& L, int nu, const double* f, const double* uin, double* uout,
                 const SweepIO& io, unsigned flags)
{
    int tx;
    const int nb = sweep_blocks(L, nu, flags, &tx);
    const dim3 grid(nb);
    if (loc == LOC_CELL) {
        if (nu == 1) sweep_flags<1, LOC_CELL>(s, grid, L, f, uin, uout, tx, io, flags);
        else sweep_flags<2, LOC_CELL>(s, grid, L, f, uin, uout, tx, io, flags);
    } else if (loc == LOC_EDGE_X) {
        if (nu == 1) sweep_flags<1, LOC_EDGE_X>(s, grid, L, f, uin, uout, tx, io, flags);
        else sweep_flags<2, LOC_EDGE_X>(s, grid, L, f, uin, uout, tx, io, flags);
    } else {
        if (nu == 1) sweep_flags<1, LOC_EDGE_Y>(s, grid, L, f, uin, uout, tx, io, flags);
        else sweep_flags<2, LOC_EDGE_Y>(s, grid, L, f, uin, uout, tx, io, flags);
    }
    return nb;
}

void launch_form_rhs(hipStream_t s, const Lev& L, const double* r, const double* u, double* f)
{
    hipLaunchKernelGGL(k_form_rhs, dim3(blocks_for((int64_t)L.nx * L.ny)), dim3(256), 0, s, L, r, u, f);
}

void launch_sum(hipStream_t s, const double* partials, int n, double* out)
{
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, partials, n, out);
}

void launch_tail(hipStream_t s, int loc, const TailArgs& A)
{
    if (loc == LOC_CELL)
        hipLaunchKernelGGL(k_tail<LOC_CELL>, dim3(1), dim3(1024), 0, s, A);
    else if (loc == LOC_EDGE_X)
        hipLaunchKernelGGL(k_tail<LOC_EDGE_X>, dim3(1), dim3(1024), 0, s, A);
    else
        hipLaunchKernelGGL(k_tail<LOC_EDGE_Y>, dim3(1), dim3(1024), 0, s, A);
}

void launch_restrict(hipStream_t s, int loc, const Lev& Lf, const double* f, const double* u, int ncx, int ncy,
                     double* uc, double* uc0, double* rc)
{
    const unsigned nb = blocks_for((int64_t)ncx * ncy);
    if (loc == LOC_CELL)
        hipLaunchKernelGGL(k_restrict<LOC_CELL>, dim3(nb), dim3(256), 0, s, Lf, f, u, ncx, ncy, uc, uc0, rc);
    else if (loc == LOC_EDGE_X)
        hipLaunchKernelGGL(k_restrict<LOC_EDGE_X>, dim3(nb), dim3(256), 0, s, Lf, f, u, ncx, ncy, uc, uc0, rc);
    else
        hipLaunchKernelGGL(k_restrict<LOC_EDGE_Y>, dim3(nb), dim3(256), 0, s, Lf, f, u, ncx, ncy, uc, uc0, rc);
}

void launch_coarse_rhs(hipStream_t s, const Lev& Lc, double* f, const double* u)
{
    hipLaunchKernelGGL(k_coarse_rhs, dim3(blocks_for((int64_t)Lc.nx * Lc.ny)), dim3(256), 0, s, Lc, f, u);
}

void launch_correct(hipStream_t s, int loc, const Lev& Lf, const double* uc, const double* uc0, int ncx, int ncy,
                    const double* usrc, double* udst)
{
    const Coarse C{uc, uc0, ncx, ncy};
    const unsigned nb = blocks_for((int64_t)Lf.nx * Lf.ny);
    if (loc == LOC_CELL)
        hipLaunchKernelGGL(k_correct<LOC_CELL>, dim3(nb), dim3(256), 0, s, Lf, C, usrc, udst);
    else if (loc == LOC_EDGE_X)
        hipLaunchKernelGGL(k_correct<LOC_EDGE_X>, dim3(nb), dim3(256), 0, s, Lf, C, usrc, udst);
    else
        hipLaunchKernelGGL(k_correct<LOC_EDGE_Y>, dim3(nb), dim3(256), 0, s, Lf, C, usrc, udst);
}

void launch_resnorm(hipStream_t s, const Lev& L, const double* f, const double* u, double* r, double* partials,
                    double* out)
{
    const int64_t n = (int64_t)L.nx * L.ny;
    const int nb = (int)std::min<int64_t>(kNormBlocks, (n + 255) / 256);
    hipLaunchKernelGGL(k_resnorm, dim3(nb), dim3(256), 0, s, L, f, u, r, partials);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, partials, nb, out);
}

void launch_copy(hipStream_t s, const double* src, double* dst, int64_t n)
{
    const unsigned nb = (unsigned)std::min<int64_t>(4096, (n + 255) / 256);
    hipLaunchKernelGGL(k_copy, dim3(nb), dim3(256), 0, s, src, dst, n);
}

void launch_rhs_u(hipStream_t s, const NsArgs& a, const double* u, const double* v, const double* p, double* fu)
{
    hipLaunchKernelGGL(k_rhs_u, dim3(blocks_for((int64_t)(a.nx - 1) * a.ny)), dim3(256), 0, s, a, u, v, p, fu);
}

void launch_rhs_v(hipStream_t s, const NsArgs& a, const double* u, const double* v, const double* p, double* fv)
{
    hipLaunchKernelGGL(k_rhs_v, dim3(blocks_for((int64_t)a.nx * (a.ny - 1))), dim3(256), 0, s, a, u, v, p, fv);
}

void launch_neg_div(hipStream_t s, const NsArgs& a, const double* ut, const double* vt, double* fp)
{
    hipLaunchKernelGGL(k_neg_div, dim3(blocks_for((int64_t)a.nx * a.ny)), dim3(256), 0, s, a, ut, vt, fp);
}

void launch_project(hipStream_t s, const NsArgs& a, const double* ut, const double* vt, const double* pt,
                    const double* p_in, double* u_out, double* v_out, double* p_out)
{
    hipLaunchKernelGGL(k_project, dim3(blocks_for((int64_t)a.nx * a.ny)), dim3(256), 0, s, a, ut, vt, pt, p_in, u_out,
                       v_out, p_out);
}

}  // namespace stag
}  // namespace fas
