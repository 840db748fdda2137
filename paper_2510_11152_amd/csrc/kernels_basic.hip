// Per-level kernels of the V-cycle, one thread per cell (or per coarse cell):
// colour-phase smoother, residual, fused residual + restriction, FAS coarse right-hand
// side, prolongation + correction, deterministic norms, kappa gradient and the
// mixed-precision helpers.  These serve every level and every configuration; the fused
// tile kernels replace them on large levels where they apply.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "fas_batch.h"
#include "fas_device.h"
#include "fas_fused.h"
#include "fas_internal.h"

namespace fas {

namespace {

constexpr int kBlock = 256;

// Batched grids: problem b = blockIdx.y; level arrays of consecutive problems are
// `fine` (this level) / `coarse` (next level) elements apart; inactive problems skip.
struct Batch {
    int64_t fine, coarse;
    const int* act;
};

__device__ __forceinline__ bool skip_problem(const Batch& bt) { return bt.act && !bt.act[blockIdx.y]; }

template <typename T>
Op<T> make_op(const fas_grid* g, int l, const Coef& c, const void* kap)
{
    Op<T> op;
    op.n0 = g->lev[l].n[0];
    op.n1 = g->lev[l].n[1];
    op.n2 = g->lev[l].n[2];
    op.bc = g->bc;
    op.k = (T)c.kd;
    for (int W = 0; W < 16; ++W) op.q[W] = (T)c.q[W];
    op.kap = (const T*)kap;
    return op;
}

inline unsigned blocks_for(int64_t work) { return (unsigned)((work + kBlock - 1) / kBlock); }

// Batch descriptor of level l (its own arrays and the next level's).
inline Batch batch_of(const fas_grid* g, int l)
{
    Batch b;
    b.fine = g->lev[l].N;
    b.coarse = l < g->L ? g->lev[l + 1].N : 0;
    b.act = active_flags(g);
    return b;
}

inline dim3 grid2(unsigned blocks, const fas_grid* g) { return dim3(blocks, (unsigned)g->batch, 1); }

inline void check_launch()
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error(FAS_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
}

// --------------------------------------------------------------------------- smoother
// One colour phase: every cell whose 0-based index sum has `parity`; one thread per
// pair of x-neighbours (exactly one of the two has the parity).
template <typename T, int DIM, bool KV>
__global__ __launch_bounds__(kBlock) void k_smooth_phase(Op<T> op, const T* __restrict__ f, T* u, int parity, Batch bt)
{
    if (skip_problem(bt)) return;
    f += blockIdx.y * bt.fine;
    u += blockIdx.y * bt.fine;
    const int half = (op.n0 + 1) >> 1;
    const int64_t total = (int64_t)half * op.n1 * op.n2;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= total) return;
    const int t = (int)(tid % half);
    const int64_t rest = tid / half;
    const int j = (int)(rest % op.n1);
    const int l = (int)(rest / op.n1);
    const int i = 2 * t + ((parity + j + l) & 1);
    if (i >= op.n0) return;
    Nbhd<T, DIM> s;
    gather<T, DIM, KV>(op, u, i, j, l, s);
    const int64_t p = cell_index(op.n0, op.n1, i, j, l);
    u[p] = gs_value<T, DIM, KV>(op, s, f[p]);
}

// One index-parity set (the multi-colour sets of Section 2.3 / Appendix B): the cells
// whose 0-based index along axis a is even exactly when bit a of `mask` is set (a 1-based
// odd index).  No two cells of a set are neighbours, so one thread per cell updates the
// set in any order.  Loads and stores are 2-strided in x: these sweeps serve the set
// orders that do not reduce to two colours (U, Z, symmetric), which are compared for
// convergence, not speed.
template <typename T, int DIM, bool KV>
__global__ __launch_bounds__(kBlock) void k_smooth_set(Op<T> op, const T* __restrict__ f, T* u, int mask, Batch bt)
{
    if (skip_problem(bt)) return;
    f += blockIdx.y * bt.fine;
    u += blockIdx.y * bt.fine;
    const int o0 = (mask & 1) ? 0 : 1, o1 = (mask & 2) ? 0 : 1, o2 = DIM == 3 && !(mask & 4) ? 1 : 0;
    const int m0 = (op.n0 - o0 + 1) >> 1, m1 = (op.n1 - o1 + 1) >> 1;
    const int m2 = DIM == 3 ? (op.n2 - o2 + 1) >> 1 : 1;
    const int64_t total = (int64_t)m0 * m1 * m2;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= total) return;
    const int i = 2 * (int)(tid % m0) + o0;
    const int64_t rest = tid / m0;
    const int j = 2 * (int)(rest % m1) + o1;
    const int l = 2 * (int)(rest / m1) + o2;
    Nbhd<T, DIM> s;
    gather<T, DIM, KV>(op, u, i, j, l, s);
    const int64_t p = cell_index(op.n0, op.n1, i, j, l);
    u[p] = gs_value<T, DIM, KV>(op, s, f[p]);
}

// --------------------------------------------------------------------------- residual
template <typename T, int DIM, bool KV>
__global__ __launch_bounds__(kBlock) void k_residual(Op<T> op, const T* __restrict__ f, const T* __restrict__ u,
                                                     T* __restrict__ r, Batch bt)
{
    if (skip_problem(bt)) return;
    f += blockIdx.y * bt.fine;
    u += blockIdx.y * bt.fine;
    r += blockIdx.y * bt.fine;
    const int64_t N = (int64_t)op.n0 * op.n1 * op.n2;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int i = (int)(p % op.n0);
    const int j = (int)((p / op.n0) % op.n1);
    const int l = (int)(p / ((int64_t)op.n0 * op.n1));
    Nbhd<T, DIM> s;
    gather<T, DIM, KV>(op, u, i, j, l, s);
    r[p] = f[p] - apply_value<T, DIM, KV>(op, s, u[p]);
}

// Fixed-order block reduction of per-thread double sums into out[idx].
__device__ void block_sum_at(double v, double* out, int idx)
{
    __shared__ double red[kBlock];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[idx] = red[0];
}

// Fixed-order block reduction of per-thread double sums into out[blockIdx.x].
__device__ void block_sum_store(double v, double* out)
{
    __shared__ double red[kBlock];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// Sum of r^2 (r = f - A u), or of f^2 when u == nullptr; grid-stride with a fixed grid.
template <typename T, int DIM, bool KV>
__global__ __launch_bounds__(kBlock) void k_resid_norm(Op<T> op, const T* __restrict__ f,
                                                       const T* __restrict__ u, double* __restrict__ partials, Batch bt)
{
    if (skip_problem(bt)) return;
    f += blockIdx.y * bt.fine;
    if (u) u += blockIdx.y * bt.fine;
    partials += (int64_t)blockIdx.y * gridDim.x;
    const int64_t N = (int64_t)op.n0 * op.n1 * op.n2;
    double acc = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
        T r;
        if (u) {
            const int i = (int)(p % op.n0);
            const int j = (int)((p / op.n0) % op.n1);
            const int l = (int)(p / ((int64_t)op.n0 * op.n1));
            Nbhd<T, DIM> s;
            gather<T, DIM, KV>(op, u, i, j, l, s);
            r = f[p] - apply_value<T, DIM, KV>(op, s, u[p]);
        } else {
            r = f[p];
        }
        acc += (double)r * (double)r;
    }
    block_sum_store(acc, partials);
}

// One block per problem: out[b] = fixed-order sum of partials[b*count .. b*count + count).
// 1024 threads, each summing a strided subsequence (loads unrolled so that several are in
// flight), then a fixed tree over the threads.
constexpr int kSumBlock = 1024;

// Fixed-order total of partials[0..count) by one block of kSumBlock threads: strided
// per-thread sums, then a binary tree in LDS.  Every thread returns the total.
__device__ __forceinline__ double sum_block(const double* __restrict__ partials, int count)
{
    double acc = 0.0;
#pragma unroll 4
    for (int b = threadIdx.x; b < count; b += kSumBlock) acc += partials[b];
    __shared__ double red[kSumBlock];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kSumBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + s];
        __syncthreads();
    }
    return red[0];
}

__global__ __launch_bounds__(kSumBlock) void k_sum_partials(const double* __restrict__ partials, int count,
                                                             double* __restrict__ out)
{
    const double t = sum_block(partials + (int64_t)blockIdx.x * count, count);
    if (threadIdx.x == 0) out[blockIdx.x] = t;
}

// One problem: the norm total of cycle k (as k_sum_partials) and its convergence update
// (as k_update_active) in one launch.
__global__ __launch_bounds__(kSumBlock) void k_sum_update(const double* __restrict__ partials, int count,
                                                           double* __restrict__ norm2, const double* __restrict__ rnorm2,
                                                           double tol2, double atol2, int k,
                                                           int* __restrict__ act, int* __restrict__ cyc,
                                                           int* __restrict__ alive, double* __restrict__ hist)
{
    const double nr = sum_block(partials, count);
    if (threadIdx.x != 0) return;
    norm2[0] = nr;
    if (act[0]) {
        if (k <= kHist) hist[k - 1] = nr;
        if (!isfinite(nr)) {
            act[0] = 0;
            cyc[0] = -k;
        } else if (nr <= tol2 * rnorm2[0] || nr <= atol2 || nr == 0.0) {
            act[0] = 0;
            cyc[0] = k;
        }
    }
    alive[0] = act[0];
}

// ----------------------------------------------------------- residual + restriction
// One thread per coarse cell: uc = R u, rc = R (f - A u) over the 2^d children.
template <typename T, int DIM, bool KV>
__global__ __launch_bounds__(kBlock) void k_resid_restrict(Op<T> op, const T* __restrict__ f,
                                                           const T* __restrict__ u, T* __restrict__ uc,
                                                           T* __restrict__ rc, Batch bt)
{
    if (skip_problem(bt)) return;
    f += blockIdx.y * bt.fine;
    u += blockIdx.y * bt.fine;
    uc += blockIdx.y * bt.coarse;
    rc += blockIdx.y * bt.coarse;
    const int m0 = op.n0 >> 1, m1 = op.n1 >> 1, m2 = DIM == 3 ? op.n2 >> 1 : 1;
    const int64_t Nc = (int64_t)m0 * m1 * m2;
    const int64_t P = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (P >= Nc) return;
    const int I = (int)(P % m0);
    const int J = (int)((P / m0) % m1);
    const int K = (int)(P / ((int64_t)m0 * m1));
    T uu[8], rr[8];
#pragma unroll
    for (int c = 0; c < (DIM == 3 ? 8 : 4); ++c) {
        const int i = 2 * I + (c & 1), j = 2 * J + ((c >> 1) & 1), l = DIM == 3 ? 2 * K + (c >> 2) : 0;
        const int64_t p = cell_index(op.n0, op.n1, i, j, l);
        Nbhd<T, DIM> s;
        gather<T, DIM, KV>(op, u, i, j, l, s);
        uu[c] = u[p];
        rr[c] = f[p] - apply_value<T, DIM, KV>(op, s, uu[c]);
    }
    if constexpr (DIM == 2) {
        uc[P] = restrict4(uu[0], uu[1], uu[2], uu[3]);
        rc[P] = restrict4(rr[0], rr[1], rr[2], rr[3]);
    } else {
        uc[P] = restrict8(uu[0], uu[1], uu[2], uu[3], uu[4], uu[5], uu[6], uu[7]);
        rc[P] = restrict8(rr[0], rr[1], rr[2], rr[3], rr[4], rr[5], rr[6], rr[7]);
    }
}

// FAS coarse right-hand side in place: fc = rc + Ac(uc) (Alg. 1 coarse source term; fc
// holds rc on entry, the paper's memory reuse).
template <typename T, int DIM, bool KV>
__global__ __launch_bounds__(kBlock) void k_coarse_rhs(Op<T> op, const T* __restrict__ uc, T* __restrict__ fc,
                                                       Batch bt)
{
    if (skip_problem(bt)) return;
    uc += blockIdx.y * bt.fine;
    fc += blockIdx.y * bt.fine;
    const int64_t N = (int64_t)op.n0 * op.n1 * op.n2;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int i = (int)(p % op.n0);
    const int j = (int)((p / op.n0) % op.n1);
    const int l = (int)(p / ((int64_t)op.n0 * op.n1));
    Nbhd<T, DIM> s;
    gather<T, DIM, KV>(op, uc, i, j, l, s);
    fc[p] = fc[p] + apply_value<T, DIM, KV>(op, s, uc[p]);
}

// ----------------------------------------------------------- transfer operators
template <typename T, int DIM>
__device__ __forceinline__ T restrict_at(const T* __restrict__ x, int n0, int n1, int I, int J, int K)
{
    const int i = 2 * I, j = 2 * J;
    if constexpr (DIM == 2) {
        return restrict4(x[cell_index(n0, n1, i, j, 0)], x[cell_index(n0, n1, i + 1, j, 0)],
                         x[cell_index(n0, n1, i, j + 1, 0)], x[cell_index(n0, n1, i + 1, j + 1, 0)]);
    } else {
        const int l = 2 * K;
        return restrict8(x[cell_index(n0, n1, i, j, l)], x[cell_index(n0, n1, i + 1, j, l)],
                         x[cell_index(n0, n1, i, j + 1, l)], x[cell_index(n0, n1, i + 1, j + 1, l)],
                         x[cell_index(n0, n1, i, j, l + 1)], x[cell_index(n0, n1, i + 1, j, l + 1)],
                         x[cell_index(n0, n1, i, j + 1, l + 1)], x[cell_index(n0, n1, i + 1, j + 1, l + 1)]);
    }
}

template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_restrict(int n0, int n1, int n2, const T* __restrict__ fine,
                                                     T* __restrict__ coarse, Batch bt)
{
    if (skip_problem(bt)) return;
    fine += blockIdx.y * bt.fine;
    coarse += blockIdx.y * bt.coarse;
    const int m0 = n0 >> 1, m1 = n1 >> 1, m2 = DIM == 3 ? n2 >> 1 : 1;
    const int64_t Nc = (int64_t)m0 * m1 * m2;
    const int64_t P = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (P >= Nc) return;
    const int I = (int)(P % m0);
    const int J = (int)((P / m0) % m1);
    const int K = (int)(P / ((int64_t)m0 * m1));
    coarse[P] = restrict_at<T, DIM>(fine, n0, n1, I, J, K);
}

// u += P(uc - R u): the old coarse value R u is recomputed from the unchanged fine cells.
// With cold != nullptr the old coarse value is read from cold instead.
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_prolong(int n0, int n1, int n2, const T* __restrict__ uc,
                                                    const T* __restrict__ cold, T* __restrict__ u, Batch bt)
{
    if (skip_problem(bt)) return;
    uc += blockIdx.y * bt.coarse;
    if (cold) cold += blockIdx.y * bt.coarse;
    u += blockIdx.y * bt.fine;
    const int m0 = n0 >> 1, m1 = n1 >> 1, m2 = DIM == 3 ? n2 >> 1 : 1;
    const int64_t Nc = (int64_t)m0 * m1 * m2;
    const int64_t P = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (P >= Nc) return;
    const int I = (int)(P % m0);
    const int J = (int)((P / m0) % m1);
    const int K = (int)(P / ((int64_t)m0 * m1));
    const T old = cold ? cold[P] : restrict_at<T, DIM>(u, n0, n1, I, J, K);
    const T c = uc[P] - old;
#pragma unroll
    for (int ch = 0; ch < (DIM == 3 ? 8 : 4); ++ch) {
        const int64_t p =
            cell_index(n0, n1, 2 * I + (ch & 1), 2 * J + ((ch >> 1) & 1), DIM == 3 ? 2 * K + (ch >> 2) : 0);
        u[p] = u[p] + c;
    }
}

// ----------------------------------------------------------- kappa gradient (FP64)
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_kappa_grad(Op<double> op, const double* __restrict__ mu,
                                                       const double* __restrict__ u, double* __restrict__ g)
{
    const int64_t N = (int64_t)op.n0 * op.n1 * op.n2;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int c[3] = {(int)(p % op.n0), (int)((p / op.n0) % op.n1), (int)(p / ((int64_t)op.n0 * op.n1))};
    const int n[3] = {op.n0, op.n1, op.n2};
    const double* kap = op.kap;
    double t[6];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            int d[3] = {c[0], c[1], c[2]};
            d[a] += side ? 1 : -1;
            bool in = d[a] >= 0 && d[a] < n[a];
            if (!in && op.bc == BC_PERIODIC) {
                d[a] = d[a] < 0 ? n[a] - 1 : 0;
                in = true;
            }
            double val;
            if (in) {
                const int64_t q = cell_index(op.n0, op.n1, d[0], d[1], d[2]);
                const double s = kap[p] + kap[q];
                const double dw = ((2.0 * kap[q]) * kap[q]) / (s * s);
                val = dw * ((mu[p] - mu[q]) * (u[p] - u[q]));
            } else {
                val = op.bc == BC_DIRICHLET ? (2.0 * mu[p]) * u[p] : 0.0;
            }
            t[2 * a + side] = val;
        }
    }
    double S = (t[0] + t[1]) + (t[2] + t[3]);
    if constexpr (DIM == 3) S = S + (t[4] + t[5]);
    g[p] = g[p] - op.k * S;
}

// ----------------------------------------------------------- mixed precision helpers
// Neighbourhood of the even (EVEN) or odd cell of the x-pair (i, i + 1) of row (j, l),
// constant kappa, from pair loads: the pair itself, the cells left of i and right of
// i + 1, and the pairs of the rows (and planes) around it.  Values and boundary-face
// count are those of gather() (a neighbour across a non-periodic boundary is 0, read
// from an in-range index first).
template <int DIM>
struct PairNbhd {
    double2 c;           // the pair
    double xl, xr;       // cells i - 1 and i + 2
    double2 ym, yp, zm, zp;
    bool uxl, uxr, uym, uyp, uzm, uzp;  // the neighbour is inside (or wrapped)
};

template <int DIM>
__device__ __forceinline__ void load_pair_nbhd(const Op<double>& op, const double* __restrict__ u, int i, int j, int l,
                                               PairNbhd<DIM>& s)
{
    const bool per = op.bc == BC_PERIODIC;
    const int64_t row = cell_index(op.n0, op.n1, 0, j, l);
    s.c = *reinterpret_cast<const double2*>(u + row + i);
    s.uxl = per || i > 0;
    s.uxr = per || i + 2 < op.n0;
    const int il = i > 0 ? i - 1 : (per ? op.n0 - 1 : i);
    const int ir = i + 2 < op.n0 ? i + 2 : (per ? 0 : i + 1);
    s.xl = u[row + il];
    s.xr = u[row + ir];
    s.uym = per || j > 0;
    s.uyp = per || j + 1 < op.n1;
    const int jm = j > 0 ? j - 1 : (per ? op.n1 - 1 : j);
    const int jp = j + 1 < op.n1 ? j + 1 : (per ? 0 : j);
    s.ym = *reinterpret_cast<const double2*>(u + cell_index(op.n0, op.n1, i, jm, l));
    s.yp = *reinterpret_cast<const double2*>(u + cell_index(op.n0, op.n1, i, jp, l));
    if constexpr (DIM == 3) {
        s.uzm = per || l > 0;
        s.uzp = per || l + 1 < op.n2;
        const int lm = l > 0 ? l - 1 : (per ? op.n2 - 1 : l);
        const int lp = l + 1 < op.n2 ? l + 1 : (per ? 0 : l);
        s.zm = *reinterpret_cast<const double2*>(u + cell_index(op.n0, op.n1, i, j, lm));
        s.zp = *reinterpret_cast<const double2*>(u + cell_index(op.n0, op.n1, i, j, lp));
    }
}

template <int DIM, bool EVEN>
__device__ __forceinline__ void pair_cell(const PairNbhd<DIM>& s, Nbhd<double, DIM>& nb)
{
    const double vxm = EVEN ? s.xl : s.c.x, vxp = EVEN ? s.c.y : s.xr;
    const bool uxm = EVEN ? s.uxl : true, uxp = EVEN ? true : s.uxr;
    nb.v[0] = uxm ? vxm : 0.0;
    nb.v[1] = uxp ? vxp : 0.0;
    nb.v[2] = s.uym ? (EVEN ? s.ym.x : s.ym.y) : 0.0;
    nb.v[3] = s.uyp ? (EVEN ? s.yp.x : s.yp.y) : 0.0;
    nb.nout = (uxm ? 0 : 1) + (uxp ? 0 : 1) + (s.uym ? 0 : 1) + (s.uyp ? 0 : 1);
    if constexpr (DIM == 3) {
        nb.v[4] = s.uzm ? (EVEN ? s.zm.x : s.zm.y) : 0.0;
        nb.v[5] = s.uzp ? (EVEN ? s.zp.x : s.zp.y) : 0.0;
        nb.nout += (s.uzm ? 0 : 1) + (s.uzp ? 0 : 1);
    }
}

// Outer step of the mixed-precision defect correction: r = f - A u (FP64), r32 = fp32(r),
// per-block sums of r^2 into rpart and (fpart != nullptr) of f^2 into fpart.  One thread
// per x-pair of cells (n0 is even on every grid), grid-stride over a fixed grid so that
// the partial sums have a fixed count and order.  act: the solve's active flag.
template <int DIM, bool KV>
__global__ __launch_bounds__(kBlock) void k_mixed_resid(Op<double> op, const double* __restrict__ f,
                                                        const double* __restrict__ u, float* __restrict__ r32,
                                                        double* __restrict__ rpart, double* __restrict__ fpart,
                                                        const int* __restrict__ act, int64_t stride)
{
    // problem b = blockIdx.y of a stacked grid: arrays b * stride apart, partial sums per
    // problem gridDim.x apart
    const int b = (int)blockIdx.y;
    if (act && !act[b]) return;
    f += b * stride;
    u += b * stride;
    r32 += b * stride;
    rpart += (int64_t)b * gridDim.x;
    if (fpart) fpart += (int64_t)b * gridDim.x;
    const int half = op.n0 >> 1;
    const int64_t pairs = (int64_t)half * op.n1 * op.n2;
    double acc = 0.0, facc = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < pairs; t += (int64_t)gridDim.x * blockDim.x) {
        const int i = 2 * (int)(t % half);
        const int64_t row = t / half;
        const int j = (int)(row % op.n1), l = (int)(row / op.n1);
        const int64_t p = cell_index(op.n0, op.n1, i, j, l);
        const double2 fp = *reinterpret_cast<const double2*>(f + p);
        double re, ro;
        if constexpr (KV) {
            Nbhd<double, DIM> nb;
            gather<double, DIM, true>(op, u, i, j, l, nb);
            re = fp.x - apply_value<double, DIM, true>(op, nb, u[p]);
            gather<double, DIM, true>(op, u, i + 1, j, l, nb);
            ro = fp.y - apply_value<double, DIM, true>(op, nb, u[p + 1]);
        } else {
            PairNbhd<DIM> s;
            load_pair_nbhd<DIM>(op, u, i, j, l, s);
            Nbhd<double, DIM> nb;
            pair_cell<DIM, true>(s, nb);
            re = fp.x - apply_value<double, DIM, false>(op, nb, s.c.x);
            pair_cell<DIM, false>(s, nb);
            ro = fp.y - apply_value<double, DIM, false>(op, nb, s.c.y);
        }
        float2 rv;
        rv.x = (float)re;
        rv.y = (float)ro;
        *reinterpret_cast<float2*>(r32 + p) = rv;
        acc += re * re;
        acc += ro * ro;
        if (fpart) {
            facc += fp.x * fp.x;
            facc += fp.y * fp.y;
        }
    }
    block_sum_store(acc, rpart);
    if (fpart) {
        __syncthreads();
        block_sum_store(facc, fpart);
    }
}

// u += fp64(e) (the outer update of the defect correction when no inner pass folds it).
// The same outer step on 2D grids with a constant coefficient, as row marches: thread t of
// block (x, y) owns the column pair 2 (x kBlock + t), 2 (x kBlock + t) + 1 and walks the
// rows of segment y in order, keeping rows j - 1, j, j + 1 of u in registers, so u is read
// about once (x-neighbours come from the same rows in cache).  Problem b = blockIdx.z; one
// partial sum per block (fixed order).  The point formulas are those of the grid-stride
// kernel above, so r32 is the same; only the partial sums are grouped differently.
constexpr int kMixedSeg = 32;  // rows per segment

__global__ __launch_bounds__(kBlock) void k_mixed_resid_rows(Op<double> op, const double* __restrict__ f,
                                                             const double* __restrict__ u, float* __restrict__ r32,
                                                             double* __restrict__ rpart, double* __restrict__ fpart,
                                                             const int* __restrict__ act, int64_t stride)
{
    const int b = (int)blockIdx.z;
    if (act && !act[b]) return;
    f += b * stride;
    u += b * stride;
    r32 += b * stride;
    const int nblk = (int)(gridDim.x * gridDim.y), blk = (int)(blockIdx.y * gridDim.x + blockIdx.x);
    rpart += (int64_t)b * nblk;
    if (fpart) fpart += (int64_t)b * nblk;
    const bool per = op.bc == BC_PERIODIC;
    const int i = 2 * (int)(blockIdx.x * kBlock + threadIdx.x);
    const bool col = i < op.n0;
    const int ic = col ? i : op.n0 - 2;  // columns past the grid load the last pair and store nothing
    const bool uxl = per || ic > 0, uxr = per || ic + 2 < op.n0;
    const int il = ic > 0 ? ic - 1 : (per ? op.n0 - 1 : ic);
    const int ir = ic + 2 < op.n0 ? ic + 2 : (per ? 0 : ic + 1);
    const int j0 = (int)blockIdx.y * kMixedSeg, j1 = min(j0 + kMixedSeg, op.n1);
    auto row = [&](int j) { return (int64_t)j * op.n0; };
    const int jm0 = j0 > 0 ? j0 - 1 : (per ? op.n1 - 1 : j0);
    double2 um = *reinterpret_cast<const double2*>(u + row(jm0) + ic);
    double2 uc = *reinterpret_cast<const double2*>(u + row(j0) + ic);
    double acc = 0.0, facc = 0.0;
#pragma unroll 4
    for (int j = j0; j < j1; ++j) {
        const int jp = j + 1 < op.n1 ? j + 1 : (per ? 0 : j);
        const double2 up = *reinterpret_cast<const double2*>(u + row(jp) + ic);
        const double2 fp = *reinterpret_cast<const double2*>(f + row(j) + ic);
        PairNbhd<2> s;
        s.c = uc;
        s.xl = u[row(j) + il];
        s.xr = u[row(j) + ir];
        s.ym = um;
        s.yp = up;
        s.uxl = uxl;
        s.uxr = uxr;
        s.uym = per || j > 0;
        s.uyp = per || j + 1 < op.n1;
        Nbhd<double, 2> nb;
        pair_cell<2, true>(s, nb);
        const double re = fp.x - apply_value<double, 2, false>(op, nb, uc.x);
        pair_cell<2, false>(s, nb);
        const double ro = fp.y - apply_value<double, 2, false>(op, nb, uc.y);
        if (col) {
            float2 rv;
            rv.x = (float)re;
            rv.y = (float)ro;
            *reinterpret_cast<float2*>(r32 + row(j) + i) = rv;
            acc += re * re;
            acc += ro * ro;
            if (fpart) {
                facc += fp.x * fp.x;
                facc += fp.y * fp.y;
            }
        }
        um = uc;
        uc = up;
    }
    block_sum_at(acc, rpart, blk);
    if (fpart) {
        __syncthreads();
        block_sum_at(facc, fpart, blk);
    }
}

// Problem b = blockIdx.y of N cells (arrays b * N apart), gated by its active flag.
__global__ __launch_bounds__(kBlock) void k_update_mixed(int64_t N, const float* __restrict__ e, double* __restrict__ u,
                                                         const int* __restrict__ act)
{
    const int b = (int)blockIdx.y;
    if (act && !act[b]) return;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    u[b * N + p] = u[b * N + p] + (double)e[b * N + p];
}

// x = 0 (FP32), problem b = blockIdx.y of N cells, gated by its active flag.
__global__ __launch_bounds__(kBlock) void k_zero_f32(int64_t N, float* __restrict__ x, const int* __restrict__ act)
{
    const int b = (int)blockIdx.y;
    if (act && !act[b]) return;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    x[b * N + p] = 0.0f;
}

__global__ __launch_bounds__(kBlock) void k_cast_f32(int64_t N, const double* __restrict__ src,
                                                     float* __restrict__ dst)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    dst[p] = (float)src[p];
}

// ----------------------------------------------------------- batched convergence flags
__global__ __launch_bounds__(kBlock) void k_init_active(int* act, int* cyc, int nb)
{
    for (int b = blockIdx.x * kBlock + threadIdx.x; b < nb; b += gridDim.x * kBlock) {
        act[b] = 1;
        cyc[b] = 0;
    }
}

__global__ __launch_bounds__(kBlock) void k_update_active(const double* __restrict__ norm2,
                                                          const double* __restrict__ rnorm2, double tol2,
                                                          double atol2, int k, int* __restrict__ act,
                                                          int* __restrict__ cyc, int nb, int* __restrict__ count,
                                                          double* __restrict__ hist)
{
    __shared__ int red[kBlock];
    int alive = 0;
    for (int b = threadIdx.x; b < nb; b += kBlock) {
        if (!act[b]) continue;
        const double nr = norm2[b];
        if (hist && k <= kHist) hist[k - 1] = nr;  // single problem: squared norm after cycle k
        if (!isfinite(nr)) {
            act[b] = 0;
            cyc[b] = -k;
        } else if (nr <= tol2 * rnorm2[b] || nr <= atol2 || nr == 0.0) {
            act[b] = 0;
            cyc[b] = k;
        } else {
            ++alive;
        }
    }
    red[threadIdx.x] = alive;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) count[0] = red[0];
}

// ----------------------------------------------------------- grain-growth right-hand side
// Fan-Chen free energy f = sum_i (-alpha eta_i^2/2 + beta eta_i^4/4) + gamma sum_{i<j}
// eta_i^2 eta_j^2: d f/d eta_i = (beta eta_i^3 - alpha eta_i) + 2 gamma eta_i (S - eta_i^2),
// S = sum_j eta_j^2 (summed in j order); semi-implicit step right-hand side
// f_i = eta_i - dt * d f/d eta_i.
// W consecutive cells per thread (W = 2: float2 accesses, N even), the field loops
// unrolled so that many fields' loads are in flight; each cell's sum over j keeps its
// order.
template <typename T, int W>
__global__ __launch_bounds__(kBlock) void k_grain_rhs(int q, int64_t N, T dt, T alpha, T beta, T gamma2,
                                                      const T* __restrict__ eta, T* __restrict__ f)
{
    using V2 = typename std::conditional<sizeof(T) == 8, double2, float2>::type;
    using V = typename std::conditional<W == 2, V2, T>::type;
    const int64_t p = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * W;
    if (p >= N) return;
    auto ld = [&](int64_t o, T* e) {
        if constexpr (W == 2) {
            const V v = *reinterpret_cast<const V*>(eta + o);
            e[0] = v.x;
            e[1] = v.y;
        } else {
            e[0] = eta[o];
        }
    };
    T S[W], e[W];
    ld(p, e);
#pragma unroll
    for (int c = 0; c < W; ++c) S[c] = e[c] * e[c];
#pragma unroll 8
    for (int j = 1; j < q; ++j) {
        ld((int64_t)j * N + p, e);
#pragma unroll
        for (int c = 0; c < W; ++c) S[c] = S[c] + e[c] * e[c];
    }
#pragma unroll 8
    for (int i = 0; i < q; ++i) {
        ld((int64_t)i * N + p, e);
        T r[W];
#pragma unroll
        for (int c = 0; c < W; ++c) {
            const T e2 = e[c] * e[c];
            const T g = ((beta * e2) * e[c] - alpha * e[c]) + (gamma2 * e[c]) * (S[c] - e2);
            r[c] = e[c] - dt * g;
        }
        if constexpr (W == 2) {
            V v;
            v.x = r[0];
            v.y = r[1];
            *reinterpret_cast<V*>(f + (int64_t)i * N + p) = v;
        } else {
            f[(int64_t)i * N + p] = r[0];
        }
    }
}

}  // namespace

// ------------------------------------------------- array-form batches (StatusDesc each)
__device__ __forceinline__ const StatusDesc& status_of(const TableLaunch& t, int p)
{
    return *reinterpret_cast<const StatusDesc*>(t.desc[p]);
}

__global__ __launch_bounds__(kBlock) void k_batch_init(TableLaunch t)
{
    const int p = (int)(blockIdx.x * kBlock + threadIdx.x);
    if (p >= t.np) return;
    const StatusDesc& d = status_of(t, p);
    d.act[0] = 1;
    d.cyc[0] = 0;
}

// One block per problem: ||rhs||^2 from the first cycle's per-tile f^2 sums.
__global__ __launch_bounds__(kSumBlock) void k_batch_fsum(TableLaunch t)
{
    const StatusDesc& d = status_of(t, (int)blockIdx.x);
    const double s = sum_block(d.fpartials, d.fcount);
    if (threadIdx.x == 0) d.rnorm[0] = s;
}

// One block per problem: the norm total of cycle k and its stopping test, as
// k_sum_update does for a single solve (the same sum, the same tests).
__global__ __launch_bounds__(kSumBlock) void k_batch_update(TableLaunch t, double tol2, int k)
{
    const StatusDesc& d = status_of(t, (int)blockIdx.x);
    if (!d.act[0]) return;  // uniform over the block
    const double nr = sum_block(d.partials, d.count);
    if (threadIdx.x != 0) return;
    d.norm_out[0] = nr;
    if (k <= kHist) d.hist[k - 1] = nr;
    if (!isfinite(nr)) {
        d.act[0] = 0;
        d.cyc[0] = -k;
    } else if (nr <= tol2 * d.rnorm[0] || nr <= d.atol2 || nr == 0.0) {
        d.act[0] = 0;
        d.cyc[0] = k;
    }
}

// One block: the problems still active, into count[0] (added to it when accumulating).
__global__ __launch_bounds__(kBlock) void k_batch_alive(TableLaunch t, int* count, int accumulate)
{
    __shared__ int red[kBlock];
    int alive = 0;
    for (int p = threadIdx.x; p < t.np; p += kBlock) alive += status_of(t, p).act[0] ? 1 : 0;
    red[threadIdx.x] = alive;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) count[0] = (accumulate ? count[0] : 0) + red[0];
}

__global__ __launch_bounds__(kBlock) void k_batch_gather(TableLaunch t, double* out, int base, int stride)
{
    const StatusDesc& d = status_of(t, (int)blockIdx.x);
    double* const o = out + (int64_t)(base + (int)blockIdx.x) * stride;
    for (int i = threadIdx.x; i < stride; i += kBlock)
        o[i] = i == 0 ? (double)d.cyc[0] : (i == 1 ? d.rnorm[0] : d.hist[i - 2]);
}

// --------------------------------------------------------------------------- dispatch
#define FAS_DISPATCH(g, kap, BODY)                                                        \
    do {                                                                                  \
        const bool kv_ = (kap) != nullptr;                                                \
        if ((g)->dtype == FAS_F64) {                                                      \
            using T = double;                                                             \
            if ((g)->dim == 2) {                                                          \
                constexpr int D = 2;                                                      \
                if (kv_) { constexpr bool KV = true; BODY; } else { constexpr bool KV = false; BODY; } \
            } else {                                                                      \
                constexpr int D = 3;                                                      \
                if (kv_) { constexpr bool KV = true; BODY; } else { constexpr bool KV = false; BODY; } \
            }                                                                             \
        } else {                                                                          \
            using T = float;                                                              \
            if ((g)->dim == 2) {                                                          \
                constexpr int D = 2;                                                      \
                if (kv_) { constexpr bool KV = true; BODY; } else { constexpr bool KV = false; BODY; } \
            } else {                                                                      \
                constexpr int D = 3;                                                      \
                if (kv_) { constexpr bool KV = true; BODY; } else { constexpr bool KV = false; BODY; } \
            }                                                                             \
        }                                                                                 \
    } while (0)

void launch_smooth_phase(const fas_grid* g, int l, const Coef& c, const void* kap, const void* f, void* u,
                         int parity)
{
    const Level& L = g->lev[l];
    const int64_t work = (int64_t)((L.n[0] + 1) / 2) * L.n[1] * L.n[2];
    FAS_DISPATCH(g, kap, (k_smooth_phase<T, D, KV><<<grid2(blocks_for(work), g), kBlock, 0, g->stream>>>(
                             make_op<T>(g, l, c, kap), (const T*)f, (T*)u, parity, batch_of(g, l))));
    check_launch();
}

void launch_batch_init(hipStream_t stream, const TableLaunch& t)
{
    k_batch_init<<<blocks_for(t.np), kBlock, 0, stream>>>(t);
    check_launch();
}

void launch_batch_fsum(hipStream_t stream, const TableLaunch& t)
{
    k_batch_fsum<<<(unsigned)t.np, kSumBlock, 0, stream>>>(t);
    check_launch();
}

void launch_batch_update(hipStream_t stream, const TableLaunch& t, double tol, int k)
{
    k_batch_update<<<(unsigned)t.np, kSumBlock, 0, stream>>>(t, tol * tol, k);
    check_launch();
}

void launch_batch_alive(hipStream_t stream, const TableLaunch& t, int* count, bool accumulate)
{
    k_batch_alive<<<1, kBlock, 0, stream>>>(t, count, accumulate ? 1 : 0);
    check_launch();
}

void launch_batch_gather(hipStream_t stream, const TableLaunch& t, double* out, int base, int stride)
{
    if (stride < 2 || stride > kHist + 2) throw Error(FAS_ERR_ARG, "internal: gather stride");
    k_batch_gather<<<(unsigned)t.np, kBlock, 0, stream>>>(t, out, base, stride);
    check_launch();
}

void launch_smooth_set(const fas_grid* g, int l, const Coef& c, const void* kap, const void* f, void* u, int mask)
{
    const Level& L = g->lev[l];
    const int64_t work = (int64_t)((L.n[0] + 1) / 2) * ((L.n[1] + 1) / 2) * (g->dim == 3 ? (L.n[2] + 1) / 2 : 1);
    FAS_DISPATCH(g, kap, (k_smooth_set<T, D, KV><<<grid2(blocks_for(work), g), kBlock, 0, g->stream>>>(
                             make_op<T>(g, l, c, kap), (const T*)f, (T*)u, mask, batch_of(g, l))));
    check_launch();
}

void launch_residual(const fas_grid* g, int l, const Coef& c, const void* kap, const void* f, const void* u,
                     void* r)
{
    FAS_DISPATCH(g, kap, (k_residual<T, D, KV><<<grid2(blocks_for(g->lev[l].N), g), kBlock, 0, g->stream>>>(
                             make_op<T>(g, l, c, kap), (const T*)f, (const T*)u, (T*)r, batch_of(g, l))));
    check_launch();
}

void launch_resid_norm(const fas_grid* g, int l, const Coef& c, const void* kap, const void* f, const void* u)
{
    const unsigned cap = (unsigned)(g->npartials / g->batch);
    // a grid-stride loop: a few thousand blocks fill the device, and keep the final sum short
    unsigned nb = blocks_for(g->lev[l].N);
    if (nb > (unsigned)fas::kPartials) nb = (unsigned)fas::kPartials;
    if (nb > cap) nb = cap;
    FAS_DISPATCH(g, kap, (k_resid_norm<T, D, KV><<<grid2(nb, g), kBlock, 0, g->stream>>>(
                             make_op<T>(g, l, c, kap), (const T*)f, (const T*)u, g->partials, batch_of(g, l))));
    check_launch();
    launch_sum_partials(g, (int)nb);
}

void launch_sum_partials(const fas_grid* g, int count, double* out, const double* src)
{
    k_sum_partials<<<(unsigned)g->batch, kSumBlock, 0, g->stream>>>(src ? src : g->partials, count,
                                                                    out ? out : g->norm_out);
    check_launch();
}

void launch_sum_update(const fas_grid* g, int count, double tol, int k)
{
    if (g->batch != 1) throw Error(FAS_ERR_ARG, "internal: the fused norm update takes one problem");
    k_sum_update<<<1, kSumBlock, 0, g->stream>>>(g->partials, count, g->norm_out, g->rnorm, tol * tol,
                                                 g->atol * g->atol, k, g->active,
                                                  g->cyc, g->count, g->hist);
    check_launch();
}

void launch_resid_restrict(const fas_grid* g, int l, const Coef& c, const void* kap, const void* f,
                           const void* u, void* uc, void* rc)
{
    FAS_DISPATCH(g, kap, (k_resid_restrict<T, D, KV><<<grid2(blocks_for(g->lev[l + 1].N), g), kBlock, 0, g->stream>>>(
                             make_op<T>(g, l, c, kap), (const T*)f, (const T*)u, (T*)uc, (T*)rc, batch_of(g, l))));
    check_launch();
}

void launch_coarse_rhs(const fas_grid* g, int lc, const Coef& c, const void* kapc, const void* uc, void* fc)
{
    FAS_DISPATCH(g, kapc, (k_coarse_rhs<T, D, KV><<<grid2(blocks_for(g->lev[lc].N), g), kBlock, 0, g->stream>>>(
                              make_op<T>(g, lc, c, kapc), (const T*)uc, (T*)fc, batch_of(g, lc))));
    check_launch();
}

void launch_prolong_correct(const fas_grid* g, int l, const void* uc, void* u)
{
    launch_prolong_add(g, l, uc, nullptr, u);
}

void launch_prolong_add(const fas_grid* g, int l, const void* cnew, const void* cold, void* fine)
{
    const Level& L = g->lev[l];
    const unsigned nb = blocks_for(g->lev[l + 1].N);
    FAS_DISPATCH(g, (const void*)nullptr, (k_prolong<T, D><<<grid2(nb, g), kBlock, 0, g->stream>>>(
                                              L.n[0], L.n[1], L.n[2], (const T*)cnew, (const T*)cold, (T*)fine,
                                              batch_of(g, l))));
    check_launch();
}

void launch_restrict(const fas_grid* g, int l, const void* fine, void* coarse)
{
    const Level& L = g->lev[l];
    const unsigned nb = blocks_for(g->lev[l + 1].N);
    FAS_DISPATCH(g, (const void*)nullptr, (k_restrict<T, D><<<grid2(nb, g), kBlock, 0, g->stream>>>(
                                              L.n[0], L.n[1], L.n[2], (const T*)fine, (T*)coarse, batch_of(g, l))));
    check_launch();
}

void launch_kappa_grad(const fas_grid* g, const Coef& c, const void* kap, const void* mu, const void* u, void* gk)
{
    const Op<double> op = make_op<double>(g, 0, c, kap);
    const unsigned nb = blocks_for(g->lev[0].N);
    if (g->dim == 2)
        k_kappa_grad<2><<<nb, kBlock, 0, g->stream>>>(op, (const double*)mu, (const double*)u, (double*)gk);
    else
        k_kappa_grad<3><<<nb, kBlock, 0, g->stream>>>(op, (const double*)mu, (const double*)u, (double*)gk);
    check_launch();
}

int launch_mixed_resid(const fas_grid* g, const Coef& c, const void* kap, const void* f, const void* u, void* r32,
                       bool fnorm)
{
    const Op<double> op = make_op<double>(g, 0, c, kap);
    const int64_t pairs = g->lev[0].N / 2;
    // a fixed grid per problem: r^2 partial sums in g->partials, f^2 in g->fpartials
    unsigned nb = (unsigned)std::min<int64_t>((pairs + kBlock - 1) / kBlock, (int64_t)(g->npartials / g->batch));
    if (nb > (unsigned)kPartials) nb = (unsigned)kPartials;
    const int* act = active_flags(g);
    auto F = (const double*)f;
    auto U = (const double*)u;
    double* fp = fnorm ? g->fpartials : nullptr;
    const bool kv = kap != nullptr;
    const int64_t stride = g->lev[0].N;
    if (g->dim == 3 && !kap) {
        // plane march: each block keeps a ring of planes, so u is read about once
        const int np = launch_march3_resid(g, c, f, u, r32, g->partials, fp);
        if (np) return np;
    }
    if (g->dim == 2 && !kap) {
        // row marches: one block per 512 columns and kMixedSeg rows
        const unsigned bx = (unsigned)((g->lev[0].n[0] / 2 + kBlock - 1) / kBlock);
        const unsigned by = (unsigned)((g->lev[0].n[1] + kMixedSeg - 1) / kMixedSeg);
        if ((int64_t)bx * by <= (int64_t)(g->npartials / g->batch)) {
            k_mixed_resid_rows<<<dim3(bx, by, (unsigned)g->batch), kBlock, 0, g->stream>>>(
                op, F, U, (float*)r32, g->partials, fp, act, stride);
            check_launch();
            return (int)(bx * by);
        }
    }
    const dim3 grid(nb, (unsigned)g->batch, 1);
#define FAS_MIXED_RESID(D_, KV_) \
    k_mixed_resid<D_, KV_><<<grid, kBlock, 0, g->stream>>>(op, F, U, (float*)r32, g->partials, fp, act, stride)
    if (g->dim == 2) {
        if (kv) FAS_MIXED_RESID(2, true);
        else FAS_MIXED_RESID(2, false);
    } else {
        if (kv) FAS_MIXED_RESID(3, true);
        else FAS_MIXED_RESID(3, false);
    }
#undef FAS_MIXED_RESID
    check_launch();
    return (int)nb;
}

void launch_update_mixed(const fas_grid* g, const void* e32, void* u)
{
    const int64_t N = g->lev[0].N;
    k_update_mixed<<<grid2(blocks_for(N), g), kBlock, 0, g->stream>>>(N, (const float*)e32, (double*)u,
                                                                      active_flags(g));
    check_launch();
}

void launch_zero_f32(const fas_grid* g, int64_t N, void* x)
{
    k_zero_f32<<<grid2(blocks_for(N), g), kBlock, 0, g->stream>>>(N, (float*)x, active_flags(g));
    check_launch();
}

void launch_cast_f32(const fas_grid* g, int64_t N, const void* src64, void* dst32)
{
    k_cast_f32<<<blocks_for(N), kBlock, 0, g->stream>>>(N, (const double*)src64, (float*)dst32);
    check_launch();
}

}  // namespace fas

namespace fas {

void launch_init_active(const fas_grid* g)
{
    k_init_active<<<blocks_for(g->batch), kBlock, 0, g->stream>>>(g->active, g->cyc, g->batch);
    check_launch();
}

void launch_update_active(const fas_grid* g, double tol, int k)
{
    k_update_active<<<1, kBlock, 0, g->stream>>>(g->norm_out, g->rnorm, tol * tol, g->atol * g->atol, k, g->active,
                                                 g->cyc, g->batch,
                                                 g->count, g->batch == 1 ? g->hist : nullptr);
    check_launch();
}

// Grain map of a multi-order-parameter state: per cell, the field with the largest value
// (the lowest index among equal maxima), as read off the order parameters to find grains.
__global__ __launch_bounds__(kBlock) void k_grain_argmax(int q, int64_t N, const float* __restrict__ eta,
                                                         int* __restrict__ label)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= N) return;
    float best = eta[p];
    int arg = 0;
#pragma unroll 8
    for (int i = 1; i < q; ++i) {
        const float v = eta[(int64_t)i * N + p];
        if (v > best) {
            best = v;
            arg = i;
        }
    }
    label[p] = arg;
}

void launch_grain_argmax(hipStream_t stream, int q, int64_t N, const float* eta, int* label)
{
    k_grain_argmax<<<blocks_for(N), kBlock, 0, stream>>>(q, N, eta, label);
    check_launch();
}

template <typename T>
void launch_grain_rhs_t(hipStream_t stream, int q, int64_t N, T dt, T alpha, T beta, T gamma2, const T* eta, T* f)
{
    // N even and pair-aligned arrays: pair accesses stay aligned in every field
    const uintptr_t al = 2 * sizeof(T);
    if (N % 2 == 0 && ((uintptr_t)eta % al) == 0 && ((uintptr_t)f % al) == 0)
        k_grain_rhs<T, 2><<<blocks_for(N / 2), kBlock, 0, stream>>>(q, N, dt, alpha, beta, gamma2, eta, f);
    else
        k_grain_rhs<T, 1><<<blocks_for(N), kBlock, 0, stream>>>(q, N, dt, alpha, beta, gamma2, eta, f);
    check_launch();
}

void launch_grain_rhs(hipStream_t stream, int dtype, int q, int64_t N, double dt, double alpha, double beta,
                      double gamma, const void* eta, void* f)
{
    // the pair term's coefficient 2 gamma is rounded once, in the arithmetic's precision
    if (dtype == FAS_F64)
        launch_grain_rhs_t<double>(stream, q, N, dt, alpha, beta, 2.0 * gamma, (const double*)eta, (double*)f);
    else
        launch_grain_rhs_t<float>(stream, q, N, (float)dt, (float)alpha, (float)beta, (float)(2.0 * gamma),
                                  (const float*)eta, (float*)f);
}

}  // namespace fas
