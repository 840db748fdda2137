// Persistent coarse tail: every level from `top` down to the coarsest, in one workgroup
// whose LDS holds u and f of all those levels (Remark 2's recursion below `top`, and
// Remark 1's smoothing on the coarsest level).  One launch replaces a dozen tiny
// launches per level; the per-point formulas are those of fas_device.h, so the values
// are bit-identical to running the per-level kernels.
#include <hip/hip_runtime.h>
#include <string.h>

#include "fas_batch.h"
#include "fas_device.h"
#include "fas_internal.h"
#include "fas_tail.h"

namespace fas {

namespace {

constexpr int kTailThreads = 1024;
constexpr int kTailLds = 96 * 1024;     // bytes of LDS for u and f of the tail levels
constexpr int kTailLdsKV = 144 * 1024;  // cell kappa: u, f and kappa of the tail levels

template <typename T>
struct TailArgs {
    int nl;                   // levels in the tail (top .. coarsest)
    int pre, post, nuc;       // sweeps
    int first;                // parity of the first phase of a sweep
    int form_rhs;             // 1: f_top = r_top + A u_top (FAS coarse right-hand side)
    int lds_off[kMaxTail];    // element offset of u of each level; f follows u
    int kap_off[kMaxTail];    // cell kappa: element offset of each level's kappa copy
    Op<T> op[kMaxTail];
    T* u_top;                 // in: initial guess of the top level; out: its new values
    const T* r_top;           // in: restricted residual (form_rhs) or the right-hand side
    int64_t stride;           // batched grids: problem b = blockIdx.x at b * stride
    const int* act;           // per-problem active flags (nullable)
};

// Cells are visited row by row: the 1024 threads form TX columns by kTailThreads / TX
// rows (x fastest), TX the smallest power of two >= the row's work items (at most 32), so
// narrow levels keep every lane busy and no thread divides by a level size.
constexpr int kTX = 32;
struct TMap {
    int tx, ty, TX, TY;
};
__device__ __forceinline__ TMap tmap(int width)
{
    int lg = 0;
    while ((1 << lg) < width && (1 << lg) < kTX) ++lg;
    return TMap{(int)threadIdx.x & ((1 << lg) - 1), (int)threadIdx.x >> lg, 1 << lg, kTailThreads >> lg};
}

// 2D, constant kappa: the neighbourhood of cell (i, j) of a level held in LDS, with the
// values and boundary-face count of fas_device.h's gather (neighbours across a periodic
// edge wrapped, across another edge 0), from 32-bit indices: every tail phase is a chain
// of these, so their index arithmetic is on its critical path.
template <typename T>
__device__ __forceinline__ void gather2(const Op<T>& op, const T* U, int i, int j, Nbhd<T, 2>& s)
{
    const bool per = op.bc == BC_PERIODIC;
    const int n0 = op.n0, n1 = op.n1, p = i + n0 * j;
    const bool xl = i > 0, xr = i < n0 - 1, yl = j > 0, yr = j < n1 - 1;
    // an in-range index for each neighbour: wrapped on periodic grids, else the cell
    const int qxm = xl ? p - 1 : (per ? p + n0 - 1 : p);
    const int qxp = xr ? p + 1 : (per ? p - n0 + 1 : p);
    const int qym = yl ? p - n0 : (per ? p + (n1 - 1) * n0 : p);
    const int qyp = yr ? p + n0 : (per ? p - (n1 - 1) * n0 : p);
    const T vxm = U[qxm], vxp = U[qxp], vym = U[qym], vyp = U[qyp];
    s.v[0] = (per || xl) ? vxm : (T)0;
    s.v[1] = (per || xr) ? vxp : (T)0;
    s.v[2] = (per || yl) ? vym : (T)0;
    s.v[3] = (per || yr) ? vyp : (T)0;
    s.nout = per ? 0 : (!xl) + (!xr) + (!yl) + (!yr);
}

// Neighbourhood of cell (i, j, l) of a level held in LDS.
template <typename T, int DIM, bool KV>
__device__ __forceinline__ void tail_gather(const Op<T>& op, const T* U, int i, int j, int l, Nbhd<T, DIM>& s)
{
    if constexpr (DIM == 2 && !KV)
        gather2<T>(op, U, i, j, s);
    else
        gather<T, DIM, KV>(op, U, i, j, l, s);
}

template <typename T, int DIM, bool KV>
__device__ void tail_smooth(const Op<T>& op, T* U, const T* F, int sweeps, int first, bool reverse)
{
    const int f0 = reverse ? 1 - first : first;
    const int half = (op.n0 + 1) >> 1;
    // 2D constant kappa: q[W] for 0, 1 and 2 boundary faces (uniform picks; a per-cell
    // index into the table would be a memory load per cell)
    const T q0 = op.q[diag_count(op.bc, DIM, 0)], q1 = op.q[diag_count(op.bc, DIM, 1)],
            q2 = op.q[diag_count(op.bc, DIM, 2)];
    const int rows = op.n1 * op.n2;
    const TMap m = tmap(half);
    for (int s = 0; s < sweeps; ++s) {
        for (int ph = 0; ph < 2; ++ph) {
            const int parity = ph == 0 ? f0 : 1 - f0;
            for (int row = m.ty; row < rows; row += m.TY) {
                const int l = DIM == 3 ? row / op.n1 : 0, j = DIM == 3 ? row - l * op.n1 : row;
                const int odd = (parity + j + l) & 1;
                for (int tt = m.tx; tt < half; tt += m.TX) {
                    const int i = 2 * tt + odd;
                    if (i >= op.n0) continue;
                    Nbhd<T, DIM> nb;
                    tail_gather<T, DIM, KV>(op, U, i, j, l, nb);
                    const int p = (int)cell_index(op.n0, op.n1, i, j, l);
                    if constexpr (DIM == 2 && !KV) {  // gs_value's tree
                        const T S = nbsum<T, DIM>(nb.v);
                        U[p] = (F[p] + op.k * S) * (nb.nout == 0 ? q0 : (nb.nout == 1 ? q1 : q2));
                    } else {
                        U[p] = gs_value<T, DIM, KV>(op, nb, F[p]);
                    }
                }
            }
            __syncthreads();
        }
    }
}

// The tail of one problem: its top level's u (in and out) and r (or f) at u_top / r_top.
template <typename T, int DIM, bool KV>
__device__ __forceinline__ void tail_body(const TailArgs<T>& a, T* const u_top, const T* const r_top)
{
    // cell kappa: every level's kappa is copied into LDS too, so the face weights of each
    // phase read it there rather than from global memory
    __shared__ __attribute__((aligned(16))) char lds[KV ? kTailLdsKV : kTailLds];
    T* base = reinterpret_cast<T*>(lds);
    auto U = [&](int l) { return base + a.lds_off[l]; };
    auto F = [&](int l) { return base + a.lds_off[l] + (a.op[l].n0 * a.op[l].n1 * a.op[l].n2); };
    // the operator of level l, its cell kappa (if any) read from the LDS copy
    auto OP = [&](int l) {
        Op<T> o = a.op[l];
        if constexpr (KV) o.kap = base + a.kap_off[l];
        return o;
    };
    const int N0 = a.op[0].n0 * a.op[0].n1 * a.op[0].n2;
    for (int p = threadIdx.x; p < N0; p += kTailThreads) {
        U(0)[p] = u_top[p];
        F(0)[p] = r_top[p];
    }
    if constexpr (KV) {
        for (int l = 0; l < a.nl; ++l) {
            const int Nl = a.op[l].n0 * a.op[l].n1 * a.op[l].n2;
            T* const kl = base + a.kap_off[l];
            const T* const kg = a.op[l].kap;
            for (int p = threadIdx.x; p < Nl; p += kTailThreads) kl[p] = kg[p];
        }
    }
    __syncthreads();
    if (a.form_rhs) {
        // f = r_c + A_c u_c
        const Op<T> op = OP(0);
        const TMap m = tmap(op.n0);
        for (int row = m.ty; row < op.n1 * op.n2; row += m.TY) {
            const int l = DIM == 3 ? row / op.n1 : 0, j = DIM == 3 ? row - l * op.n1 : row;
            for (int i = m.tx; i < op.n0; i += m.TX) {
                const int p = (int)cell_index(op.n0, op.n1, i, j, l);
                Nbhd<T, DIM> nb;
                tail_gather<T, DIM, KV>(op, U(0), i, j, l, nb);
                F(0)[p] = F(0)[p] + apply_value<T, DIM, KV>(op, nb, U(0)[p]);
            }
        }
        __syncthreads();
    }
    const bool rev = false;
    // descend: pre-smoothing, then u_c = R u, f_c = R (f - A u) + A_c u_c
    for (int lv = 0; lv + 1 < a.nl; ++lv) {
        const Op<T> op = OP(lv);
        const Op<T> oc = OP(lv + 1);
        T* u = U(lv);
        const T* f = F(lv);
        tail_smooth<T, DIM, KV>(op, u, f, a.pre, a.first, rev);
        const TMap m = tmap(oc.n0);
        for (int crow = m.ty; crow < oc.n1 * oc.n2; crow += m.TY)
        for (int I = m.tx; I < oc.n0; I += m.TX) {
            const int K = DIM == 3 ? crow / oc.n1 : 0, J = DIM == 3 ? crow - K * oc.n1 : crow;
            const int P = (int)cell_index(oc.n0, oc.n1, I, J, K);
            T uu[8], rr[8];
#pragma unroll
            for (int c = 0; c < (DIM == 3 ? 8 : 4); ++c) {
                const int i = 2 * I + (c & 1), j = 2 * J + ((c >> 1) & 1), l = DIM == 3 ? 2 * K + (c >> 2) : 0;
                const int p = (int)cell_index(op.n0, op.n1, i, j, l);
                Nbhd<T, DIM> nb;
                tail_gather<T, DIM, KV>(op, u, i, j, l, nb);
                uu[c] = u[p];
                rr[c] = f[p] - apply_value<T, DIM, KV>(op, nb, uu[c]);
            }
            if constexpr (DIM == 2) {
                U(lv + 1)[P] = restrict4(uu[0], uu[1], uu[2], uu[3]);
                F(lv + 1)[P] = restrict4(rr[0], rr[1], rr[2], rr[3]);
            } else {
                U(lv + 1)[P] = restrict8(uu[0], uu[1], uu[2], uu[3], uu[4], uu[5], uu[6], uu[7]);
                F(lv + 1)[P] = restrict8(rr[0], rr[1], rr[2], rr[3], rr[4], rr[5], rr[6], rr[7]);
            }
        }
        __syncthreads();
        for (int crow = m.ty; crow < oc.n1 * oc.n2; crow += m.TY)
        for (int I = m.tx; I < oc.n0; I += m.TX) {
            const int K = DIM == 3 ? crow / oc.n1 : 0, J = DIM == 3 ? crow - K * oc.n1 : crow;
            const int P = (int)cell_index(oc.n0, oc.n1, I, J, K);
            Nbhd<T, DIM> nb;
            tail_gather<T, DIM, KV>(oc, U(lv + 1), I, J, K, nb);
            F(lv + 1)[P] = F(lv + 1)[P] + apply_value<T, DIM, KV>(oc, nb, U(lv + 1)[P]);
        }
        __syncthreads();
    }
    // coarsest level: smoothing only (Remark 1)
    tail_smooth<T, DIM, KV>(OP(a.nl - 1), U(a.nl - 1), F(a.nl - 1), a.nuc, a.first, rev);
    // ascend: u += P(u_c - R u), post-smoothing
    for (int lv = a.nl - 2; lv >= 0; --lv) {
        const Op<T> op = OP(lv);
        const Op<T> oc = OP(lv + 1);
        T* u = U(lv);
        const TMap m = tmap(oc.n0);
        for (int crow = m.ty; crow < oc.n1 * oc.n2; crow += m.TY)
        for (int I = m.tx; I < oc.n0; I += m.TX) {
            const int K = DIM == 3 ? crow / oc.n1 : 0, J = DIM == 3 ? crow - K * oc.n1 : crow;
            const int P = (int)cell_index(oc.n0, oc.n1, I, J, K);
            const int i = 2 * I, j = 2 * J, l = 2 * K;
            T old;
            if constexpr (DIM == 2) {
                old = restrict4(u[cell_index(op.n0, op.n1, i, j, 0)], u[cell_index(op.n0, op.n1, i + 1, j, 0)],
                                u[cell_index(op.n0, op.n1, i, j + 1, 0)], u[cell_index(op.n0, op.n1, i + 1, j + 1, 0)]);
            } else {
                old = restrict8(u[cell_index(op.n0, op.n1, i, j, l)], u[cell_index(op.n0, op.n1, i + 1, j, l)],
                                u[cell_index(op.n0, op.n1, i, j + 1, l)], u[cell_index(op.n0, op.n1, i + 1, j + 1, l)],
                                u[cell_index(op.n0, op.n1, i, j, l + 1)], u[cell_index(op.n0, op.n1, i + 1, j, l + 1)],
                                u[cell_index(op.n0, op.n1, i, j + 1, l + 1)],
                                u[cell_index(op.n0, op.n1, i + 1, j + 1, l + 1)]);
            }
            const T c = U(lv + 1)[P] - old;
#pragma unroll
            for (int ch = 0; ch < (DIM == 3 ? 8 : 4); ++ch) {
                const int p = (int)cell_index(op.n0, op.n1, i + (ch & 1), j + ((ch >> 1) & 1), DIM == 3 ? l + (ch >> 2) : 0);
                u[p] = u[p] + c;
            }
        }
        __syncthreads();
        tail_smooth<T, DIM, KV>(op, u, F(lv), a.post, a.first, rev);
    }
    for (int p = threadIdx.x; p < N0; p += kTailThreads) u_top[p] = U(0)[p];
}

// Problem b = blockIdx.x of a stacked batch (arrays b * stride apart).
template <typename T, int DIM, bool KV>
__global__ __launch_bounds__(kTailThreads) void k_tail(TailArgs<T> a)
{
    if (a.act && !a.act[blockIdx.x]) return;
    tail_body<T, DIM, KV>(a, a.u_top + blockIdx.x * a.stride, a.r_top + blockIdx.x * a.stride);
}

// Table launch (array-form batches): problem blockIdx.x's descriptor.
template <typename T, int DIM, bool KV>
__global__ __launch_bounds__(kTailThreads) void k_tail_table(TableLaunch tl)
{
    const TailArgs<T>& a = *reinterpret_cast<const TailArgs<T>*>(tl.desc[blockIdx.x]);
    if (a.act && !a.act[0]) return;
    tail_body<T, DIM, KV>(a, a.u_top, a.r_top);
}

template <typename T>
TailArgs<T> make_tail_args(const fas_grid* g, int top, const Coef* coef, int pre, int post, int first)
{
    TailArgs<T> a{};
    a.nl = g->L - top + 1;
    a.pre = pre;
    a.post = post;
    a.nuc = g->nuc;
    a.first = first;
    int off = 0;
    for (int i = 0; i < a.nl; ++i) {
        const int l = top + i;
        Op<T>& op = a.op[i];
        op.n0 = g->lev[l].n[0];
        op.n1 = g->lev[l].n[1];
        op.n2 = g->lev[l].n[2];
        op.bc = g->bc;
        op.k = (T)coef[l].kd;
        for (int W = 0; W < 16; ++W) op.q[W] = (T)coef[l].q[W];
        op.kap = (const T*)g->lev[l].kap;
        a.lds_off[i] = off;
        off += 2 * (int)g->lev[l].N;
    }
    const bool kv = g->lev[top].kap != nullptr;
    for (int i = 0; i < a.nl; ++i) {  // cell kappa: copies after every level's u and f
        a.kap_off[i] = off;
        if (kv) off += (int)g->lev[top + i].N;
    }
    if ((size_t)off * sizeof(T) > (size_t)(kv ? kTailLdsKV : kTailLds))
        throw Error(FAS_ERR_ARG, "internal: tail levels exceed the tail's LDS");
    return a;
}

inline void check_launch()
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error(FAS_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
}

template <typename T>
void launch_t(const fas_grid* g, int top, const Coef* coef, int pre, int post, int first, void* u, const void* r,
              int form_rhs)
{
    TailArgs<T> a = make_tail_args<T>(g, top, coef, pre, post, first);
    a.u_top = (T*)u;
    a.r_top = (const T*)r;
    a.form_rhs = form_rhs;
    a.stride = g->lev[top].N;
    a.act = active_flags(g);
    const unsigned nb = (unsigned)g->batch;
    const bool kv = g->lev[top].kap != nullptr;
    if (g->dim == 2) {
        if (kv)
            k_tail<T, 2, true><<<nb, kTailThreads, 0, g->stream>>>(a);
        else
            k_tail<T, 2, false><<<nb, kTailThreads, 0, g->stream>>>(a);
    } else {
        if (kv)
            k_tail<T, 3, true><<<nb, kTailThreads, 0, g->stream>>>(a);
        else
            k_tail<T, 3, false><<<nb, kTailThreads, 0, g->stream>>>(a);
    }
    check_launch();
}

}  // namespace

int tail_top(const fas_grid* g)
{
    // the largest level from which every coarser level's u and f (and the cell kappa on a
    // grid that may take one) fit the tail's LDS; the two budgets admit the same levels
    const size_t s = g->elem();
    const bool kv = (g->flags & FAS_FLAG_VARIABLE_KAPPA) != 0;
    const size_t cap = kv ? (size_t)kTailLdsKV : (size_t)kTailLds;
    size_t bytes = 0;
    int top = g->L + 1;
    for (int l = g->L; l >= 0; --l) {
        bytes += (kv ? 3 : 2) * (size_t)g->lev[l].N * s;
        if (bytes > cap || g->L - l + 1 > kMaxTail) break;
        top = l;
    }
    return top;  // L + 1: not even the coarsest level fits
}

size_t tail_desc_bytes(int dtype)
{
    return dtype == FAS_F64 ? sizeof(TailArgs<double>) : sizeof(TailArgs<float>);
}

template <typename T>
void fill_tail_desc_t(const fas_grid* g, int top, const Coef* coef, int pre, int post, int first, void* u,
                      const void* r, bool form_rhs, const int* act, void* out)
{
    TailArgs<T> a = make_tail_args<T>(g, top, coef, pre, post, first);
    a.u_top = (T*)u;
    a.r_top = (const T*)r;
    a.form_rhs = form_rhs ? 1 : 0;
    a.stride = 0;
    a.act = act;
    memcpy(out, &a, sizeof(a));
}

void fill_tail_desc(const fas_grid* g, int top, const Coef* coef, int pre, int post, int first, void* u, const void* r,
                    bool form_rhs, const int* act, void* out)
{
    if (!u || !r || !act || top < 0 || top > g->L || g->L - top + 1 > kMaxTail)
        throw Error(FAS_ERR_ARG, "internal: tail descriptor with a missing array or level");
    if (g->dtype == FAS_F64)
        fill_tail_desc_t<double>(g, top, coef, pre, post, first, u, r, form_rhs, act, out);
    else
        fill_tail_desc_t<float>(g, top, coef, pre, post, first, u, r, form_rhs, act, out);
}

void launch_tail_table(hipStream_t stream, int dtype, int dim, bool kv, const TableLaunch& t)
{
    if (t.np < 1 || t.np > kBatchChunk) throw Error(FAS_ERR_ARG, "internal: table launch size");
    const unsigned nb = (unsigned)t.np;
#define FAS_TAIL_T(T_)                                                                         \
    do {                                                                                       \
        if (dim == 2) {                                                                        \
            if (kv) k_tail_table<T_, 2, true><<<nb, kTailThreads, 0, stream>>>(t);             \
            else k_tail_table<T_, 2, false><<<nb, kTailThreads, 0, stream>>>(t);               \
        } else {                                                                               \
            if (kv) k_tail_table<T_, 3, true><<<nb, kTailThreads, 0, stream>>>(t);             \
            else k_tail_table<T_, 3, false><<<nb, kTailThreads, 0, stream>>>(t);               \
        }                                                                                      \
    } while (0)
    if (dtype == FAS_F64)
        FAS_TAIL_T(double);
    else
        FAS_TAIL_T(float);
#undef FAS_TAIL_T
    check_launch();
}

void launch_tail(const fas_grid* g, int top, const Coef* coef, int pre, int post, int first, void* u, const void* r,
                 bool form_rhs)
{
    if (g->dtype == FAS_F64)
        launch_t<double>(g, top, coef, pre, post, first, u, r, form_rhs ? 1 : 0);
    else
        launch_t<float>(g, top, coef, pre, post, first, u, r, form_rhs ? 1 : 0);
}

}  // namespace fas
