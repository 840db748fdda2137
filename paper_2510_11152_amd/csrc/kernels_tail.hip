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
constexpr int kTailLdsKV = 156 * 1024;  // cell kappa: u and f of the tail levels, and in 2D
                                        // the face weights of one level (3D: kappa per level)

template <typename T>
struct TailArgs {
    int nl;                   // levels in the tail (top .. coarsest)
    int pre, post, nuc;       // sweeps
    int first;                // parity of the first phase of a sweep
    int form_rhs;             // 1: f_top = r_top + A u_top (FAS coarse right-hand side)
    int lds_off[kMaxTail];    // element offset of u of each level; f follows u
    int kap_off[kMaxTail];    // 3D cell kappa: element offset of each level's kappa copy
    int face_off;             // 2D cell kappa: element offset of the face-weight tables
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

// 2D cell kappa: the face weights of one level, built in LDS once per visit of the level,
// so that a phase reads each face's harmonic mean instead of recomputing it (a division)
// for both of its cells.  wx[j (n0 + 1) + i] is the face between cells i - 1 and i of row j
// (i = 0 and n0: the boundary faces), wy[j n0 + i] the face between rows j - 1 and j of
// column i.  The values and argument orders are those of the per-cell gather (fas_device.h):
// across a periodic edge the face of the wrapped pair, across another edge 2 kappa of the
// cell (Dirichlet) or 0 (Neumann).
template <typename T>
__device__ void build_faces2(const Op<T>& op, const T* __restrict__ kap, T* wx, T* wy)
{
    const int n0 = op.n0, n1 = op.n1;
    const bool per = op.bc == BC_PERIODIC, dir = op.bc == BC_DIRICHLET;
    const TMap m = tmap(n0 + 1);
    for (int j = m.ty; j < n1; j += m.TY) {
        const T* const kr = kap + (size_t)j * n0;
        for (int i = m.tx; i <= n0; i += m.TX) {
            T w;
            if (i > 0 && i < n0)
                w = face_w(kr[i - 1], kr[i]);
            else if (per)
                w = face_w(kr[n0 - 1], kr[0]);
            else
                w = dir ? (T)2 * kr[i == 0 ? 0 : n0 - 1] : (T)0;
            wx[j * (n0 + 1) + i] = w;
        }
    }
    for (int j = m.ty; j <= n1; j += m.TY) {
        for (int i = m.tx; i < n0; i += m.TX) {
            T w;
            if (j > 0 && j < n1)
                w = face_w(kap[(size_t)(j - 1) * n0 + i], kap[(size_t)j * n0 + i]);
            else if (per)
                w = face_w(kap[(size_t)(n1 - 1) * n0 + i], kap[i]);
            else
                w = dir ? (T)2 * kap[(size_t)(j == 0 ? 0 : n1 - 1) * n0 + i] : (T)0;
            wy[j * n0 + i] = w;
        }
    }
}

// 2D cell kappa: neighbour values as gather2, face weights from the level's tables.
template <typename T>
__device__ __forceinline__ void gather2kv(const Op<T>& op, const T* U, const T* wx, const T* wy, int i, int j,
                                          Nbhd<T, 2>& s)
{
    gather2<T>(op, U, i, j, s);
    const int fx = j * (op.n0 + 1) + i, fy = j * op.n0 + i;
    s.w[0] = wx[fx];
    s.w[1] = wx[fx + 1];
    s.w[2] = wy[fy];
    s.w[3] = wy[fy + op.n0];
}

// Neighbourhood of cell (i, j, l) of a level held in LDS (wx, wy: the 2D cell-kappa face
// tables of that level).
template <typename T, int DIM, bool KV>
__device__ __forceinline__ void tail_gather(const Op<T>& op, const T* U, const T* wx, const T* wy, int i, int j,
                                            int l, Nbhd<T, DIM>& s)
{
    if constexpr (DIM == 2 && !KV)
        gather2<T>(op, U, i, j, s);
    else if constexpr (DIM == 2 && KV)
        gather2kv<T>(op, U, wx, wy, i, j, s);
    else
        gather<T, DIM, KV>(op, U, i, j, l, s);
}

template <typename T, int DIM, bool KV>
__device__ void tail_smooth(const Op<T>& op, T* U, const T* F, const T* wx, const T* wy, int sweeps, int first,
                            bool reverse)
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
                    tail_gather<T, DIM, KV>(op, U, wx, wy, i, j, l, nb);
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
    // cell kappa: in 2D each level's face weights are built in LDS when the level is
    // visited (from its kappa in global memory); in 3D every level's kappa is copied into
    // LDS, so the face weights of each phase read it there rather than from global memory
    constexpr bool KV2 = KV && DIM == 2;
    __shared__ __attribute__((aligned(16))) char lds[KV ? kTailLdsKV : kTailLds];
    T* base = reinterpret_cast<T*>(lds);
    auto U = [&](int l) { return base + a.lds_off[l]; };
    auto F = [&](int l) { return base + a.lds_off[l] + (a.op[l].n0 * a.op[l].n1 * a.op[l].n2); };
    // the operator of level l, its cell kappa (if any) read from the LDS copy (3D)
    auto OP = [&](int l) {
        Op<T> o = a.op[l];
        if constexpr (KV && DIM == 3) o.kap = base + a.kap_off[l];
        return o;
    };
    T* const wx = KV2 ? base + a.face_off : nullptr;  // x faces of the current level
    int faces_of = -1;  // level whose face tables are in LDS
    auto faces = [&](int l) {
        if constexpr (KV2) {
            if (faces_of != l) {
                __syncthreads();  // the previous tables' readers are done
                build_faces2<T>(a.op[l], a.op[l].kap, wx, wx + (a.op[l].n0 + 1) * a.op[l].n1);
                __syncthreads();
                faces_of = l;
            }
        }
    };
    // the y-face table of level l starts after its x faces
    auto WY = [&](int l) { return KV2 ? wx + (a.op[l].n0 + 1) * a.op[l].n1 : nullptr; };
    const int N0 = a.op[0].n0 * a.op[0].n1 * a.op[0].n2;
    for (int p = threadIdx.x; p < N0; p += kTailThreads) {
        U(0)[p] = u_top[p];
        F(0)[p] = r_top[p];
    }
    if constexpr (KV && DIM == 3) {
        for (int l = 0; l < a.nl; ++l) {
            const int Nl = a.op[l].n0 * a.op[l].n1 * a.op[l].n2;
            T* const kl = base + a.kap_off[l];
            const T* const kg = a.op[l].kap;
            for (int p = threadIdx.x; p < Nl; p += kTailThreads) kl[p] = kg[p];
        }
    }
    __syncthreads();
    faces(0);
    if (a.form_rhs) {
        // f = r_c + A_c u_c
        const Op<T> op = OP(0);
        const TMap m = tmap(op.n0);
        for (int row = m.ty; row < op.n1 * op.n2; row += m.TY) {
            const int l = DIM == 3 ? row / op.n1 : 0, j = DIM == 3 ? row - l * op.n1 : row;
            for (int i = m.tx; i < op.n0; i += m.TX) {
                const int p = (int)cell_index(op.n0, op.n1, i, j, l);
                Nbhd<T, DIM> nb;
                tail_gather<T, DIM, KV>(op, U(0), wx, WY(0), i, j, l, nb);
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
        faces(lv);
        tail_smooth<T, DIM, KV>(op, u, f, wx, WY(lv), a.pre, a.first, rev);
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
                tail_gather<T, DIM, KV>(op, u, wx, WY(lv), i, j, l, nb);
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
        faces(lv + 1);
        for (int crow = m.ty; crow < oc.n1 * oc.n2; crow += m.TY)
        for (int I = m.tx; I < oc.n0; I += m.TX) {
            const int K = DIM == 3 ? crow / oc.n1 : 0, J = DIM == 3 ? crow - K * oc.n1 : crow;
            const int P = (int)cell_index(oc.n0, oc.n1, I, J, K);
            Nbhd<T, DIM> nb;
            tail_gather<T, DIM, KV>(oc, U(lv + 1), wx, WY(lv + 1), I, J, K, nb);
            F(lv + 1)[P] = F(lv + 1)[P] + apply_value<T, DIM, KV>(oc, nb, U(lv + 1)[P]);
        }
        __syncthreads();
    }
    // coarsest level: smoothing only (Remark 1)
    faces(a.nl - 1);
    tail_smooth<T, DIM, KV>(OP(a.nl - 1), U(a.nl - 1), F(a.nl - 1), wx, WY(a.nl - 1), a.nuc, a.first, rev);
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
        faces(lv);
        tail_smooth<T, DIM, KV>(op, u, F(lv), wx, WY(lv), a.post, a.first, rev);
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
    a.face_off = off;
    if (kv && g->dim == 2) {
        // 2D cell kappa: the face tables of one level, sized for the top level
        off += (int)((g->lev[top].n[0] + 1) * g->lev[top].n[1] + g->lev[top].n[0] * (g->lev[top].n[1] + 1));
    } else {
        for (int i = 0; i < a.nl; ++i) {  // 3D cell kappa: copies after every level's u and f
            a.kap_off[i] = off;
            if (kv) off += (int)g->lev[top + i].N;
        }
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
    // the largest level from which every coarser level's u and f (and, on a grid that may
    // take a cell kappa, the top level's face tables in 2D or every level's kappa in 3D) fit
    // the tail's LDS; the budgets admit the same levels
    const size_t s = g->elem();
    const bool kv = (g->flags & FAS_FLAG_VARIABLE_KAPPA) != 0;
    const size_t cap = kv ? (size_t)kTailLdsKV : (size_t)kTailLds;
    size_t bytes = 0;
    int top = g->L + 1;
    for (int l = g->L; l >= 0; --l) {
        bytes += (kv && g->dim == 3 ? 3 : 2) * (size_t)g->lev[l].N * s;
        const int64_t n0 = g->lev[l].n[0], n1 = g->lev[l].n[1];
        const size_t faces = kv && g->dim == 2 ? (size_t)((n0 + 1) * n1 + n0 * (n1 + 1)) * s : 0;
        if (bytes + faces > cap || g->L - l + 1 > kMaxTail) break;
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
