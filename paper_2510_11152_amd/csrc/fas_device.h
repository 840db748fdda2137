// Device-side point formulas of the FAS V-cycle (arXiv 2510.11152, Section 2.2-2.3,
// Appendix C), shared by every kernel of the library.
//
// Each formula is one fixed evaluation tree; the library is compiled with
// -ffp-contract=off, so every kernel that evaluates a given point rounds identically,
// whatever the fusion or tiling around it.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fas {

enum { BC_NEUMANN = 0, BC_DIRICHLET = 1, BC_PERIODIC = 2 };

// Operator of one level, passed by value to kernels.
//   constant kappa: A u = u + k (W u - S),   k = dt*kappa/h_l^2, S = neighbour sum,
//                   W = interior faces + 2 * Dirichlet faces; q[W] = 1/(1 + k W)
//   cell kappa:     A u = u + k (Wt u - Sw), k = dt/h_l^2, Sw = sum_f w_f u_f,
//                   Wt = sum_f w_f, w_f harmonic mean (2 kappa_p on a Dirichlet face)
template <typename T>
struct Op {
    int n0, n1, n2;  // cells per axis (n2 = 1 in 2D)
    int bc;
    T k;
    T q[16];
    const T* kap;    // cell field of this level, or nullptr
};

// Workgroups are dealt round-robin over the 8 XCDs, each with its own L2.  This renumbers
// block b of n so that each XCD takes one contiguous range of the work: neighbouring
// tiles, which read each other's halo cells, then share an L2.  A bijection on [0, n).
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned n)
{
    const unsigned per = (n + 7u) / 8u, xcd = b % 8u, idx = b / 8u;
    const unsigned full = n % 8u == 0 ? 8u : n % 8u;  // XCDs that receive `per` blocks
    return xcd < full ? xcd * per + idx : full * per + (xcd - full) * (per - 1u) + idx;
}

// Streaming store of a cell pair: outputs are written once and read by a later launch, so
// they need not displace the rows that neighbouring waves still read from the caches.
__device__ __forceinline__ void store_pair_nt(double* p, double x, double y)
{
    typedef double v2 __attribute__((ext_vector_type(2)));
    v2 v;
    v.x = x;
    v.y = y;
    __builtin_nontemporal_store(v, reinterpret_cast<v2*>(p));
}
__device__ __forceinline__ void store_pair_nt(float* p, float x, float y)
{
    typedef float v2 __attribute__((ext_vector_type(2)));
    v2 v;
    v.x = x;
    v.y = y;
    __builtin_nontemporal_store(v, reinterpret_cast<v2*>(p));
}

__device__ __forceinline__ int64_t cell_index(int n0, int n1, int i, int j, int l)
{
    return (int64_t)i + (int64_t)n0 * ((int64_t)j + (int64_t)n1 * l);
}

// Face weight between the cell on the minus side (lo) and the plus side (hi).
template <typename T>
__device__ __forceinline__ T face_w(T lo, T hi)
{
    T t = (T)2 * lo;
    t = t * hi;
    return t / (lo + hi);
}

// Neighbourhood of one cell: values v (0 across a non-periodic boundary), face weights w
// (cell kappa only) and the number of boundary faces.  Slot order: x-, x+, y-, y+, z-, z+.
template <typename T, int DIM>
struct Nbhd {
    T v[2 * DIM];
    T w[2 * DIM];
    int nout;
};

// Gather from a full level array (global memory or LDS).  Branch-free: every neighbour is
// loaded from an in-range index (wrapped on periodic grids, clamped otherwise) and a
// neighbour across a non-periodic boundary is then replaced by 0 (weight 0, or 2 kappa_p
// on a Dirichlet face) by selects, which give the same values as skipping it.
template <typename T, int DIM, bool KV>
__device__ __forceinline__ void gather(const Op<T>& op, const T* __restrict__ u, int i, int j, int l,
                                       Nbhd<T, DIM>& s)
{
    const int c[3] = {i, j, l};
    const int n[3] = {op.n0, op.n1, op.n2};
    const bool periodic = op.bc == BC_PERIODIC;
    const int64_t p = cell_index(op.n0, op.n1, i, j, l);
    T kp = (T)0;
    if constexpr (KV) kp = op.kap[p];
    const T wb = op.bc == BC_DIRICHLET ? (T)2 * kp : (T)0;  // weight of a boundary face
    s.nout = 0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int slot = 2 * a + side;
            int d[3] = {c[0], c[1], c[2]};
            const int e = c[a] + (side ? 1 : -1);
            const bool in = e >= 0 && e < n[a];
            const int wrapped = e < 0 ? n[a] - 1 : (e >= n[a] ? 0 : e);
            d[a] = periodic ? wrapped : (in ? e : c[a]);
            const bool use = periodic || in;
            const int64_t q = cell_index(op.n0, op.n1, d[0], d[1], d[2]);
            const T v = u[q];
            s.v[slot] = use ? v : (T)0;
            s.nout += use ? 0 : 1;
            if constexpr (KV) {
                const T kq = op.kap[q];
                const T w = side ? face_w(kp, kq) : face_w(kq, kp);
                s.w[slot] = use ? w : wb;
            }
        }
    }
}

template <typename T, int DIM>
__device__ __forceinline__ T nbsum(const T* v)
{
    T S = (v[0] + v[1]) + (v[2] + v[3]);
    if constexpr (DIM == 3) S = S + (v[4] + v[5]);
    return S;
}

template <typename T, int DIM>
__device__ __forceinline__ T wsum(const T* v, const T* w)
{
    T S = (w[0] * v[0] + w[1] * v[1]) + (w[2] * v[2] + w[3] * v[3]);
    if constexpr (DIM == 3) S = S + (w[4] * v[4] + w[5] * v[5]);
    return S;
}

template <typename T, int DIM>
__device__ __forceinline__ T wtot(const T* w)
{
    T S = (w[0] + w[1]) + (w[2] + w[3]);
    if constexpr (DIM == 3) S = S + (w[4] + w[5]);
    return S;
}

__device__ __forceinline__ int diag_count(int bc, int dim, int nout)
{
    return (2 * dim - nout) + (bc == BC_DIRICHLET ? 2 * nout : 0);
}

// Gauss-Seidel point update: row p of A u = f solved for u_p (eqs. FCGS-1..4 generalised).
template <typename T, int DIM, bool KV>
__device__ __forceinline__ T gs_value(const Op<T>& op, const Nbhd<T, DIM>& s, T f)
{
    if constexpr (!KV) {
        const T S = nbsum<T, DIM>(s.v);
        return (f + op.k * S) * op.q[diag_count(op.bc, DIM, s.nout)];
    } else {
        const T Sw = wsum<T, DIM>(s.v, s.w);
        const T Wt = wtot<T, DIM>(s.w);
        return (f + op.k * Sw) / ((T)1 + op.k * Wt);
    }
}

// (A u)_p.
template <typename T, int DIM, bool KV>
__device__ __forceinline__ T apply_value(const Op<T>& op, const Nbhd<T, DIM>& s, T up)
{
    if constexpr (!KV) {
        const T S = nbsum<T, DIM>(s.v);
        const T W = (T)diag_count(op.bc, DIM, s.nout);
        return up + op.k * (W * up - S);
    } else {
        const T Sw = wsum<T, DIM>(s.v, s.w);
        const T Wt = wtot<T, DIM>(s.w);
        return up + op.k * (Wt * up - Sw);
    }
}

// Restriction R (Appendix C): children summed along x, then y, then z, times 2^-d.
template <typename T>
__device__ __forceinline__ T restrict4(T x00, T x10, T x01, T x11)
{
    return ((x00 + x10) + (x01 + x11)) * (T)0.25;
}

template <typename T>
__device__ __forceinline__ T restrict8(T x000, T x100, T x010, T x110, T x001, T x101, T x011, T x111)
{
    return (((x000 + x100) + (x010 + x110)) + ((x001 + x101) + (x011 + x111))) * (T)0.125;
}

// Parity of the 0-based index sum updated first in a forward sweep: the paper's first
// sets (1-2 in 2D, 1-4 in 3D) have an odd 1-based sum; the 0-based sum differs by DIM.
template <int DIM>
__device__ __host__ __forceinline__ int first_parity()
{
    return (DIM + 1) & 1;
}

}  // namespace fas
