// Fused, temporally blocked 2D tile kernels for large levels (constant kappa).
//
// pre  (Alg. 1 pre-smoothing, fine residual, restriction): one pass reads u and f once,
//      runs nu X-MCGS sweeps on an LDS tile with a halo, writes the smoothed u to a
//      second buffer, and writes u_c = R u and r_c = R (f - A u) for the coarse level.
// post (fine grid correction and post-smoothing): one pass reads the pre-smoothed u, f
//      and the new coarse values, applies u += P(u_c - R u), runs nu sweeps, writes u
//      back, and (finest level) emits per-tile partial sums of the residual squares.
//
// Each sweep is two colour phases; a phase at radius R around the tile needs the
// previous phase valid at radius R + 1, so a tile loads a halo of H = 2 nu + 2 cells
// (even, so local and global index parity agree) and recomputes the halo cells
// redundantly.  Point formulas are those of fas_device.h, so every cell gets the same
// bits as in the one-phase-per-launch kernels.
//
// LDS layout: every row is split by the parity of the local x index, su[p][y][x >> 1]
// with p = x & 1.  A colour phase touches one x-parity per row, so lanes access
// consecutive words (no bank conflicts).
#include <hip/hip_runtime.h>

#include "fas_device.h"
#include "fas_fused.h"
#include "fas_internal.h"

namespace fas {

namespace {

constexpr int kThreads = 256;

template <typename T>
struct TileShape;
template <>
struct TileShape<double> {
    static constexpr int TX = 64, TY = 32;
};
template <>
struct TileShape<float> {
    static constexpr int TX = 64, TY = 64;
};

template <typename T>
struct FusedArgs {
    int n0, n1;        // level size
    int bc;
    T k;               // dt*kappa/h^2 of the level
    T q[16];           // 1/(1 + k W)
    int first;         // parity (0-based index sum) of the first phase of a sweep
    int tiles_x, tiles_y, per_xcd;
    const T* f;
    const T* u_in;
    T* u_out;
    T* uc;             // pre: R u out;  post: new coarse values in
    T* rc;             // pre: R r out
    double* partials;  // post: per-tile sum of r^2 (nullable)
};

// Map the block to a tile so that each XCD (blocks are dealt round-robin over 8 XCDs)
// walks a contiguous band of tiles and neighbouring tiles share its L2.
__device__ __forceinline__ int tile_of_block(int per_xcd)
{
    return (int)(blockIdx.x % 8u) * per_xcd + (int)(blockIdx.x / 8u);
}

template <typename T, int TX, int TY, int H>
struct Tile {
    static constexpr int WL = TX + 2 * H;  // loaded width (even)
    static constexpr int HL = TY + 2 * H;
    static constexpr int WH = WL / 2;
    static constexpr int WF = WL - 2;      // f is loaded one cell less on each side
    static constexpr int HF = HL - 2;
    static constexpr int WFH = WF / 2;
    T u[2][HL][WH];
    T f[2][HF][WFH];
    __device__ __forceinline__ T& U(int ly, int lx) { return u[lx & 1][ly][lx >> 1]; }
    __device__ __forceinline__ T& F(int ly, int lx) { return f[(lx - 1) & 1][ly - 1][(lx - 1) >> 1]; }
};

// Global cell of a local coordinate; periodic grids wrap, others report out-of-domain.
__device__ __forceinline__ bool map_cell(int g, int n, int bc, int& out)
{
    if (g >= 0 && g < n) {
        out = g;
        return true;
    }
    if (bc == BC_PERIODIC) {
        out = g < 0 ? g + n : g - n;
        if (out < 0 || out >= n) out = ((g % n) + n) % n;
        return true;
    }
    return false;
}

template <typename T, int TX, int TY, int H>
__device__ __forceinline__ void load_tile(Tile<T, TX, TY, H>& t, const FusedArgs<T>& a, const T* __restrict__ src,
                                          int x0, int y0)
{
    using TT = Tile<T, TX, TY, H>;
    for (int idx = threadIdx.x; idx < TT::WL * TT::HL; idx += kThreads) {
        const int ly = idx / TT::WL, lx = idx % TT::WL;
        int gx, gy;
        T v = (T)0;
        if (map_cell(x0 - H + lx, a.n0, a.bc, gx) && map_cell(y0 - H + ly, a.n1, a.bc, gy))
            v = src[(int64_t)gy * a.n0 + gx];
        t.U(ly, lx) = v;
    }
    for (int idx = threadIdx.x; idx < TT::WF * TT::HF; idx += kThreads) {
        const int ly = idx / TT::WF + 1, lx = idx % TT::WF + 1;
        int gx, gy;
        T v = (T)0;
        if (map_cell(x0 - H + lx, a.n0, a.bc, gx) && map_cell(y0 - H + ly, a.n1, a.bc, gy))
            v = a.f[(int64_t)gy * a.n0 + gx];
        t.F(ly, lx) = v;
    }
}

// Diagonal count of a cell on a non-periodic boundary tile (out-of-domain neighbours
// hold 0 in LDS, so the neighbour sum needs no change).
__device__ __forceinline__ int edge_w(const int gx, const int gy, const int n0, const int n1, const int bc)
{
    const int nout = (gx == 0) + (gx == n0 - 1) + (gy == 0) + (gy == n1 - 1);
    return (4 - nout) + (bc == BC_DIRICHLET ? 2 * nout : 0);
}

// nstage colour phases on the tile, phase s covering radius H - 1 - s.
template <typename T, int TX, int TY, int H, bool EDGE>
__device__ __forceinline__ void run_phases(Tile<T, TX, TY, H>& t, const FusedArgs<T>& a, int x0, int y0, int nstage)
{
    using TT = Tile<T, TX, TY, H>;
    const T k = a.k;
    const T q4 = a.q[4];
    for (int s = 0; s < nstage; ++s) {
        const int par = (s & 1) ? 1 - a.first : a.first;
        const int R = H - 1 - s;
        const int ylo = H - R, yhi = H + TY + R;  // rows [ylo, yhi)
        const int xlo = H - R, xhi = H + TX + R;
        const int rows = yhi - ylo;
        for (int idx = threadIdx.x; idx < rows * TT::WH; idx += kThreads) {
            const int ly = ylo + idx / TT::WH;
            const int kk = idx % TT::WH;
            const int lx = 2 * kk + ((par + ly) & 1);
            if (lx < xlo || lx >= xhi) continue;
            const int gx = x0 - H + lx, gy = y0 - H + ly;
            if constexpr (EDGE) {
                if (gx < 0 || gx >= a.n0 || gy < 0 || gy >= a.n1) continue;
            }
            const T S = (t.U(ly, lx - 1) + t.U(ly, lx + 1)) + (t.U(ly - 1, lx) + t.U(ly + 1, lx));
            T qv = q4;
            if constexpr (EDGE) qv = a.q[edge_w(gx, gy, a.n0, a.n1, a.bc)];
            t.U(ly, lx) = (t.F(ly, lx) + k * S) * qv;
        }
        __syncthreads();
    }
}

template <typename T, int TX, int TY, int H, bool EDGE>
__device__ __forceinline__ T resid_at(Tile<T, TX, TY, H>& t, const FusedArgs<T>& a, int ly, int lx, int gx, int gy)
{
    const T up = t.U(ly, lx);
    const T S = (t.U(ly, lx - 1) + t.U(ly, lx + 1)) + (t.U(ly - 1, lx) + t.U(ly + 1, lx));
    int W = 4;
    if constexpr (EDGE) W = edge_w(gx, gy, a.n0, a.n1, a.bc);
    return t.F(ly, lx) - (up + a.k * ((T)W * up - S));
}

template <typename T, int TX, int TY, int H>
__device__ __forceinline__ void store_interior(Tile<T, TX, TY, H>& t, const FusedArgs<T>& a, int x0, int y0)
{
    for (int idx = threadIdx.x; idx < TX * TY; idx += kThreads) {
        const int iy = idx / TX, ix = idx % TX;
        const int gx = x0 + ix, gy = y0 + iy;
        if (gx < a.n0 && gy < a.n1) a.u_out[(int64_t)gy * a.n0 + gx] = t.U(H + iy, H + ix);
    }
}

// A tile takes the boundary-aware path when a non-periodic boundary is within its halo.
template <int TX, int TY, int H, typename A>
__device__ __forceinline__ bool edge_tile(const A& a, int x0, int y0)
{
    return a.bc != BC_PERIODIC && (x0 - H < 0 || y0 - H < 0 || x0 + TX + H > a.n0 || y0 + TY + H > a.n1);
}

template <typename T, int TX, int TY, int H, int NU, bool EDGE>
__device__ __forceinline__ void pre_body(Tile<T, TX, TY, H>& t, const FusedArgs<T>& a, int x0, int y0)
{
    run_phases<T, TX, TY, H, EDGE>(t, a, x0, y0, 2 * NU);
    store_interior<T, TX, TY, H>(t, a, x0, y0);
    // residual at the 4 children of each coarse cell of the tile, then R u and R r
    const int mc0 = a.n0 >> 1;
    for (int idx = threadIdx.x; idx < (TX / 2) * (TY / 2); idx += kThreads) {
        const int J = idx / (TX / 2), I = idx % (TX / 2);
        const int gx = x0 + 2 * I, gy = y0 + 2 * J;
        if (gx >= a.n0 || gy >= a.n1) continue;
        const int lx = H + 2 * I, ly = H + 2 * J;
        const T r00 = resid_at<T, TX, TY, H, EDGE>(t, a, ly, lx, gx, gy);
        const T r10 = resid_at<T, TX, TY, H, EDGE>(t, a, ly, lx + 1, gx + 1, gy);
        const T r01 = resid_at<T, TX, TY, H, EDGE>(t, a, ly + 1, lx, gx, gy + 1);
        const T r11 = resid_at<T, TX, TY, H, EDGE>(t, a, ly + 1, lx + 1, gx + 1, gy + 1);
        const int64_t P = (int64_t)(gy >> 1) * mc0 + (gx >> 1);
        a.uc[P] = restrict4(t.U(ly, lx), t.U(ly, lx + 1), t.U(ly + 1, lx), t.U(ly + 1, lx + 1));
        a.rc[P] = restrict4(r00, r10, r01, r11);
    }
}

template <typename T, int NU>
__global__ __launch_bounds__(kThreads) void k_fused_pre(FusedArgs<T> a)
{
    constexpr int TX = TileShape<T>::TX, TY = TileShape<T>::TY, H = 2 * NU + 2;
    __shared__ Tile<T, TX, TY, H> t;
    const int tile = tile_of_block(a.per_xcd);
    if (tile >= a.tiles_x * a.tiles_y) return;
    const int x0 = (tile % a.tiles_x) * TX, y0 = (tile / a.tiles_x) * TY;
    load_tile<T, TX, TY, H>(t, a, a.u_in, x0, y0);
    __syncthreads();
    if (edge_tile<TX, TY, H>(a, x0, y0))
        pre_body<T, TX, TY, H, NU, true>(t, a, x0, y0);
    else
        pre_body<T, TX, TY, H, NU, false>(t, a, x0, y0);
}

template <typename T, int TX, int TY, int H, int NU, bool EDGE, bool NORM>
__device__ __forceinline__ void post_body(Tile<T, TX, TY, H>& t, const FusedArgs<T>& a, int x0, int y0, int tile,
                                          double* red)
{
    run_phases<T, TX, TY, H, EDGE>(t, a, x0, y0, 2 * NU);
    store_interior<T, TX, TY, H>(t, a, x0, y0);
    if constexpr (NORM) {
        double acc = 0.0;
        for (int idx = threadIdx.x; idx < TX * TY; idx += kThreads) {
            const int iy = idx / TX, ix = idx % TX;
            const int gx = x0 + ix, gy = y0 + iy;
            if (gx >= a.n0 || gy >= a.n1) continue;
            const T r = resid_at<T, TX, TY, H, EDGE>(t, a, H + iy, H + ix, gx, gy);
            acc += (double)r * (double)r;
        }
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int s = kThreads / 2; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) a.partials[tile] = red[0];
    }
}

template <typename T, int NU, bool NORM>
__global__ __launch_bounds__(kThreads) void k_fused_post(FusedArgs<T> a)
{
    constexpr int TX = TileShape<T>::TX, TY = TileShape<T>::TY, H = 2 * NU + 2;
    using TT = Tile<T, TX, TY, H>;
    __shared__ TT t;
    __shared__ double red[NORM ? kThreads : 1];
    const int tile = tile_of_block(a.per_xcd);
    if (tile >= a.tiles_x * a.tiles_y) return;
    const int x0 = (tile % a.tiles_x) * TX, y0 = (tile / a.tiles_x) * TY;
    load_tile<T, TX, TY, H>(t, a, a.u_in, x0, y0);
    __syncthreads();
    // u += P(u_c - R u) on every loaded coarse cell (H even: coarse cells are whole)
    const int mc0 = a.n0 >> 1, mc1 = a.n1 >> 1;
    for (int idx = threadIdx.x; idx < TT::WH * (TT::HL / 2); idx += kThreads) {
        const int cy = idx / TT::WH, cx = idx % TT::WH;
        const int lx = 2 * cx, ly = 2 * cy;
        int GX, GY;
        if (!map_cell(((x0 - H) >> 1) + cx, mc0, a.bc, GX) || !map_cell(((y0 - H) >> 1) + cy, mc1, a.bc, GY)) continue;
        const T old = restrict4(t.U(ly, lx), t.U(ly, lx + 1), t.U(ly + 1, lx), t.U(ly + 1, lx + 1));
        const T c = a.uc[(int64_t)GY * mc0 + GX] - old;
        t.U(ly, lx) = t.U(ly, lx) + c;
        t.U(ly, lx + 1) = t.U(ly, lx + 1) + c;
        t.U(ly + 1, lx) = t.U(ly + 1, lx) + c;
        t.U(ly + 1, lx + 1) = t.U(ly + 1, lx + 1) + c;
    }
    __syncthreads();
    if (edge_tile<TX, TY, H>(a, x0, y0))
        post_body<T, TX, TY, H, NU, true, NORM>(t, a, x0, y0, tile, red);
    else
        post_body<T, TX, TY, H, NU, false, NORM>(t, a, x0, y0, tile, red);
}

template <typename T>
FusedArgs<T> make_args(const fas_grid* g, int l, const Coef& c, int first)
{
    FusedArgs<T> a{};
    a.n0 = g->lev[l].n[0];
    a.n1 = g->lev[l].n[1];
    a.bc = g->bc;
    a.k = (T)c.kd;
    for (int W = 0; W < 16; ++W) a.q[W] = (T)c.q[W];
    a.first = first;
    a.tiles_x = (a.n0 + TileShape<T>::TX - 1) / TileShape<T>::TX;
    a.tiles_y = (a.n1 + TileShape<T>::TY - 1) / TileShape<T>::TY;
    a.per_xcd = (a.tiles_x * a.tiles_y + 7) / 8;
    return a;
}

inline void check_launch()
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error(FAS_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
}

template <typename T, int NU>
void pre_nu(const fas_grid* g, FusedArgs<T>& a)
{
    k_fused_pre<T, NU><<<(unsigned)a.per_xcd * 8u, kThreads, 0, g->stream>>>(a);
}

template <typename T, int NU>
void post_nu(const fas_grid* g, FusedArgs<T>& a, bool norm)
{
    if (norm)
        k_fused_post<T, NU, true><<<(unsigned)a.per_xcd * 8u, kThreads, 0, g->stream>>>(a);
    else
        k_fused_post<T, NU, false><<<(unsigned)a.per_xcd * 8u, kThreads, 0, g->stream>>>(a);
}

template <typename T>
void pre_dispatch(const fas_grid* g, FusedArgs<T>& a, int nu)
{
    switch (nu) {
        case 0: pre_nu<T, 0>(g, a); break;
        case 1: pre_nu<T, 1>(g, a); break;
        case 2: pre_nu<T, 2>(g, a); break;
        case 3: pre_nu<T, 3>(g, a); break;
        default: throw Error(FAS_ERR_ARG, "fused kernels take nu <= 3");
    }
}

template <typename T>
void post_dispatch(const fas_grid* g, FusedArgs<T>& a, int nu, bool norm)
{
    switch (nu) {
        case 0: post_nu<T, 0>(g, a, norm); break;
        case 1: post_nu<T, 1>(g, a, norm); break;
        case 2: post_nu<T, 2>(g, a, norm); break;
        case 3: post_nu<T, 3>(g, a, norm); break;
        default: throw Error(FAS_ERR_ARG, "fused kernels take nu <= 3");
    }
}

}  // namespace

bool fused_ok(const fas_grid* g, int l, int nu_pre, int nu_post, bool variable)
{
    if (!g->fused || g->dim != 2 || variable || l >= g->L) return false;
    if (nu_pre > 3 || nu_post > 3) return false;
    // worthwhile once the level spans a few tiles
    return g->lev[l].n[0] >= 64 && g->lev[l].n[1] >= 32;
}

int fused_tiles(const fas_grid* g, int l)
{
    const int TX = g->dtype == FAS_F64 ? TileShape<double>::TX : TileShape<float>::TX;
    const int TY = g->dtype == FAS_F64 ? TileShape<double>::TY : TileShape<float>::TY;
    const int tx = (g->lev[l].n[0] + TX - 1) / TX, ty = (g->lev[l].n[1] + TY - 1) / TY;
    return tx * ty;
}

void launch_fused_pre(const fas_grid* g, int l, const Coef& c, int first, int nu, const void* f, const void* u_in,
                      void* u_out, void* uc, void* rc)
{
    if (g->dtype == FAS_F64) {
        auto a = make_args<double>(g, l, c, first);
        a.f = (const double*)f, a.u_in = (const double*)u_in, a.u_out = (double*)u_out;
        a.uc = (double*)uc, a.rc = (double*)rc;
        pre_dispatch<double>(g, a, nu);
    } else {
        auto a = make_args<float>(g, l, c, first);
        a.f = (const float*)f, a.u_in = (const float*)u_in, a.u_out = (float*)u_out;
        a.uc = (float*)uc, a.rc = (float*)rc;
        pre_dispatch<float>(g, a, nu);
    }
    check_launch();
}

void launch_fused_post(const fas_grid* g, int l, const Coef& c, int first, int nu, const void* f, const void* u_in,
                       const void* uc, void* u_out, double* partials)
{
    if (g->dtype == FAS_F64) {
        auto a = make_args<double>(g, l, c, first);
        a.f = (const double*)f, a.u_in = (const double*)u_in, a.u_out = (double*)u_out;
        a.uc = (double*)uc, a.partials = partials;
        post_dispatch<double>(g, a, nu, partials != nullptr);
    } else {
        auto a = make_args<float>(g, l, c, first);
        a.f = (const float*)f, a.u_in = (const float*)u_in, a.u_out = (float*)u_out;
        a.uc = (float*)uc, a.partials = partials;
        post_dispatch<float>(g, a, nu, partials != nullptr);
    }
    check_launch();
}

}  // namespace fas
