// Fused 2D pre/post passes as block tiles: the default fused pass on every 2D level
// (constant or cell kappa).
//
// A block of WV waves holds a whole tile in registers at once: the 128-column window of
// a strip (one cell pair per lane, x-neighbours by DPP, 112 columns written) and four
// (FP64) or eight (FP32) consecutive rows per wave.  The pass runs colour phase by colour
// phase; before each phase every wave trades the top and bottom rows of its band through
// LDS (one barrier), then updates its cells of that colour.  All loads of a tile are issued together, so
// the tile waits on memory once, and the halo rows that neighbouring tiles share are
// read close together in time from the same XCD's L2.  The wave-strip marches
// (strip_march.h) instead visit a segment's rows one after another, so their launches
// last at least (segment + halo) dependent row steps, which on small levels is most of
// their time; on large levels they keep only a few rows of loads in flight per wave.
// The marches remain for passes without sweeps.
//
// Halo: the values valid after colour phase s are those at least s cells inside the
// loaded window (the residual needs one more), so the tile recomputes H rows above and
// below (2nu + 2 for passes that take the residual, else 2nu) and 8 columns on each side.
//
// The passes are those of the strips (Alg. 1): pre = nu X-MCGS sweeps, then
// u_c = R u and r_c = R(f - A u), optionally forming the FAS right-hand side f = r + A u
// first, or summing f^2 per tile (a solve's first pass), or starting from u = 0 without
// reading it (the first inner cycle of a defect correction); post = u += P(u_c - R u), nu
// sweeps, optionally one sum of r^2 per tile, and in its accumulating form (FP32 only)
// adding the result into an FP64 array instead of storing it (the last inner cycle of a
// defect correction: the outer update u64 += fp64(e)).  The point formulas and their evaluation
// trees are those of fas_device.h, so every value is bit-identical to the strip and
// per-phase kernels.
#include <hip/hip_runtime.h>
#include <string.h>

#include "fas_batch.h"
#include "fas_device.h"
#include "fas_fused.h"
#include "fas_internal.h"
#include "march_util.h"

namespace fas {

namespace {

// Rows of the tile each wave holds: 4 in FP64, 8 in FP32 (half the registers per row).
// Taller tiles recompute fewer halo rows; FP64 has the registers for 4 rows at three
// 8-wave blocks per compute unit.
template <typename T>
constexpr int rows_per_wave()
{
    return sizeof(T) == 8 ? 4 : 8;
}
constexpr int kTileHX = 8;                  // halo columns each side

// Halo rows above and below a tile: 2nu phases, one more for a residual, rounded up to
// even (row pairs form coarse rows, and a row's parity fixes its colour).
constexpr int tile_halo(int nu, bool residual)
{
    return residual ? 2 * nu + 2 : 2 * nu;
}
constexpr int kTileCols = 128 - 2 * kTileHX;
static_assert(kTileCols == kStripCols, "tile columns match the strips");
constexpr int kMaxTileWaves = 16;
constexpr int kMaxTileWavesKV = 8;  // cell kappa: more registers per lane

template <typename T>
struct TileArgs {
    int n0, n1;          // level size (even)
    int bc;
    T k;                 // dt*kappa/h^2 of the level
    T q[16];             // 1/(1 + k W)
    int strips, tiles_y; // tiles across x and along y
    int group;           // strips per group of the tile order (tile_coords)
    int tile_rows;       // rows written per tile: WV * rows_per_wave - 2 * halo (even)
    const T* f;
    const T* u_in;
    T* u_out;
    T* uc;               // pre: R u out;  post: new coarse values in
    T* rc;               // pre: R r out
    T* fout;             // pre forming the right-hand side (f then holds r): f = r + A u out
    double* partials;    // one sum per tile (nullable): post r^2, pre f^2
    double* u64;         // accumulating post pass: u64 += fp64(result) on the written cells
    const T* kap;        // cell kappa of the level (single-problem grids), else nullptr
    int batch;           // problems; problem b's arrays start b * stride (b * cstride coarse)
    int64_t stride, cstride;
    const int* act;      // per-problem active flags (nullable)
};

// Tile t of a problem -> (strip, tile row).  Tiles are walked in groups of up to `group`
// strips, down the tile rows of a group, so the tiles that share halo rows above and
// below run within a few tiles of each other (and, with xcd_block, on the same XCD)
// rather than a whole row of tiles apart.  A bijection on [0, strips * tiles_y).
constexpr int kTileGroup = 16;  // strips per group unless tuned

__device__ __forceinline__ void tile_coords(int t, int strips, int tiles_y, int group, int& strip, int& ty)
{
    const int K = strips < group ? strips : group;
    const int span = K * tiles_y, gi = t / span, within = t % span;
    const int width = strips - gi * K < K ? strips - gi * K : K;  // the last group may be narrower
    ty = within / width;
    strip = gi * K + within % width;
}

// LDS of a block: two exchange buffers of WV x (top, bottom) rows of u, one of kappa
// (cell kappa), then WV wave sums.
template <typename T>
size_t tile_lds_bytes(int wv, bool kv)
{
    return (kv ? 3 : 2) * (size_t)wv * 128 * sizeof(typename Pair<T>::V) + (size_t)wv * sizeof(double);
}

// Pass kinds: MODE 0 pre, 1 post, 2 accumulating post; IN selects how the pre pass
// starts: from u_in (IN_U), forming the right-hand side first (IN_RHS) or from zero
// (IN_ZERO, u_in not read).
enum { IN_U = 0, IN_RHS = 1, IN_ZERO = 2 };

// One tile of problem b (tile t of per).  XE: the window reaches past a domain x-edge
// (columns are wrapped, or zero and never updated, and edge cells have their own
// diagonal counts); the other tiles run without any of that, which keeps the diagonal
// coefficients in scalar registers.
template <typename T, int NU, int MODE, bool NORM, int IN, bool KV, int FIRST, bool XE>
__device__ __forceinline__ void tile_pass(const TileArgs<T>& a, int b, int t, int per)
{
    using V = typename Pair<T>::V;
    constexpr bool RHS = IN == IN_RHS;
    constexpr bool POST = MODE >= 1;
    static_assert(IN == IN_U || MODE == 0, "only a pre pass forms f or starts from zero");
    static_assert(MODE != 2 || sizeof(T) == 4, "the accumulating pass adds FP32 results into FP64");
    constexpr bool RES = MODE == 0 || NORM;  // the pass takes the residual
    constexpr int S = 2 * NU, H = tile_halo(NU, RES), B = rows_per_wave<T>();
    static_assert(NU >= 1 && H <= kTileHX, "halo columns");
    extern __shared__ __attribute__((aligned(16))) char tile_lds[];
    const int WV = blockDim.x >> 6;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    V* const xch = reinterpret_cast<V*>(tile_lds);
    V* const kxch = xch + 2 * WV * 128;  // cell kappa: band edges (traded once)
    double* const red = reinterpret_cast<double*>(tile_lds + (KV ? 3 : 2) * (size_t)WV * 128 * sizeof(V));

    const T* const f = a.f + b * a.stride;
    const T* const u_in = a.u_in + b * a.stride;
    T* const u_out = a.u_out + b * a.stride;

    int strip, ty;
    tile_coords(t, a.strips, a.tiles_y, a.group, strip, ty);
    const int x0 = strip * kTileCols, y0 = ty * a.tile_rows;
    const int yend = min(y0 + a.tile_rows, a.n1);  // rows written: [y0, yend)
    const int gxe = x0 - kTileHX + 2 * lane;       // even cell of this lane
    const int rb = y0 - H + w * B;                 // row of the wave's first row (even)
    const bool periodic = a.bc == BC_PERIODIC;
    // A window reaches at most 8 columns / H rows before the domain and less than one
    // domain size past it (levels are at least 128 x 64), so one wrap step is enough.
    const bool xin = !XE || periodic || (gxe >= 0 && gxe < a.n0);
    const int gxl = !XE ? gxe
                        : periodic ? gxe + (gxe < 0 ? a.n0 : 0) - (gxe >= a.n0 ? a.n0 : 0)
                                   : min(max(gxe, 0), a.n0 - 2);
    const bool own = lane >= kTileHX / 2 && lane < 64 - kTileHX / 2 && (!XE || gxe < a.n0);  // writes this pair
    // boundary faces across x of the even / odd cell (n0 even: a pair is in or out)
    const bool bxe = XE && !periodic && gxe == 0;
    const bool bxo = XE && !periodic && gxe + 2 == a.n0;
    const bool dir = a.bc == BC_DIRICHLET;
    const T k = a.k;
    // diagonal count W (and q[W]) of a cell with no, one or two boundary faces
    const T qA = a.q[4], qB = dir ? a.q[5] : a.q[3], qC = dir ? a.q[6] : a.q[2];
    const T wA = (T)4, wB = dir ? (T)5 : (T)3, wC = dir ? (T)6 : (T)2;
    const T kdir = dir ? (T)2 : (T)0;  // cell kappa: a boundary face weighs kdir * kappa_p
    const int mc0 = a.n0 >> 1;

    T ue[B], uo[B], fe[B], fo[B];
    T ke[KV ? B : 1], ko[KV ? B : 1];
    T cr[B / 2];
    bool yin[B], yb[B], ys[B], yn[B];
#pragma unroll
    for (int r = 0; r < B; ++r) {
        const int gy = rb + r;
        const bool in = periodic || (gy >= 0 && gy < a.n1);
        const int gl = periodic ? gy + (gy < 0 ? a.n1 : 0) - (gy >= a.n1 ? a.n1 : 0) : min(max(gy, 0), a.n1 - 1);
        yin[r] = in;
        ys[r] = !periodic && gy == 0;
        yn[r] = !periodic && gy == a.n1 - 1;
        yb[r] = ys[r] || yn[r];
        // uniform row base plus a 32-bit lane offset
        const int64_t row = (int64_t)gl * a.n0;
        V zu;
        if constexpr (IN == IN_ZERO) {
            zu.x = (T)0;
            zu.y = (T)0;
        } else {
            zu = *reinterpret_cast<const V*>(u_in + row + (unsigned)gxl);
        }
        const V zf = *reinterpret_cast<const V*>(f + row + (unsigned)gxl);
        const bool c = in && xin;  // outside a non-periodic domain: 0, never updated
        ue[r] = c ? zu.x : (T)0;
        uo[r] = c ? zu.y : (T)0;
        fe[r] = c ? zf.x : (T)0;
        fo[r] = c ? zf.y : (T)0;
        if constexpr (KV) {
            const V zk = *reinterpret_cast<const V*>(a.kap + row + (unsigned)gxl);
            ke[r] = c ? zk.x : (T)0;
            ko[r] = c ? zk.y : (T)0;
        }
        if constexpr (POST) {
            if ((r & 1) == 0) cr[r >> 1] = a.uc[b * a.cstride + (int64_t)(gl >> 1) * mc0 + (gxl >> 1)];
        }
    }
    if constexpr (POST) {
        // fine grid correction u += P(u_c - R u) on every 2 x 2 block held (rows 2m, 2m + 1)
#pragma unroll
        for (int m = 0; m < B / 2; ++m) {
            const T old = restrict4(ue[2 * m], uo[2 * m], ue[2 * m + 1], uo[2 * m + 1]);
            const T c = cr[m] - old;
            const bool apply = yin[2 * m] && xin;
            ue[2 * m] = apply ? ue[2 * m] + c : ue[2 * m];
            uo[2 * m] = apply ? uo[2 * m] + c : uo[2 * m];
            ue[2 * m + 1] = apply ? ue[2 * m + 1] + c : ue[2 * m + 1];
            uo[2 * m + 1] = apply ? uo[2 * m + 1] + c : uo[2 * m + 1];
        }
    }

    // The row above the wave's band (bottom row of wave w - 1) and the row below it (top
    // row of wave w + 1), as they stand after the last phase.  Exchange e writes buffer
    // e & 1: a wave can only overwrite a buffer after the next barrier, which every wave
    // passes only once it has read that buffer.
    V up, dn;
    auto exchange = [&](int e) {
        V* const buf = xch + (e & 1) * (WV * 128);
        V top, bot;
        top.x = ue[0];
        top.y = uo[0];
        bot.x = ue[B - 1];
        bot.y = uo[B - 1];
        buf[w * 128 + lane] = top;
        buf[w * 128 + 64 + lane] = bot;
        __syncthreads();
        up.x = (T)0;
        up.y = (T)0;
        dn = up;
        if (w > 0) up = buf[(w - 1) * 128 + 64 + lane];
        if (w < WV - 1) dn = buf[(w + 1) * 128 + lane];
    };
    // Cell kappa: the kappa rows above and below the band, read once.
    V kup, kdn;
    if constexpr (KV) {
        V top, bot;
        top.x = ke[0];
        top.y = ko[0];
        bot.x = ke[B - 1];
        bot.y = ko[B - 1];
        kxch[w * 128 + lane] = top;
        kxch[w * 128 + 64 + lane] = bot;
    }
    // Cell kappa: weighted neighbour sum Sw and weight total Wt of the even (EVEN) or odd
    // cell of row r, with the face weights and boundary faces of fas_device.h's gather
    // (slot order x-, x+, y-, y+; a boundary face weighs kdir * kappa_p).
    auto kv_terms = [&](bool even, int r, T& Sw, T& Wt) {
        if (even) {
            const T kp = ke[r], uw = dpp_move<kShr1>(uo[r]), kw = dpp_move<kShr1>(ko[r]);
            const T uem = r > 0 ? ue[r - 1] : up.x, uep = r < B - 1 ? ue[r + 1] : dn.x;
            const T kem = r > 0 ? ke[r - 1] : kup.x, kep = r < B - 1 ? ke[r + 1] : kdn.x;
            const T wb = kdir * kp;
            const T w0 = bxe ? wb : face_w(kw, kp);
            const T w1 = face_w(kp, ko[r]);
            const T w2 = ys[r] ? wb : face_w(kem, kp);
            const T w3 = yn[r] ? wb : face_w(kp, kep);
            Sw = (w0 * uw + w1 * uo[r]) + (w2 * uem + w3 * uep);
            Wt = (w0 + w1) + (w2 + w3);
        } else {
            const T kp = ko[r], uE = dpp_move<kShl1>(ue[r]), kE = dpp_move<kShl1>(ke[r]);
            const T uom = r > 0 ? uo[r - 1] : up.y, uop = r < B - 1 ? uo[r + 1] : dn.y;
            const T kom = r > 0 ? ko[r - 1] : kup.y, kop = r < B - 1 ? ko[r + 1] : kdn.y;
            const T wb = kdir * kp;
            const T w0 = face_w(ke[r], kp);
            const T w1 = bxo ? wb : face_w(kp, kE);
            const T w2 = ys[r] ? wb : face_w(kom, kp);
            const T w3 = yn[r] ? wb : face_w(kp, kop);
            Sw = (w0 * ue[r] + w1 * uE) + (w2 * uom + w3 * uop);
            Wt = (w0 + w1) + (w2 + w3);
        }
    };
    // Neighbour sums and diagonal counts (weighted, with cell kappa) of both cells of
    // row r: A u = u + k (W u - S).
    auto terms = [&](int r, T& Se, T& So, T& We, T& Wo) {
        if constexpr (KV) {
            kv_terms(true, r, Se, We);
            kv_terms(false, r, So, Wo);
        } else {
            const T uem = r > 0 ? ue[r - 1] : up.x, uep = r < B - 1 ? ue[r + 1] : dn.x;
            const T uom = r > 0 ? uo[r - 1] : up.y, uop = r < B - 1 ? uo[r + 1] : dn.y;
            const T wv = dpp_move<kShr1>(uo[r]);
            const T ev = dpp_move<kShl1>(ue[r]);
            Se = (wv + uo[r]) + (uem + uep);
            So = (ue[r] + ev) + (uom + uop);
            We = sel3(bxe, yb[r], wA, wB, wC);
            Wo = sel3(bxo, yb[r], wA, wB, wC);
        }
    };

    exchange(0);  // its barrier also publishes the kappa edges
    if constexpr (KV) {
        kup.x = (T)0;
        kup.y = (T)0;
        kdn = kup;
        if (w > 0) kup = kxch[(w - 1) * 128 + 64 + lane];
        if (w < WV - 1) kdn = kxch[(w + 1) * 128 + lane];
    }
    if constexpr (RHS) {
        // FAS right-hand side from the initial values: f = r + A u
#pragma unroll
        for (int r = 0; r < B; ++r) {
            T Se, So, We, Wo;
            terms(r, Se, So, We, Wo);
            fe[r] = fe[r] + (ue[r] + k * (We * ue[r] - Se));
            fo[r] = fo[r] + (uo[r] + k * (Wo * uo[r] - So));
            const int gy = rb + r;
            if (gy >= y0 && gy < yend && own)
                store_pair_nt(a.fout + b * a.stride + (int64_t)gy * a.n0 + gxe, fe[r], fo[r]);
        }
    }
    // colour phases; phase s updates the cells with (i + j) & 1 == colour
#pragma unroll
    for (int s = 1; s <= S; ++s) {
        if (s > 1) exchange(s - 1);
        const int colour = ((s - 1) & 1) ^ FIRST;
#pragma unroll
        for (int r = 0; r < B; ++r) {
            const bool upd = yin[r] && xin;
            if constexpr (KV) {
                const bool even = ((r & 1) ^ colour) == 0;
                T Sw, Wt;
                kv_terms(even, r, Sw, Wt);
                if (even) {
                    const T nv = (fe[r] + k * Sw) / ((T)1 + k * Wt);
                    ue[r] = upd ? nv : ue[r];
                } else {
                    const T nv = (fo[r] + k * Sw) / ((T)1 + k * Wt);
                    uo[r] = upd ? nv : uo[r];
                }
            } else if (((r & 1) ^ colour) == 0) {  // the even cell of the pair (rb is even)
                const T uem = r > 0 ? ue[r - 1] : up.x, uep = r < B - 1 ? ue[r + 1] : dn.x;
                const T wv = dpp_move<kShr1>(uo[r]);
                const T Ssum = (wv + uo[r]) + (uem + uep);
                const T qv = sel3(bxe, yb[r], qA, qB, qC);
                const T nv = (fe[r] + k * Ssum) * qv;
                ue[r] = upd ? nv : ue[r];
            } else {
                const T uom = r > 0 ? uo[r - 1] : up.y, uop = r < B - 1 ? uo[r + 1] : dn.y;
                const T ev = dpp_move<kShl1>(ue[r]);
                const T Ssum = (ue[r] + ev) + (uom + uop);
                const T qv = sel3(bxo, yb[r], qA, qB, qC);
                const T nv = (fo[r] + k * Ssum) * qv;
                uo[r] = upd ? nv : uo[r];
            }
        }
    }
    // final rows: write them, and take the residual (restriction or norm) row by row
    if constexpr (RES) exchange(S);
    double acc = 0.0;
    T re_prev = (T)0, ro_prev = (T)0;
#pragma unroll
    for (int r = 0; r < B; ++r) {
        T re = (T)0, ro = (T)0;
        if constexpr (RES) {
            T Se, So, We, Wo;
            terms(r, Se, So, We, Wo);
            re = fe[r] - (ue[r] + k * (We * ue[r] - Se));
            ro = fo[r] - (uo[r] + k * (Wo * uo[r] - So));
        }
        const int gy = rb + r;
        if (gy >= y0 && gy < yend && own) {
            if constexpr (MODE == 2) {
                // u64 += fp64(u) on the written cells (no other tile writes them)
                double* const q = a.u64 + b * a.stride + (int64_t)gy * a.n0 + gxe;
                const double2 o = *reinterpret_cast<const double2*>(q);
                store_pair_nt(q, o.x + (double)ue[r], o.y + (double)uo[r]);
            } else {
                store_pair_nt(u_out + (int64_t)gy * a.n0 + gxe, ue[r], uo[r]);
            }
            if constexpr (MODE == 0) {
                // rows (r - 1, r) form coarse row gy / 2 when r is odd (y0, yend even)
                if (r & 1) {
                    const T ucv = restrict4(ue[r - 1], uo[r - 1], ue[r], uo[r]);
                    const T rcv = restrict4(re_prev, ro_prev, re, ro);
                    const int64_t P = b * a.cstride + (int64_t)(gy >> 1) * mc0 + (gxe >> 1);
                    __builtin_nontemporal_store(ucv, a.uc + P);
                    __builtin_nontemporal_store(rcv, a.rc + P);
                }
            }
            if constexpr (NORM && MODE == 0) {  // pre: the right-hand side's f^2
                acc += (double)fe[r] * (double)fe[r];
                acc += (double)fo[r] * (double)fo[r];
            } else if constexpr (NORM) {
                acc += (double)re * (double)re;
                acc += (double)ro * (double)ro;
            }
        }
        re_prev = re;
        ro_prev = ro;
    }
    if constexpr (NORM) {
        // fixed butterfly over the lanes, then the waves in order
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (lane == 0) red[w] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int i = 0; i < WV; ++i) s += red[i];
            a.partials[(int64_t)b * per + t] = s;
        }
    }
}

template <typename T, int NU, int MODE, bool NORM, int IN, bool KV, int FIRST>
__global__ __launch_bounds__(64 * (KV ? kMaxTileWavesKV : kMaxTileWaves)) void k_tile(TileArgs<T> a)
{
    // neighbouring tiles, which share halo cells, run on one XCD
    const int blk = (int)xcd_block(blockIdx.x, gridDim.x);
    const int per = a.strips * a.tiles_y;
    const int b = blk / per, t = blk % per;
    if (b >= a.batch || (a.act && !a.act[b])) return;  // uniform over the block
    int strip, ty;
    tile_coords(t, a.strips, a.tiles_y, a.group, strip, ty);
    const int x0 = strip * kTileCols;
    if (x0 - kTileHX < 0 || x0 - kTileHX + 128 >= a.n0)
        tile_pass<T, NU, MODE, NORM, IN, KV, FIRST, true>(a, b, t, per);
    else
        tile_pass<T, NU, MODE, NORM, IN, KV, FIRST, false>(a, b, t, per);
}

// Table launches (array-form batches, fas_batch.h): the launch's blocks are renumbered
// over the XCDs as one range, the problem is the one whose block range holds the block,
// and its arguments come from its descriptor.  A pre-pass descriptor with fout forms the
// FAS right-hand side, one with partials sums f^2 per tile; a post-pass descriptor with
// partials sums the residual's squares per tile.
template <typename T, int NU, bool POSTP, bool KV, int FIRST>
__global__ __launch_bounds__(64 * (KV ? kMaxTileWavesKV : kMaxTileWaves)) void k_tile_table(TableLaunch tl)
{
    const int blk = (int)xcd_block(blockIdx.x, gridDim.x);
    int lo = 0, hi = tl.np - 1;  // the problem p with first[p] <= blk < first[p + 1]
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (blk >= tl.first[mid])
            lo = mid;
        else
            hi = mid - 1;
    }
    const TileArgs<T> a = *reinterpret_cast<const TileArgs<T>*>(tl.desc[lo]);
    if (a.act && !a.act[0]) return;  // uniform over the block
    const int per = a.strips * a.tiles_y;
    const int t = blk - tl.first[lo];
    int strip, ty;
    tile_coords(t, a.strips, a.tiles_y, a.group, strip, ty);
    const int x0 = strip * kTileCols;
    const bool xe = x0 - kTileHX < 0 || x0 - kTileHX + 128 >= a.n0;
#define FAS_TILE_PASS(MODE_, NORM_, IN_)                                        \
    do {                                                                        \
        if (xe)                                                                 \
            tile_pass<T, NU, MODE_, NORM_, IN_, KV, FIRST, true>(a, 0, t, per);  \
        else                                                                    \
            tile_pass<T, NU, MODE_, NORM_, IN_, KV, FIRST, false>(a, 0, t, per); \
    } while (0)
    if constexpr (POSTP) {
        if (a.partials)
            FAS_TILE_PASS(1, true, IN_U);
        else
            FAS_TILE_PASS(1, false, IN_U);
    } else {
        if (a.fout)
            FAS_TILE_PASS(0, false, IN_RHS);
        else if (a.partials)
            FAS_TILE_PASS(0, true, IN_U);
        else
            FAS_TILE_PASS(0, false, IN_U);
    }
#undef FAS_TILE_PASS
}

inline void check_launch()
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error(FAS_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
}

template <typename T, bool POSTP, bool KV>
void launch_tile_table_t(hipStream_t stream, int nu, int first, int wv, const TableLaunch& t)
{
    const unsigned blocks = (unsigned)t.first[t.np];
    const unsigned threads = 64u * (unsigned)wv;
    const size_t lds = tile_lds_bytes<T>(wv, KV);
#define FAS_TT_LAUNCH(NU_)                                                                       \
    (first ? k_tile_table<T, NU_, POSTP, KV, 1><<<blocks, threads, lds, stream>>>(t)             \
           : k_tile_table<T, NU_, POSTP, KV, 0><<<blocks, threads, lds, stream>>>(t))
    switch (nu) {
        case 1: FAS_TT_LAUNCH(1); break;
        case 2: FAS_TT_LAUNCH(2); break;
        case 3: FAS_TT_LAUNCH(3); break;
        default: throw Error(FAS_ERR_ARG, "tile kernels take 1 <= nu <= 3");
    }
#undef FAS_TT_LAUNCH
    check_launch();
}

template <typename T, int MODE, bool NORM, int IN, bool KV>
void launch_tile_kv(const fas_grid* g, const TileArgs<T>& a, int nu, int first, int wv)
{
    const unsigned blocks = (unsigned)((int64_t)a.batch * a.strips * a.tiles_y);
    const unsigned threads = 64u * (unsigned)wv;
    const size_t lds = tile_lds_bytes<T>(wv, KV);
#define FAS_TILE_LAUNCH(NU_)                                                                     \
    (first ? k_tile<T, NU_, MODE, NORM, IN, KV, 1><<<blocks, threads, lds, g->stream>>>(a)       \
           : k_tile<T, NU_, MODE, NORM, IN, KV, 0><<<blocks, threads, lds, g->stream>>>(a))
    switch (nu) {
        case 1: FAS_TILE_LAUNCH(1); break;
        case 2: FAS_TILE_LAUNCH(2); break;
        case 3: FAS_TILE_LAUNCH(3); break;
        default: throw Error(FAS_ERR_ARG, "tile kernels take 1 <= nu <= 3");
    }
#undef FAS_TILE_LAUNCH
    check_launch();
}

template <typename T, int MODE, bool NORM, int IN>
void launch_tile(const fas_grid* g, const TileArgs<T>& a, int nu, int first, int wv)
{
    if (a.kap)
        launch_tile_kv<T, MODE, NORM, IN, true>(g, a, nu, first, wv);
    else
        launch_tile_kv<T, MODE, NORM, IN, false>(g, a, nu, first, wv);
}

// Strips per group of level l: tuned, else the rule.
int tile_group(const fas_grid* g, int l) { return g->tile_grp[l] ? g->tile_grp[l] : kTileGroup; }

int tile_rows_of(const fas_grid* g, int wv, int nu, bool residual)
{
    return wv * (g->dtype == FAS_F64 ? rows_per_wave<double>() : rows_per_wave<float>()) - 2 * tile_halo(nu, residual);
}

template <typename T>
TileArgs<T> make_tile_args(const fas_grid* g, int l, const Coef& c, int nu, int wv, bool residual)
{
    TileArgs<T> a{};
    a.n0 = g->lev[l].n[0];
    a.n1 = g->lev[l].n[1];
    a.bc = g->bc;
    a.k = (T)c.kd;
    for (int W = 0; W < 16; ++W) a.q[W] = (T)c.q[W];
    a.strips = (a.n0 + kTileCols - 1) / kTileCols;
    a.tile_rows = tile_rows_of(g, wv, nu, residual);
    a.tiles_y = (a.n1 + a.tile_rows - 1) / a.tile_rows;
    a.group = tile_group(g, l);
    a.batch = g->batch;
    a.stride = g->lev[l].N;
    a.cstride = l < g->L ? g->lev[l + 1].N : 0;
    a.act = active_flags(g);
    a.kap = (const T*)g->lev[l].kap;  // cell kappa: single-problem grids only
    return a;
}

}  // namespace

bool tile_ok(const fas_grid* g, int l, int nu_pre, int nu_post, bool variable)
{
    if (!fused_ok(g, l, nu_pre, nu_post, variable)) return false;
    if (nu_pre < 1 || nu_post < 1) return false;
    return (int64_t)g->lev[l].n[0] * g->lev[l].n[1] <= g->tile_max;
}

int tile_waves(const fas_grid* g, int l, int nu)
{
    (void)nu;
    // forced (FAS_OPT_TILE_WAVES), else tuned (FAS_OPT_AUTOTUNE), else the rule: 8 waves,
    // two per SIMD; in FP64 (about 70 VGPRs) three blocks per compute unit
    const int w = g->tile_waves ? g->tile_waves : (g->tile_wv[l] ? g->tile_wv[l] : 8);
    if (g->lev[l].kap) return w < kMaxTileWavesKV ? w : kMaxTileWavesKV;
    return w;
}

int tile_count_with(const fas_grid* g, int l, int nu, int wv)
{
    const int rows = tile_rows_of(g, wv, nu, true);
    if (rows < 2) return -1;
    return ((g->lev[l].n[0] + kTileCols - 1) / kTileCols) * ((g->lev[l].n[1] + rows - 1) / rows);
}

int tile_count(const fas_grid* g, int l, int nu)
{
    const int rows = tile_rows_of(g, tile_waves(g, l, nu), nu, true);
    return ((g->lev[l].n[0] + kTileCols - 1) / kTileCols) * ((g->lev[l].n[1] + rows - 1) / rows);
}

void launch_tile_pre(const fas_grid* g, int l, const Coef& c, int first, int nu, const void* f, const void* u_in,
                     void* u_out, void* uc, void* rc, void* fout, double* fpartials, bool zero)
{
    if (fout && fpartials) throw Error(FAS_ERR_ARG, "internal: a pre pass forms f or sums f^2, not both");
    if (zero && (fout || fpartials || g->dtype != FAS_F32))
        throw Error(FAS_ERR_ARG, "internal: a zero-start pre pass is an FP32 pass that forms nothing else");
    const int wv = tile_waves(g, l, nu);
    if (g->dtype == FAS_F64) {
        auto a = make_tile_args<double>(g, l, c, nu, wv, true);
        a.f = (const double*)f, a.u_in = (const double*)u_in, a.u_out = (double*)u_out;
        a.uc = (double*)uc, a.rc = (double*)rc, a.fout = (double*)fout, a.partials = fpartials;
        if (fout)
            launch_tile<double, 0, false, IN_RHS>(g, a, nu, first, wv);
        else if (fpartials)
            launch_tile<double, 0, true, IN_U>(g, a, nu, first, wv);
        else
            launch_tile<double, 0, false, IN_U>(g, a, nu, first, wv);
    } else {
        auto a = make_tile_args<float>(g, l, c, nu, wv, true);
        a.f = (const float*)f, a.u_in = (const float*)u_in, a.u_out = (float*)u_out;
        a.uc = (float*)uc, a.rc = (float*)rc, a.fout = (float*)fout, a.partials = fpartials;
        if (fout)
            launch_tile<float, 0, false, IN_RHS>(g, a, nu, first, wv);
        else if (fpartials)
            launch_tile<float, 0, true, IN_U>(g, a, nu, first, wv);
        else if (zero)
            launch_tile<float, 0, false, IN_ZERO>(g, a, nu, first, wv);
        else
            launch_tile<float, 0, false, IN_U>(g, a, nu, first, wv);
    }
}

size_t tile_desc_bytes(int dtype)
{
    return dtype == FAS_F64 ? sizeof(TileArgs<double>) : sizeof(TileArgs<float>);
}

template <typename T>
int fill_tile_desc_t(const fas_grid* g, int l, const Coef& c, int nu, int wv, bool post, const void* f,
                     const void* u_in, void* u_out, void* uc, void* rc, void* fout, double* partials, const int* act,
                     void* out)
{
    TileArgs<T> a = make_tile_args<T>(g, l, c, nu, wv, !post || partials != nullptr);
    a.batch = 1;
    a.stride = 0;
    a.cstride = 0;
    a.act = act;
    a.f = (const T*)f;
    a.u_in = (const T*)u_in;
    a.u_out = (T*)u_out;
    a.uc = (T*)uc;
    a.rc = (T*)rc;
    a.fout = (T*)fout;
    a.partials = partials;
    a.u64 = nullptr;
    memcpy(out, &a, sizeof(a));
    return a.strips * a.tiles_y;
}

int fill_tile_desc(const fas_grid* g, int l, const Coef& c, int nu, int wv, bool post, const void* f,
                   const void* u_in, void* u_out, void* uc, void* rc, void* fout, double* partials, const int* act,
                   void* out)
{
    if (post && (fout || rc)) throw Error(FAS_ERR_ARG, "internal: a post pass forms no right-hand side");
    if (fout && partials) throw Error(FAS_ERR_ARG, "internal: a pre pass forms f or sums f^2, not both");
    // every array the pass reads or writes must be there (a kernel would dereference it)
    if (!f || !u_in || !u_out || !uc || (!post && !rc) || !act || u_in == u_out)
        throw Error(FAS_ERR_ARG, "internal: tile-pass descriptor with a missing or aliased array");
    if (l < 0 || l >= g->L) throw Error(FAS_ERR_ARG, "internal: tile-pass descriptor level");
    if (g->dtype == FAS_F64)
        return fill_tile_desc_t<double>(g, l, c, nu, wv, post, f, u_in, u_out, uc, rc, fout, partials, act, out);
    return fill_tile_desc_t<float>(g, l, c, nu, wv, post, f, u_in, u_out, uc, rc, fout, partials, act, out);
}

void launch_tile_table(hipStream_t stream, int dtype, bool post, int nu, int first, bool kv, int wv,
                       const TableLaunch& t)
{
    if (t.np < 1 || t.np > kBatchChunk) throw Error(FAS_ERR_ARG, "internal: table launch size");
    if (wv < 6 || wv > (kv ? kMaxTileWavesKV : kMaxTileWaves)) throw Error(FAS_ERR_ARG, "internal: tile waves");
    if (t.first[t.np] <= 0) return;
#define FAS_TT(T_, P_, K_) launch_tile_table_t<T_, P_, K_>(stream, nu, first, wv, t)
    if (dtype == FAS_F64) {
        if (post) { if (kv) FAS_TT(double, true, true); else FAS_TT(double, true, false); }
        else { if (kv) FAS_TT(double, false, true); else FAS_TT(double, false, false); }
    } else {
        if (post) { if (kv) FAS_TT(float, true, true); else FAS_TT(float, true, false); }
        else { if (kv) FAS_TT(float, false, true); else FAS_TT(float, false, false); }
    }
#undef FAS_TT
}

void launch_tile_post(const fas_grid* g, int l, const Coef& c, int first, int nu, const void* f, const void* u_in,
                      const void* uc, void* u_out, double* partials, double* u64)
{
    if (u64 && (partials || g->dtype != FAS_F32))
        throw Error(FAS_ERR_ARG, "internal: the accumulating post pass is an FP32 pass without a norm");
    const int wv = tile_waves(g, l, nu);
    if (g->dtype == FAS_F64) {
        auto a = make_tile_args<double>(g, l, c, nu, wv, partials != nullptr);
        a.f = (const double*)f, a.u_in = (const double*)u_in, a.u_out = (double*)u_out;
        a.uc = (double*)uc, a.partials = partials;
        if (partials)
            launch_tile<double, 1, true, IN_U>(g, a, nu, first, wv);
        else
            launch_tile<double, 1, false, IN_U>(g, a, nu, first, wv);
    } else {
        auto a = make_tile_args<float>(g, l, c, nu, wv, partials != nullptr);
        a.f = (const float*)f, a.u_in = (const float*)u_in, a.u_out = (float*)u_out;
        a.uc = (float*)uc, a.partials = partials, a.u64 = u64;
        if (partials)
            launch_tile<float, 1, true, IN_U>(g, a, nu, first, wv);
        else if (u64)
            launch_tile<float, 2, false, IN_U>(g, a, nu, first, wv);
        else
            launch_tile<float, 1, false, IN_U>(g, a, nu, first, wv);
    }
}

}  // namespace fas
