// Fused, temporally blocked 2D kernels for large levels (constant or cell kappa), built
// as wave-strip marches.
//
// pre  (Alg. 1 pre-smoothing, fine residual, restriction): one pass reads u and f once,
//      runs nu X-MCGS sweeps, writes the smoothed u to a second buffer, and writes
//      u_c = R u and r_c = R (f - A u) for the coarse level.  On a coarse level the
//      pass may instead read r = R(f_fine - A_fine u_fine) and form the FAS right-hand
//      side f = r + A u itself from the rows it holds (and write f for the post pass).
// post (fine grid correction and post-smoothing): one pass reads the pre-smoothed u, f
//      and the new coarse values, applies u += P(u_c - R u), runs nu sweeps, writes u
//      back and, on the finest level, one partial sum of the squared residual per wave.
//
// Geometry.  One wavefront owns a strip of 128 columns (lane k holds the cell pair
// 2k, 2k+1 of every row) and a segment of rows, which it visits top to bottom keeping
// a ring of rows in registers.  Horizontal neighbours come from the adjacent lane by a
// DPP lane shift, vertical ones from the ring, so no LDS is used.  The nu sweeps are
// pipelined over rows: when row t arrives, colour phase s (s = 1..2nu) updates row
// t - s - 1, in increasing s, which reproduces exactly the values of running the
// phases one after the other over the whole grid (the lag of one row lets the row below
// receive its coarse correction, or lets the right-hand side of a row be formed while
// its neighbours still hold their initial values).  The outer 8 columns
// on each side of the strip and H = 2nu + 2 rows above the segment are recomputed as
// halo; a strip writes 112 columns (whole 128-byte lines in FP64) and neighbouring strips
// overlap.
// Point formulas are those of fas_device.h (same bits as every other kernel).
#pragma once
#include <hip/hip_runtime.h>

#include "fas_device.h"
#include "fas_fused.h"
#include "fas_internal.h"
#include "march_util.h"

namespace fas {

namespace {

constexpr int kWaves = 4;  // independent wavefronts per block
constexpr int kThreads = 64 * kWaves;

template <typename T>
struct StripArgs {
    int n0, n1;        // level size
    int bc;
    T k;               // dt*kappa/h^2 of the level
    T q[16];           // 1/(1 + k W)
    int strips, segs;  // strips across x, row segments along y
    int seg_rows;      // rows per segment (even)
    const T* f;
    const T* u_in;
    T* u_out;
    T* uc;             // pre: R u out;  post: new coarse values in
    T* rc;             // pre: R r out
    T* fout;           // pre forming the right-hand side (f then holds r): f = r + A u out
    const T* kap;      // cell kappa of the level (variable-kappa kernels), else nullptr
    double* partials;  // post: one sum of r^2 per wave (nullable)
    int batch;         // problems; problem b's arrays start b * stride (b * cstride coarse)
    int64_t stride, cstride;
    const int* act;    // per-problem active flags (nullable)
};

template <int NU, bool KV, bool EDGE, bool FULLPF>
struct StripGeom {
    static constexpr int S = 2 * NU;         // colour phases per pass
    static constexpr int H = 2 * NU + 2;     // halo rows above the segment
    static constexpr int HX = 8;             // halo columns each side (>= H; keeps the
                                             // written columns on 128-byte lines)
    static constexpr int TXS = 128 - 2 * HX; // columns written per strip (112)
    static_assert(TXS == kStripCols, "strip width");
    static constexpr int LAG = 1;            // phases trail the newest row by one (see header)
    // rows loaded ahead: 4; 2 where kappa rows take registers, and on the few waves at a
    // domain edge of the coarser-level passes, whose selects would otherwise set the
    // register count (and so the occupancy, 3 instead of 4) of the whole kernel.  The
    // finest-level passes (FULLPF) keep 4 everywhere: there the edge waves, which finish
    // last, would cost more than the occupancy gains.
    static constexpr int PF = KV ? 2 : (EDGE && !FULLPF) ? 2 : 4;
    static constexpr int RING = S + 4 + PF;  // rows held: S + 3 + LAG + PF, even
    // rows visited per full segment: H above, the segment, S + 1 + LAG below
    static constexpr int extra = H + S + 1 + LAG;
};

// The march of one wavefront.  EDGE: the strip or segment reaches past a domain edge
// (rows/columns are wrapped for periodic grids, or zero and never updated otherwise;
// boundary cells need their own diagonal counts).  Interior waves run without any of
// that.  Loads are unconditional (boundary waves load a clamped address and select),
// so each row's loads stay in flight for PF rows.
// Per-problem arrays of a batched launch (the kernel arguments stay in place).
template <typename T>
struct Arrays {
    const T* f;
    const T* u_in;
    T* u_out;
    T* uc;
    T* rc;
    T* fout;
    const T* kap;
    double* partials;
};

template <typename T, int NU, int MODE, bool NORM, bool RHS, bool KV, bool EDGE, int FIRST>
__device__ __forceinline__ void march(const StripArgs<T>& a, const Arrays<T> A, int strip, int seg, int seg_rows,
                                      int wave_id)
{
    using G = StripGeom<NU, KV, EDGE, (MODE == 0 && !RHS) || NORM>;
    using V = typename Pair<T>::V;
    constexpr int S = G::S, H = G::H, RING = G::RING, PF = G::PF, LAG = G::LAG;
    const int lane = threadIdx.x & 63;
    const bool periodic = a.bc == BC_PERIODIC;
    const int x0 = strip * G::TXS;              // first written column
    const int gxe = x0 - G::HX + 2 * lane;      // even cell of this lane (global x)
    const int y0 = seg * seg_rows;
    const int rA = y0 - H;                      // first row visited (even)
    const int yend = min(y0 + seg_rows, a.n1);  // rows written: [y0, yend)
    const int nsteps = yend - rA + S + 1 + LAG;
    const bool own = lane >= G::HX / 2 && lane < 64 - G::HX / 2 && gxe < a.n0;  // writes this pair
    bool xin = true;
    int gxl = gxe;
    if constexpr (EDGE) {
        if (periodic) {
            gxl = wrap(gxe, a.n0);
        } else {
            xin = gxe >= 0 && gxe < a.n0;
            gxl = min(max(gxe, 0), a.n0 - 2);
        }
    }
    // boundary faces across x of the even / odd cell (n0 even: a pair is in or out)
    const bool bxe = EDGE && !periodic && gxe == 0;
    const bool bxo = EDGE && !periodic && gxe + 2 == a.n0;
    const int dsgn = a.bc == BC_DIRICHLET ? 1 : -1;
    const T k = a.k;
    const T q4 = a.q[4];
    const int mc0 = a.n0 >> 1;
    const int gcx = gxl >> 1;  // coarse column of the pair

    T ue[RING], uo[RING], fe[RING], fo[RING];
    T cr[RING];                                 // post: new coarse value of the coarse row
                                                // completed by an odd row
    T ke[KV ? RING : 1], ko[KV ? RING : 1];     // cell kappa
    T re_prev = (T)0, ro_prev = (T)0;
    double acc = 0.0;

    // global row of visited row rho and whether it is inside a non-periodic domain
    auto row_of = [&](int rho, int& gy) -> bool {
        gy = rA + rho;
        if constexpr (!EDGE) return true;
        if (gy >= 0 && gy < a.n1) return true;
        if (periodic) {
            gy = wrap(gy, a.n1);
            return true;
        }
        gy = min(max(gy, 0), a.n1 - 1);
        return false;
    };
    // load visited row rho into ring slot p (ODD: rho is odd)
    auto load_row = [&](int rho, int p, bool odd) {
        int gy;
        const bool yin = row_of(rho, gy);
        const int64_t off = (int64_t)gy * a.n0 + gxl;
        V zu = *reinterpret_cast<const V*>(A.u_in + off);
        V zf = *reinterpret_cast<const V*>(A.f + off);
        V zk{};
        if constexpr (KV) zk = *reinterpret_cast<const V*>(A.kap + off);
        T c = (T)0;
        if constexpr (MODE == 1) {
            if (odd) c = A.uc[(int64_t)(gy >> 1) * mc0 + gcx];
        }
        if constexpr (EDGE) {
            const bool in = yin && xin;
            zu.x = in ? zu.x : (T)0;
            zu.y = in ? zu.y : (T)0;
            zf.x = in ? zf.x : (T)0;
            zf.y = in ? zf.y : (T)0;
            zk.x = in ? zk.x : (T)0;
            zk.y = in ? zk.y : (T)0;
        }
        ue[p] = zu.x;
        uo[p] = zu.y;
        fe[p] = zf.x;
        fo[p] = zf.y;
        if constexpr (KV) {
            ke[p] = zk.x;
            ko[p] = zk.y;
        }
        if constexpr (MODE == 1) cr[p] = c;
    };
    // Diagonal count W of a cell (and q[W] = 1/(1 + k W)): 4, plus dsgn per boundary face
    // (n1 >= 64, so a row has at most one y-boundary face).  Only three values occur, held
    // as scalars; a cell picks one by its x-boundary face (per lane) and its row's y-boundary
    // face (uniform), which keeps these out of vector registers.
    const bool npe = EDGE && !periodic;
    const bool dir = a.bc == BC_DIRICHLET;  // uniform: constant-index picks only
    const T qA = q4, qB = npe ? (dir ? a.q[5] : a.q[3]) : q4, qC = npe ? (dir ? a.q[6] : a.q[2]) : q4;
    const T wA = (T)4, wB = npe ? (T)(4 + dsgn) : (T)4, wC = npe ? (T)(4 + 2 * dsgn) : (T)4;
    auto ybound = [&](int gy) -> bool { return EDGE && !periodic && (gy == 0 || gy == a.n1 - 1); };
    // Cell kappa: weighted neighbour sum Sw and weight total Wt of the even (EVEN) or odd
    // cell of ring slot a0 (rows am above, ap below), with the face weights and the
    // boundary faces of fas_device.h's gather (slot order x-, x+, y-, y+).
    const T kdir = a.bc == BC_DIRICHLET ? (T)2 : (T)0;  // boundary face: 2 kappa_p (Dirichlet)
    auto kv_terms = [&](bool even, int a0, int am, int ap, int gy, T& Sw, T& Wt) {
        const bool ys = EDGE && !periodic && gy == 0, yn = EDGE && !periodic && gy == a.n1 - 1;
        if (even) {
            const T kp = ke[a0], uw = dpp_move<kShr1>(uo[a0]), kw = dpp_move<kShr1>(ko[a0]);
            const T wb = kdir * kp;
            const T w0 = bxe ? wb : face_w(kw, kp);
            const T w1 = face_w(kp, ko[a0]);
            const T w2 = ys ? wb : face_w(ke[am], kp);
            const T w3 = yn ? wb : face_w(kp, ke[ap]);
            Sw = (w0 * uw + w1 * uo[a0]) + (w2 * ue[am] + w3 * ue[ap]);
            Wt = (w0 + w1) + (w2 + w3);
        } else {
            const T kp = ko[a0], ue_ = dpp_move<kShl1>(ue[a0]), kE = dpp_move<kShl1>(ke[a0]);
            const T wb = kdir * kp;
            const T w0 = face_w(ke[a0], kp);
            const T w1 = bxo ? wb : face_w(kp, kE);
            const T w2 = ys ? wb : face_w(ko[am], kp);
            const T w3 = yn ? wb : face_w(kp, ko[ap]);
            Sw = (w0 * ue[a0] + w1 * ue_) + (w2 * uo[am] + w3 * uo[ap]);
            Wt = (w0 + w1) + (w2 + w3);
        }
    };

#pragma unroll
    for (int p = 0; p < PF; ++p) load_row(p, p, p & 1);

    // whole ring turns; loads past the last visited row repeat that row (no new memory
    // traffic), and the steps past it only touch rows that are never written
    const int nturns = (nsteps + RING - 1) / RING;
    for (int turn = 0; turn < nturns; ++turn) {
        const int rb = turn * RING;
#pragma unroll
        for (int j = 0; j < RING; ++j) {
            const int rho = rb + j;
            // prefetch row rho + PF
            load_row(min(rho + PF, nsteps - 1), (j + PF) % RING, ((j + PF) & 1) != 0);
            if constexpr (RHS) {
                // FAS right-hand side of row rho - LAG (f held r): its upper neighbour is
                // first smoothed by phase 1 of this step, so every neighbour still holds
                // its initial value here
                const int r = rho - LAG;
                int gy;
                const bool yin = row_of(r, gy);
                if (r >= 1 && (!EDGE || yin)) {
                    constexpr int sh = 2 * RING;
                    const int a0 = (j - LAG + sh) % RING;
                    const int am = (j - LAG - 1 + sh) % RING;
                    const int ap = (j - LAG + 1 + sh) % RING;
                    T Se, So, We, Wo;
                    if constexpr (KV) {
                        kv_terms(true, a0, am, ap, gy, Se, We);
                        kv_terms(false, a0, am, ap, gy, So, Wo);
                    } else {
                        const T w = dpp_move<kShr1>(uo[a0]);
                        const T e = dpp_move<kShl1>(ue[a0]);
                        Se = (w + uo[a0]) + (ue[am] + ue[ap]);
                        So = (ue[a0] + e) + (uo[am] + uo[ap]);
                        const bool yb = ybound(gy);
                        We = sel3(bxe, yb, wA, wB, wC);
                        Wo = sel3(bxo, yb, wA, wB, wC);
                    }
                    fe[a0] = fe[a0] + (ue[a0] + k * (We * ue[a0] - Se));
                    fo[a0] = fo[a0] + (uo[a0] + k * (Wo * uo[a0] - So));
                    const int graw = rA + r;
                    if (graw >= y0 && graw < yend && own) {
                        store_pair_nt(A.fout + (int64_t)graw * a.n0 + gxe, fe[a0], fo[a0]);
                    }
                }
            }
            if constexpr (MODE == 1) {
                // fine grid correction u += P(u_c - R u) once both rows of a coarse row
                // are present (rho odd: rows rho - 1 and rho)
                if (j & 1) {
                    int gy;
                    const bool yin = row_of(rho, gy);
                    const int jp = (j + RING - 1) % RING;
                    const T old = restrict4(ue[jp], uo[jp], ue[j], uo[j]);
                    const T c = cr[j] - old;
                    const bool apply = !EDGE || (yin && xin);
                    ue[jp] = apply ? ue[jp] + c : ue[jp];
                    uo[jp] = apply ? uo[jp] + c : uo[jp];
                    ue[j] = apply ? ue[j] + c : ue[j];
                    uo[j] = apply ? uo[j] + c : uo[j];
                }
            }
            // colour phases: phase s updates row rho - s - LAG
#pragma unroll
            for (int s = 1; s <= S; ++s) {
                const int r = rho - s - LAG;
                if (r < 1) continue;
                int gy;
                const bool yin = row_of(r, gy);
                if (EDGE && !yin) continue;
                constexpr int sh = 2 * RING;
                const int a0 = (j - s - LAG + sh) % RING;      // row r
                const int am = (j - s - LAG - 1 + sh) % RING;  // row r - 1
                const int ap = (j - s - LAG + 1 + sh) % RING;  // row r + 1
                // colour of phase s; the pair's cell of that colour in row r is the even
                // one when the row parity equals the colour (rA and x0 - H are even)
                const int colour = ((s - 1) & 1) ^ FIRST;
                const bool even_cell = (((j - s - LAG + sh) & 1) ^ colour) == 0;
                if constexpr (KV) {
                    T Sw, Wt;
                    kv_terms(even_cell, a0, am, ap, gy, Sw, Wt);
                    if (even_cell) {
                        const T nv = (fe[a0] + k * Sw) / ((T)1 + k * Wt);
                        ue[a0] = (!EDGE || xin) ? nv : ue[a0];
                    } else {
                        const T nv = (fo[a0] + k * Sw) / ((T)1 + k * Wt);
                        uo[a0] = (!EDGE || xin) ? nv : uo[a0];
                    }
                } else if (even_cell) {
                    const T w = dpp_move<kShr1>(uo[a0]);
                    const T Ssum = (w + uo[a0]) + (ue[am] + ue[ap]);
                    const T qv = sel3(bxe, ybound(gy), qA, qB, qC);
                    const T nv = (fe[a0] + k * Ssum) * qv;
                    ue[a0] = (!EDGE || xin) ? nv : ue[a0];
                } else {
                    const T e = dpp_move<kShl1>(ue[a0]);
                    const T Ssum = (ue[a0] + e) + (uo[am] + uo[ap]);
                    const T qv = sel3(bxo, ybound(gy), qA, qB, qC);
                    const T nv = (fo[a0] + k * Ssum) * qv;
                    uo[a0] = (!EDGE || xin) ? nv : uo[a0];
                }
            }
            // row r = rho - S - 1 - LAG is final: write it, take its residual
            {
                const int r = rho - S - 1 - LAG;
                if (r >= 1) {
                    int gy;
                    row_of(r, gy);
                    const int graw = rA + r;
                    const bool inseg = graw >= y0 && graw < yend;
                    constexpr int sh = 2 * RING;
                    const int a0 = (j - S - 1 - LAG + sh) % RING;
                    const int am = (j - S - 2 - LAG + sh) % RING;
                    const int ap = (j - S - LAG + sh) % RING;
                    T Se, So, We, Wo;
                    if constexpr (KV) {
                        kv_terms(true, a0, am, ap, gy, Se, We);
                        kv_terms(false, a0, am, ap, gy, So, Wo);
                    } else {
                        const T w = dpp_move<kShr1>(uo[a0]);
                        const T e = dpp_move<kShl1>(ue[a0]);
                        Se = (w + uo[a0]) + (ue[am] + ue[ap]);
                        So = (ue[a0] + e) + (uo[am] + uo[ap]);
                        const bool yb = ybound(gy);
                        We = sel3(bxe, yb, wA, wB, wC);
                        Wo = sel3(bxo, yb, wA, wB, wC);
                    }
                    const T re = fe[a0] - (ue[a0] + k * (We * ue[a0] - Se));
                    const T ro = fo[a0] - (uo[a0] + k * (Wo * uo[a0] - So));
                    if (inseg && own) {
                        store_pair_nt(A.u_out + (int64_t)graw * a.n0 + gxe, ue[a0], uo[a0]);
                        if constexpr (MODE == 0) {
                            // rows (r - 1, r) form coarse row graw / 2 when r is odd
                            if (((j - S - 1 - LAG + sh) & 1) && graw - 1 >= y0) {
                                const T ucv = restrict4(ue[am], uo[am], ue[a0], uo[a0]);
                                const T rcv = restrict4(re_prev, ro_prev, re, ro);
                                const int64_t P = (int64_t)(graw >> 1) * mc0 + (gxe >> 1);
                                __builtin_nontemporal_store(ucv, A.uc + P);
                                __builtin_nontemporal_store(rcv, A.rc + P);
                            }
                        }
                        if constexpr (NORM) {
                            acc += (double)re * (double)re;
                            acc += (double)ro * (double)ro;
                        }
                    }
                    re_prev = re;
                    ro_prev = ro;
                }
            }
        }
    }
    if constexpr (NORM) {
        // fixed butterfly over the 64 lanes (same order on every run)
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (lane == 0) A.partials[wave_id] = acc;
    }
}

template <typename T, int NU, int MODE, bool NORM, bool RHS, bool KV>
__global__ __launch_bounds__(kThreads) void k_strip(StripArgs<T> a, int first)
{
    using G = StripGeom<NU, KV, false, false>;  // HX, H, extra: the same for every wave
    // neighbouring strips, which share halo columns, run on one XCD
    const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
    // the wave index is uniform across the wave: keep it (and all row bookkeeping) scalar
    const int gw = (int)blk * kWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int per = a.strips * a.segs;
    const int b = gw / per, wave_id = gw % per;
    if (b >= a.batch || (a.act && !a.act[b])) return;
    Arrays<T> A;
    A.f = a.f + b * a.stride;
    A.u_in = a.u_in + b * a.stride;
    A.u_out = a.u_out + b * a.stride;
    A.uc = a.uc + b * a.cstride;
    A.rc = a.rc ? a.rc + b * a.cstride : nullptr;
    A.fout = a.fout ? a.fout + b * a.stride : nullptr;
    A.kap = a.kap;  // cell kappa: single-problem grids only
    A.partials = a.partials ? a.partials + (int64_t)b * per : nullptr;
    const int strip = wave_id % a.strips, seg = wave_id / a.strips;
    const int x0 = strip * G::TXS, y0 = seg * a.seg_rows;
    // rows read: [y0 - H, y0 - H + seg_rows + extra), columns [x0 - HX, x0 - HX + 128)
    const bool edge = x0 - G::HX < 0 || x0 - G::HX + 128 > a.n0 || y0 - G::H < 0 ||
                      y0 - G::H + a.seg_rows + G::extra > a.n1;
    if (edge) {
        if (first)
            march<T, NU, MODE, NORM, RHS, KV, true, 1>(a, A, strip, seg, a.seg_rows, wave_id);
        else
            march<T, NU, MODE, NORM, RHS, KV, true, 0>(a, A, strip, seg, a.seg_rows, wave_id);
    } else {
        if (first)
            march<T, NU, MODE, NORM, RHS, KV, false, 1>(a, A, strip, seg, a.seg_rows, wave_id);
        else
            march<T, NU, MODE, NORM, RHS, KV, false, 0>(a, A, strip, seg, a.seg_rows, wave_id);
    }
}

// Blocks of the pre kernel resident per compute unit (its register count sets it).
template <typename T, int NU>
int blocks_per_cu()
{
    static const int nb = [] {
        int v = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, reinterpret_cast<const void*>(&k_strip<T, NU, 0, false, false, false>),
                                                         kThreads, 0) != hipSuccess || v < 1)
            v = 1;
        return v;
    }();
    return nb;
}

template <typename T>
StripArgs<T> make_args(const fas_grid* g, int l, const Coef& c, int nu)
{
    StripArgs<T> a{};
    a.n0 = g->lev[l].n[0];
    a.n1 = g->lev[l].n[1];
    a.bc = g->bc;
    a.k = (T)c.kd;
    for (int W = 0; W < 16; ++W) a.q[W] = (T)c.q[W];
    a.strips = (a.n0 + kStripCols - 1) / kStripCols;
    a.seg_rows = fused_seg_rows(g, l, nu);
    a.segs = (a.n1 + a.seg_rows - 1) / a.seg_rows;
    a.batch = g->batch;
    a.stride = g->lev[l].N;
    a.cstride = l < g->L ? g->lev[l + 1].N : 0;
    a.act = active_flags(g);
    a.kap = (const T*)g->lev[l].kap;
    return a;
}

inline void check_launch()
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error(FAS_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
}

template <typename T, int MODE, bool NORM, bool RHS, bool KV>
void launch_kv(const fas_grid* g, const StripArgs<T>& a, int nu, int first)
{
    const unsigned blocks = (unsigned)(((int64_t)a.batch * a.strips * a.segs + kWaves - 1) / kWaves);
    switch (nu) {
        case 0: k_strip<T, 0, MODE, NORM, RHS, KV><<<blocks, kThreads, 0, g->stream>>>(a, first); break;
        case 1: k_strip<T, 1, MODE, NORM, RHS, KV><<<blocks, kThreads, 0, g->stream>>>(a, first); break;
        case 2: k_strip<T, 2, MODE, NORM, RHS, KV><<<blocks, kThreads, 0, g->stream>>>(a, first); break;
        case 3: k_strip<T, 3, MODE, NORM, RHS, KV><<<blocks, kThreads, 0, g->stream>>>(a, first); break;
        default: throw Error(FAS_ERR_ARG, "fused kernels take nu <= 3");
    }
}

template <typename T, int MODE, bool NORM, bool RHS>
void launch_nu(const fas_grid* g, const StripArgs<T>& a, int nu, int first)
{
    if (a.kap)
        launch_kv<T, MODE, NORM, RHS, true>(g, a, nu, first);
    else
        launch_kv<T, MODE, NORM, RHS, false>(g, a, nu, first);
}

}  // namespace

template <typename T>
void strip_pre(const fas_grid* g, int l, const Coef& c, int first, int nu, const void* f, const void* u_in, void* u_out,
               void* uc, void* rc, void* fout)
{
    auto a = make_args<T>(g, l, c, nu);
    a.f = (const T*)f, a.u_in = (const T*)u_in, a.u_out = (T*)u_out;
    a.uc = (T*)uc, a.rc = (T*)rc, a.fout = (T*)fout;
    if (fout)
        launch_nu<T, 0, false, true>(g, a, nu, first);
    else
        launch_nu<T, 0, false, false>(g, a, nu, first);
}

template <typename T>
void strip_post(const fas_grid* g, int l, const Coef& c, int first, int nu, const void* f, const void* u_in,
                const void* uc, void* u_out, double* partials)
{
    auto a = make_args<T>(g, l, c, nu);
    a.f = (const T*)f, a.u_in = (const T*)u_in, a.u_out = (T*)u_out;
    a.uc = (T*)uc, a.partials = partials;
    if (partials)
        launch_nu<T, 1, true, false>(g, a, nu, first);
    else
        launch_nu<T, 1, false, false>(g, a, nu, first);
}

template <typename T>
int strip_waves_per_cu(int nu)
{
    int b = 1;
    switch (nu) {
        case 0: b = blocks_per_cu<T, 0>(); break;
        case 1: b = blocks_per_cu<T, 1>(); break;
        case 2: b = blocks_per_cu<T, 2>(); break;
        default: b = blocks_per_cu<T, 3>(); break;
    }
    return b * kWaves;
}

}  // namespace fas
