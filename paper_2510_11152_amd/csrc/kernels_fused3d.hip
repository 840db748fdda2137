// Fused 3D plane-march kernels for large levels (constant kappa): one or two X-MCGS
// sweeps (each both colour phases, Appendix B sets 1-4 then 5-8) per pass, fused with the
// residual and restriction, or with the prolongation correction, or with the residual norm.
//
// Geometry.  A 1024-thread block owns an x-y tile of 64 x 32 cells (thread (px, py) holds
// the cell pair 2px, 2px+1 of row py) and marches along z through a segment of planes,
// keeping a ring of planes in registers.  x-neighbours come from the adjacent lane by a
// DPP shift (a wavefront holds two tile rows; the lanes where the shift crosses a row are
// halo columns), y-neighbours through a double-buffered LDS exchange (one barrier per
// plane), z-neighbours from the ring.  Phase s = 1 .. S (S = 2 per sweep) updates plane
// t - s - LAG when plane t arrives; the residual follows on plane t - S - 1 - LAG.  A halo
// of H cells on each side of the tile and H planes below the segment are recomputed
// (neighbouring tiles overlap): each phase reaches one cell further, so H = S covers the
// phases, and a pass that also takes the residual needs S + 1, rounded up to even to keep
// 2 x 2 x 2 blocks aligned (one sweep: H = 2 or 4; two sweeps: 4 or 6).  Point formulas
// are those of fas_device.h.
//
// Modes: 0 = sweep + residual + restriction (u_c = R u, r_c = R r);
//        1 = correction u += P(u_c - R u) + sweep;  2 = sweep only;
//        3 = no sweep (FP64): the residual r = f - A u cast to FP32 for the inner solve of
//            the mixed form, with the partial sums of r^2 (and of f^2 if asked).
// RHS (the first pass of a coarse level, mode 2): f holds r = R(f - A u) of the finer
// level, and the pass first forms the FAS right-hand side f = r + A u, one plane ahead of
// the sweep while every neighbour still holds its initial value, then uses it and writes
// it for the level's later passes.
// Any mode with NORM leaves one partial sum of the squared residual per block.
// Inner solves of the mixed form (FP32 only): zero_in makes a pass start from u = 0 without
// reading u; acc64 makes a pass add its result into an FP64 iterate (acc64 += fp64(u))
// instead of storing u.
#include <hip/hip_runtime.h>

#include "fas_device.h"
#include "fas_fused.h"
#include "fas_internal.h"

namespace fas {

namespace {

constexpr int kTPX = 32, kTPY = 32;        // pairs per row, rows per tile
constexpr int kThreads3 = kTPX * kTPY;     // 1024
constexpr int kWX = 2 * kTPX;              // tile width in cells (64)
constexpr int kSegPlanes = 64;

template <typename T>
struct March3Args {
    int n0, n1, n2;
    int bc;
    T k;
    T q[16];
    int tiles_x, tiles_y, segs, seg_planes;
    int batch;
    int64_t stride, cstride;
    const int* act;
    const T* f;
    const T* u_in;
    T* u_out;
    T* uc;
    T* rc;
    T* fout;  // RHS passes: the formed right-hand side
    double* partials;
    float* r32;          // mode 3: the FP32 residual
    double* fpartials;   // mode 3 (nullable): partial sums of f^2
    int zero_in;         // FP32: 1: u_in is taken as 0 and not read (modes 0 and 2)
    double* acc64;       // FP32 (nullable): acc64 += fp64(u) in place of storing u_out
};

constexpr int kShr1 = 0x138;  // wave_shr:1 (lane i gets lane i - 1)
constexpr int kShl1 = 0x130;  // wave_shl:1 (lane i gets lane i + 1)

template <int CTRL>
__device__ __forceinline__ float dpp3(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

template <int CTRL>
__device__ __forceinline__ double dpp3(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

template <typename T>
struct Pair3;
template <>
struct Pair3<double> {
    using V = double2;
};
template <>
struct Pair3<float> {
    using V = float2;
};

__device__ __forceinline__ int wrap3(int g, int n)
{
    int w = g < 0 ? g + n : g - n;
    if (w < 0 || w >= n) w = ((g % n) + n) % n;
    return w;
}

template <typename T>
__device__ __forceinline__ T pick_q3(const March3Args<T>& a, int W)
{
    T v = a.q[6];
    v = W == 3 ? a.q[3] : v;
    v = W == 4 ? a.q[4] : v;
    v = W == 5 ? a.q[5] : v;
    v = W == 7 ? a.q[7] : v;
    v = W == 8 ? a.q[8] : v;
    v = W == 9 ? a.q[9] : v;
    return v;
}

// halo of a pass: even, >= the phases' reach (one cell per phase), +1 when the residual
// is taken
constexpr int halo3(int ns, int mode, bool norm)
{
    return (2 * ns + ((mode == 0 || mode == 3 || norm) ? 1 : 0) + 1) & ~1;
}

template <typename T, int NS, int MODE, bool NORM, bool RHS>
struct Geom3 {
    static constexpr int S = 2 * NS;            // colour phases in the pass
    static constexpr int H = halo3(NS, MODE, NORM);
    static constexpr bool RES = MODE == 0 || MODE == 3 || NORM;  // residual of the final plane
    // the correction (mode 1) and the right-hand side (RHS) need the plane below untouched
    static constexpr int LAG = (MODE == 1 || RHS) ? 1 : 0;
    // planes loaded ahead: one for two FP64 sweeps, whose ring of planes fills the 128
    // VGPRs of a 1024-lane block (with two, the FP64 two-sweep passes spill)
    static constexpr int PF = (NS == 2 && sizeof(T) == 8) ? 1 : 2;
    static constexpr int RING = (S + 3 + LAG + PF + 1) & ~1;  // planes held: >= S + 3 + LAG + PF, even
    static constexpr int SLOTS = S + 4;         // LDS exchange slots per buffer
    static constexpr int UX = kWX - 2 * H;      // cells written per tile in x
    static constexpr int UY = kTPY - 2 * H;     // rows written per tile
};

// LDS exchange area: two buffers of S + 4 slots: one per colour phase, residual even and
// odd, and two for the correction pair sums (mode 1) or the initial values (RHS).  The
// restriction of mode 0 (which uses neither) takes those last two slots of both buffers;
// the norm reduction reuses the area after the march.
template <typename T, int SLOTS>
struct Xchg {
    T buf[2][SLOTS][kThreads3];
};

// Per-problem arrays of a batched launch (the kernel arguments stay in place).
template <typename T>
struct Arrays3 {
    const T* f;
    const T* u_in;
    T* u_out;
    T* uc;
    T* rc;
    T* fout;
    float* r32;
    double* acc64;
};

template <typename T, int NS, int MODE, bool NORM, bool RHS, bool EDGE, int FIRST>
__device__ __forceinline__ void march3(const March3Args<T>& a, const Arrays3<T> A,
                                       Xchg<T, Geom3<T, NS, MODE, NORM, RHS>::SLOTS>& X, int tx, int ty, int seg,
                                       double* red)
{
    using G = Geom3<T, NS, MODE, NORM, RHS>;
    using V = typename Pair3<T>::V;
    static_assert(!RHS || MODE == 2, "the right-hand side is formed by a level's first, sweep-only pass");
    constexpr int S = G::S, H = G::H, RING = G::RING, PF = G::PF, LAG = G::LAG;
    const int tid = threadIdx.x;
    const int px = tid % kTPX, py = tid / kTPX;
    const bool periodic = a.bc == BC_PERIODIC;
    const int x0 = tx * G::UX, y0 = ty * G::UY;
    const int gxe = x0 - H + 2 * px;
    const int gy0 = y0 - H + py;
    const int z0 = seg * a.seg_planes;
    const int rA = z0 - H;
    const int zend = min(z0 + a.seg_planes, a.n2);
    const int nsteps = zend - rA + S + 1 + LAG;
    // x / y position of the pair: wrapped (periodic) or in / out of the domain
    bool xyin = true;
    int gxl = gxe, gyl = gy0;
    if constexpr (EDGE) {
        if (periodic) {
            gxl = wrap3(gxe, a.n0);
            gyl = wrap3(gy0, a.n1);
        } else {
            xyin = gxe >= 0 && gxe < a.n0 && gy0 >= 0 && gy0 < a.n1;
            gxl = min(max(gxe, 0), a.n0 - 2);
            gyl = min(max(gy0, 0), a.n1 - 1);
        }
    }
    const bool own = px >= H / 2 && px < kTPX - H / 2 && py >= H && py < kTPY - H && gxe < a.n0 && gy0 < a.n1;
    // diagonal data: x and y boundary faces of the even / odd cell (z faces per plane)
    const int dsgn = a.bc == BC_DIRICHLET ? 1 : -1;
    int bye = 0;
    if (EDGE && !periodic) bye = (gy0 == 0) + (gy0 == a.n1 - 1);
    const int be = (EDGE && !periodic) ? (gxe == 0) + bye : 0;
    const int bo = (EDGE && !periodic) ? (gxe + 2 == a.n0) + bye : 0;
    const T k = a.k;
    T qe_in = a.q[6], qe_zb = a.q[6], qo_in = a.q[6], qo_zb = a.q[6];
    T we_in = (T)6, we_zb = (T)6, wo_in = (T)6, wo_zb = (T)6;
    if constexpr (EDGE) {
        if (!periodic) {
            const int ce = 6 + dsgn * be, co = 6 + dsgn * bo;
            qe_in = pick_q3(a, ce);
            qe_zb = pick_q3(a, ce + dsgn);
            qo_in = pick_q3(a, co);
            qo_zb = pick_q3(a, co + dsgn);
            we_in = (T)ce;
            we_zb = (T)(ce + dsgn);
            wo_in = (T)co;
            wo_zb = (T)(co + dsgn);
        }
    }
    const int64_t plane = (int64_t)a.n0 * a.n1;
    const int mc0 = a.n0 >> 1, mc1 = a.n1 >> 1;
    const int64_t cplane = (int64_t)mc0 * mc1;
    const int ym = py > 0 ? tid - kTPX : tid;              // neighbours in the tile (edge rows
    const int yp = py < kTPY - 1 ? tid + kTPX : tid;       // read themselves: halo rows)

    T ue[RING], uo[RING], fe[RING], fo[RING], cr[RING];
    T su_prev = 0, sr_prev = 0;  // restriction: pair sums of the previous plane
    double acc = 0.0, facc = 0.0;

    auto plane_of = [&](int rho, int& gz) -> bool {
        gz = rA + rho;
        if constexpr (!EDGE) return true;
        if (gz >= 0 && gz < a.n2) return true;
        if (periodic) {
            gz = wrap3(gz, a.n2);
            return true;
        }
        gz = min(max(gz, 0), a.n2 - 1);
        return false;
    };
    auto load_plane = [&](int rho, int p, bool odd) {
        int gz;
        const bool zin = plane_of(rho, gz);
        const int64_t off = (int64_t)gz * plane + (int64_t)gyl * a.n0 + gxl;
        V zu;
        if (sizeof(T) == 4 && a.zero_in) {
            zu.x = (T)0;
            zu.y = (T)0;
        } else {
            zu = *reinterpret_cast<const V*>(A.u_in + off);
        }
        V zf = *reinterpret_cast<const V*>(A.f + off);
        T c = (T)0;
        if constexpr (MODE == 1) {
            if (odd) c = A.uc[(int64_t)(gz >> 1) * cplane + (int64_t)(gyl >> 1) * mc0 + (gxl >> 1)];
        }
        if constexpr (EDGE) {
            const bool in = zin && xyin;
            zu.x = in ? zu.x : (T)0;
            zu.y = in ? zu.y : (T)0;
            zf.x = in ? zf.x : (T)0;
            zf.y = in ? zf.y : (T)0;
        }
        ue[p] = zu.x;
        uo[p] = zu.y;
        fe[p] = zf.x;
        fo[p] = zf.y;
        cr[p] = c;
    };
    auto zbound = [&](int gz) -> bool { return EDGE && !periodic && (gz == 0 || gz == a.n2 - 1); };

#pragma unroll
    for (int p = 0; p < PF; ++p) load_plane(p, p, p & 1);

    // whole ring turns; loads past the last visited plane repeat that plane (no new
    // memory traffic), and the steps past it only touch planes that are never written
    const int nturns = (nsteps + RING - 1) / RING;
    for (int turn = 0; turn < nturns; ++turn) {
        const int rb = turn * RING;
#pragma unroll
        for (int j = 0; j < RING; ++j) {
            const int rho = rb + j;
            load_plane(min(rho + PF, nsteps - 1), (j + PF) % RING, ((j + PF) & 1) != 0);
            constexpr int sh = 4 * RING;
            T* B2 = X.buf[j & 1][S];      // residual: even / odd cells of the final plane
            T* B3 = X.buf[j & 1][S + 1];
            T* B4 = X.buf[j & 1][S + 2];  // correction pair sums / initial values (RHS)
            T* B5 = X.buf[j & 1][S + 3];
            // publish the values the neighbouring rows read in this step
            // (colour of a cell: (x + y + z) parity with x, y, z local; all origins even)
#pragma unroll
            for (int s = 1; s <= S; ++s) {
                const int a0 = (j - s - LAG + sh) % RING;
                const int colour = ((s - 1) & 1) ^ FIRST;
                // the other colour's cell of this pair in plane rho - s - LAG
                const bool other_even = (((py + j - s - LAG + sh) & 1) ^ (1 - colour)) == 0;
                X.buf[j & 1][s - 1][tid] = other_even ? ue[a0] : uo[a0];
            }
            if constexpr (G::RES) {
                const int a0 = (j - S - 1 - LAG + sh) % RING;
                B2[tid] = ue[a0];
                B3[tid] = uo[a0];
            }
            if constexpr (MODE == 1) {
                if (j & 1) {
                    const int jp = (j + RING - 1) % RING;
                    B4[tid] = ue[jp] + uo[jp];  // pair sums along x of planes rho - 1, rho
                    B5[tid] = ue[j] + uo[j];
                }
            }
            if constexpr (RHS) {
                const int a0 = (j - LAG + sh) % RING;  // plane rho - 1, initial values
                B4[tid] = ue[a0];
                B5[tid] = uo[a0];
            }
            __syncthreads();
            if constexpr (RHS) {
                // FAS right-hand side of plane rho - LAG (f held r)
                const int r = rho - LAG;
                int gz;
                const bool zin = plane_of(r, gz);
                if (r >= 1 && (!EDGE || zin)) {
                    const int a0 = (j - LAG + sh) % RING;
                    const int am = (j - LAG - 1 + sh) % RING;
                    const int ap = (j - LAG + 1 + sh) % RING;
                    const T w = dpp3<kShr1>(uo[a0]);
                    const T e = dpp3<kShl1>(ue[a0]);
                    const T Se = ((w + uo[a0]) + (B4[ym] + B4[yp])) + (ue[am] + ue[ap]);
                    const T So = ((ue[a0] + e) + (B5[ym] + B5[yp])) + (uo[am] + uo[ap]);
                    const bool zb = zbound(gz);
                    const T We = zb ? we_zb : we_in;
                    const T Wo = zb ? wo_zb : wo_in;
                    fe[a0] = fe[a0] + (ue[a0] + k * (We * ue[a0] - Se));
                    fo[a0] = fo[a0] + (uo[a0] + k * (Wo * uo[a0] - So));
                    const int graw = rA + r;
                    if (graw >= z0 && graw < zend && own)
                        store_pair_nt(A.fout + (int64_t)graw * plane + (int64_t)gy0 * a.n0 + gxe, fe[a0], fo[a0]);
                }
            }
            if constexpr (MODE == 1) {
                // fine grid correction on planes (rho - 1, rho) when rho is odd
                if (j & 1) {
                    int gz;
                    const bool zin = plane_of(rho, gz);
                    const int pr = tid ^ kTPX;  // partner row of the coarse cell
                    const bool even_row = (py & 1) == 0;
                    const T s00 = even_row ? B4[tid] : B4[pr];  // plane rho-1, rows 2J / 2J+1
                    const T s10 = even_row ? B4[pr] : B4[tid];
                    const T s01 = even_row ? B5[tid] : B5[pr];  // plane rho
                    const T s11 = even_row ? B5[pr] : B5[tid];
                    const T old = ((s00 + s10) + (s01 + s11)) * (T)0.125;
                    const T c = cr[j] - old;
                    const int jp = (j + RING - 1) % RING;
                    const bool apply = !EDGE || (zin && xyin);
                    ue[jp] = apply ? ue[jp] + c : ue[jp];
                    uo[jp] = apply ? uo[jp] + c : uo[jp];
                    ue[j] = apply ? ue[j] + c : ue[j];
                    uo[j] = apply ? uo[j] + c : uo[j];
                }
            }
            // colour phases
#pragma unroll
            for (int s = 1; s <= S; ++s) {
                const int r = rho - s - LAG;
                if (r < 1) continue;
                int gz;
                const bool zin = plane_of(r, gz);
                if (EDGE && !zin) continue;
                const int a0 = (j - s - LAG + sh) % RING;
                const int am = (j - s - LAG - 1 + sh) % RING;
                const int ap = (j - s - LAG + 1 + sh) % RING;
                const int colour = ((s - 1) & 1) ^ FIRST;
                const T* Bs = X.buf[j & 1][s - 1];
                const bool even_cell = (((py + j - s - LAG + sh) & 1) ^ colour) == 0;
                const bool zb = zbound(gz);
                if (even_cell) {
                    const T w = dpp3<kShr1>(uo[a0]);
                    const T Ssum = ((w + uo[a0]) + (Bs[ym] + Bs[yp])) + (ue[am] + ue[ap]);
                    const T qv = zb ? qe_zb : qe_in;
                    const T nv = (fe[a0] + k * Ssum) * qv;
                    ue[a0] = (!EDGE || xyin) ? nv : ue[a0];
                } else {
                    const T e = dpp3<kShl1>(ue[a0]);
                    const T Ssum = ((ue[a0] + e) + (Bs[ym] + Bs[yp])) + (uo[am] + uo[ap]);
                    const T qv = zb ? qo_zb : qo_in;
                    const T nv = (fo[a0] + k * Ssum) * qv;
                    uo[a0] = (!EDGE || xyin) ? nv : uo[a0];
                }
            }
            // plane rho - S - 1 - LAG is final: write, residual, restriction / norm
            {
                const int r = rho - S - 1 - LAG;
                if (r >= 1) {
                    int gz;
                    plane_of(r, gz);
                    const int graw = rA + r;
                    const bool inseg = graw >= z0 && graw < zend;
                    const int a0 = (j - S - 1 - LAG + sh) % RING;
                    const int am = (j - S - 2 - LAG + sh) % RING;
                    const int ap = (j - S - LAG + sh) % RING;
                    T re = (T)0, ro = (T)0;
                    if constexpr (G::RES) {
                        const T w = dpp3<kShr1>(uo[a0]);
                        const T e = dpp3<kShl1>(ue[a0]);
                        const T Se = ((w + uo[a0]) + (B2[ym] + B2[yp])) + (ue[am] + ue[ap]);
                        const T So = ((ue[a0] + e) + (B3[ym] + B3[yp])) + (uo[am] + uo[ap]);
                        const bool zb = zbound(gz);
                        const T We = zb ? we_zb : we_in;
                        const T Wo = zb ? wo_zb : wo_in;
                        re = fe[a0] - (ue[a0] + k * (We * ue[a0] - Se));
                        ro = fo[a0] - (uo[a0] + k * (Wo * uo[a0] - So));
                    }
                    if (inseg && own) {
                        const int64_t o = (int64_t)graw * plane + (int64_t)gy0 * a.n0 + gxe;
                        if constexpr (MODE == 3) {
                            float2 rv;
                            rv.x = (float)re;
                            rv.y = (float)ro;
                            *reinterpret_cast<float2*>(A.r32 + o) = rv;
                            if (a.fpartials) {
                                facc += (double)fe[a0] * (double)fe[a0];
                                facc += (double)fo[a0] * (double)fo[a0];
                            }
                        } else if (sizeof(T) == 4 && A.acc64) {
                            double2* const d = reinterpret_cast<double2*>(A.acc64 + o);
                            double2 v = *d;
                            v.x = v.x + (double)ue[a0];
                            v.y = v.y + (double)uo[a0];
                            *d = v;
                        } else {
                            store_pair_nt(A.u_out + o, ue[a0], uo[a0]);
                        }
                        if constexpr (NORM) {
                            acc += (double)re * (double)re;
                            acc += (double)ro * (double)ro;
                        }
                    }
                    if constexpr (MODE == 0) {
                        const T su = ue[a0] + uo[a0];
                        const T sr = re + ro;
                        // planes (r - 1, r) form coarse plane graw / 2 when r is odd
                        if (((j - S - 1 - LAG + sh) & 1) && graw - 1 >= z0 && inseg) {
                            T* R0 = X.buf[0][S + 2];  // slots mode 0 leaves unused
                            T* R1 = X.buf[0][S + 3];
                            T* R2 = X.buf[1][S + 2];
                            T* R3 = X.buf[1][S + 3];
                            R0[tid] = su_prev;
                            R1[tid] = sr_prev;
                            R2[tid] = su;
                            R3[tid] = sr;
                            __syncthreads();
                            const int pr = tid ^ kTPX;
                            if ((py & 1) == 0 && own) {
                                // children summed along x (pair), then y (rows), then z
                                const T ucv = ((R0[tid] + R0[pr]) + (R2[tid] + R2[pr])) * (T)0.125;
                                const T rcv = ((R1[tid] + R1[pr]) + (R3[tid] + R3[pr])) * (T)0.125;
                                const int64_t P = (int64_t)(graw >> 1) * cplane + (int64_t)(gy0 >> 1) * mc0 + (gxe >> 1);
                                __builtin_nontemporal_store(ucv, A.uc + P);
                                __builtin_nontemporal_store(rcv, A.rc + P);
                            }
                        }
                        su_prev = su;
                        sr_prev = sr;
                    }
                }
            }
        }
    }
    if constexpr (NORM) {
        // red aliases the exchange area; mode 3 sums f^2 beside r^2 in red[kThreads3 ..)
        __syncthreads();
        red[tid] = acc;
        if constexpr (MODE == 3) red[kThreads3 + tid] = facc;
        __syncthreads();
        for (int s = kThreads3 / 2; s > 0; s >>= 1) {
            if (tid < s) {
                red[tid] = red[tid] + red[tid + s];
                if constexpr (MODE == 3) red[kThreads3 + tid] = red[kThreads3 + tid] + red[kThreads3 + tid + s];
            }
            __syncthreads();
        }
    }
}

template <typename T, int NS, int MODE, bool NORM, bool RHS>
__global__ __launch_bounds__(kThreads3) void k_march3(March3Args<T> a, int first)
{
    using G = Geom3<T, NS, MODE, NORM, RHS>;
    static_assert(sizeof(Xchg<T, G::SLOTS>) >= (MODE == 3 ? 2 : 1) * kThreads3 * sizeof(double),
                  "norm reductions fit the exchange area");
    static_assert(MODE != 3 || (NS == 0 && NORM && !RHS && sizeof(T) == 8), "mode 3: FP64 residual pass");
    __shared__ Xchg<T, G::SLOTS> X;
    double* red = reinterpret_cast<double*>(&X.buf[0][0][0]);
    // (dispatch order, tile x fastest: the blocks resident at one time cover one z-segment
    // of neighbouring tiles across all XCDs; an XCD-contiguous renumbering measured slower)
    const int per = a.tiles_x * a.tiles_y * a.segs;
    const int b = blockIdx.x / per, w = blockIdx.x % per;
    if (a.act && !a.act[b]) return;
    Arrays3<T> A;
    A.f = a.f + b * a.stride;
    A.u_in = a.u_in + b * a.stride;
    A.u_out = a.u_out + b * a.stride;
    A.uc = a.uc ? a.uc + b * a.cstride : nullptr;
    A.rc = a.rc ? a.rc + b * a.cstride : nullptr;
    A.fout = a.fout ? a.fout + b * a.stride : nullptr;
    A.r32 = a.r32 ? a.r32 + b * a.stride : nullptr;
    A.acc64 = a.acc64 ? a.acc64 + b * a.stride : nullptr;
    const int tx = w % a.tiles_x, ty = (w / a.tiles_x) % a.tiles_y, seg = w / (a.tiles_x * a.tiles_y);
    const int x0 = tx * G::UX, y0 = ty * G::UY, z0 = seg * a.seg_planes;
    const int planes_read = a.seg_planes + G::H + G::S + 1 + G::LAG;  // the steps of a full segment
    const bool edge = x0 - G::H < 0 || x0 - G::H + kWX > a.n0 || y0 - G::H < 0 || y0 - G::H + kTPY > a.n1 ||
                      z0 - G::H < 0 || z0 - G::H + planes_read > a.n2;
    if (edge) {
        if (first)
            march3<T, NS, MODE, NORM, RHS, true, 1>(a, A, X, tx, ty, seg, red);
        else
            march3<T, NS, MODE, NORM, RHS, true, 0>(a, A, X, tx, ty, seg, red);
    } else {
        if (first)
            march3<T, NS, MODE, NORM, RHS, false, 1>(a, A, X, tx, ty, seg, red);
        else
            march3<T, NS, MODE, NORM, RHS, false, 0>(a, A, X, tx, ty, seg, red);
    }
    if constexpr (NORM) {
        if (threadIdx.x == 0) {
            a.partials[(int64_t)b * per + w] = red[0];
            if constexpr (MODE == 3) {
                if (a.fpartials) a.fpartials[(int64_t)b * per + w] = red[kThreads3];
            }
        }
    }
}

template <typename T>
March3Args<T> make_args3(const fas_grid* g, int l, const Coef& c, int ns, int mode, bool norm)
{
    March3Args<T> a{};
    a.n0 = g->lev[l].n[0];
    a.n1 = g->lev[l].n[1];
    a.n2 = g->lev[l].n[2];
    a.bc = g->bc;
    a.k = (T)c.kd;
    for (int W = 0; W < 16; ++W) a.q[W] = (T)c.q[W];
    const int H = halo3(ns, mode, norm);
    a.tiles_x = (a.n0 + (kWX - 2 * H) - 1) / (kWX - 2 * H);
    a.tiles_y = (a.n1 + (kTPY - 2 * H) - 1) / (kTPY - 2 * H);
    a.seg_planes = kSegPlanes;
    while (a.seg_planes > 8 && (int64_t)g->batch * a.tiles_x * a.tiles_y * ((a.n2 + a.seg_planes - 1) / a.seg_planes) < 512)
        a.seg_planes >>= 1;
    if (g->seg_rows[l]) a.seg_planes = g->seg_rows[l];
    if (g->seg_force) a.seg_planes = g->seg_force < a.n2 ? g->seg_force : a.n2;
    a.segs = (a.n2 + a.seg_planes - 1) / a.seg_planes;
    a.batch = g->batch;
    a.stride = g->lev[l].N;
    a.cstride = l < g->L ? g->lev[l + 1].N : 0;
    a.act = active_flags(g);
    return a;
}

inline void check_launch3()
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error(FAS_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
}

template <typename T, int NS, int MODE, bool NORM, bool RHS = false>
void go3(const fas_grid* g, const March3Args<T>& a, int first)
{
    const unsigned blocks = (unsigned)((int64_t)a.batch * a.tiles_x * a.tiles_y * a.segs);
    k_march3<T, NS, MODE, NORM, RHS><<<blocks, kThreads3, 0, g->stream>>>(a, first);
}

template <typename T>
void dispatch3(const fas_grid* g, int l, const Coef& c, int first, int mode, int ns, bool norm, const void* f,
               const void* u_in, void* u_out, void* uc, void* rc, double* partials, void* fout, bool zero_in,
               double* acc64)
{
    if ((zero_in && (sizeof(T) != 4 || mode == 1 || fout)) || (acc64 && (sizeof(T) != 4 || mode == 0)))
        throw Error(FAS_ERR_ARG, "internal: zero start / FP64 accumulation on a pass that cannot take it");
    March3Args<T> a = make_args3<T>(g, l, c, ns, mode, norm && mode != 0);
    a.zero_in = zero_in ? 1 : 0;
    a.acc64 = acc64;
    a.f = (const T*)f;
    a.u_in = (const T*)u_in;
    a.u_out = (T*)u_out;
    a.uc = (T*)uc;
    a.rc = (T*)rc;
    a.partials = partials;
    a.fout = (T*)fout;
    if (ns != 1 && ns != 2) throw Error(FAS_ERR_ARG, "internal: 3D march kernels run one or two sweeps per pass");
    if (fout && (mode != 2 || norm || ns != 1))
        throw Error(FAS_ERR_ARG, "internal: right-hand side formed by a one-sweep, sweep-only pass");
    if (fout) {
        go3<T, 1, 2, false, true>(g, a, first);
    } else if (ns == 1) {
        if (mode == 0) go3<T, 1, 0, false>(g, a, first);
        else if (mode == 1) norm ? go3<T, 1, 1, true>(g, a, first) : go3<T, 1, 1, false>(g, a, first);
        else norm ? go3<T, 1, 2, true>(g, a, first) : go3<T, 1, 2, false>(g, a, first);
    } else {
        if (mode == 0) go3<T, 2, 0, false>(g, a, first);
        else if (mode == 1) norm ? go3<T, 2, 1, true>(g, a, first) : go3<T, 2, 1, false>(g, a, first);
        else norm ? go3<T, 2, 2, true>(g, a, first) : go3<T, 2, 2, false>(g, a, first);
    }
    check_launch3();
}

}  // namespace

bool fused3_ok(const fas_grid* g, int l, bool variable)
{
    if (!g->fused || g->dim != 3 || variable || l >= g->L) return false;
    return g->lev[l].n[0] >= 64 && g->lev[l].n[1] >= 32 && g->lev[l].n[2] >= 16;
}

int fused3_partials(const fas_grid* g, int l, int ns)
{
    const March3Args<double> a = make_args3<double>(g, l, g->coef[l], ns, 2, true);
    return a.tiles_x * a.tiles_y * a.segs;
}

int launch_march3_resid(const fas_grid* g, const Coef& c, const void* f, const void* u, void* r32, double* partials,
                        double* fpartials)
{
    if (g->dtype != FAS_F64 || !fused3_ok(g, 0, g->lev[0].kap != nullptr)) return 0;
    March3Args<double> a = make_args3<double>(g, 0, c, 0, 3, true);
    const int per = a.tiles_x * a.tiles_y * a.segs;
    if (per > g->npartials / g->batch) return 0;
    a.f = (const double*)f;
    a.u_in = (const double*)u;
    a.r32 = (float*)r32;
    a.partials = partials;
    a.fpartials = fpartials;
    go3<double, 0, 3, true>(g, a, 0);
    check_launch3();
    return per;
}

void launch_march3(const fas_grid* g, int l, const Coef& c, int first, int mode, int ns, bool norm, const void* f,
                   const void* u_in, void* u_out, void* uc, void* rc, double* partials, void* fout, bool zero_in,
                   double* acc64)
{
    if (g->dtype == FAS_F64)
        dispatch3<double>(g, l, c, first, mode, ns, norm, f, u_in, u_out, uc, rc, partials, fout, zero_in, acc64);
    else
        dispatch3<float>(g, l, c, first, mode, ns, norm, f, u_in, u_out, uc, rc, partials, fout, zero_in, acc64);
}

}  // namespace fas
