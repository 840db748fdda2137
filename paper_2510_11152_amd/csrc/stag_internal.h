// Internal interface of the staggered-grid solver and the projection step
// (kernels_stag.hip: kernels and launchers; stag_api.hip: the C ABI of include/fas_stag.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace fas {
namespace stag {

// Kind of one axis of a variable's index set (Section 2.1).
enum { K_CN = 0,   // cell-centred, even ghost (homogeneous Neumann)
       K_CD = 1,   // cell-centred, odd ghost (homogeneous Dirichlet)
       K_V = 2 };  // edge-centred: the wall points hold 0
enum { LOC_CELL = 0, LOC_EDGE_X = 1, LOC_EDGE_Y = 2 };

// One level of one variable: a w - c Lap_h w, unknowns nx x ny (row-major, x fastest).
struct Lev {
    int nx, ny;
    int kx, ky;
    double a, c, h2, ih2;
};

// Red-black sweep windows: 2 * kTile columns (a column pair per lane) x kWinRows rows in
// LDS, nu sweeps (1 or 2) per launch.
constexpr int kTile = 64;
constexpr int kWinRows = 32;
constexpr int kNormBlocks = 1024;

// The coarse iterate after the coarse solve and its restricted copy from before it: the FAS
// correction is e = uc - uc0 (coarse unknowns ncx x ncy).
struct Coarse {
    const double* uc;
    const double* uc0;
    int ncx, ncy;
    __host__ __device__ __forceinline__ double e(int K, int J) const
    {
        const size_t i = (size_t)J * ncx + K;
        return uc[i] - uc0[i];
    }
};

// Window of a sweep launch: rows, margins of the written region along x and y (the sweeps
// reach 2 nu; the norm needs one more ring, the fused restriction two, since an edge axis
// takes a third tap one past the region; x margins and the row margin of the restriction
// stay even, keeping 2 x 2 blocks aligned), and the written extents.
struct SweepGeom {
    int wy, hx, hy, ox, oy;
};
constexpr SweepGeom sweep_geom(int nu, bool norm, bool res)
{
    return SweepGeom{kWinRows, 2 * nu + (norm || res ? 2 : 0),
                     2 * nu + (res ? 2 : (norm ? 1 : 0)), 2 * kTile - 2 * (2 * nu + (norm || res ? 2 : 0)),
                     kWinRows - 2 * (2 * nu + (res ? 2 : (norm ? 1 : 0)))};
}

// Fused work of a sweep launch (flags), and its arrays.
enum { SW_CORR = 1, SW_NORM = 2, SW_RHS = 4, SW_RES = 8 };
struct SweepIO {
    Coarse C;           // SW_CORR: the window is loaded as uin + P e
    double* partials;   // SW_NORM: per block, the sum of the squared residuals written
    double* fout;       // SW_RHS: f (the input) holds r; f = r + L u is formed and written here
    double* uc;         // SW_RES: uc = uc0 = R u and rc = R (f - L u) of the written region
    double* uc0;
    double* rc;
    int ncx, ncy;
};

// nu (1 or 2) full sweeps of level L: reads uin, writes uout (distinct buffers), with the
// fused work of `flags` (allowed: none, CORR, CORR | NORM, RHS, RES, RHS | RES).  Returns the
// number of blocks (the partial sums of SW_NORM).
int launch_sweep(hipStream_t s, int loc, const Lev& L, int nu, const double* f, const double* uin, double* uout,
                 const SweepIO& io, unsigned flags);
// Blocks of such a launch (tiles_x may be NULL).
int sweep_blocks(const Lev& L, int nu, unsigned flags, int* tiles_x);
// out[0] = sum of partials[0 .. n) in a fixed order.
void launch_sum(hipStream_t s, const double* partials, int n, double* out);
// f = r + L u on level L (out of place).
void launch_form_rhs(hipStream_t s, const Lev& L, const double* r, const double* u, double* f);

// Persistent tail: levels top .. coarsest in one workgroup's LDS.
constexpr int kTailMaxLevels = 12;
constexpr int kTailDoubles = 16384;  // 128 KiB of LDS
constexpr int kTailTopMax = 4096;    // unknowns of the tail's top level (4 per thread)
struct TailArgs {
    int nlev;                                   // levels in the tail (top first)
    Lev op[kTailMaxLevels];
    int ou[kTailMaxLevels], of[kTailMaxLevels], ou0[kTailMaxLevels];  // LDS offsets (doubles)
    double* u;                                  // top level iterate (in and out)
    const double* f;                            // top level right-hand side, or
    const double* r;                            // its restricted residual (f = r + L u formed here)
    int nu1, nu2, nuc;
};
void launch_tail(hipStream_t s, int loc, const TailArgs& A);
// Coarse iterate, its copy and the restricted residual of fine level Lf (location loc):
// uc = uc0 = R u, rc = R (f - L u); coarse sizes ncx x ncy.
void launch_restrict(hipStream_t s, int loc, const Lev& Lf, const double* f, const double* u, int ncx, int ncy,
                     double* uc, double* uc0, double* rc);
// f = f + L_c u on level Lc, in place (the FAS coarse right-hand side from R r).
void launch_coarse_rhs(hipStream_t s, const Lev& Lc, double* f, const double* u);
// udst = usrc + P (uc - uc0) on fine level Lf (udst may equal usrc).
void launch_correct(hipStream_t s, int loc, const Lev& Lf, const double* uc, const double* uc0, int ncx, int ncy,
                    const double* usrc, double* udst);
// sum (f - L u)^2 into out[0] (fixed order); r (optional) receives the residual.
void launch_resnorm(hipStream_t s, const Lev& L, const double* f, const double* u, double* r, double* partials,
                    double* out);
void launch_copy(hipStream_t s, const double* src, double* dst, int64_t n);

// ---- projection step (Section 4.2) ---------------------------------------------------------
struct NsArgs {
    int nx, ny;              // cells
    double dt, ih, ih2, lift;  // lift = (2 c lid) / h^2 with c = dt / Re
    double lid;
    int nforce;
    const double* fu[4];
    const double* fv[4];
    double coef[4];
};
// f_u (ny x (nx-1)) from u^n, v^n, p^n; f_v ((ny-1) x nx).
void launch_rhs_u(hipStream_t s, const NsArgs& a, const double* u, const double* v, const double* p, double* fu);
void launch_rhs_v(hipStream_t s, const NsArgs& a, const double* u, const double* v, const double* p, double* fv);
// f_p = -div(ut, vt) per cell.
void launch_neg_div(hipStream_t s, const NsArgs& a, const double* ut, const double* vt, double* fp);
// u_out = ut - dt d_x pt, v_out = vt - dt d_y pt, p_out = p_in + pt (p_out may equal p_in).
void launch_project(hipStream_t s, const NsArgs& a, const double* ut, const double* vt, const double* pt,
                    const double* p_in, double* u_out, double* v_out, double* p_out);

}  // namespace stag
}  // namespace fas
