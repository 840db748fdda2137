// Host-side internals of libfas: the grid plan and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <stdexcept>
#include <string>

#include "../../include/fas.h"

namespace fas {

constexpr int kMaxLevels = 24;
constexpr int kMaxEvents = 256;  // profiler event pairs held before a flush
constexpr int kPartials = 2048;  // blocks of a norm reduction (fixed: deterministic order)
constexpr int kHist = 64;        // cycles whose squared residual norms a solve keeps

// Error carried to the C ABI boundary.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// Message returned by fas_last_error() for the calling thread (set by every entry point
// that fails).
void set_last_error(const std::string& msg);

#define FAS_HIP_CHECK(expr)                                                                         \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            throw ::fas::Error(FAS_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));     \
    } while (0)

struct Level {
    int n[3];      // cells per axis, n[2] = 1 in 2D
    int64_t N;
    double h;      // h * 2^l
    void* u;       // level arrays (level 0: caller's, set per call)
    void* f;
    void* x;       // second buffer of the same size (out-of-place kernels)
    void* r;       // 2D, l >= 1: restricted residual R(f - A u) of the finer level, read by
                   // a march pre pass that forms f = r + A u itself (nullptr otherwise)
    void* kap;     // active cell kappa of this level for the current call, or nullptr
    void* kap_slot;  // workspace storage for kappa of this level (nullptr if none)
};

// Per-call operator coefficients of one level, computed on the host in double:
//   kd = dt*kappa/h_l^2 (constant kappa) or dt/h_l^2 (cell kappa); q[W] = 1/(1 + kd W)
struct Coef {
    double kd;
    double q[16];
    bool variable;
};

}  // namespace fas

struct fas_grid {
    int dim, bc, dtype, coarsest, flags, L;
    int64_t n[3];
    double h;
    fas::Level lev[fas::kMaxLevels];
    hipStream_t stream;
    double* partials;    // per-block / per-wave partial sums of a norm (npartials), device
    double* fpartials;   // array-form batched solve: per-tile sums of rhs^2 (npartials), device
    void* desc;          // array-form batched solve: launch descriptors (kDescBytes), device
    int desc_valid;      // the pinned host copy holds what desc holds
    double* norm_out;    // reduced sum of squares, one per problem, device
    int npartials;
    // batched grids: `batch` same-shape problems, level arrays contiguous across problems
    int batch;
    int* active;         // per-problem flag: still iterating (device)
    int* cyc;            // per-problem cycle count at convergence (device)
    double* rnorm;       // per-problem ||rhs||^2 (device)
    int* count;          // number of active problems (device, 1 int)
    double* hist;        // single problem: ||f - A u||^2 after cycles 1..kHist (device); the
                         // regions rnorm .. hist + kHist are one span in this order
    int last_cycles;     // cycles of the last converged solve (0: none yet)
    int fnorm_pending;   // the next finest-level tile pre pass also sums f^2 into rnorm
    int defer_norm;      // a cycle leaves its norm partials for the caller to sum ...
    int deferred_np;     // ... and reports how many (0: the norm is already in norm_out)
    double* host;        // pinned host scalars
    void* mix_e;         // FP32 inner grid: correction e and residual r32 (finest size)
    void* mix_r;
    int zero_start;      // the next finest-level tile pre pass starts from u = 0 (no read)
    double* accum64;     // non-null: the finest-level tile post pass adds its result into
                         // this FP64 array instead of storing it (nor the u argument)
    double atol;            // FAS_OPT_ATOL: absolute stopping tolerance on ||f - A u||_2 (0: none)
    int mixed_next;         // FAS_OPT_MIXED_INNER_NEXT: inner cycles of corrections 2.. (0: as the first)
    int kmax, nuc, fused;   // fused: fused kernels in use (fused_opt with a two-colour order)
    int fused_opt;          // FAS_OPT_FUSED as set
    int order, symmetric;   // FAS_OPT_ORDER / FAS_OPT_SYMMETRIC
    fas::Coef coef[fas::kMaxLevels];
    fas_stats_t stats;
    // HIP graph of one V-cycle (FAS_OPT_GRAPH) and march segment heights (FAS_OPT_AUTOTUNE)
    int use_graph, autotune, tuned;
    void* graph_cache;            // GraphCache (fas_api.hip)
    int seg_rows[fas::kMaxLevels];  // 0: default rule; else rows (2D) / planes (3D) per segment
    int seg_force;                  // FAS_OPT_SEG_ROWS: > 0 overrides rule and autotuner
    int cus;                        // compute units of the device (0: not queried yet)
    int64_t tile_max;               // FAS_OPT_TILE: largest 2D level (cells) run as block tiles
    int tile_waves;                 // FAS_OPT_TILE_WAVES: waves per tile block (0: rule)
    int march3_ns;                  // FAS_OPT_MARCH3_SWEEPS: most sweeps per 3D march pass
    int tile_wv[fas::kMaxLevels];   // FAS_OPT_AUTOTUNE: tuned waves per tile block (0: rule)
    int tile_grp[fas::kMaxLevels];  // FAS_OPT_AUTOTUNE: tuned strips per tile group (0: rule)
    int gate;                       // a solve is running its cycle loop: kernels of a single
                                    // problem check the active flag too
    hipEvent_t cyc_ev[2];           // cycle loop: one event per cycle in flight
    int cyc_ev_created;
    // profiler (FAS_OPT_PROFILE): event pairs around finest-level launches
    int profile;
    hipEvent_t ev[2 * fas::kMaxEvents];
    int ev_kind[fas::kMaxEvents];
    int ev_n, ev_created;
    fas_profile_t prof;
    size_t elem() const { return dtype == FAS_F64 ? 8 : 4; }
};

namespace fas {

// Per-problem active flags the kernels check (a batched grid, or any grid inside a
// solve's cycle loop, where a cycle already enqueued must do nothing once the solve has
// converged), or nullptr.
inline const int* active_flags(const fas_grid* g) { return g->batch > 1 || g->gate ? g->active : nullptr; }

// ---- launchers (kernels_basic.hip) ----------------------------------------------------
// All act on level `l` of grid g with coefficients c, on g->stream.
void launch_smooth_phase(const fas_grid* g, int l, const Coef& c, const void* kap, const void* f, void* u,
                         int parity);
// One index-parity set: cells whose 0-based index along axis a is even exactly when bit
// a of mask is set.
void launch_smooth_set(const fas_grid* g, int l, const Coef& c, const void* kap, const void* f, void* u, int mask);
void launch_residual(const fas_grid* g, int l, const Coef& c, const void* kap, const void* f, const void* u,
                     void* r);
// Partial sums of r^2 (r = f - A u) into g->partials then a fixed-order total into
// g->norm_out[0]; rhs-only mode (u == nullptr) sums f^2.
void launch_resid_norm(const fas_grid* g, int l, const Coef& c, const void* kap, const void* f, const void* u);
// Fixed-order total of src[b * count .. (b + 1) * count) (default g->partials) into out[b]
// (default g->norm_out), for every problem b of g.
void launch_sum_partials(const fas_grid* g, int count, double* out = nullptr, const double* src = nullptr);
void launch_resid_restrict(const fas_grid* g, int l, const Coef& c, const void* kap, const void* f,
                           const void* u, void* uc, void* rc);
void launch_coarse_rhs(const fas_grid* g, int lc, const Coef& c, const void* kapc, const void* uc, void* fc);
void launch_prolong_correct(const fas_grid* g, int l, const void* uc, void* u);
void launch_restrict(const fas_grid* g, int l, const void* fine, void* coarse);
void launch_prolong_add(const fas_grid* g, int l, const void* cnew, const void* cold, void* fine);
void launch_kappa_grad(const fas_grid* g, const Coef& c, const void* kap, const void* mu, const void* u,
                       void* gk);
// Mixed precision, outer step (FP64 grid g, gated by its active flags; problem b of a
// stacked grid at b * cells): r = f - A u, r32 = fp32(r), partial sums of r^2 in
// g->partials[b * count .. (b + 1) * count) and with fnorm of f^2 at the same places of
// g->fpartials; returns count.
int launch_mixed_resid(const fas_grid* g, const Coef& c, const void* kap, const void* f, const void* u, void* r32,
                       bool fnorm);
// u += fp64(e32) on the finest level of g, every problem (gated).
void launch_update_mixed(const fas_grid* g, const void* e32, void* u);
// x = 0 in FP32, N cells per problem of g (gated by g's active flags).
void launch_zero_f32(const fas_grid* g, int64_t N, void* x);
void launch_cast_f32(const fas_grid* g, int64_t N, const void* src64, void* dst32);
// Batched solves: every problem active, cycle counts zero.
void launch_init_active(const fas_grid* g);
// After cycle k: problems with norm_out <= tol^2 * rnorm (or 0) stop and record k;
// a non-finite norm stops with -k; g->count gets the number still active; a single
// problem also records norm_out in g->hist[k - 1] (k <= kHist) while active.
void launch_update_active(const fas_grid* g, double tol, int k);
// One problem: launch_sum_partials(g, count) and launch_update_active(g, tol, k) in one
// launch (the same norm bits, the same flags).
void launch_sum_update(const fas_grid* g, int count, double tol, int k);
// Allen-Cahn grain-growth right-hand side for q fields of N cells (FP32 or FP64):
// S = sum_j eta_j^2; f_i = eta_i - dt*((beta eta_i^3 - alpha eta_i) + 2 gamma eta_i (S - eta_i^2)).
void launch_grain_rhs(hipStream_t stream, int dtype, int q, int64_t N, double dt, double alpha, double beta,
                      double gamma, const void* eta, void* f);
// label[p] = the index of the largest of eta_0[p] .. eta_{q-1}[p] (lowest among equals).
void launch_grain_argmax(hipStream_t stream, int q, int64_t N, const float* eta, int* label);

}  // namespace fas
