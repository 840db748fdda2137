/*
 * fas.h - C ABI of the MI355X matrix-free FAS multigrid library (libfas.so).
 *
 * Method: the matrix-free Full Approximation Storage multigrid of arXiv 2510.11152,
 * Section 2 (Alg. 1 applied recursively as in Remark 2), on cell-centred grids, with the
 * X-shape multi-colour Gauss-Seidel smoother of Section 2.3 / Appendix B, the 2^d-cell
 * average restriction and piecewise-constant prolongation of Appendix C, and smoothing
 * (not a direct solve) on the coarsest level (Remark 1).  The operator is one
 * backward-Euler heat step
 *
 *     A u = u - dt * div(kappa grad u) = f          (eq. PDE_discret with dt, kappa)
 *
 * discretised with the 5-point (2D) / 7-point (3D) stencil, spacing h equal on every
 * axis (Section 2.1).  Boundary conditions: homogeneous Neumann (default), Dirichlet
 * u = 0 through a ghost value equal to minus the adjacent cell (the reading that
 * reproduces the paper's Tables 2-3), or periodic.  kappa is a constant or a cell field;
 * face values of a cell field are harmonic means, and the coarse-level field is the
 * restricted fine field.
 *
 * Conventions for every entry point
 *   - Arrays are device pointers to contiguous storage of the grid's dtype, x fastest:
 *     index = i + n0*(j + n1*k).  The caller owns all device memory, including the
 *     workspace handed to fas_grid_create; the library never calls hipMalloc and keeps
 *     no pointer after fas_grid_destroy.  Its own runtime objects are a 4 KiB pinned
 *     host buffer (norm and convergence read-back, on first use), HIP events (the solve
 *     loop, FAS_OPT_PROFILE and the FAS_OPT_AUTOTUNE timing), and a private capture
 *     stream with the instantiated graph (FAS_OPT_GRAPH), all released by
 *     fas_grid_destroy.
 *   - All work is enqueued on the grid's HIP stream (fas_grid_create / fas_set_stream).
 *     Entry points that report a norm or a convergence status synchronise that stream;
 *     the others return as soon as the work is enqueued.
 *   - Return value: FAS_OK (0), FAS_NOT_CONVERGED (+1, u holds the last iterate) or a
 *     negative FAS_ERR_* code.  fas_last_error() gives a message for the calling
 *     thread.  Nothing throws or aborts across the ABI.
 *   - A grid is not thread-safe: calls that share a grid (hence a workspace) must not
 *     overlap in time, on any stream.
 */
#ifndef FAS_H
#define FAS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define FAS_OK 0
#define FAS_NOT_CONVERGED 1
#define FAS_ERR_ARG (-1)       /* null/aliased pointer, bad option or parameter       */
#define FAS_ERR_SHAPE (-2)     /* sizes not coarsest*2^L with L >= 1, or too large     */
#define FAS_ERR_NOMEM (-3)     /* workspace smaller than fas_workspace_size()          */
#define FAS_ERR_HIP (-4)       /* a HIP runtime call failed                            */
#define FAS_ERR_NONFINITE (-5) /* a residual norm became NaN or Inf                    */

/* boundary conditions */
#define FAS_BC_NEUMANN 0
#define FAS_BC_DIRICHLET 1
#define FAS_BC_PERIODIC 2

/* storage / arithmetic type of a grid */
#define FAS_F64 0
#define FAS_F32 1

/* fas_grid_create flags */
#define FAS_FLAG_VARIABLE_KAPPA 1 /* reserve coarse-level storage for a cell kappa field   */
#define FAS_FLAG_MIXED_INNER 2    /* FP32 grid used as the inner solver of fas_solve_mixed */

/* fas_grid_set options */
#define FAS_OPT_KMAX 1          /* maximum V-cycles of a solve (default 100; Table 1 kMax) */
#define FAS_OPT_COARSE_SWEEPS 2 /* sweeps on the coarsest level (default 2; Remark 1)      */
#define FAS_OPT_FUSED 3         /* 1 (default): fused tile kernels where available;
                                   0: one kernel per colour phase everywhere              */
#define FAS_OPT_PROFILE 4       /* 1: time every finest-level kernel launch with HIP events
                                   recorded on the grid's stream (read with
                                   fas_get_profile); 0 (default): off                     */

#define FAS_OPT_GRAPH 5         /* 1: capture each V-cycle in a HIP graph (replayed while the
                                   arrays, coefficients and sweep counts stay the same);
                                   0 (default): launch kernels one by one                 */
#define FAS_OPT_AUTOTUNE 6      /* 1: on a level's first fused pass, time the candidates
                                   and keep the fastest (cached per process): for block
                                   tiles the waves per block (6, 8, 12, 16; cell kappa 6,
                                   8) and the strips per group of the tile order (4, 8,
                                   16, 32), for row marches the segment height;
                                   0 (default): fixed rules                               */
#define FAS_OPT_SEG_ROWS 7       /* > 0 (even, >= 8): rows (2D) / planes (3D) per segment of
                                   every march launch, overriding rule and autotuner;
                                   0 (default): rule or autotuner                         */
#define FAS_OPT_TILE 8           /* >= 0: 2D levels of at most this many cells per problem run
                                   their fused passes as block tiles (1..3 sweeps), the
                                   others as row marches; 0: row marches
                                   only; default: every level                             */
#define FAS_OPT_TILE_WAVES 9     /* 6..16: waves per tile workgroup (rows written per tile
                                   4 * waves - 4 nu - 4 in FP64, 8 * waves - 4 nu - 4 in
                                   FP32; cell kappa: at most 8); 0 (default): 8           */
#define FAS_OPT_ORDER 10         /* set order of every smoothing sweep (Section 2.3): FAS_ORDER_X
                                   (default; the paper's sets 1-4, Appendix B's sets 1-8 in
                                   3D), FAS_ORDER_U or FAS_ORDER_Z.  Orders other than X, and
                                   the symmetric sequence, run one launch per index-parity set
                                   (no fused passes)                                       */
#define FAS_OPT_SYMMETRIC 11     /* 1: every second sweep of a smoothing step visits the sets
                                   in reverse order (the 1234-4321 sequence of Section 2.3);
                                   0 (default): every sweep in order (1234-1234)          */

#define FAS_OPT_ATOL 12          /* >= 0 (any double): a solve also stops once ||f - A u||_2 <= atol
                                   (Algorithm 1 tests an absolute residual; the relative test
                                   of fas_solve is this library's default); 0 (default): none.
                                   For every solve form; stacked problems share the grid's value */
#define FAS_OPT_MIXED_INNER_NEXT 13 /* >= 0, set on the FP64 grid of a mixed solve: FP32 cycles in
                                   every correction after the first (the first takes the
                                   inner_cycles argument, whose correction starts from the full
                                   residual); 0 (default): inner_cycles for all */
#define FAS_OPT_MARCH3_SWEEPS 14 /* 1 or 2 (default): most sweeps one pass of the 3D plane
                                   marches runs (constant kappa, levels from 64 x 32 x 16
                                   up); with 2, V(2, 2) makes one pre- and one post-smoothing
                                   pass per level instead of two each.  Results are
                                   identical                                              */

/* FAS_OPT_ORDER values.  A set is written by the parities of its cells' 1-based indices
 * along x, y (, z), o = odd, e = even:
 *   X: 2D oe eo ee oo;  3D oee eoe eeo ooo oeo eoo eee ooe (Appendix B, sets 1-8)
 *   U: 2D oo eo ee oe;  3D ooo eoo eeo oeo oee eee eoe ooe (Gray-code path, x first)
 *   Z: 2D oo oe eo ee;  3D ooo ooe oeo oee eoo eoe eeo eee (lexicographic, z fastest)
 * The paper draws the 2D U and Z partitions only; the 3D U and Z paths extend them. */
#define FAS_ORDER_X 0
#define FAS_ORDER_U 1
#define FAS_ORDER_Z 2

/* kernel classes reported by fas_get_profile */
#define FAS_K_SMOOTH 0 /* stand-alone smoothing launches on the finest level              */
#define FAS_K_PRE 1    /* residual + restriction (fused with pre-smoothing when fused)     */
#define FAS_K_POST 2   /* prolongation + correction (fused with post-smoothing when fused) */
#define FAS_K_NORM 3   /* residual-norm reduction                                          */
#define FAS_K_COUNT 4

typedef struct fas_grid* fas_grid_t;

typedef struct {
    int cycles;             /* V-cycles (or outer corrections) of the last solve        */
    int status;             /* FAS_OK / FAS_NOT_CONVERGED / error of the last solve      */
    double rhs_norm;        /* ||f||_2 of the last solve                                 */
    double rel_res[64];     /* ||f - A u||_2 / ||f||_2 after cycle c (c < 64)            */
} fas_stats_t;

/* Bytes of device workspace a grid needs.  dim = 2 or 3; n[0..dim-1] cells per axis; the
 * shortest axis must be coarsest * 2^L with L >= 1 and every axis divisible by 2^L
 * (Section 2.1: M_0 = M_1/2, h_0 = 2 h_1).  coarsest: cells along the shortest axis of
 * the coarsest level (even, >= 2).  Returns 0 for an invalid shape. */
size_t fas_workspace_size(int dim, const int64_t n[3], int dtype, int coarsest, int flags);

/* Create a grid plan over a caller-owned workspace of at least fas_workspace_size()
 * bytes (256-byte aligned).  h: finest spacing.  bc: FAS_BC_*.  stream: hipStream_t
 * (NULL = default stream).  *out receives the handle. */
int fas_grid_create(int dim, const int64_t n[3], double h, int bc, int dtype, int coarsest, int flags,
                    void* workspace, size_t ws_bytes, void* stream, fas_grid_t* out);
int fas_grid_destroy(fas_grid_t grid);
int fas_grid_set(fas_grid_t grid, int option, double value);
int fas_set_stream(fas_grid_t grid, void* stream);
/* Number of coarsenings L (levels 0..L, level 0 finest) and the cells of level `level`. */
int fas_grid_levels(fas_grid_t grid);
int64_t fas_level_cells(fas_grid_t grid, int level);

/* Coefficient arguments (kappa, kappa_cell) of the entry points below: kappa_cell NULL
 * selects the constant kappa; otherwise kappa_cell is the finest-level cell field (grid
 * dtype, finest size, all values > 0) and kappa is ignored.  A cell field requires a grid
 * created with FAS_FLAG_VARIABLE_KAPPA. */

/* Solve A u = rhs by V(nu1,nu2)-cycles (Alg. 1 outer loop) until
 * ||rhs - A u||_2 <= tol * ||rhs||_2 or FAS_OPT_KMAX cycles.  u: initial guess in,
 * iterate out.  rhs and u must not alias (FAS_ERR_ARG).  The test runs on the device
 * after every cycle (squared norms compared); the call returns once the iterate is final.
 * The host waits on the stream only near the expected end: after a solve on the grid that
 * took c cycles, cycles 1..c-2 are enqueued without a wait (cycles enqueued after
 * convergence do nothing).  fas_get_stats reports every cycle's relative residual. */
int fas_solve(fas_grid_t grid, double dt, double kappa, const void* kappa_cell, const void* rhs, void* u,
              double tol, int nu1, int nu2);

/* One V(nu1,nu2)-cycle on u in place.  rel_res (nullable): if given, the stream is
 * synchronised and ||rhs - A u||_2/||rhs||_2 after the cycle is written there. */
int fas_vcycle(fas_grid_t grid, double dt, double kappa, const void* kappa_cell, const void* rhs, void* u,
               int nu1, int nu2, double* rel_res);

/* Transposed cycle/solve (the adjoint of the cycle as a linear map of rhs): every sweep
 * runs its two colours in reverse order and the pre/post sweep counts are swapped.  A is
 * symmetric, so fas_solve_transposed converges to the same A^{-1} rhs. */
int fas_vcycle_transposed(fas_grid_t grid, double dt, double kappa, const void* kappa_cell, const void* rhs,
                          void* u, int nu1, int nu2, double* rel_res);
int fas_solve_transposed(fas_grid_t grid, double dt, double kappa, const void* kappa_cell, const void* rhs,
                         void* u, double tol, int nu1, int nu2);

/* Building blocks on one level (0 = finest).  Arrays are that level's size.  For these
 * calls with a cell field, kappa_cell is the field ON THAT LEVEL (the restricted field
 * for level > 0).
 *   fas_smooth:    `sweeps` X-MCGS sweeps in place (Section 2.3; reverse = 1 runs the
 *                  colours in reverse order).
 *   fas_residual:  r = rhs - A u (eq. residual); norm2 (nullable, synchronises) gets
 *                  ||r||_2.
 *   fas_restrict:  coarse = R fine, average of the 2^d children (Appendix C); level is
 *                  the fine level.
 *   fas_prolong_add: fine += P(c_new - c_old), piecewise constant (Appendix C, Alg. 1
 *                  fine grid correction); level is the fine level. */
int fas_smooth(fas_grid_t grid, int level, double dt, double kappa, const void* kappa_cell, const void* rhs,
               void* u, int sweeps, int reverse);
int fas_residual(fas_grid_t grid, int level, double dt, double kappa, const void* kappa_cell, const void* rhs,
                 const void* u, void* r, double* norm2);
int fas_restrict(fas_grid_t grid, int level, const void* fine, void* coarse);
int fas_prolong_add(fas_grid_t grid, int level, const void* c_new, const void* c_old, void* fine);

/* Gradient of a loss through one solve A(kappa) u = b given mu = A^{-T} dLoss/du:
 * gkappa -= mu^T (dA/dkappa) u on the finest level (FP64 grid, cell kappa).  Face
 * weight w = 2 ka kb/(ka + kb), dw/dka = 2 kb^2/(ka + kb)^2; a Dirichlet face of cell p
 * contributes 2 mu_p u_p.  gkappa is accumulated (+=) in place. */
int fas_kappa_grad(fas_grid_t grid, double dt, const void* kappa_cell, const void* mu, const void* u,
                   void* gkappa);

/* Mixed precision (FP32 storage and smoothing inside FP64 defect correction; the paper is
 * silent on precision beyond FP64):
 *   loop: r = rhs - A u (FP64); rho = ||r||_2; stop if rho <= tol*||rhs||_2;
 *         r32 = fp32(r); e = 0; `inner` FP32 V-cycles on A e = r32; u += fp64(e)
 * (r is not divided by rho before the cast: FP32 arithmetic is exact under power-of-two
 * scaling away from overflow and subnormals, so such a scale changes no bit, and a
 * norm-valued one would only round once more).  One FP64 pass per correction forms r,
 * its norm partial sums and r32; the stopping test runs on the device; the first inner
 * cycle starts from e = 0 without reading it and the last adds e into u in its final pass.
 * g64: FP64 grid; g32: FP32 grid of the same shape, bc and h, created with
 * FAS_FLAG_MIXED_INNER (and FAS_FLAG_VARIABLE_KAPPA for a cell field, which is given in
 * FP64 and rounded to FP32 for the inner cycle).  Stats on g64 count outer corrections. */
int fas_solve_mixed(fas_grid_t g64, fas_grid_t g32, double dt, double kappa, const void* kappa_cell,
                    const void* rhs, void* u, double tol, int nu1, int nu2, int inner);

typedef struct {
    int launches[FAS_K_COUNT]; /* finest-level launches per kernel class since the last reset */
    double ms[FAS_K_COUNT];    /* summed HIP-event durations of those launches (ms)         */
} fas_profile_t;

/* Batched solves (the paper solves its q grain-growth fields one
 * after the other): `batch` independent problems of one shape, bc, h and dtype, kappa
 * constant.  Every array argument holds the whole batch contiguously: problem b's
 * array starts b * (cells per problem) elements in.  Each kernel launch serves every
 * unconverged problem at once; the coarse tail is one workgroup per problem in a
 * single launch.  Problem b stops once ||rhs_b - A u_b|| <= tol ||rhs_b|| (its later
 * launches skip it), so each member's iterates equal those of solving it alone. */
size_t fas_workspace_size_batched(int dim, const int64_t n[3], int dtype, int coarsest, int flags, int batch);
int fas_grid_create_batched(int dim, const int64_t n[3], double h, int bc, int dtype, int coarsest, int flags,
                            int batch, void* workspace, size_t ws_bytes, void* stream, fas_grid_t* out);
/* status_out / cycles_out (nullable, batch entries each): per-problem status and
 * V-cycles.  Returns FAS_OK if all converged, else FAS_NOT_CONVERGED or
 * FAS_ERR_NONFINITE.  The host waits on the stream near the expected end, as fas_solve. */
int fas_solve_stacked(fas_grid_t grid, double dt, double kappa, const void* rhs, void* u, double tol, int nu1,
                      int nu2, int* status_out, int* cycles_out);

/* The mixed-precision defect correction of fas_solve_mixed over every problem of stacked
 * grids: g64 an FP64 grid and g32 an FP32 grid (FAS_FLAG_MIXED_INNER) of the same shape,
 * spacing, boundary condition and batch, kappa constant.  Every evaluation of the FP64
 * residuals, norms and stopping tests and every pass of the inner FP32 cycles serves all
 * problems still iterating in one launch; problem b stops once
 * ||rhs_b - A u_b|| <= tol ||rhs_b||, so its iterates are those of solving it alone.
 * status_out / cycles_out (nullable, batch entries): status and outer corrections per
 * problem.  Returns FAS_OK if all converged, else FAS_NOT_CONVERGED or FAS_ERR_NONFINITE. */
int fas_solve_stacked_mixed(fas_grid_t g64, fas_grid_t g32, double dt, double kappa, const void* rhs, void* u,
                            double tol, int nu1, int nu2, int inner, int* status_out, int* cycles_out);

/* Coefficient of one problem of an array-form batch: cell == NULL selects the constant
 * kappa = scalar, else cell is the finest-level cell field (grid dtype). */
typedef struct {
    double scalar;
    const void* cell;
} fas_kappa_t;

/* Array-form batched solve (the paper solves its grain-growth fields one after the other;
 * here independent problems advance together): problem p solves A_p u[p] = rhs[p] on its
 * own grid grids[p] (any sizes, spacings and boundary conditions; one dtype; kappa[p]
 * constant for every problem or a cell field for every problem) to
 * ||rhs_p - A_p u_p|| <= tol ||rhs_p||, each with the stopping test of fas_solve and at
 * most grids[0]'s FAS_OPT_KMAX cycles.  Every pass of a V-cycle is one launch over all
 * problems still iterating at that pass: a block finds its problem from the launch's
 * block ranges and reads that problem's arrays and coefficients from a descriptor in the
 * problem's own workspace (written when the arrays or coefficients change).  So each
 * problem's iterates, norms and cycle count equal those of fas_solve on its own grid.
 * This needs 2D grids whose levels above the coarse tail all take the tile passes
 * (1 <= nu1, nu2 <= 3; the default options) and one tile shape (FAS_OPT_TILE_WAVES) for
 * all; otherwise the problems are solved one after another with fas_solve.  All work is
 * enqueued on grids[0]'s stream; grids must be distinct; rhs[p] and u[p] must not alias.
 * status_out (nullable, nprob entries) gets each problem's status, fas_get_stats of grid
 * p its cycles, ||rhs|| and relative residuals.  Returns FAS_OK when all converged, else
 * FAS_NOT_CONVERGED or FAS_ERR_NONFINITE. */
int fas_solve_batched(int nprob, const fas_grid_t* grids, double dt, const fas_kappa_t* kappa, const void* const* rhs,
                      void* const* u, double tol, int nu1, int nu2, int* status_out);

/* Right-hand side of one semi-implicit step of the multi-order-parameter grain-growth
 * model (Section 3.3.1, eq. grain-growth-equations with L = 1): free energy
 * sum_i (-alpha eta_i^2/2 + beta eta_i^4/4) + gamma sum_{i<j} eta_i^2 eta_j^2, so
 *     f_i = eta_i - dt * ((beta eta_i^3 - alpha eta_i) + 2 gamma eta_i (S - eta_i^2)),
 *     S = sum_j eta_j^2,
 * and (I - dt kappa Lap) eta_i^{n+1} = f_i is then one batched solve (the paper's
 * coefficients: alpha = beta = gamma = 1; the grain workload here: gamma = 1.5).  eta, f:
 * q fields of ncells values of `dtype` (FAS_F32 or FAS_F64) each, contiguous, device; S is
 * summed in field order and every operation rounds in that precision (2 gamma rounded
 * once); stream: hipStream_t. */
int fas_grain_rhs(void* stream, int dtype, int q, int64_t ncells, double dt, double alpha, double beta, double gamma,
                  const void* eta, void* f);

/* Grain map of a grain-growth state (Section 3.3.1: a grain is a region where one order
 * parameter dominates): label[p] = the index i of the largest eta_i at cell p, the lowest
 * index among equal values.  eta: q fields of ncells FP32 values, contiguous; label:
 * ncells int32; device; stream: hipStream_t. */
int fas_grain_argmax(void* stream, int q, int64_t ncells, const void* eta, void* label);

/* Measurement helper (not part of the method): the attainable HBM bandwidth the stencil
 * passes are compared with.  kind 0 reads `bytes` of a (per-block sums into part[0..blocks)),
 * 1 copies a to c, 2 writes c = a + b (two streams in, one out, like a smoothing pass).
 * Arrays: device, 16-byte aligned, `bytes` each (a multiple of 16), FP64 contents.
 * `blocks` workgroups of 256 lanes, 16 bytes per lane per step.  One warm-up launch, then
 * `reps` launches timed with HIP events on `stream`; *ms_out gets the mean duration.
 * Synchronises the stream. */
int fas_stream_probe(void* stream, int kind, int64_t bytes, const void* a, const void* b, void* c, double* part,
                     int blocks, int reps, double* ms_out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): fas_solve on a single problem whose
 * grid is planned inside the call and whose workspace is a static device buffer of the
 * library, FAS_NOALLOC_MAX_BYTES per GPU, held by every GPU the library runs on until the
 * process ends.  The call allocates nothing: no hipMalloc/hipFree, no pinned host memory,
 * no events.  Arguments as fas_grid_create (without flags and workspace) plus fas_solve's;
 * the stream must belong to the calling thread's current device; kmax: maximum V-cycles;
 * cycles_out (nullable) gets the cycles run.  A grid whose workspace
 * (fas_workspace_size, with FAS_FLAG_VARIABLE_KAPPA when kappa_cell is given) exceeds
 * FAS_NOALLOC_MAX_BYTES is rejected with FAS_ERR_NOMEM (FP64 2048^2 and 128^3 fit).  The
 * host waits on the stream after every cycle.  All calls on one GPU share its buffer:
 * calls that overlap in time on one GPU (any streams or threads) race and must not be
 * made.  Nothing a call reads from the buffer is left over from an earlier call. */
#define FAS_NOALLOC_MAX_BYTES (96u << 20)
int fas_solve_noalloc(int dim, const int64_t n[3], double h, int bc, int dtype, int coarsest, void* stream, double dt,
                      double kappa, const void* kappa_cell, const void* rhs, void* u, double tol, int nu1, int nu2,
                      int kmax, int* cycles_out);

int fas_get_stats(fas_grid_t grid, fas_stats_t* out);
/* Accumulated kernel times of a grid with FAS_OPT_PROFILE on (synchronises the stream);
 * reset != 0 clears the counters afterwards. */
int fas_get_profile(fas_grid_t grid, fas_profile_t* out, int reset);
const char* fas_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FAS_H */
