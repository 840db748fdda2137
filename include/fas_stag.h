/* Staggered-grid FAS multigrid and the first-order projection step of the incompressible
 * Navier-Stokes equations (arXiv 2510.11152, Sections 2.1, 4.1-4.2, Appendices C-D).
 *
 * Part of libfas (same library, status codes and fas_last_error() as include/fas.h).
 *
 * Conventions shared by every entry point below.
 *   - A 2D grid of nx x ny square cells of side h (Section 2.1).  Variables live at the
 *     cell centres (FAS_LOC_CELL: pressure), at the interior east-west edge centres
 *     x = i h, i = 1 .. nx-1 (FAS_LOC_EDGE_X: u) or at the interior north-south edge
 *     centres y = j h (FAS_LOC_EDGE_Y: v).  Arrays are FP64, row-major with x fastest:
 *     CELL ny x nx, EDGE_X ny x (nx-1), EDGE_Y (ny-1) x nx values, no padding, device
 *     memory, owned by the caller.
 *   - nx and ny must both be coarsest * 2^L with L >= 1 (coarsest >= 2): every level
 *     halves both axes, down to `coarsest` cells on the shorter axis.
 *   - Every call is enqueued on the stream given at creation (NULL: the default stream).
 *     Calls that report a residual or a cycle count wait for that stream.
 *   - Two handles must not run on one workspace at the same time.
 */
#ifndef FAS_STAG_H
#define FAS_STAG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FAS_LOC_CELL 0
#define FAS_LOC_EDGE_X 1
#define FAS_LOC_EDGE_Y 2

typedef struct fas_stag fas_stag_t;

/* ---- staggered FAS solver (Section 4.1; Algorithm 1 on each variable) -------------------
 * Solves a w - c Lap_h w = f for one variable with homogeneous boundary data: wall points
 * of an edge axis hold 0; a cell-centred axis has odd ghosts (cell_bc = 1, Dirichlet) or
 * even ghosts (cell_bc = 0, Neumann; CELL only, edge locations are always Dirichlet).
 * Smoother: X-MCGS (eqs. FCGS-1..4; for this operator a red-black sweep with the points
 * whose 0-based indices have an odd sum first).  Transfers: Appendix C for cells (mean of
 * four, injection), Appendix D for edges (six-point restriction, linear prolongation).
 * The coarsest level gets FAS_OPT_COARSE_SWEEPS sweeps (default 16).
 *
 * Workspace: per level a second buffer of the iterate (the sweeps read one buffer and write
 * the other), and on levels >= 1 the iterate, its restricted copy and the right-hand side,
 * plus the norm partial sums.  fas_stag_workspace_size() returns its size in bytes (0 for
 * an unsupported shape). */
size_t fas_stag_workspace_size(int loc, int64_t nx, int64_t ny, int coarsest);

/* Creates a handle over a caller-owned device workspace of at least
 * fas_stag_workspace_size() bytes (FAS_ERR_NOMEM otherwise; FAS_ERR_SHAPE for bad sizes,
 * FAS_ERR_ARG for a bad location, h <= 0 or cell_bc outside {0, 1}). */
int fas_stag_create(int loc, int64_t nx, int64_t ny, double h, int cell_bc, int coarsest, void* workspace,
                    size_t workspace_bytes, void* stream, fas_stag_t** out);
int fas_stag_destroy(fas_stag_t* s);
/* Options (FAS_ERR_ARG for any other): FAS_OPT_COARSE_SWEEPS (>= 1); FAS_OPT_FUSED (1, the
 * default: the levels from 64 x 64 unknowns down run as one persistent workgroup with every
 * array in LDS, the restriction and the coarse right-hand side are formed inside the
 * pre-smoothing launches and the FAS correction and the residual norm inside the
 * post-smoothing ones; 0: one kernel per step and level; both give identical results);
 * FAS_OPT_PROFILE (1: HIP events time the finest level's pre- and post-smoothing launches of
 * the fused path, one cycle in every synchronised stretch; read with fas_stag_profile). */
int fas_stag_set(fas_stag_t* s, int option, double value);
/* Average microseconds of the profiled finest-level pre-smoothing launches (smoothing,
 * residual and restriction) and post-smoothing launches (correction, smoothing and, in a
 * solve, the residual norm), and the number of cycles timed.  Synchronises the stream.
 * FAS_ERR_ARG if FAS_OPT_PROFILE is off. */
int fas_stag_profile(fas_stag_t* s, double* pre_us, double* post_us, int* cycles);
int fas_stag_levels(const fas_stag_t* s);

/* Algorithm 1's loop: V(nu1, nu2) cycles until res = h ||f - L w||_2 <= tol (eq.
 * residual; absolute) or kmax cycles (0 cycles if the initial guess already meets tol).
 * w: initial guess in, iterate out.  f and w must not alias.  cycles_out and res_out may
 * be NULL.  Returns FAS_OK, FAS_NOT_CONVERGED (w holds the last iterate) or
 * FAS_ERR_NONFINITE (res became NaN or Inf). */
int fas_stag_solve(fas_stag_t* s, double a, double c, const void* f, void* w, double tol, int nu1, int nu2,
                   int kmax, int* cycles_out, double* res_out);
/* One V(nu1, nu2) cycle, w in place. */
int fas_stag_vcycle(fas_stag_t* s, double a, double c, const void* f, void* w, int nu1, int nu2);
/* nu X-MCGS sweeps on the finest level, w in place. */
int fas_stag_smooth(fas_stag_t* s, double a, double c, const void* f, void* w, int nu);
/* r = f - L w on the finest level (r may be NULL: only the norm); res_out (may be NULL)
 * gets h ||r||_2. */
int fas_stag_residual(fas_stag_t* s, double a, double c, const void* f, const void* w, void* r, double* res_out);

/* ---- first-order projection scheme (Section 4.2, Scheme 1) ------------------------------
 * Incompressible Navier-Stokes on [0, nx h] x [0, ny h] with no-slip walls; the top wall
 * may slide with a constant tangential speed `lid` (u = lid there).  One step:
 *   f_u = u^n + dt ((F_u - conv_u) - d_x p^n)        conv: third-order WENO upwinding
 *   (1 - (dt/Re) Lap_h) u~ = f_u,  likewise v~      (staggered FAS, EDGE_X / EDGE_Y)
 *   -dt Lap_h p~ = -div(u~, v~)                      (CELL, homogeneous Neumann)
 *   u^{n+1} = u~ - dt d_x p~,  v^{n+1} = v~ - dt d_y p~,  p^{n+1} = p^n + p~
 * The caller may add a separable source F = sum_k coef[k] Phi_k (k < nforce <= 4), with
 * Phi fields at the u and at the v points (Section 4.4.3's manufactured solution is such a
 * sum of three terms).
 *
 * Field layouts (the caller allocates every field, zero-filled before the first step):
 *   FAS_NS_MEMORY_EFFICIENT: 6 fields U_old, U_new, V_old, V_new, P_old, P_new (the 2D
 *     subset of the eight GPU-resident variables of the memory-efficient table): u~ is
 *     written into U_new and u^{n+1} into U_old, so no copy new -> old is needed.
 *   FAS_NS_CLASSICAL: 9 fields U_new, U_old, U~, V_new, V_old, V~, P_new, P_old, P~ (the 2D
 *     subset of the twelve of the classical table), with the copies new -> old at the end
 *     of every step.
 * Both give identical results.  The state u^n, v^n, p^n is always in U_old, V_old, P_old
 * (before and after a step); U_new/U~ etc. keep the last u~, v~, p~, which start the next
 * step's solves.  Field shapes: U* ny x (nx-1), V* (ny-1) x nx, P* ny x nx.
 *
 * Workspace (scratch, not a resident variable): one right-hand side of ny x nx values and
 * the coarse levels, shared by the three solves. */
#define FAS_NS_MEMORY_EFFICIENT 0
#define FAS_NS_CLASSICAL 1

typedef struct fas_ns fas_ns_t;

int fas_ns_fields(int layout); /* 6, 9, or 0 for an unknown layout */
size_t fas_ns_workspace_size(int64_t nx, int64_t ny, int coarsest);
/* fields: fas_ns_fields(layout) device pointers in the order above (distinct, not NULL). */
int fas_ns_create(int64_t nx, int64_t ny, double h, double re, int layout, int coarsest, void* const* fields,
                  void* workspace, size_t workspace_bytes, void* stream, fas_ns_t** out);
int fas_ns_destroy(fas_ns_t* ns);
/* Applies an option of fas_stag_set to the three solvers. */
int fas_ns_set(fas_ns_t* ns, int option, double value);
/* One step of size dt.  force_u / force_v: nforce device fields each (NULL if nforce = 0),
 * coef: nforce host doubles.  Each solve stops at h ||r||_2 <= tol or kmax cycles.
 * cycles_out[3] and res_out[3] (may be NULL): the u, v and p solves.  Returns FAS_OK,
 * FAS_NOT_CONVERGED (the step completed with a solve short of tol) or an error; after
 * FAS_ERR_NONFINITE (a solve's residual became NaN or Inf) the step stops there and the
 * fields hold its intermediate state (u~, v~ or p~ partly solved, u^n, v^n, p^n intact). */
int fas_ns_step(fas_ns_t* ns, double dt, double lid, int nforce, const void* const* force_u,
                const void* const* force_v, const double* coef, double tol, int nu1, int nu2, int kmax,
                int* cycles_out, double* res_out);
/* Bytes of the fields of this layout, and of the workspace. */
int fas_ns_memory(const fas_ns_t* ns, size_t* field_bytes, size_t* workspace_bytes);

#ifdef __cplusplus
}
#endif

#endif
