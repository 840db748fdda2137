// Array-form batched solves (fas_solve_batched): independent problems of any sizes, each
// on its own grid, advanced together.  Every pass of a V-cycle is one launch that serves
// each problem still iterating at that pass; a block finds its problem from the launch's
// block ranges and reads that problem's arguments (arrays, sizes, coefficients, active
// flag) from a descriptor kept in the problem's own workspace.
#pragma once
#include "fas_internal.h"

namespace fas {

constexpr int kBatchChunk = 64;           // problems per table launch (kernel-argument arrays)
constexpr size_t kDescBytes = 32 * 1024;  // descriptor region of a grid's workspace

// One table launch: np problems, problem p's descriptor at desc[p] (device address) and
// its blocks [first[p], first[p + 1]).
struct TableLaunch {
    int np;
    const void* desc[kBatchChunk];
    int first[kBatchChunk + 1];
};

// Per-problem status of a batched solve (its own grid's buffers).
struct StatusDesc {
    const double* partials;   // residual-norm partial sums of the finest post pass
    const double* fpartials;  // ||rhs||^2 partial sums of the first finest pre pass
    int count, fcount;
    double* rnorm;            // ||rhs||^2
    double* norm_out;         // ||rhs - A u||^2 after the last cycle
    int* act;                 // still iterating
    int* cyc;                 // cycle of the stop (0: none yet; -k: not finite at k)
    double* hist;             // squared norms after cycles 1..kHist
    double atol2;             // absolute stopping tolerance, squared (0: none)
};

// ---- 2D tile passes (kernels_tile2d.hip) -------------------------------------------------
// Bytes of one tile-pass descriptor of a grid of this dtype.
size_t tile_desc_bytes(int dtype);
// Waves per tile block of level l with nu sweeps (the launch shape of the tile kernels).
int tile_waves(const fas_grid* g, int l, int nu);
// Writes the descriptor of one tile pass on level l of g into host memory `out` and
// returns its block count.  post == false: pre pass (nu sweeps, then u_c = R u and
// r_c = R(f - A u); with fout, f holds the restricted residual and f = r + A u is formed
// and written first; with partials, one sum of f^2 per tile).  post == true: correction
// from uc and nu sweeps (with partials, one sum of the residual's squares per tile).
// wv: waves per block of the launch.  act: the problem's active flag.
int fill_tile_desc(const fas_grid* g, int l, const Coef& c, int nu, int wv, bool post, const void* f,
                   const void* u_in, void* u_out, void* uc, void* rc, void* fout, double* partials, const int* act,
                   void* out);
// One launch of the tile pass (pre or post) over the problems of t, all of g's dtype.
void launch_tile_table(hipStream_t stream, int dtype, bool post, int nu, int first, bool kv, int wv,
                       const TableLaunch& t);

// ---- persistent coarse tails (kernels_tail.hip) -----------------------------------------
size_t tail_desc_bytes(int dtype);
// Descriptor of the tail of g from level `top` (as launch_tail), into host memory `out`.
void fill_tail_desc(const fas_grid* g, int top, const Coef* coef, int pre, int post, int first, void* u, const void* r,
                    bool form_rhs, const int* act, void* out);
// One workgroup per problem of t.
void launch_tail_table(hipStream_t stream, int dtype, int dim, bool kv, const TableLaunch& t);

// ---- status (kernels_basic.hip); descriptors are StatusDesc ------------------------------
void launch_batch_init(hipStream_t stream, const TableLaunch& t);  // act = 1, cyc = 0
void launch_batch_fsum(hipStream_t stream, const TableLaunch& t);  // rnorm = sum of fpartials
// norm_out = sum of partials; the stopping test of cycle k and the history, per problem.
void launch_batch_update(hipStream_t stream, const TableLaunch& t, double tol, int k);
// count (one int) = problems of t still active, added to the value there if accumulate.
void launch_batch_alive(hipStream_t stream, const TableLaunch& t, int* count, bool accumulate);
// Per problem p of t: out[(base + p) * stride ..] = {cyc, rnorm, hist[0 .. stride - 2)}.
void launch_batch_gather(hipStream_t stream, const TableLaunch& t, double* out, int base, int stride);

}  // namespace fas
