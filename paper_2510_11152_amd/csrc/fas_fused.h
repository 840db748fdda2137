// Launchers of the fused tile kernels (kernels_fused2d.hip).
#pragma once
#include "fas_internal.h"

namespace fas {

constexpr int kStripCols = 112;  // columns a 2D march wavefront writes
constexpr int kMinSegRows = 8;   // shortest 2D march segment (bounds the partial sums)

// Whether level l (not the coarsest) runs the fused pre/post kernels.
bool fused_ok(const fas_grid* g, int l, int nu_pre, int nu_post, bool variable);
// Number of norm partial sums a fused post launch on level l leaves (one per wave).
int fused_tiles(const fas_grid* g, int l, int nu_post);
// Rows per march segment on level l with nu sweeps per pass: the forced or tuned value,
// else the rule (as few segments as fill the device's wave slots once).
int fused_seg_rows(const fas_grid* g, int l, int nu);
// pre: nu sweeps on u_in -> u_out, then uc = R u_out, rc = R(f - A u_out).
// first: parity of the 0-based index sum updated first in each sweep.  fout != nullptr:
// f holds r = R(f_fine - A_fine u_fine) and the pass first forms the FAS right-hand side
// f = r + A u_in, which it uses and writes to fout.
void launch_fused_pre(const fas_grid* g, int l, const Coef& c, int first, int nu, const void* f, const void* u_in,
                      void* u_out, void* uc, void* rc, void* fout = nullptr);
// post: u_out = nu sweeps of (u_in + P(uc - R u_in)); partials (nullable) gets one sum
// of r^2 per tile, r = f - A u_out.
void launch_fused_post(const fas_grid* g, int l, const Coef& c, int first, int nu, const void* f, const void* u_in,
                       const void* uc, void* u_out, double* partials);

// Per-precision entry points of the 2D marches (strip_march.h, instantiated in
// kernels_fused2d_f64.hip / kernels_fused2d_f32.hip); the launchers above dispatch here.
template <typename T>
void strip_pre(const fas_grid* g, int l, const Coef& c, int first, int nu, const void* f, const void* u_in, void* u_out,
               void* uc, void* rc, void* fout);
template <typename T>
void strip_post(const fas_grid* g, int l, const Coef& c, int first, int nu, const void* f, const void* u_in,
                const void* uc, void* u_out, double* partials);
// Waves of the pre kernel with nu sweeps resident per compute unit.
template <typename T>
int strip_waves_per_cu(int nu);

// Block-tile passes of the 2D levels (kernels_tile2d.hip): the same passes and arguments
// as launch_fused_pre / launch_fused_post, one tile per workgroup.  tile_ok: level l takes
// them (a fused constant-kappa level of at most g->tile_max cells, both passes with 1..3
// sweeps).  tile_count: norm partial sums a post launch leaves per problem.
bool tile_ok(const fas_grid* g, int l, int nu_pre, int nu_post, bool variable);
int tile_count(const fas_grid* g, int l, int nu);
// Norm partial sums of a post launch on level l with wv waves per block (-1: no rows left
// to write).
int tile_count_with(const fas_grid* g, int l, int nu, int wv);
// Waves per block, and strips per group of the tile order, of level l's tile passes.
int tile_waves(const fas_grid* g, int l, int nu);
int tile_group(const fas_grid* g, int l);
constexpr int kTileWaveChoices[] = {6, 8, 12, 16};  // candidates of the autotuner
constexpr int kTileGroupChoices[] = {4, 8, 16, 32};
// fpartials (nullable, not with fout): one sum of f^2 per tile as well (tile_count(g, l,
// nu) of them).  zero (FP32, neither fout nor fpartials): the pass starts from u = 0 and
// does not read u_in.
void launch_tile_pre(const fas_grid* g, int l, const Coef& c, int first, int nu, const void* f, const void* u_in,
                     void* u_out, void* uc, void* rc, void* fout = nullptr, double* fpartials = nullptr,
                     bool zero = false);
// u64 (FP32 grid, no partials): instead of storing the result in u_out, add it to the FP64
// array u64 of the level's size (u64 += fp64(u)).
void launch_tile_post(const fas_grid* g, int l, const Coef& c, int first, int nu, const void* f, const void* u_in,
                      const void* uc, void* u_out, double* partials, double* u64 = nullptr);

// 3D plane-march kernels (kernels_fused3d.hip): one or two sweeps per pass.
bool fused3_ok(const fas_grid* g, int l, bool variable);
// Norm partial sums that a pass of ns sweeps with a norm leaves per problem on level l.
int fused3_partials(const fas_grid* g, int l, int ns);
// mode 0: sweeps, then uc = R u_out, rc = R(f - A u_out); mode 1: u_in + P(uc - R u_in),
// then the sweeps; mode 2: the sweeps.  ns = sweeps in the pass (1 or 2).  norm: per-block
// sums of r^2 (r = f - A u_out) into partials.  fout != nullptr (mode 2, ns 1, no norm): f
// holds r = R(f_fine - A_fine u_fine) and the pass first forms f = r + A u_in into fout.
// zero_in (FP32, modes 0 and 2, no fout): u_in is taken as 0 and not read.  acc64 (FP32, modes 1
// and 2): acc64 += fp64(result) replaces the store into u_out.
void launch_march3(const fas_grid* g, int l, const Coef& c, int first, int mode, int ns, bool norm, const void* f,
                   const void* u_in, void* u_out, void* uc, void* rc, double* partials, void* fout = nullptr,
                   bool zero_in = false, double* acc64 = nullptr);
// The mixed form's FP64 pass on the finest level of an FP64 grid that runs plane marches:
// r32 = fp32(f - A u), r^2 partial sums into partials and, if fpartials is given, f^2 into
// fpartials (per problem, one per block).  Returns the partial sums per problem, or 0 (no
// launch) when the grid has no such march or too many blocks.
int launch_march3_resid(const fas_grid* g, const Coef& c, const void* f, const void* u, void* r32, double* partials,
                        double* fpartials);

}  // namespace fas
