// Launcher of the persistent coarse-tail kernel (kernels_tail.hip).
#pragma once
#include "fas_internal.h"

namespace fas {

constexpr int kMaxTail = 10;  // levels one tail launch may hold

// Highest level (smallest index) from which all coarser levels fit one tail launch;
// g->L + 1 if none does.
int tail_top(const fas_grid* g);
// One V-cycle of levels top..L in a single workgroup.  u: that level's u (in: initial
// guess, out: result).  r: the restricted residual when form_rhs (the FAS right-hand
// side f = r + A u is formed first), else the right-hand side itself.  first: parity of
// the first phase of every sweep (already reversed for a transposed cycle).
void launch_tail(const fas_grid* g, int top, const Coef* coef, int pre, int post, int first, void* u, const void* r,
                 bool form_rhs);

}  // namespace fas
