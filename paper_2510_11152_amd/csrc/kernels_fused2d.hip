// Host side of the 2D wave-strip marches: which levels take them, segment heights,
// and the launches (the kernels themselves are in strip_march.h, instantiated once per
// precision in kernels_fused2d_f64.hip and kernels_fused2d_f32.hip).
#include <hip/hip_runtime.h>

#include <atomic>

#include "fas_fused.h"
#include "fas_internal.h"

namespace fas {

namespace {

// Compute units of the current device (queried once per device).
int device_cus()
{
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int v = cache[dev].load(std::memory_order_relaxed);
    if (!v) {
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v < 1) v = 256;
        cache[dev].store(v, std::memory_order_relaxed);
    }
    return v;
}

// Rows per segment.  Every segment reads H + S + 2 rows beyond its own, so segments
// should be long; a launch whose waves all fit the device at once has no tail of late
// waves.  The rule takes the fewest segments that fill the wave slots once (at least
// kMinSegRows rows each; a batch with more strips than slots gets whole columns).
int seg_rule(const fas_grid* g, int l, int nu)
{
    const int n0 = g->lev[l].n[0], n1 = g->lev[l].n[1];
    const int64_t per = (int64_t)g->batch * ((n0 + kStripCols - 1) / kStripCols);
    const int64_t slots =
        (int64_t)device_cus() * (g->dtype == FAS_F64 ? strip_waves_per_cu<double>(nu) : strip_waves_per_cu<float>(nu));
    int64_t segs = slots / per;
    if (segs < 1) segs = 1;
    int rows = (int)((n1 + segs - 1) / segs);
    rows += rows & 1;
    return rows < kMinSegRows ? kMinSegRows : rows;
}

inline void check_launch()
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error(FAS_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
}

}  // namespace

bool fused_ok(const fas_grid* g, int l, int nu_pre, int nu_post, bool variable)
{
    (void)variable;  // constant and cell kappa alike (cell kappa only on single grids)
    if (!g->fused || g->dim != 2 || l >= g->L) return false;
    if (nu_pre > 3 || nu_post > 3) return false;
    // at least one full strip wide (so a periodic halo wraps at most once) and a few
    // rows per segment
    return g->lev[l].n[0] >= 128 && g->lev[l].n[1] >= 64;
}

int fused_seg_rows(const fas_grid* g, int l, int nu)
{
    const int n1 = g->lev[l].n[1];
    int rows = g->seg_force ? g->seg_force : g->seg_rows[l] ? g->seg_rows[l] : seg_rule(g, l, nu);
    if (rows > n1) rows = n1;  // n1 is even
    return rows;
}

int fused_tiles(const fas_grid* g, int l, int nu_post)
{
    const int n0 = g->lev[l].n[0], n1 = g->lev[l].n[1];
    const int strips = (n0 + kStripCols - 1) / kStripCols;
    const int rows = fused_seg_rows(g, l, nu_post);
    return strips * ((n1 + rows - 1) / rows);
}

void launch_fused_pre(const fas_grid* g, int l, const Coef& c, int first, int nu, const void* f, const void* u_in,
                      void* u_out, void* uc, void* rc, void* fout)
{
    if (g->dtype == FAS_F64)
        strip_pre<double>(g, l, c, first, nu, f, u_in, u_out, uc, rc, fout);
    else
        strip_pre<float>(g, l, c, first, nu, f, u_in, u_out, uc, rc, fout);
    check_launch();
}

void launch_fused_post(const fas_grid* g, int l, const Coef& c, int first, int nu, const void* f, const void* u_in,
                       const void* uc, void* u_out, double* partials)
{
    if (g->dtype == FAS_F64)
        strip_post<double>(g, l, c, first, nu, f, u_in, uc, u_out, partials);
    else
        strip_post<float>(g, l, c, first, nu, f, u_in, uc, u_out, partials);
    check_launch();
}

}  // namespace fas
