// C ABI of libfas: grid plan, workspace layout, the V-cycle / solve drivers
// (Alg. 1 applied recursively, Remarks 1-2) and the mixed-precision defect correction.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fas_batch.h"
#include "fas_fused.h"
#include "fas_tail.h"
#include "fas_internal.h"

using fas::Error;

// Device workspace of fas_solve_noalloc (one copy per GPU the library runs on).
static __device__ __align__(256) char scratch[FAS_NOALLOC_MAX_BYTES];

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg)
{
    g_last_error = msg;
    return code;
}

template <typename F>
int guarded(F&& body)
{
    try {
        return body();
    } catch (const Error& e) {
        return fail(e.code, e.what());
    } catch (const std::exception& e) {
        return fail(FAS_ERR_ARG, e.what());
    } catch (...) {
        return fail(FAS_ERR_ARG, "unknown error");
    }
}

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Workspace of fas_solve_noalloc, one per GPU (see static_workspace).
constexpr size_t kStaticWorkspace = (size_t)FAS_NOALLOC_MAX_BYTES;

// Workspace layout (offsets from the workspace base, each 256-byte aligned):
//   level 0: x                      (second buffer of the finest level)
//   level l >= 1: u, f, x           (paper's two arrays per level plus the second buffer)
//   kappa levels 1..L, and level 0 of an FP32 grid (FAS_FLAG_VARIABLE_KAPPA)
//   e, r32 of the finest level       (FAS_FLAG_MIXED_INNER)
//   norm partial sums                (kPartials + 8 doubles)
struct Layout {
    int L;
    int n[fas::kMaxLevels][3];
    size_t x[fas::kMaxLevels], u[fas::kMaxLevels], f[fas::kMaxLevels], r[fas::kMaxLevels], kap[fas::kMaxLevels];
    size_t mix_e, mix_r, partials, fpartials, norm_out, active, cyc, rnorm, count, hist, desc, total;
    int npartials;
};

// Returns 0 or an error code (FAS_ERR_SHAPE / FAS_ERR_ARG) with a message.
int plan(int dim, const int64_t n[3], int dtype, int coarsest, int flags, int batch, Layout* lay, std::string* why)
{
    if (batch < 1) return *why = "batch must be >= 1", FAS_ERR_ARG;
    if (batch > 1 && (flags & FAS_FLAG_VARIABLE_KAPPA))
        return *why = "batched grids take a constant kappa", FAS_ERR_ARG;
    if (dim != 2 && dim != 3) return *why = "dim must be 2 or 3", FAS_ERR_ARG;
    if (dtype != FAS_F64 && dtype != FAS_F32) return *why = "dtype must be FAS_F64 or FAS_F32", FAS_ERR_ARG;
    if (flags & ~(FAS_FLAG_VARIABLE_KAPPA | FAS_FLAG_MIXED_INNER)) return *why = "unknown flags", FAS_ERR_ARG;
    if ((flags & FAS_FLAG_MIXED_INNER) && dtype != FAS_F32)
        return *why = "FAS_FLAG_MIXED_INNER needs an FP32 grid", FAS_ERR_ARG;
    if (coarsest < 2 || (coarsest & 1)) return *why = "coarsest must be even and >= 2", FAS_ERR_SHAPE;
    int64_t nmin = n[0];
    for (int a = 0; a < dim; ++a) {
        if (n[a] < 1) return *why = "sizes must be positive", FAS_ERR_SHAPE;
        if (n[a] < nmin) nmin = n[a];
    }
    if (nmin % coarsest) return *why = "shortest axis must be coarsest * 2^L", FAS_ERR_SHAPE;
    int64_t ratio = nmin / coarsest;
    int L = 0;
    while (((int64_t)1 << L) < ratio) ++L;
    if (((int64_t)1 << L) != ratio || L < 1) return *why = "shortest axis must be coarsest * 2^L, L >= 1", FAS_ERR_SHAPE;
    if (L >= fas::kMaxLevels) return *why = "too many levels", FAS_ERR_SHAPE;
    for (int a = 0; a < dim; ++a)
        if (n[a] % ((int64_t)1 << L)) return *why = "every axis must be divisible by 2^L", FAS_ERR_SHAPE;
    int64_t N0 = 1;
    for (int a = 0; a < dim; ++a) N0 *= n[a];
    if (N0 >= ((int64_t)1 << 31)) return *why = "grid too large (>= 2^31 cells)", FAS_ERR_SHAPE;
    const size_t s = (dtype == FAS_F64 ? 8 : 4) * (size_t)batch;  // level arrays hold the whole batch
    lay->L = L;
    size_t off = 0;
    for (int l = 0; l <= L; ++l) {
        int64_t Nl = 1;
        for (int a = 0; a < 3; ++a) {
            lay->n[l][a] = a < dim ? (int)(n[a] >> l) : 1;
            Nl *= lay->n[l][a];
        }
        lay->u[l] = lay->f[l] = lay->r[l] = 0;
        lay->x[l] = off;
        off = align_up(off + Nl * s);
        if (l >= 1) {
            lay->u[l] = off;
            off = align_up(off + Nl * s);
            lay->f[l] = off;
            off = align_up(off + Nl * s);
            lay->r[l] = off;
            off = align_up(off + Nl * s);
        }
        lay->kap[l] = 0;
        const bool need_kap = (flags & FAS_FLAG_VARIABLE_KAPPA) && (l >= 1 || dtype == FAS_F32);
        if (need_kap) {
            lay->kap[l] = off;
            off = align_up(off + Nl * s);
        }
    }
    lay->mix_e = lay->mix_r = 0;
    if (flags & FAS_FLAG_MIXED_INNER) {
        lay->mix_e = off;
        off = align_up(off + N0 * s);
        lay->mix_r = off;
        off = align_up(off + N0 * s);
    }
    // one partial sum per fused tile (3D tiles write at least 52 x 20 cells of a plane,
    // segments of 64 planes, 32 when the grid is small), per 2D march wave (kStripCols x
    // kMinSegRows cells at least) or per block of the stand-alone norm kernel
    int64_t tiles = 1;
    if (dim == 3)
        tiles = ((n[0] + 51) / 52) * ((n[1] + 19) / 20) * ((n[2] + 31) / 32);
    else
        for (int a = 0; a < dim; ++a) tiles *= (n[a] + (a == 0 ? 63 : 31)) / (a == 0 ? 64 : 32);
    if (dim == 2) {
        const int64_t waves = ((n[0] + fas::kStripCols - 1) / fas::kStripCols) *
                              ((n[1] + fas::kMinSegRows - 1) / fas::kMinSegRows);
        if (waves > tiles) tiles = waves;
    }
    const int64_t per = tiles > fas::kPartials ? tiles : fas::kPartials;
    if (per * batch >= ((int64_t)1 << 31)) return *why = "batch too large", FAS_ERR_SHAPE;
    lay->npartials = (int)(per * batch);
    lay->partials = off;
    off = align_up(off + (size_t)lay->npartials * sizeof(double));
    lay->fpartials = off;  // ||rhs||^2 partial sums of an array-form batched solve
    off = align_up(off + (size_t)lay->npartials * sizeof(double));
    lay->norm_out = off;
    off = align_up(off + (size_t)(batch + 8) * sizeof(double));
    lay->rnorm = off;
    off = align_up(off + (size_t)batch * sizeof(double));
    lay->active = off;
    off = align_up(off + (size_t)batch * sizeof(int));
    lay->cyc = off;
    off = align_up(off + (size_t)batch * sizeof(int));
    lay->count = off;
    off = align_up(off + 8 * sizeof(int));
    lay->hist = off;  // after rnorm, active, cyc and count: one span for a single problem
    off = align_up(off + fas::kHist * sizeof(double));
    lay->desc = off;  // launch descriptors of an array-form batched solve
    off = align_up(off + fas::kDescBytes);
    lay->total = off;
    return 0;
}

void check_grid(const fas_grid* g)
{
    if (!g) throw Error(FAS_ERR_ARG, "null grid");
}

void check_level(const fas_grid* g, int level, bool need_coarse)
{
    if (level < 0 || level > g->L || (need_coarse && level >= g->L))
        throw Error(FAS_ERR_ARG, "level out of range");
}

// Operator coefficients for one call (Section 2.1: h_l = 2^l h).
void set_coefs(fas_grid* g, double dt, double kappa, bool variable)
{
    if (!(dt > 0.0) || !isfinite(dt)) throw Error(FAS_ERR_ARG, "dt must be positive and finite");
    if (!variable && (!(kappa > 0.0) || !isfinite(kappa))) throw Error(FAS_ERR_ARG, "kappa must be positive");
    for (int l = 0; l <= g->L; ++l) {
        const double hl = g->lev[l].h;
        const double c = variable ? dt : dt * kappa;
        fas::Coef& C = g->coef[l];
        C.kd = c / (hl * hl);
        for (int W = 0; W < 16; ++W) C.q[W] = 1.0 / (1.0 + C.kd * (double)W);
        C.variable = variable;
    }
}

// Cell-kappa hierarchy: level 0 is the caller's field (rounded to FP32 for an FP32
// grid); level l+1 = R(level l).
// Only level 0 is set up when coarse == false (callers that only evaluate the operator
// on the finest level).
void set_kappa(fas_grid* g, const void* kcell, bool source_is_f64, bool coarse = true)
{
    for (int l = 0; l <= g->L; ++l) g->lev[l].kap = nullptr;
    if (!kcell) return;
    if (!(g->flags & FAS_FLAG_VARIABLE_KAPPA))
        throw Error(FAS_ERR_ARG, "cell kappa needs a grid created with FAS_FLAG_VARIABLE_KAPPA");
    if (g->dtype == FAS_F32 && source_is_f64) {
        g->lev[0].kap = g->lev[0].kap_slot;
        fas::launch_cast_f32(g, g->lev[0].N, kcell, g->lev[0].kap);
    } else {
        g->lev[0].kap = const_cast<void*>(kcell);
    }
    if (!coarse) return;
    for (int l = 0; l < g->L; ++l) {
        g->lev[l + 1].kap = g->lev[l + 1].kap_slot;
        fas::launch_restrict(g, l, g->lev[l].kap, g->lev[l + 1].kap);
    }
}

void ensure_host(fas_grid* g);

double read_norm(fas_grid* g)
{
    ensure_host(g);
    FAS_HIP_CHECK(hipMemcpyAsync(g->host, g->norm_out, sizeof(double), hipMemcpyDeviceToHost,
                                 g->stream));
    FAS_HIP_CHECK(hipStreamSynchronize(g->stream));
    return sqrt(g->host[0]);
}

// ---- profiler: HIP events recorded on the grid stream around finest-level launches ----
void prof_flush(fas_grid* g)
{
    if (!g->ev_n) return;
    FAS_HIP_CHECK(hipEventSynchronize(g->ev[2 * g->ev_n - 1]));
    for (int i = 0; i < g->ev_n; ++i) {
        float ms = 0.f;
        FAS_HIP_CHECK(hipEventElapsedTime(&ms, g->ev[2 * i], g->ev[2 * i + 1]));
        g->prof.ms[g->ev_kind[i]] += ms;
        g->prof.launches[g->ev_kind[i]] += 1;
    }
    g->ev_n = 0;
}

struct ProfScope {
    fas_grid* g;
    bool on;
    ProfScope(fas_grid* g_, int level, int kind) : g(g_), on(g_->profile && level == 0)
    {
        if (!on) return;
        if (g->ev_n == fas::kMaxEvents) prof_flush(g);
        const int i = g->ev_n;
        while (g->ev_created < 2 * (i + 1)) FAS_HIP_CHECK(hipEventCreate(&g->ev[g->ev_created++]));
        g->ev_kind[i] = kind;
        FAS_HIP_CHECK(hipEventRecord(g->ev[2 * i], g->stream));
    }
    void end()
    {
        if (!on) return;
        FAS_HIP_CHECK(hipEventRecord(g->ev[2 * g->ev_n + 1], g->stream));
        ++g->ev_n;
        on = false;
    }
};

// Set orders of one sweep (Section 2.3 and its figure of the X, U and Z partitions; the
// 3D X order is the sets 1-8 of Appendix B).  A set is written by the parities of its
// cells' 1-based indices along x, y (, z): 'o' odd, 'e' even.  The paper draws only the
// 2D U and Z partitions; in 3D, U is read as the Gray-code path that extends the 2D U
// (x flips first) and Z as the lexicographic path that extends the 2D Z (z fastest).
const char* const kSetOrders[2][3] = {
    {"oe eo ee oo", "oo eo ee oe", "oo oe eo ee"},
    {"oee eoe eeo ooo oeo eoo eee ooe", "ooo eoo eeo oeo oee eee eoe ooe", "ooo ooe oeo oee eoo eoe eeo eee"},
};

// The sets of g's order as masks for launch_smooth_set (bit a: odd 1-based index along
// axis a); returns their number, 2^dim.
int set_masks(const fas_grid* g, int masks[8])
{
    const char* s = kSetOrders[g->dim - 2][g->order];
    int n = 0;
    while (*s) {
        int m = 0;
        for (int a = 0; a < g->dim; ++a, ++s) m |= (*s == 'o' ? 1 : 0) << a;
        masks[n++] = m;
        if (*s == ' ') ++s;
    }
    return n;
}

// Whether every sweep of g reduces to two colours: the X sets 1-2 (1-4 in 3D) are exactly
// the cells with an odd 1-based index sum and no two of them are neighbours, so the X
// order is red-black Gauss-Seidel with that colour first, which the fused kernels run.
bool two_colour(const fas_grid* g) { return g->order == FAS_ORDER_X && !g->symmetric; }

// `sweeps` smoothing sweeps of level l with cell field kap (nullptr: constant kappa).
// reverse runs every sweep backwards (the transpose of the forward sweep); with the
// symmetric sequence every second sweep is reversed as well.
void smooth_kap(fas_grid* g, int l, const void* kap, const void* f, void* u, int sweeps, bool reverse)
{
    if (!two_colour(g)) {
        int masks[8];
        const int ns = set_masks(g, masks);
        for (int s = 0; s < sweeps; ++s) {
            const bool rev = (g->symmetric && (s & 1)) != reverse;
            for (int t = 0; t < ns; ++t) {
                ProfScope ps(g, l, FAS_K_SMOOTH);
                fas::launch_smooth_set(g, l, g->coef[l], kap, f, u, masks[rev ? ns - 1 - t : t]);
                ps.end();
            }
        }
        return;
    }
    const int first = (g->dim + 1) & 1;
    for (int s = 0; s < sweeps; ++s)
        for (int ph = 0; ph < 2; ++ph) {
            const int parity = ((ph == 0) != reverse) ? first : 1 - first;
            ProfScope ps(g, l, FAS_K_SMOOTH);
            fas::launch_smooth_phase(g, l, g->coef[l], kap, f, u, parity);
            ps.end();
        }
}

void smooth(fas_grid* g, int l, const void* f, void* u, int sweeps, bool reverse)
{
    smooth_kap(g, l, g->lev[l].kap, f, u, sweeps, reverse);
}

// FAS V-cycle below level l (Alg. 1 with the coarse steps replaced by recursion).
// partials != nullptr asks the finest-level post-smoothing to leave per-tile residual
// partial sums there; returns the number written (0 if it could not).
// rc_in (level >= 1, march levels only): the restricted residual from which the first pass
// forms f itself.
void autotune_level(fas_grid* g, int l, int first, int pre, int post, const void* f, const void* u,
                    const void* rc_in = nullptr, void* scratch = nullptr);

void autotune_tile(fas_grid* g, int l, int first, int pre, int post, const void* f, const void* u,
                   const void* rc_in);

// Whether coarse level lc forms its FAS right-hand side inside its first march pass (2D
// strips or 3D planes); the finer level then leaves R(f - A u) in lev[lc].r (the pass
// reads it while writing f, so it cannot be f itself).
// Sweeps of each 3D march pass of one smoothing step of nu sweeps, in order: up to
// march3_ns each.  pre: the step ends with the residual-restriction pass, which takes the
// full count, the passes before it split the rest; post: the correction pass comes first
// and takes the full count.  form (pre, nu >= 2): the first pass forms the right-hand
// side, which the one-sweep kernel does.
std::vector<int> march3_split(const fas_grid* g, int nu, bool form, bool pre)
{
    if (nu < 1 || (form && (!pre || nu < 2))) throw Error(FAS_ERR_ARG, "internal: 3D march pass split");
    const int m = g->march3_ns;
    std::vector<int> ns;
    int rem = nu;
    if (form) ns.push_back(1), --rem;
    const int end = std::min(m, rem);  // the restriction pass (pre) / the correction pass (post)
    rem -= end;
    if (!pre) ns.push_back(end);
    while (rem > 0) {
        const int k = std::min(m, rem);
        ns.push_back(k);
        rem -= k;
    }
    if (pre) ns.push_back(end);
    return ns;
}

bool rhs_in_pre(const fas_grid* g, int lc, int pre, int post)
{
    if (lc < 1 || lc > g->L || !g->lev[lc].r || !g->fused || lc == fas::tail_top(g)) return false;
    const bool kv = g->lev[lc].kap != nullptr;
    // 3D: formed by the first sweep-only pass, so the level needs two pre-sweeps (the
    // sweep-residual-restriction pass has no registers to spare for it)
    return fas::fused_ok(g, lc, pre, post, kv) || (fas::fused3_ok(g, lc, kv) && pre >= 2 && post >= 1);
}

// Whether coarse level lc runs its 3D march passes from the level's second buffer: a level
// whose passes form the right-hand side takes an odd number of passes when the post
// passes are one fewer than the pre passes; the finer level then leaves the restricted
// iterate in lev[lc].x, so that the last pass ends in lev[lc].u and no copy is needed.
bool march3_from_x(const fas_grid* g, int lc, int pre, int post)
{
    if (!rhs_in_pre(g, lc, pre, post) || !fas::fused3_ok(g, lc, g->lev[lc].kap != nullptr) || post < 1) return false;
    return (march3_split(g, pre, true, true).size() + march3_split(g, post, false, false).size()) % 2 == 1;
}

// Where level l leaves the restricted residual for level l + 1.
void* rc_dst(const fas_grid* g, int l, int pre, int post)
{
    return rhs_in_pre(g, l + 1, pre, post) ? g->lev[l + 1].r : g->lev[l + 1].f;
}

// Coarse part of a cycle below level l: the persistent tail when level l + 1 is its top
// (the FAS right-hand side is formed inside it), else the recursion, with the coarse
// right-hand side formed by level l + 1's pre pass or by its own kernel.
int vcycle_level(fas_grid* g, int l, const void* f, void* u, int pre, int post, bool rev, double* partials,
                 const void* rc_in = nullptr);

void coarse_part(fas_grid* g, int l, int pre, int post, bool rev)
{
    fas::Level& C = g->lev[l + 1];
    const int first = ((g->dim + 1) & 1) ^ (rev ? 1 : 0);
    if (g->fused && l + 1 == fas::tail_top(g)) {
        fas::launch_tail(g, l + 1, g->coef, pre, post, first, C.u, C.f, true);
        return;
    }
    if (rhs_in_pre(g, l + 1, pre, post)) {
        vcycle_level(g, l + 1, C.f, C.u, pre, post, rev, nullptr, C.r);
        return;
    }
    fas::launch_coarse_rhs(g, l + 1, g->coef[l + 1], C.kap, C.u, C.f);
    vcycle_level(g, l + 1, C.f, C.u, pre, post, rev, nullptr);
}

int vcycle_level(fas_grid* g, int l, const void* f, void* u, int pre, int post, bool rev, double* partials,
                 const void* rc_in)
{
    if (l == g->L) {
        smooth(g, l, f, u, g->nuc, rev);  // Remark 1: coarsest level smoothed, no direct solve
        return 0;
    }
    fas::Level& C = g->lev[l + 1];
    const int first = ((g->dim + 1) & 1) ^ (rev ? 1 : 0);
    if (l == 0 && g->fused && fas::tail_top(g) == 0) {
        // the whole hierarchy fits one tail launch
        fas::launch_tail(g, 0, g->coef, pre, post, first, u, f, false);
        return 0;
    }
    if (fas::fused3_ok(g, l, g->lev[l].kap != nullptr) && pre >= 1 && post >= 1) {
        // 3D: passes of up to march3_ns sweeps, ping-pong between u and the level's second
        // buffer; with rc_in the first pass sweeps once, reading it and forming f
        // (= lev[l].f) for the passes after it
        const std::vector<int> pre_ns = march3_split(g, pre, rc_in != nullptr, true);
        const std::vector<int> post_ns = march3_split(g, post, false, false);
        const int npre = (int)pre_ns.size(), npost = (int)post_ns.size();
        const int norm_ns = post_ns.back();
        // the iterate starts in the second buffer when the finer level left it there
        const bool from_x = rc_in && march3_from_x(g, l, pre, post);
        void* bufs[2] = {from_x ? g->lev[l].x : u, from_x ? u : g->lev[l].x};
        int cur = 0;
        // times the sweep-residual-restriction pass (input bufs[0], output bufs[1])
        autotune_level(g, l, first, pre, post, f, bufs[0], rc_in, bufs[1]);
        if (partials && fas::fused3_partials(g, l, norm_ns) > g->npartials / g->batch) partials = nullptr;
        void* const rcd = rc_dst(g, l, pre, post);
        void* const ucd = march3_from_x(g, l + 1, pre, post) ? C.x : C.u;
        // a defect correction's first inner cycle starts from zero; its last adds the
        // finest-level result into the FP64 iterate instead of storing it
        const bool zero = l == 0 && g->zero_start;
        double* const acc64 = l == 0 ? g->accum64 : nullptr;
        if (acc64 && partials) throw Error(FAS_ERR_ARG, "internal: accumulation with a norm");
        {
            ProfScope ps(g, l, FAS_K_PRE);
            for (int i = 0; i < npre - 1; ++i, cur ^= 1) {
                const bool form = rc_in && i == 0;
                fas::launch_march3(g, l, g->coef[l], first, 2, pre_ns[i], false, form ? rc_in : f, bufs[cur],
                                   bufs[cur ^ 1], nullptr, nullptr, nullptr, form ? g->lev[l].f : nullptr,
                                   zero && i == 0);
            }
            fas::launch_march3(g, l, g->coef[l], first, 0, pre_ns[npre - 1], false, f, bufs[cur], bufs[cur ^ 1], ucd,
                               rcd, nullptr, nullptr, zero && npre == 1);
            cur ^= 1;
            ps.end();
        }
        coarse_part(g, l, pre, post, rev);
        {
            ProfScope ps(g, l, FAS_K_POST);
            for (int i = 0; i < npost; ++i, cur ^= 1)
                fas::launch_march3(g, l, g->coef[l], first, i == 0 ? 1 : 2, post_ns[i], partials && i == npost - 1, f,
                                   bufs[cur], bufs[cur ^ 1], i == 0 ? C.u : nullptr, nullptr, partials, nullptr, false,
                                   i == npost - 1 ? acc64 : nullptr);
            ps.end();
        }
        if (acc64) return 0;  // the result went into the FP64 iterate; the FP32 one is dead
        if (bufs[cur] != u)
            FAS_HIP_CHECK(hipMemcpyAsync(u, bufs[cur], (size_t)g->lev[l].N * g->elem() * g->batch,
                                         hipMemcpyDeviceToDevice, g->stream));
        return partials ? fas::fused3_partials(g, l, norm_ns) : 0;
    }
    if (fas::fused_ok(g, l, pre, post, g->lev[l].kap != nullptr)) {
        void* x = g->lev[l].x;
        // block tiles on the smaller levels, row marches on the larger ones
        const bool tile = fas::tile_ok(g, l, pre, post, g->lev[l].kap != nullptr);
        if (tile)
            autotune_tile(g, l, first, pre, post, f, u, rc_in);
        else
            autotune_level(g, l, first, pre, post, f, u, rc_in);
        const int np = tile ? fas::tile_count(g, l, post) : fas::fused_tiles(g, l, post);
        if (partials && np > g->npartials / g->batch) partials = nullptr;
        // rc_in: f = rc_in + A u, formed and written by the pre pass
        const void* const fin = rc_in ? rc_in : f;
        void* const fout = rc_in ? g->lev[l].f : nullptr;
        // a solve's first pass also sums f^2 (its ||rhs||^2) per tile
        const bool fnorm = tile && l == 0 && g->fnorm_pending;
        // a defect correction's first inner cycle starts from zero; its last adds the
        // finest-level result into the FP64 iterate (tile passes on level 0 only)
        const bool zero = tile && l == 0 && g->zero_start;
        double* const acc64 = tile && l == 0 ? g->accum64 : nullptr;
        {
            ProfScope ps(g, l, FAS_K_PRE);
            if (tile)
                fas::launch_tile_pre(g, l, g->coef[l], first, pre, fin, u, x, C.u, rc_dst(g, l, pre, post), fout,
                                     fnorm ? g->partials : nullptr, zero);
            else
                fas::launch_fused_pre(g, l, g->coef[l], first, pre, fin, u, x, C.u, rc_dst(g, l, pre, post), fout);
            ps.end();
        }
        if (fnorm) {
            fas::launch_sum_partials(g, fas::tile_count(g, 0, pre), g->rnorm);
            g->fnorm_pending = 0;
        }
        coarse_part(g, l, pre, post, rev);
        {
            ProfScope ps(g, l, FAS_K_POST);
            if (tile)
                fas::launch_tile_post(g, l, g->coef[l], first, post, f, x, C.u, u, partials, acc64);
            else
                fas::launch_fused_post(g, l, g->coef[l], first, post, f, x, C.u, u, partials);
            ps.end();
        }
        return partials ? np : 0;
    }
    if (rc_in) throw Error(FAS_ERR_ARG, "internal: coarse right-hand side expected from a fused pass");
    smooth(g, l, f, u, pre, rev);
    // r = f - A u;  u_c = R u;  f_c = R r + A_c u_c
    {
        ProfScope ps(g, l, FAS_K_PRE);
        fas::launch_resid_restrict(g, l, g->coef[l], g->lev[l].kap, f, u, C.u, rc_dst(g, l, pre, post));
        ps.end();
    }
    coarse_part(g, l, pre, post, rev);
    // u += P(u_c - R u)
    {
        ProfScope ps(g, l, FAS_K_POST);
        fas::launch_prolong_correct(g, l, C.u, u);
        ps.end();
    }
    smooth(g, l, f, u, post, rev);
    return 0;
}

// Whether a V(pre, post)-cycle of g runs its finest level as tile passes (the passes that
// can start from zero and add their result into an FP64 array).
bool finest_is_tile(const fas_grid* g, int pre, int post, bool kv)
{
    if (g->fused && fas::tail_top(g) == 0) return false;
    if (fas::fused3_ok(g, 0, kv) && pre >= 1 && post >= 1) return false;
    return fas::fused_ok(g, 0, pre, post, kv) && fas::tile_ok(g, 0, pre, post, kv);
}

// Whether a V(pre, post)-cycle of g runs its finest level as 3D plane-march passes (which
// can also start from zero and add their result into an FP64 array).
bool finest_is_march3(const fas_grid* g, int pre, int post, bool kv)
{
    if (g->fused && fas::tail_top(g) == 0) return false;
    return fas::fused3_ok(g, 0, kv) && pre >= 1 && post >= 1;
}

// One cycle on the finest level; with want_norm the squared residual norm of the result
// is left in g->norm_out (reduced from the fused kernel's partials when available).
void vcycle_top(fas_grid* g, const void* f, void* u, int nu1, int nu2, bool transposed, bool want_norm = false)
{
    const int np = vcycle_level(g, 0, f, u, transposed ? nu2 : nu1, transposed ? nu1 : nu2, transposed,
                                want_norm ? g->partials : nullptr);
    if (!want_norm) return;
    if (np > 0 && g->defer_norm) {  // summed by the caller's convergence update
        g->deferred_np = np;
        return;
    }
    ProfScope ps(g, 0, FAS_K_NORM);
    if (np > 0)
        fas::launch_sum_partials(g, np);
    else
        fas::launch_resid_norm(g, 0, g->coef[0], g->lev[0].kap, f, u);
    ps.end();
}

// ---- autotuner: segment height of the march kernels ------------------------------------
// Candidates are timed on the level's own data (the pre pass is out of place, so running
// it again recomputes the same outputs); the fastest is kept per grid and per process.
// Shared by every grid of the process (grids on different threads included): guarded.
std::mutex& tune_mutex()
{
    static std::mutex m;
    return m;
}

std::map<std::string, int>& tune_cache()
{
    static std::map<std::string, int> cache;
    return cache;
}

void autotune_level(fas_grid* g, int l, int first, int pre, int post, const void* f, const void* u,
                    const void* rc_in, void* scratch)
{
    // the timed passes read u and write scratch (default: the level's second buffer)
    if (!scratch) scratch = g->lev[l].x;
    if (!g->autotune || g->seg_force || g->seg_rows[l]) return;
    const bool d3 = g->dim == 3;
    char key[160];
    snprintf(key, sizeof key, "%d:%d:%d:%d:%d:%d:%d:%d:%d:%d", g->dim, g->lev[l].n[0], g->lev[l].n[1], g->lev[l].n[2],
             g->dtype, g->batch, pre, post, rc_in ? 1 : 0, d3 ? g->march3_ns : 0);
    {
        std::lock_guard<std::mutex> lock(tune_mutex());
        auto it = tune_cache().find(key);
        if (it != tune_cache().end()) {
            g->seg_rows[l] = it->second;
            return;
        }
    }
    // 3D: planes per segment.  2D: the rule's rows (one round of waves), half and twice
    // that, and a few fixed heights.
    std::vector<int> cands;
    const int extent = d3 ? g->lev[l].n[2] : g->lev[l].n[1];
    if (d3) {
        cands = {8, 16, 32, 64, 128};
    } else {
        const int rule = fas::fused_seg_rows(g, l, pre);
        for (int r : {rule, (rule / 2 + 1) & ~1, 2 * rule, 64, 128, 256})
            if (r >= fas::kMinSegRows && std::find(cands.begin(), cands.end(), r) == cands.end()) cands.push_back(r);
    }
    hipEvent_t e0, e1;
    FAS_HIP_CHECK(hipEventCreate(&e0));
    FAS_HIP_CHECK(hipEventCreate(&e1));
    float best = 1e30f;
    int best_rows = 0;
    fas::Level& C = g->lev[l + 1];
    for (int rows : cands) {
        if (rows > extent && rows != cands.front()) continue;
        g->seg_rows[l] = rows;
        float total = 0.f;
        for (int rep = 0; rep < 3; ++rep) {
            FAS_HIP_CHECK(hipEventRecord(e0, g->stream));
            if (d3)
                fas::launch_march3(g, l, g->coef[l], first, 0, march3_split(g, pre, rc_in != nullptr, true).back(), false, f, u,
                                   scratch, C.u, rc_dst(g, l, pre, post), nullptr);
            else if (rc_in)
                fas::launch_fused_pre(g, l, g->coef[l], first, pre, rc_in, u, scratch, C.u,
                                      rc_dst(g, l, pre, post), g->lev[l].f);
            else
                fas::launch_fused_pre(g, l, g->coef[l], first, pre, f, u, scratch, C.u, rc_dst(g, l, pre, post));
            FAS_HIP_CHECK(hipEventRecord(e1, g->stream));
            FAS_HIP_CHECK(hipEventSynchronize(e1));
            float ms = 0.f;
            FAS_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
            if (rep) total += ms;  // the first launch warms caches
        }
        if (total < best) {
            best = total;
            best_rows = rows;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    g->seg_rows[l] = best_rows;
    {
        std::lock_guard<std::mutex> lock(tune_mutex());
        tune_cache()[key] = best_rows;
    }
}

// ---- autotuner: tile shape of the 2D block-tile passes ------------------------------------
// On a level's first tile pass, times the pre pass (out of place: running it again
// recomputes the same outputs) for every pair of waves per block and strips per group of
// the tile order, and keeps the fastest, per grid and per process (keyed by level shape,
// dtype, batch, sweeps, coefficient kind and pass form).  The values a pass computes do
// not depend on the shape; only the grouping of the per-tile norm sums does.
void autotune_tile(fas_grid* g, int l, int first, int pre, int post, const void* f, const void* u,
                   const void* rc_in)
{
    if (!g->autotune || g->tile_waves || g->tile_wv[l]) return;
    const bool kv = g->lev[l].kap != nullptr;
    char key[160];
    snprintf(key, sizeof key, "tile:%d:%d:%d:%d:%d:%d:%d:%d:%d", g->dim, g->lev[l].n[0], g->lev[l].n[1], g->dtype,
             g->batch, pre, post, kv ? 1 : 0, rc_in ? 1 : 0);
    {
        std::lock_guard<std::mutex> lock(tune_mutex());
        auto it = tune_cache().find(key);
        if (it != tune_cache().end()) {
            g->tile_wv[l] = it->second >> 8;
            g->tile_grp[l] = it->second & 255;
            return;
        }
    }
    hipEvent_t e0, e1;
    FAS_HIP_CHECK(hipEventCreate(&e0));
    FAS_HIP_CHECK(hipEventCreate(&e1));
    fas::Level& C = g->lev[l + 1];
    const void* fin = rc_in ? rc_in : f;
    void* const fout = rc_in ? g->lev[l].f : nullptr;
    float best = 1e30f;
    int best_wv = 8, best_grp = 16;
    const int cap = g->npartials / g->batch;
    for (int wv : fas::kTileWaveChoices) {
        if (kv && wv > 8) continue;
        const int cp = fas::tile_count_with(g, l, pre, wv), cq = fas::tile_count_with(g, l, post, wv);
        if (cp < 1 || cq < 1 || cp > cap || cq > cap) continue;
        for (int grp : fas::kTileGroupChoices) {
            g->tile_wv[l] = wv;
            g->tile_grp[l] = grp;
            float total = 0.f;
            for (int rep = 0; rep < 3; ++rep) {
                FAS_HIP_CHECK(hipEventRecord(e0, g->stream));
                fas::launch_tile_pre(g, l, g->coef[l], first, pre, fin, u, g->lev[l].x, C.u, rc_dst(g, l, pre, post),
                                     fout);
                FAS_HIP_CHECK(hipEventRecord(e1, g->stream));
                FAS_HIP_CHECK(hipEventSynchronize(e1));
                float ms = 0.f;
                FAS_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
                if (rep) total += ms;  // the first launch warms caches
            }
            if (total < best) {
                best = total;
                best_wv = wv;
                best_grp = grp;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    g->tile_wv[l] = best_wv;
    g->tile_grp[l] = best_grp;
    std::lock_guard<std::mutex> lock(tune_mutex());
    tune_cache()[key] = (best_wv << 8) | best_grp;
}

// ---- HIP graph of one V-cycle ------------------------------------------------------------
// Captured on a private stream (the caller's may be the legacy default stream, which
// cannot be captured) and replayed on the grid's stream; valid while the arrays,
// coefficients and sweep counts are those it was captured with.
struct GraphCache {
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void* rhs = nullptr;
    void* u = nullptr;
    const void* kap = nullptr;
    double kd0 = 0.0;
    int nu1 = -1, nu2 = -1, batch_active = 0;
    int nuc = -1;  // coarsest-level sweeps baked into the captured launches
    bool transposed = false, want_norm = false;
    int np = 0;
    void drop()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
};

// Drops the captured V-cycle of a grid: called whenever an option that selects kernels,
// their launch shapes or their arguments changes (a replay would keep the old ones).
void drop_graph(fas_grid* g)
{
    if (g->graph_cache) ((GraphCache*)g->graph_cache)->drop();
}

void vcycle_top(fas_grid* g, const void* f, void* u, int nu1, int nu2, bool transposed, bool want_norm);

void vcycle_run(fas_grid* g, const void* f, void* u, int nu1, int nu2, bool transposed, bool want_norm)
{
    // (a solve's first cycle, which also sums ||f||^2, is not the cycle a graph replays)
    if (!g->use_graph || g->profile || (g->autotune && !g->tuned) || g->fnorm_pending) {
        // the first cycle of an autotuned grid times its kernels, which cannot be captured
        vcycle_top(g, f, u, nu1, nu2, transposed, want_norm);
        if (g->autotune) g->tuned = 1;
        return;
    }
    if (!g->graph_cache) g->graph_cache = new GraphCache();
    GraphCache& gc = *(GraphCache*)g->graph_cache;
    const bool same = gc.exec && gc.rhs == f && gc.u == u && gc.kap == g->lev[0].kap && gc.kd0 == g->coef[0].kd &&
                      gc.nu1 == nu1 && gc.nu2 == nu2 && gc.transposed == transposed && gc.want_norm == want_norm &&
                      gc.batch_active == (fas::active_flags(g) != nullptr) && gc.nuc == g->nuc;
    if (!same) {
        // the captured cycle sums its own norm
        struct NoDefer {
            fas_grid* g;
            int saved;
            ~NoDefer() { g->defer_norm = saved; }
        } nd{g, g->defer_norm};
        g->defer_norm = 0;
        gc.drop();
        if (!gc.cap) FAS_HIP_CHECK(hipStreamCreateWithFlags(&gc.cap, hipStreamNonBlocking));
        hipStream_t saved = g->stream;
        g->stream = gc.cap;
        FAS_HIP_CHECK(hipStreamBeginCapture(gc.cap, hipStreamCaptureModeThreadLocal));
        try {
            vcycle_top(g, f, u, nu1, nu2, transposed, want_norm);
        } catch (...) {
            hipGraph_t dead = nullptr;
            (void)hipStreamEndCapture(gc.cap, &dead);
            if (dead) (void)hipGraphDestroy(dead);
            g->stream = saved;
            throw;
        }
        g->stream = saved;
        FAS_HIP_CHECK(hipStreamEndCapture(gc.cap, &gc.graph));
        FAS_HIP_CHECK(hipGraphInstantiate(&gc.exec, gc.graph, nullptr, nullptr, 0));
        gc.rhs = f;
        gc.u = u;
        gc.kap = g->lev[0].kap;
        gc.kd0 = g->coef[0].kd;
        gc.nu1 = nu1;
        gc.nu2 = nu2;
        gc.transposed = transposed;
        gc.want_norm = want_norm;
        gc.batch_active = fas::active_flags(g) != nullptr;
        gc.nuc = g->nuc;
    }
    FAS_HIP_CHECK(hipGraphLaunch(gc.exec, g->stream));
}

void check_solve_args(const fas_grid* g, const void* rhs, const void* u, int nu1, int nu2, double tol,
                      bool batched = false)
{
    check_grid(g);
    if (g->batch > 1 && !batched) throw Error(FAS_ERR_ARG, "stacked grid: use fas_solve_stacked");
    if (!rhs || !u) throw Error(FAS_ERR_ARG, "null rhs or u");
    if (rhs == u) throw Error(FAS_ERR_ARG, "rhs and u must not alias");
    if (nu1 < 0 || nu2 < 0 || nu1 + nu2 == 0) throw Error(FAS_ERR_ARG, "need nu1, nu2 >= 0 and nu1 + nu2 > 0");
    if (!(tol >= 0.0)) throw Error(FAS_ERR_ARG, "tol must be >= 0");
}

struct GateScope {
    fas_grid* g;
    explicit GateScope(fas_grid* g_) : g(g_) { g->gate = 1; }
    ~GateScope() { g->gate = 0; }
};

constexpr size_t kHostStatus = 4096;                          // status read-back
constexpr size_t kHostBytes = kHostStatus + fas::kDescBytes;  // + descriptors of a batched solve

void ensure_host(fas_grid* g)
{
    if (!g->host) FAS_HIP_CHECK(hipHostMalloc((void**)&g->host, kHostBytes, hipHostMallocDefault));
}

// The single-problem solve.  Cycle k's stopping test (Alg. 1: ||f - A u|| <= tol ||f||,
// squared) runs on the device, which clears the active flag on convergence and keeps the
// squared norms in g->hist.  Making a result visible to the host stalls the GPU for tens
// of microseconds (measured), so the host looks only at some cycles: after a solve that
// took c cycles, the next one enqueues cycles 1 .. c - 2 without looking and then checks
// every cycle.  A cycle enqueued after convergence does nothing (every kernel checks the
// active flag; its profiler timings are dropped), so results never depend on this.
int solve_impl(fas_grid* g, double dt, double kappa, const void* kcell, const void* rhs, void* u, double tol,
               int nu1, int nu2, bool transposed)
{
    check_solve_args(g, rhs, u, nu1, nu2, tol);
    set_coefs(g, dt, kappa, kcell != nullptr);
    set_kappa(g, kcell, g->dtype == FAS_F64);
    memset(&g->stats, 0, sizeof(g->stats));
    ensure_host(g);
    // status span: rnorm, active, cyc, count, hist (one problem) in workspace order
    char* const span = (char*)g->rnorm;
    const size_t span_bytes = (size_t)((char*)(g->hist + fas::kHist) - span);
    if (span_bytes > kHostStatus) throw Error(FAS_ERR_ARG, "internal: status span exceeds the pinned buffer");
    auto host_at = [&](const void* dev) { return (char*)g->host + ((const char*)dev - span); };
    fas::launch_init_active(g);
    // ||f||^2: summed by the first cycle's finest tile pre pass, which reads f anyway
    // (the tile partial sums fit the partials buffer), else by a pass of its own
    const int pre0 = transposed ? nu2 : nu1, post0 = transposed ? nu1 : nu2;
    g->fnorm_pending = g->batch == 1 && fas::tail_top(g) > 0 && fas::tile_ok(g, 0, pre0, post0, kcell != nullptr) &&
                       fas::tile_count(g, 0, pre0) <= g->npartials;
    if (!g->fnorm_pending) {
        fas::launch_resid_norm(g, 0, g->coef[0], g->lev[0].kap, rhs, nullptr);
        FAS_HIP_CHECK(hipMemcpyAsync(g->rnorm, g->norm_out, sizeof(double), hipMemcpyDeviceToDevice, g->stream));
    }
    struct Pending {
        fas_grid* g;
        ~Pending()
        {
            g->fnorm_pending = 0;
            g->defer_norm = 0;
            g->deferred_np = 0;
        }
    } pending{g};
    g->defer_norm = 1;  // a cycle's norm total and its convergence update: one launch
    g->deferred_np = 0;
    while (g->cyc_ev_created < 2)
        FAS_HIP_CHECK(hipEventCreateWithFlags(&g->cyc_ev[g->cyc_ev_created++], hipEventDisableTiming));
    GateScope gate(g);
    const int horizon = g->last_cycles > 2 ? g->last_cycles - 2 : 0;  // cycles run without a look
    g->last_cycles = 0;
    std::vector<int> mark((size_t)g->kmax + 2, 0);  // profiler pairs recorded before cycle k
    int end = 0, verified = 0;                        // cycle the solve stopped at; last cycle seen live
    // copy the status span to the host after the last enqueued cycle; true if stopped
    auto look = [&](int k) -> bool {
        FAS_HIP_CHECK(hipMemcpyAsync(g->host, span, span_bytes, hipMemcpyDeviceToHost, g->stream));
        FAS_HIP_CHECK(hipEventRecord(g->cyc_ev[0], g->stream));
        FAS_HIP_CHECK(hipEventSynchronize(g->cyc_ev[0]));
        if (*(const int*)host_at(g->count) != 0) {
            verified = k;
            return false;
        }
        end = *(const int*)host_at(g->cyc);  // k of the stop, -k if the norm was not finite
        const int stop = end < 0 ? -end : end;
        if (g->profile && stop < k) g->ev_n = mark[(size_t)stop + 1];  // cycles after it did nothing
        return true;
    };
    bool stopped = false;
    // profiler pairs one cycle may record (finest-level launches; per phase without fusion)
    const int reserve = std::min(fas::kMaxEvents / 2, 2 * (nu1 + nu2) + 8);
    for (int k = 1; k <= g->kmax && !stopped; ++k) {
        if (g->profile && g->ev_n > fas::kMaxEvents - reserve) {
            // before the profiler flushes, every cycle enqueued must be known to have run
            if (k - 1 > verified && look(k - 1)) {
                stopped = true;
                break;
            }
            prof_flush(g);
        }
        mark[(size_t)k] = g->ev_n;
        vcycle_run(g, rhs, u, nu1, nu2, transposed, true);
        if (g->deferred_np > 0)
            fas::launch_sum_update(g, g->deferred_np, tol, k);
        else
            fas::launch_update_active(g, tol, k);
        g->deferred_np = 0;
        if (k > horizon || k == g->kmax) stopped = look(k);
    }
    const double nf = sqrt(*(const double*)host_at(g->rnorm));
    const double* hist = (const double*)host_at(g->hist);
    const int cycles = !stopped ? g->kmax : (end < 0 ? -end : end);
    g->stats.rhs_norm = nf;
    for (int i = 0; i < cycles && i < 64 && i < fas::kHist; ++i) {
        const double nr = sqrt(hist[i]);
        g->stats.rel_res[i] = nf > 0.0 ? nr / nf : nr;
    }
    g->stats.cycles = cycles;
    if (stopped && end < 0) {
        g->stats.status = FAS_ERR_NONFINITE;
        throw Error(FAS_ERR_NONFINITE, "residual norm is not finite");
    }
    const int status = stopped ? FAS_OK : FAS_NOT_CONVERGED;
    g->stats.status = status;
    if (status == FAS_OK) g->last_cycles = cycles;
    if (status != FAS_OK) g_last_error = "not converged within kmax cycles";
    return status;
}

// Mixed precision (FP32 storage and smoothing inside FP64 defect correction).  Evaluation
// k = 1, 2, ... computes r = f - A u in FP64 with ||r||^2 (and, first, ||f||^2) and
// r32 = fp32(r); the device tests ||r|| <= tol ||f|| as a solve's cycle does (the same
// active flag, history and status span).  Unless it has stopped, `inner` FP32 V-cycles
// solve A e = r32 from e = 0 and u += fp64(e).  On tile levels the first inner cycle's
// pre pass starts from zero without reading e, and the last inner cycle's post pass adds
// its result into u itself.  Every kernel, FP32 cycles included, checks the outer active
// flag, so the host looks at the status only near the expected end, as in solve_impl.
int solve_mixed_stacked(fas_grid* g64, fas_grid* g32, const void* rhs, void* u, double tol, int nu1, int nu2,
                        int inner, bool fold_top, int* status_out, int* cycles_out);

int solve_mixed_impl(fas_grid* g64, fas_grid* g32, double dt, double kappa, const void* kcell, const void* rhs,
                     void* u, double tol, int nu1, int nu2, int inner, bool stacked = false, int* status_out = nullptr,
                     int* cycles_out = nullptr)
{
    check_solve_args(g64, rhs, u, nu1, nu2, tol, stacked);
    check_grid(g32);
    if (g32->batch != g64->batch) throw Error(FAS_ERR_ARG, "the two grids must hold the same number of problems");
    if (stacked && kcell) throw Error(FAS_ERR_ARG, "stacked grids take a constant kappa");
    if (g64->dtype != FAS_F64 || g32->dtype != FAS_F32 || !(g32->flags & FAS_FLAG_MIXED_INNER))
        throw Error(FAS_ERR_ARG, "need an FP64 grid and an FP32 grid created with FAS_FLAG_MIXED_INNER");
    if (g64->dim != g32->dim || g64->bc != g32->bc || g64->h != g32->h || g64->L != g32->L)
        throw Error(FAS_ERR_ARG, "the two grids must describe the same hierarchy");
    for (int a = 0; a < 3; ++a)
        if (g64->n[a] != g32->n[a]) throw Error(FAS_ERR_ARG, "the two grids must have the same shape");
    if (inner < 1) throw Error(FAS_ERR_ARG, "inner must be >= 1");
    // the inner grid runs on the outer grid's stream and checks the outer active flag
    struct InnerScope {
        fas_grid* g;
        hipStream_t stream;
        int* active;
        ~InnerScope()
        {
            g->stream = stream;
            g->active = active;
            g->gate = 0;
            g->zero_start = 0;
            g->accum64 = nullptr;
        }
    } inner_scope{g32, g32->stream, g32->active};
    g32->stream = g64->stream;
    set_coefs(g64, dt, kappa, kcell != nullptr);
    set_kappa(g64, kcell, true, false);
    set_coefs(g32, dt, kappa, kcell != nullptr);
    set_kappa(g32, kcell, true);
    memset(&g64->stats, 0, sizeof(g64->stats));
    ensure_host(g64);
    while (g64->cyc_ev_created < 2)
        FAS_HIP_CHECK(hipEventCreateWithFlags(&g64->cyc_ev[g64->cyc_ev_created++], hipEventDisableTiming));
    fas::launch_init_active(g64);
    GateScope gate(g64);
    g32->active = g64->active;
    g32->gate = 1;
    // the finest FP32 passes start from zero and add into u themselves (tile passes, 3D
    // plane marches); else the inner iterate is zeroed and added by kernels of their own
    const bool fold_top = finest_is_tile(g32, nu1, nu2, kcell != nullptr) ||
                          finest_is_march3(g32, nu1, nu2, kcell != nullptr);
    if (stacked) return solve_mixed_stacked(g64, g32, rhs, u, tol, nu1, nu2, inner, fold_top, status_out, cycles_out);
    char* const span = (char*)g64->rnorm;
    const size_t span_bytes = (size_t)((char*)(g64->hist + fas::kHist) - span);
    if (span_bytes > kHostStatus) throw Error(FAS_ERR_ARG, "internal: status span exceeds the pinned buffer");
    auto host_at = [&](const void* dev) { return (char*)g64->host + ((const char*)dev - span); };
    const int kmax = std::min(g64->kmax, fas::kHist - 1);  // corrections
    // after a solve that took c corrections, evaluations 1 .. c are enqueued without a look
    const int horizon = g64->last_cycles > 0 ? g64->last_cycles : 0;
    g64->last_cycles = 0;
    int end = 0;
    auto look = [&]() -> bool {
        FAS_HIP_CHECK(hipMemcpyAsync(g64->host, span, span_bytes, hipMemcpyDeviceToHost, g64->stream));
        FAS_HIP_CHECK(hipEventRecord(g64->cyc_ev[0], g64->stream));
        FAS_HIP_CHECK(hipEventSynchronize(g64->cyc_ev[0]));
        if (*(const int*)host_at(g64->count) != 0) return false;
        end = *(const int*)host_at(g64->cyc);  // evaluation of the stop, -k if not finite
        return true;
    };
    bool stopped = false;
    for (int k = 1; k <= kmax + 1; ++k) {
        const int np = fas::launch_mixed_resid(g64, g64->coef[0], g64->lev[0].kap, rhs, u, g32->mix_r, k == 1);
        if (k == 1) fas::launch_sum_partials(g64, np, g64->rnorm, g64->fpartials);
        fas::launch_sum_update(g64, np, tol, k);
        if ((k > horizon || k == kmax + 1) && (stopped = look())) break;
        if (k == kmax + 1) break;
        // correction k: `inner` cycles for the first, FAS_OPT_MIXED_INNER_NEXT for the later
        const int cyc_k = (k == 1 || g64->mixed_next <= 0) ? inner : g64->mixed_next;
        for (int m = 0; m < cyc_k; ++m) {
            g32->zero_start = m == 0 && fold_top;
            g32->accum64 = m == cyc_k - 1 && fold_top ? (double*)u : nullptr;
            if (m == 0 && !fold_top) fas::launch_zero_f32(g32, g32->lev[0].N, g32->mix_e);
            vcycle_top(g32, g32->mix_r, g32->mix_e, nu1, nu2, false);
        }
        g32->zero_start = 0;
        g32->accum64 = nullptr;
        if (!fold_top) fas::launch_update_mixed(g64, g32->mix_e, u);
    }
    const double nf = sqrt(*(const double*)host_at(g64->rnorm));
    const double* hist = (const double*)host_at(g64->hist);
    const int evals = !stopped ? kmax + 1 : (end < 0 ? -end : end);
    const int corrections = evals - 1;
    g64->stats.rhs_norm = nf;
    for (int i = 0; i < evals && i < 64; ++i) {
        const double nr = sqrt(hist[i]);
        g64->stats.rel_res[i] = nf > 0.0 ? nr / nf : nr;
    }
    g64->stats.cycles = corrections;
    if (stopped && end < 0) {
        g64->stats.status = FAS_ERR_NONFINITE;
        throw Error(FAS_ERR_NONFINITE, "residual norm is not finite");
    }
    const int status = stopped ? FAS_OK : FAS_NOT_CONVERGED;
    g64->stats.status = status;
    if (status == FAS_OK) g64->last_cycles = corrections;
    if (status != FAS_OK) g_last_error = "not converged within kmax outer iterations";
    return status;
}

// The defect correction of solve_mixed_impl over every problem of stacked grids: each
// evaluation's residual, norms and stopping tests, and each inner cycle, serve all
// problems still iterating in one launch per pass.  The host reads the number still
// active near the expected end (after a solve whose slowest problem took c corrections,
// evaluations 1 .. c run without a look).  Every problem's iterates are those of its own
// mixed solve.
int solve_mixed_stacked(fas_grid* g64, fas_grid* g32, const void* rhs, void* u, double tol, int nu1, int nu2,
                        int inner, bool fold_top, int* status_out, int* cycles_out)
{
    const int kmax = std::min(g64->kmax, fas::kHist - 1);
    const int horizon = g64->last_cycles > 0 ? g64->last_cycles : 0;
    g64->last_cycles = 0;
    int* const hcount = (int*)g64->host;
    for (int k = 1; k <= kmax + 1; ++k) {
        const int np = fas::launch_mixed_resid(g64, g64->coef[0], nullptr, rhs, u, g32->mix_r, k == 1);
        if (k == 1) fas::launch_sum_partials(g64, np, g64->rnorm, g64->fpartials);
        fas::launch_sum_partials(g64, np);
        fas::launch_update_active(g64, tol, k);
        if (k > horizon || k == kmax + 1) {
            FAS_HIP_CHECK(hipMemcpyAsync(hcount, g64->count, sizeof(int), hipMemcpyDeviceToHost, g64->stream));
            FAS_HIP_CHECK(hipStreamSynchronize(g64->stream));
            if (hcount[0] == 0) break;
        }
        if (k == kmax + 1) break;
        // correction k: `inner` cycles for the first, FAS_OPT_MIXED_INNER_NEXT for the later
        const int cyc_k = (k == 1 || g64->mixed_next <= 0) ? inner : g64->mixed_next;
        for (int m = 0; m < cyc_k; ++m) {
            g32->zero_start = m == 0 && fold_top;
            g32->accum64 = m == cyc_k - 1 && fold_top ? (double*)u : nullptr;
            if (m == 0 && !fold_top) fas::launch_zero_f32(g32, g32->lev[0].N, g32->mix_e);
            vcycle_top(g32, g32->mix_r, g32->mix_e, nu1, nu2, false);
        }
        g32->zero_start = 0;
        g32->accum64 = nullptr;
        if (!fold_top) fas::launch_update_mixed(g64, g32->mix_e, u);
    }
    // cyc[b]: evaluation at which problem b stopped (0: none, -k: not finite)
    std::vector<int> cyc((size_t)g64->batch);
    FAS_HIP_CHECK(hipMemcpyAsync(cyc.data(), g64->cyc, cyc.size() * sizeof(int), hipMemcpyDeviceToHost, g64->stream));
    FAS_HIP_CHECK(hipStreamSynchronize(g64->stream));
    int worst = FAS_OK, maxc = 0;
    for (int b = 0; b < g64->batch; ++b) {
        const int c = cyc[(size_t)b];
        const int st = c > 0 ? FAS_OK : (c < 0 ? FAS_ERR_NONFINITE : FAS_NOT_CONVERGED);
        const int corrections = (c > 0 ? c : (c < 0 ? -c : kmax + 1)) - 1;
        if (status_out) status_out[b] = st;
        if (cycles_out) cycles_out[b] = corrections;
        if (st == FAS_ERR_NONFINITE) worst = FAS_ERR_NONFINITE;
        else if (st == FAS_NOT_CONVERGED && worst == FAS_OK) worst = FAS_NOT_CONVERGED;
        maxc = std::max(maxc, corrections);
    }
    g64->stats.cycles = maxc;
    g64->stats.status = worst;
    if (worst == FAS_OK) g64->last_cycles = maxc;
    if (worst == FAS_ERR_NONFINITE) throw Error(FAS_ERR_NONFINITE, "a residual norm is not finite");
    if (worst == FAS_NOT_CONVERGED) g_last_error = "some problems did not converge within kmax outer iterations";
    return worst;
}

int vcycle_impl(fas_grid* g, double dt, double kappa, const void* kcell, const void* rhs, void* u, int nu1, int nu2,
                double* rel_res, bool transposed)
{
    check_solve_args(g, rhs, u, nu1, nu2, 0.0);
    set_coefs(g, dt, kappa, kcell != nullptr);
    set_kappa(g, kcell, g->dtype == FAS_F64);
    double nf = 0.0;
    if (rel_res) {
        fas::launch_resid_norm(g, 0, g->coef[0], g->lev[0].kap, rhs, nullptr);
        nf = read_norm(g);
    }
    vcycle_top(g, rhs, u, nu1, nu2, transposed, rel_res != nullptr);
    if (rel_res) {
        const double nr = read_norm(g);
        *rel_res = nf > 0.0 ? nr / nf : nr;
    }
    return FAS_OK;
}

// Fills *g (host memory owned by the caller) with the plan of a grid over `workspace`;
// allocates nothing.  Returns FAS_OK or an error code with the message set.
int setup_grid(fas_grid* g, int dim, const int64_t n[3], double h, int bc, int dtype, int coarsest, int flags,
               int batch, void* workspace, size_t ws_bytes, void* stream)
{
    if (!n) return fail(FAS_ERR_ARG, "null argument");
    if (!(h > 0.0) || !isfinite(h)) return fail(FAS_ERR_ARG, "h must be positive");
    if (bc != FAS_BC_NEUMANN && bc != FAS_BC_DIRICHLET && bc != FAS_BC_PERIODIC)
        return fail(FAS_ERR_ARG, "unknown boundary condition");
    Layout lay;
    std::string why;
    int rc = plan(dim, n, dtype, coarsest, flags, batch, &lay, &why);
    if (rc) return fail(rc, why);
    if (bc == FAS_BC_PERIODIC)
        for (int a = 0; a < dim; ++a)
            if (lay.n[lay.L][a] & 1) return fail(FAS_ERR_SHAPE, "periodic grids need even sizes on every level");
    if (!workspace) return fail(FAS_ERR_ARG, "null workspace");
    if ((uintptr_t)workspace % kAlign) return fail(FAS_ERR_ARG, "workspace must be 256-byte aligned");
    if (ws_bytes < lay.total)
        return fail(FAS_ERR_NOMEM, "workspace too small: need " + std::to_string(lay.total) + " bytes");
    memset(g, 0, sizeof(*g));
    g->dim = dim;
    g->bc = bc;
    g->dtype = dtype;
    g->coarsest = coarsest;
    g->flags = flags;
    g->L = lay.L;
    g->h = h;
    for (int a = 0; a < 3; ++a) g->n[a] = a < dim ? n[a] : 1;
    char* base = (char*)workspace;
    for (int l = 0; l <= lay.L; ++l) {
        fas::Level& Lv = g->lev[l];
        Lv.N = 1;
        for (int a = 0; a < 3; ++a) {
            Lv.n[a] = lay.n[l][a];
            Lv.N *= Lv.n[a];
        }
        Lv.h = h * (double)((int64_t)1 << l);
        Lv.x = base + lay.x[l];
        Lv.u = l ? base + lay.u[l] : nullptr;
        Lv.f = l ? base + lay.f[l] : nullptr;
        Lv.r = lay.r[l] ? base + lay.r[l] : nullptr;
        Lv.kap_slot = lay.kap[l] ? base + lay.kap[l] : nullptr;
        Lv.kap = nullptr;
    }
    g->mix_e = (flags & FAS_FLAG_MIXED_INNER) ? base + lay.mix_e : nullptr;
    g->mix_r = (flags & FAS_FLAG_MIXED_INNER) ? base + lay.mix_r : nullptr;
    g->partials = (double*)(base + lay.partials);
    g->fpartials = (double*)(base + lay.fpartials);
    g->desc = base + lay.desc;
    g->norm_out = (double*)(base + lay.norm_out);
    g->npartials = lay.npartials;
    g->batch = batch;
    g->rnorm = (double*)(base + lay.rnorm);
    g->active = (int*)(base + lay.active);
    g->cyc = (int*)(base + lay.cyc);
    g->count = (int*)(base + lay.count);
    g->hist = (double*)(base + lay.hist);
    g->stream = (hipStream_t)stream;
    g->kmax = 100;
    g->nuc = 2;
    g->fused = 1;
    g->fused_opt = 1;
    g->order = FAS_ORDER_X;
    g->symmetric = 0;
    g->tile_max = INT64_MAX;
    g->tile_waves = 0;
    g->march3_ns = 2;
    g->host = nullptr;  // pinned scalar for norm read-back, allocated on first use
    return FAS_OK;
}

// ---- the solve without allocation: workspace in a static device buffer ------------------
// Callers that cannot allocate (HIP graph capture, serving loops) get fas_solve_noalloc: the
// grid plan lives on the host stack and its workspace is `scratch`, one per GPU, held until
// the process ends.  In host code `scratch` names a host-side stand-in, so the device address
// is looked up once per device (hipGetSymbolAddress, with that device current) and only that
// address is handed to kernels.
constexpr int kStaticDevices = 64;

std::mutex& static_mutex()
{
    static std::mutex m;
    return m;
}

void* static_workspace()
{
    static void* addr[kStaticDevices] = {};
    int dev = 0;
    FAS_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kStaticDevices) throw Error(FAS_ERR_ARG, "device index out of range");
    std::lock_guard<std::mutex> lock(static_mutex());
    if (!addr[dev]) {
        void* p = nullptr;
        FAS_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || (uintptr_t)p % kAlign) throw Error(FAS_ERR_HIP, "static workspace has no usable device address");
        addr[dev] = p;
    }
    return addr[dev];
}

// fas_solve on a grid planned inside the call over the static workspace.  The loop is
// solve_impl's without its pinned buffer, events and look-ahead: after each cycle the
// device-side stopping test runs and the host reads the number of active problems (one
// int into pageable memory) before enqueuing the next cycle.  Every workspace region a
// cycle reads is written earlier in the same call (level arrays by restriction and the
// coarse right-hand side, partial sums by the passes, flags and counts by
// launch_init_active), so nothing left by an earlier call is ever read.
int solve_noalloc_impl(int dim, const int64_t n[3], double h, int bc, int dtype, int coarsest, void* stream,
                       double dt, double kappa, const void* kcell, const void* rhs, void* u, double tol, int nu1,
                       int nu2, int kmax, int* cycles_out)
{
    if (!n) throw Error(FAS_ERR_ARG, "null argument");
    if (kmax < 1) throw Error(FAS_ERR_ARG, "kmax must be >= 1");
    const int flags = kcell ? FAS_FLAG_VARIABLE_KAPPA : 0;
    Layout lay;
    std::string why;
    if (const int rc = plan(dim, n, dtype, coarsest, flags, 1, &lay, &why)) throw Error(rc, why);
    if (lay.total > kStaticWorkspace)
        throw Error(FAS_ERR_NOMEM, "grid needs " + std::to_string(lay.total) + " bytes of workspace; the static buffer "
                                   "holds " + std::to_string(kStaticWorkspace));
    fas_grid g{};
    if (const int rc = setup_grid(&g, dim, n, h, bc, dtype, coarsest, flags, 1, static_workspace(), kStaticWorkspace,
                                  stream))
        throw Error(rc, g_last_error);
    g.kmax = kmax;
    check_solve_args(&g, rhs, u, nu1, nu2, tol);
    set_coefs(&g, dt, kappa, kcell != nullptr);
    set_kappa(&g, kcell, dtype == FAS_F64);
    fas::launch_init_active(&g);
    fas::launch_resid_norm(&g, 0, g.coef[0], g.lev[0].kap, rhs, nullptr);
    FAS_HIP_CHECK(hipMemcpyAsync(g.rnorm, g.norm_out, sizeof(double), hipMemcpyDeviceToDevice, g.stream));
    GateScope gate(&g);
    g.defer_norm = 1;
    int alive = 1, k = 0;
    while (alive && k < kmax) {
        ++k;
        g.deferred_np = 0;
        vcycle_top(&g, rhs, u, nu1, nu2, false, true);
        if (g.deferred_np > 0)
            fas::launch_sum_update(&g, g.deferred_np, tol, k);
        else
            fas::launch_update_active(&g, tol, k);
        FAS_HIP_CHECK(hipMemcpyAsync(&alive, g.count, sizeof(int), hipMemcpyDeviceToHost, g.stream));
        FAS_HIP_CHECK(hipStreamSynchronize(g.stream));
    }
    int stop = 0;
    FAS_HIP_CHECK(hipMemcpyAsync(&stop, g.cyc, sizeof(int), hipMemcpyDeviceToHost, g.stream));
    FAS_HIP_CHECK(hipStreamSynchronize(g.stream));
    if (cycles_out) *cycles_out = stop > 0 ? stop : (stop < 0 ? -stop : k);
    if (stop < 0) throw Error(FAS_ERR_NONFINITE, "residual norm is not finite");
    if (stop == 0) {
        g_last_error = "not converged within kmax cycles";
        return FAS_NOT_CONVERGED;
    }
    return FAS_OK;
}


// ---- array-form batched solve ------------------------------------------------------------
// Problems of any sizes, each on its own grid, advanced together: per V-cycle, the pre
// passes from the tallest hierarchy's finest level down (one table launch per height,
// serving every problem with a tile level at that height: height = levels below), the
// tails (one workgroup per problem), the post passes back up, then the norm totals and
// stopping tests of all problems in one launch.  Every problem's passes are those of its
// single solve with the same arguments, so its iterates, norms and cycle count are the
// single solve's.

// Whether problem grid g takes the table path: 2D, two-colour fused passes, a tile pass
// (1..3 sweeps) on every level above its tail, and the tile partial sums in its buffers.
bool table_ok(const fas_grid* g, int nu1, int nu2, bool kv)
{
    if (g->dim != 2 || g->batch != 1 || !g->fused) return false;
    const int T = fas::tail_top(g);
    if (T < 1 || T > g->L) return false;
    for (int l = 0; l < T; ++l)
        if (!fas::tile_ok(g, l, nu1, nu2, kv)) return false;
    return fas::tile_count(g, 0, nu1) <= g->npartials && fas::tile_count(g, 0, nu2) <= g->npartials;
}

struct TableProblem {
    fas_grid* g;
    int T;                  // tile levels 0..T-1, tail from level T
    int height;             // levels below the finest (L)
    size_t tile_bytes;
    int blocks[3][fas::kMaxLevels];  // blocks of pre, first-cycle pre and post launches per level
    char* host;             // staging of the descriptors (pinned)
    // device addresses in the grid's descriptor region
    const void* status() const { return g->desc; }
    const void* tail() const { return (const char*)g->desc + 256; }
    const void* tile(int kind, int l) const
    {
        return (const char*)g->desc + 256 + 2048 + (size_t)(3 * l + kind) * tile_bytes;
    }
};

// Builds problem p's descriptors in its pinned staging area and uploads them when they
// differ from what the grid's descriptor region already holds.
void build_table_problem(TableProblem& P, const void* rhs, void* u, int nu1, int nu2, int wv, hipStream_t stream)
{
    fas_grid* g = P.g;
    ensure_host(g);
    const size_t tb = fas::tile_desc_bytes(g->dtype);
    P.tile_bytes = tb;
    if (256 + 2048 + (size_t)3 * P.T * tb > fas::kDescBytes || fas::tail_desc_bytes(g->dtype) > 2048 ||
        sizeof(fas::StatusDesc) > 256)
        throw Error(FAS_ERR_ARG, "internal: batched-solve descriptors exceed their region");
    std::vector<char> d(fas::kDescBytes, 0);
    const int first = (g->dim + 1) & 1;
    const int* act = g->active;
    for (int l = 0; l < P.T; ++l) {
        fas::Level& F = g->lev[l];
        fas::Level& C = g->lev[l + 1];
        void* const rc = l + 1 == P.T ? C.f : C.r;  // the tail forms f from C.f in place
        const void* fin = l == 0 ? rhs : F.r;
        void* const fout = l == 0 ? nullptr : F.f;
        void* const uin = l == 0 ? u : F.u;
        char* const base = d.data() + 256 + 2048;
        P.blocks[0][l] = fas::fill_tile_desc(g, l, g->coef[l], nu1, wv, false, fin, uin, F.x, C.u, rc, fout, nullptr,
                                             act, base + (size_t)(3 * l + 0) * tb);
        P.blocks[1][l] = l == 0 ? fas::fill_tile_desc(g, l, g->coef[l], nu1, wv, false, fin, uin, F.x, C.u, rc, nullptr,
                                                      g->fpartials, act, base + (size_t)(3 * l + 1) * tb)
                                : P.blocks[0][l];
        // post: f, u_in = the pre pass's output, u_out, uc = the coarse level's new values
        P.blocks[2][l] = fas::fill_tile_desc(g, l, g->coef[l], nu2, wv, true, l == 0 ? rhs : F.f, F.x,
                                             l == 0 ? u : F.u, C.u, nullptr, nullptr,
                                             l == 0 ? g->partials : nullptr, act, base + (size_t)(3 * l + 2) * tb);
    }
    fas::fill_tail_desc(g, P.T, g->coef, nu1, nu2, first, g->lev[P.T].u, g->lev[P.T].f, true, act, d.data() + 256);
    fas::StatusDesc sd{};
    sd.partials = g->partials;
    sd.fpartials = g->fpartials;
    sd.count = P.blocks[2][0];
    sd.fcount = P.blocks[1][0];
    sd.rnorm = g->rnorm;
    sd.norm_out = g->norm_out;
    sd.act = g->active;
    sd.cyc = g->cyc;
    sd.hist = g->hist;
    sd.atol2 = g->atol * g->atol;
    memcpy(d.data(), &sd, sizeof(sd));
    P.host = (char*)g->host + kHostStatus;
    if (!g->desc_valid || memcmp(P.host, d.data(), fas::kDescBytes) != 0) {
        memcpy(P.host, d.data(), fas::kDescBytes);
        FAS_HIP_CHECK(hipMemcpyAsync(g->desc, P.host, fas::kDescBytes, hipMemcpyHostToDevice, stream));
        g->desc_valid = 1;
    }
}

// Table launches over a list of (descriptor, blocks) entries, in chunks of kBatchChunk.
template <typename Launch>
void for_chunks(const std::vector<std::pair<const void*, int>>& items, Launch&& launch)
{
    for (size_t i0 = 0; i0 < items.size(); i0 += fas::kBatchChunk) {
        fas::TableLaunch t;
        memset(&t, 0, sizeof(t));
        t.np = (int)std::min(items.size() - i0, (size_t)fas::kBatchChunk);
        int acc = 0;
        for (int p = 0; p < t.np; ++p) {
            t.desc[p] = items[i0 + p].first;
            t.first[p] = acc;
            acc += items[i0 + p].second;
        }
        t.first[t.np] = acc;
        launch(t, i0);
    }
}

int solve_table_impl(int nprob, fas_grid* const* grids, double dt, const fas_kappa_t* kappa,
                     const void* const* rhs, void* const* u, double tol, int nu1, int nu2, int* status_out)
{
    fas_grid* const lead = grids[0];
    hipStream_t stream = lead->stream;
    const bool kv = kappa[0].cell != nullptr;
    const int dtype = lead->dtype;
    // every problem's work runs on the first grid's stream
    struct StreamScope {
        int n;
        fas_grid* const* g;
        std::vector<hipStream_t> saved;
        ~StreamScope()
        {
            for (int p = 0; p < n; ++p) g[p]->stream = saved[(size_t)p];
        }
    } scope{nprob, grids, {}};
    for (int p = 0; p < nprob; ++p) scope.saved.push_back(grids[p]->stream);
    for (int p = 0; p < nprob; ++p) grids[p]->stream = stream;
    const int wv = fas::tile_waves(lead, 0, nu1);
    std::vector<TableProblem> P((size_t)nprob);
    int hmax = 0;
    for (int p = 0; p < nprob; ++p) {
        fas_grid* g = grids[p];
        set_coefs(g, dt, kappa[p].scalar, kv);
        set_kappa(g, kappa[p].cell, dtype == FAS_F64);
        memset(&g->stats, 0, sizeof(g->stats));
        TableProblem& Q = P[(size_t)p];
        Q.g = g;
        Q.T = fas::tail_top(g);
        Q.height = g->L;
        hmax = std::max(hmax, g->L);
        if (fas::tile_waves(g, 0, nu1) != wv || fas::tile_waves(g, 0, nu2) != wv)
            throw Error(FAS_ERR_ARG, "batched problems must share the tile shape (FAS_OPT_TILE_WAVES)");
        build_table_problem(Q, rhs[p], u[p], nu1, nu2, wv, stream);
    }
    // launch lists per height (pre, first-cycle pre, post) and tails per height
    typedef std::vector<std::pair<const void*, int>> Items;
    std::vector<Items> pre((size_t)hmax + 1), pre1((size_t)hmax + 1), post((size_t)hmax + 1), tail((size_t)hmax + 1);
    Items status;
    for (const TableProblem& Q : P) {
        for (int l = 0; l < Q.T; ++l) {
            const size_t h = (size_t)(Q.height - l);
            pre[h].push_back({Q.tile(0, l), Q.blocks[0][l]});
            pre1[h].push_back({Q.tile(l == 0 ? 1 : 0, l), Q.blocks[1][l]});
            post[h].push_back({Q.tile(2, l), Q.blocks[2][l]});
        }
        tail[(size_t)(Q.height - Q.T)].push_back({Q.tail(), 1});
        status.push_back({Q.status(), 1});
    }
    const int first = (lead->dim + 1) & 1;
    for_chunks(status, [&](const fas::TableLaunch& t, size_t) { fas::launch_batch_init(stream, t); });
    ensure_host(lead);
    const int horizon = lead->last_cycles > 2 ? lead->last_cycles - 2 : 0;
    lead->last_cycles = 0;
    const int kmax = lead->kmax;
    int* const hcount = (int*)lead->host;
    for (int k = 1; k <= kmax; ++k) {
        for (int h = hmax; h >= 0; --h) {
            for_chunks(k == 1 ? pre1[(size_t)h] : pre[(size_t)h], [&](const fas::TableLaunch& t, size_t) {
                fas::launch_tile_table(stream, dtype, false, nu1, first, kv, wv, t);
            });
            for_chunks(tail[(size_t)h],
                       [&](const fas::TableLaunch& t, size_t) { fas::launch_tail_table(stream, dtype, 2, kv, t); });
        }
        for (int h = 0; h <= hmax; ++h)
            for_chunks(post[(size_t)h], [&](const fas::TableLaunch& t, size_t) {
                fas::launch_tile_table(stream, dtype, true, nu2, first, kv, wv, t);
            });
        if (k == 1) for_chunks(status, [&](const fas::TableLaunch& t, size_t) { fas::launch_batch_fsum(stream, t); });
        for_chunks(status, [&](const fas::TableLaunch& t, size_t) { fas::launch_batch_update(stream, t, tol, k); });
        for_chunks(status, [&](const fas::TableLaunch& t, size_t i0) {
            fas::launch_batch_alive(stream, t, lead->count, i0 > 0);
        });
        if (k <= horizon && k < kmax) continue;
        FAS_HIP_CHECK(hipMemcpyAsync(hcount, lead->count, sizeof(int), hipMemcpyDeviceToHost, stream));
        FAS_HIP_CHECK(hipStreamSynchronize(stream));
        if (hcount[0] == 0) break;
    }
    // per problem: {cycle of the stop, ||rhs||^2, squared norms after each cycle} gathered
    // into the first grid's partial-sum buffer, free once the cycles are done
    const int stride = (int)std::min<int64_t>(fas::kHist + 2, lead->npartials / nprob);
    if (stride < 2) throw Error(FAS_ERR_ARG, "internal: batch status does not fit the partial-sum buffer");
    for_chunks(status, [&](const fas::TableLaunch& t, size_t i0) {
        fas::launch_batch_gather(stream, t, lead->partials, (int)i0, stride);
    });
    std::vector<double> gat((size_t)nprob * stride);
    FAS_HIP_CHECK(hipMemcpyAsync(gat.data(), lead->partials, gat.size() * sizeof(double), hipMemcpyDeviceToHost,
                                 stream));
    FAS_HIP_CHECK(hipStreamSynchronize(stream));
    int worst = FAS_OK, maxc = 0;
    for (int p = 0; p < nprob; ++p) {
        const double* r = gat.data() + (size_t)p * stride;
        const int c = (int)r[0];
        const int st = c > 0 ? FAS_OK : (c < 0 ? FAS_ERR_NONFINITE : FAS_NOT_CONVERGED);
        const int cycles = c > 0 ? c : (c < 0 ? -c : kmax);
        fas_stats_t& S = grids[p]->stats;
        S.cycles = cycles;
        S.status = st;
        S.rhs_norm = sqrt(r[1]);
        for (int i = 0; i < cycles && i < stride - 2; ++i) {
            const double nr = sqrt(r[2 + i]);
            S.rel_res[i] = S.rhs_norm > 0.0 ? nr / S.rhs_norm : nr;
        }
        if (status_out) status_out[p] = st;
        if (st == FAS_ERR_NONFINITE) worst = FAS_ERR_NONFINITE;
        else if (st == FAS_NOT_CONVERGED && worst == FAS_OK) worst = FAS_NOT_CONVERGED;
        maxc = std::max(maxc, cycles);
    }
    if (worst == FAS_OK) lead->last_cycles = maxc;
    if (worst == FAS_ERR_NONFINITE) throw Error(FAS_ERR_NONFINITE, "a residual norm is not finite");
    if (worst == FAS_NOT_CONVERGED) g_last_error = "some problems did not converge within kmax cycles";
    return worst;
}

int solve_batched_impl(int nprob, const fas_grid_t* grids, double dt, const fas_kappa_t* kappa,
                       const void* const* rhs, void* const* u, double tol, int nu1, int nu2, int* status_out)
{
    if (nprob < 1 || !grids || !kappa || !rhs || !u) throw Error(FAS_ERR_ARG, "bad batch arguments");
    std::vector<fas_grid*> gs((size_t)nprob);
    for (int p = 0; p < nprob; ++p) {
        fas_grid* g = grids[p];
        check_solve_args(g, rhs[p], u[p], nu1, nu2, tol);
        if (g->dtype != grids[0]->dtype) throw Error(FAS_ERR_ARG, "batched problems must share the dtype");
        if ((kappa[p].cell != nullptr) != (kappa[0].cell != nullptr))
            throw Error(FAS_ERR_ARG, "batched problems take all constant kappa or all cell kappa");
        gs[(size_t)p] = g;
    }
    {
        std::vector<fas_grid*> sorted = gs;
        std::sort(sorted.begin(), sorted.end());
        if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
            throw Error(FAS_ERR_ARG, "a grid appears twice in one batch");
    }
    const bool kv = kappa[0].cell != nullptr;
    bool table = true;
    for (int p = 0; p < nprob && table; ++p) table = table_ok(gs[(size_t)p], nu1, nu2, kv);
    if (table) return solve_table_impl(nprob, gs.data(), dt, kappa, rhs, u, tol, nu1, nu2, status_out);
    // otherwise (3D grids, levels without tile passes, other set orders): one solve after
    // another, each on its own grid's stream
    int worst = FAS_OK;
    for (int p = 0; p < nprob; ++p) {
        int st;
        try {
            st = solve_impl(gs[(size_t)p], dt, kappa[p].scalar, kappa[p].cell, rhs[p], u[p], tol, nu1, nu2, false);
        } catch (const Error& e) {
            if (e.code != FAS_ERR_NONFINITE) throw;
            st = FAS_ERR_NONFINITE;
        }
        if (status_out) status_out[p] = st;
        if (st == FAS_ERR_NONFINITE) worst = FAS_ERR_NONFINITE;
        else if (st == FAS_NOT_CONVERGED && worst == FAS_OK) worst = FAS_NOT_CONVERGED;
    }
    if (worst == FAS_ERR_NONFINITE) throw Error(FAS_ERR_NONFINITE, "a residual norm is not finite");
    if (worst == FAS_NOT_CONVERGED) g_last_error = "some problems did not converge within kmax cycles";
    return worst;
}

}  // namespace

void fas::set_last_error(const std::string& msg) { g_last_error = msg; }

extern "C" {

size_t fas_workspace_size(int dim, const int64_t n[3], int dtype, int coarsest, int flags)
{
    return fas_workspace_size_batched(dim, n, dtype, coarsest, flags, 1);
}

size_t fas_workspace_size_batched(int dim, const int64_t n[3], int dtype, int coarsest, int flags, int batch)
{
    if (!n) return 0;
    Layout lay;
    std::string why;
    if (plan(dim, n, dtype, coarsest, flags, batch, &lay, &why)) return 0;
    return lay.total;
}

int fas_grid_create(int dim, const int64_t n[3], double h, int bc, int dtype, int coarsest, int flags, void* workspace,
                    size_t ws_bytes, void* stream, fas_grid_t* out)
{
    return fas_grid_create_batched(dim, n, h, bc, dtype, coarsest, flags, 1, workspace, ws_bytes, stream, out);
}

int fas_grid_create_batched(int dim, const int64_t n[3], double h, int bc, int dtype, int coarsest, int flags,
                            int batch, void* workspace, size_t ws_bytes, void* stream, fas_grid_t* out)
{
    return guarded([&]() -> int {
        if (!out || !n) return fail(FAS_ERR_ARG, "null argument");
        *out = nullptr;
        fas_grid* g = new fas_grid();
        const int rc = setup_grid(g, dim, n, h, bc, dtype, coarsest, flags, batch, workspace, ws_bytes, stream);
        if (rc) {
            delete g;
            return rc;
        }
        *out = g;
        return FAS_OK;
    });
}

int fas_grid_destroy(fas_grid_t g)
{
    if (!g) return FAS_OK;
    if (g->graph_cache) {
        GraphCache* gc = (GraphCache*)g->graph_cache;
        gc->drop();
        if (gc->cap) (void)hipStreamDestroy(gc->cap);
        delete gc;
    }
    if (g->host) (void)hipHostFree(g->host);
    for (int i = 0; i < g->ev_created; ++i) (void)hipEventDestroy(g->ev[i]);
    for (int i = 0; i < g->cyc_ev_created; ++i) (void)hipEventDestroy(g->cyc_ev[i]);
    delete g;
    return FAS_OK;
}

int fas_grid_set(fas_grid_t g, int option, double value)
{
    return guarded([&]() -> int {
        check_grid(g);
        if (option == FAS_OPT_ATOL) {
            if (!(value >= 0.0) || !isfinite(value)) return fail(FAS_ERR_ARG, "atol must be finite and >= 0");
            g->atol = value;
            g->desc_valid = 0;  // the batched solve's status descriptor holds it
            return FAS_OK;
        }
        const int v = (int)value;
        if ((double)v != value) return fail(FAS_ERR_ARG, "option value must be an integer");
        // options that change no captured launch keep the graph
        if (option != FAS_OPT_KMAX && option != FAS_OPT_PROFILE && option != FAS_OPT_MIXED_INNER_NEXT) drop_graph(g);
        switch (option) {
            case FAS_OPT_KMAX:
                if (v < 1) return fail(FAS_ERR_ARG, "kmax must be >= 1");
                g->kmax = v;
                return FAS_OK;
            case FAS_OPT_COARSE_SWEEPS:
                if (v < 1) return fail(FAS_ERR_ARG, "coarse sweeps must be >= 1");
                g->nuc = v;
                return FAS_OK;
            case FAS_OPT_MIXED_INNER_NEXT:
                if (v < 0 || v > 1000) return fail(FAS_ERR_ARG, "mixed inner cycles must be 0..1000");
                g->mixed_next = v;
                return FAS_OK;
            case FAS_OPT_PROFILE:
                if (v != 0 && v != 1) return fail(FAS_ERR_ARG, "profile must be 0 or 1");
                g->profile = v;
                return FAS_OK;
            case FAS_OPT_GRAPH:
                if (v != 0 && v != 1) return fail(FAS_ERR_ARG, "graph must be 0 or 1");
                g->use_graph = v;
                return FAS_OK;
            case FAS_OPT_AUTOTUNE:
                if (v != 0 && v != 1) return fail(FAS_ERR_ARG, "autotune must be 0 or 1");
                g->autotune = v;
                g->tuned = 0;
                if (!v)
                    for (int l = 0; l < fas::kMaxLevels; ++l) g->seg_rows[l] = g->tile_wv[l] = g->tile_grp[l] = 0;
                return FAS_OK;
            case FAS_OPT_FUSED:
                if (v != 0 && v != 1) return fail(FAS_ERR_ARG, "fused must be 0 or 1");
                g->fused_opt = v;
                g->fused = v && two_colour(g);
                return FAS_OK;
            case FAS_OPT_ORDER:
                if (v != FAS_ORDER_X && v != FAS_ORDER_U && v != FAS_ORDER_Z)
                    return fail(FAS_ERR_ARG, "order must be FAS_ORDER_X, FAS_ORDER_U or FAS_ORDER_Z");
                g->order = v;
                g->fused = g->fused_opt && two_colour(g);
                return FAS_OK;
            case FAS_OPT_SYMMETRIC:
                if (v != 0 && v != 1) return fail(FAS_ERR_ARG, "symmetric must be 0 or 1");
                g->symmetric = v;
                g->fused = g->fused_opt && two_colour(g);
                return FAS_OK;
            case FAS_OPT_SEG_ROWS:
                if (v != 0 && (v < fas::kMinSegRows || (v & 1)))
                    return fail(FAS_ERR_ARG, "segment height must be 0 or an even number >= 8");
                g->seg_force = v;
                return FAS_OK;
            case FAS_OPT_TILE:
                if (value < 0) return fail(FAS_ERR_ARG, "tile level size must be >= 0");
                g->tile_max = v;
                return FAS_OK;
            case FAS_OPT_TILE_WAVES:
                if (v != 0 && (v < 6 || v > 16)) return fail(FAS_ERR_ARG, "tile waves must be 0 or 6..16");
                g->tile_waves = v;
                return FAS_OK;
            case FAS_OPT_MARCH3_SWEEPS:
                if (v != 1 && v != 2) return fail(FAS_ERR_ARG, "3D march sweeps per pass must be 1 or 2");
                g->march3_ns = v;
                return FAS_OK;
        }
        return fail(FAS_ERR_ARG, "unknown option");
    });
}

int fas_set_stream(fas_grid_t g, void* stream)
{
    if (!g) return fail(FAS_ERR_ARG, "null grid");
    g->stream = (hipStream_t)stream;
    return FAS_OK;
}

int fas_grid_levels(fas_grid_t g) { return g ? g->L : fail(FAS_ERR_ARG, "null grid"); }

int64_t fas_level_cells(fas_grid_t g, int level)
{
    if (!g || level < 0 || level > g->L) return fail(FAS_ERR_ARG, "bad grid or level");
    return g->lev[level].N;
}

int fas_solve(fas_grid_t g, double dt, double kappa, const void* kappa_cell, const void* rhs, void* u, double tol,
              int nu1, int nu2)
{
    return guarded([&] { return solve_impl(g, dt, kappa, kappa_cell, rhs, u, tol, nu1, nu2, false); });
}

int fas_solve_transposed(fas_grid_t g, double dt, double kappa, const void* kappa_cell, const void* rhs, void* u,
                         double tol, int nu1, int nu2)
{
    return guarded([&] { return solve_impl(g, dt, kappa, kappa_cell, rhs, u, tol, nu1, nu2, true); });
}

int fas_vcycle(fas_grid_t g, double dt, double kappa, const void* kappa_cell, const void* rhs, void* u, int nu1,
               int nu2, double* rel_res)
{
    return guarded([&] { return vcycle_impl(g, dt, kappa, kappa_cell, rhs, u, nu1, nu2, rel_res, false); });
}

int fas_vcycle_transposed(fas_grid_t g, double dt, double kappa, const void* kappa_cell, const void* rhs, void* u,
                          int nu1, int nu2, double* rel_res)
{
    return guarded([&] { return vcycle_impl(g, dt, kappa, kappa_cell, rhs, u, nu1, nu2, rel_res, true); });
}

int fas_smooth(fas_grid_t g, int level, double dt, double kappa, const void* kappa_cell, const void* rhs, void* u,
               int sweeps, int reverse)
{
    return guarded([&]() -> int {
        check_grid(g);
        if (g->batch > 1) return fail(FAS_ERR_ARG, "building blocks take a single-problem grid");
        check_level(g, level, false);
        if (!rhs || !u || rhs == u || sweeps < 0) return fail(FAS_ERR_ARG, "bad smoother arguments");
        if (kappa_cell && !(g->flags & FAS_FLAG_VARIABLE_KAPPA))
            return fail(FAS_ERR_ARG, "cell kappa needs FAS_FLAG_VARIABLE_KAPPA");
        set_coefs(g, dt, kappa, kappa_cell != nullptr);
        smooth_kap(g, level, kappa_cell, rhs, u, sweeps, reverse != 0);
        return FAS_OK;
    });
}

int fas_residual(fas_grid_t g, int level, double dt, double kappa, const void* kappa_cell, const void* rhs,
                 const void* u, void* r, double* norm2)
{
    return guarded([&]() -> int {
        check_grid(g);
        if (g->batch > 1) return fail(FAS_ERR_ARG, "building blocks take a single-problem grid");
        check_level(g, level, false);
        if (!rhs || !u || !r || r == u || r == rhs) return fail(FAS_ERR_ARG, "bad residual arguments");
        if (kappa_cell && !(g->flags & FAS_FLAG_VARIABLE_KAPPA))
            return fail(FAS_ERR_ARG, "cell kappa needs FAS_FLAG_VARIABLE_KAPPA");
        set_coefs(g, dt, kappa, kappa_cell != nullptr);
        fas::launch_residual(g, level, g->coef[level], kappa_cell, rhs, u, r);
        if (norm2) {
            fas::launch_resid_norm(g, level, g->coef[level], kappa_cell, r, nullptr);
            *norm2 = read_norm(g);
        }
        return FAS_OK;
    });
}

int fas_restrict(fas_grid_t g, int level, const void* fine, void* coarse)
{
    return guarded([&]() -> int {
        check_grid(g);
        if (g->batch > 1) return fail(FAS_ERR_ARG, "building blocks take a single-problem grid");
        check_level(g, level, true);
        if (!fine || !coarse || fine == coarse) return fail(FAS_ERR_ARG, "bad restriction arguments");
        fas::launch_restrict(g, level, fine, coarse);
        return FAS_OK;
    });
}

int fas_prolong_add(fas_grid_t g, int level, const void* c_new, const void* c_old, void* fine)
{
    return guarded([&]() -> int {
        check_grid(g);
        if (g->batch > 1) return fail(FAS_ERR_ARG, "building blocks take a single-problem grid");
        check_level(g, level, true);
        if (!c_new || !c_old || !fine) return fail(FAS_ERR_ARG, "bad prolongation arguments");
        fas::launch_prolong_add(g, level, c_new, c_old, fine);
        return FAS_OK;
    });
}

int fas_kappa_grad(fas_grid_t g, double dt, const void* kappa_cell, const void* mu, const void* u, void* gkappa)
{
    return guarded([&]() -> int {
        check_grid(g);
        if (g->dtype != FAS_F64 || g->batch > 1) return fail(FAS_ERR_ARG, "fas_kappa_grad needs a single FP64 grid");
        if (!kappa_cell || !mu || !u || !gkappa) return fail(FAS_ERR_ARG, "null argument");
        if (gkappa == mu || gkappa == u || gkappa == kappa_cell) return fail(FAS_ERR_ARG, "gkappa must not alias");
        set_coefs(g, dt, 1.0, true);
        fas::launch_kappa_grad(g, g->coef[0], kappa_cell, mu, u, gkappa);
        return FAS_OK;
    });
}

int fas_solve_mixed(fas_grid_t g64, fas_grid_t g32, double dt, double kappa, const void* kappa_cell, const void* rhs,
                    void* u, double tol, int nu1, int nu2, int inner)
{
    return guarded([&]() -> int { return solve_mixed_impl(g64, g32, dt, kappa, kappa_cell, rhs, u, tol, nu1, nu2, inner); });
}

int fas_solve_stacked_mixed(fas_grid_t g64, fas_grid_t g32, double dt, double kappa, const void* rhs, void* u,
                            double tol, int nu1, int nu2, int inner, int* status_out, int* cycles_out)
{
    return guarded([&]() -> int {
        return solve_mixed_impl(g64, g32, dt, kappa, nullptr, rhs, u, tol, nu1, nu2, inner, true, status_out,
                                cycles_out);
    });
}

int fas_solve_stacked(fas_grid_t g, double dt, double kappa, const void* rhs, void* u, double tol, int nu1, int nu2,
                      int* status_out, int* cycles_out)
{
    return guarded([&]() -> int {
        check_solve_args(g, rhs, u, nu1, nu2, tol, true);
        set_coefs(g, dt, kappa, false);
        set_kappa(g, nullptr, false);
        memset(&g->stats, 0, sizeof(g->stats));
        fas::launch_init_active(g);
        // ||rhs||^2 per problem: summed by the first cycle's finest tile pre pass (one
        // partial per tile and problem), else by a pass of its own
        g->fnorm_pending = fas::tail_top(g) > 0 && fas::tile_ok(g, 0, nu1, nu2, false) &&
                           (int64_t)fas::tile_count(g, 0, nu1) * g->batch <= g->npartials;
        struct Pending {
            fas_grid* g;
            ~Pending() { g->fnorm_pending = 0; }
        } pending{g};
        if (!g->fnorm_pending) {
            fas::launch_resid_norm(g, 0, g->coef[0], nullptr, rhs, nullptr);
            FAS_HIP_CHECK(hipMemcpyAsync(g->rnorm, g->norm_out, (size_t)g->batch * sizeof(double),
                                         hipMemcpyDeviceToDevice, g->stream));
        }
        ensure_host(g);
        // as the single solve: after a batched solve whose slowest problem took c cycles,
        // cycles 1..c-2 run without a look (a problem that has converged skips them)
        GateScope gate(g);
        const int horizon = g->last_cycles > 2 && !g->profile ? g->last_cycles - 2 : 0;
        g->last_cycles = 0;
        int* const hcount = (int*)g->host;
        for (int k = 1; k <= g->kmax; ++k) {
            vcycle_run(g, rhs, u, nu1, nu2, false, true);
            fas::launch_update_active(g, tol, k);
            if (k <= horizon && k < g->kmax) continue;
            FAS_HIP_CHECK(hipMemcpyAsync(hcount, g->count, sizeof(int), hipMemcpyDeviceToHost, g->stream));
            FAS_HIP_CHECK(hipStreamSynchronize(g->stream));
            if (hcount[0] == 0) break;
        }
        std::vector<int> cyc((size_t)g->batch);
        FAS_HIP_CHECK(hipMemcpyAsync(cyc.data(), g->cyc, cyc.size() * sizeof(int), hipMemcpyDeviceToHost, g->stream));
        FAS_HIP_CHECK(hipStreamSynchronize(g->stream));
        int worst = FAS_OK, maxc = 0;
        for (int b = 0; b < g->batch; ++b) {
            const int c = cyc[(size_t)b];
            const int st = c > 0 ? FAS_OK : (c < 0 ? FAS_ERR_NONFINITE : FAS_NOT_CONVERGED);
            const int cycles = c > 0 ? c : (c < 0 ? -c : g->kmax);
            if (status_out) status_out[b] = st;
            if (cycles_out) cycles_out[b] = cycles;
            if (st == FAS_ERR_NONFINITE) worst = FAS_ERR_NONFINITE;
            else if (st == FAS_NOT_CONVERGED && worst == FAS_OK) worst = FAS_NOT_CONVERGED;
            maxc = cycles > maxc ? cycles : maxc;
        }
        g->stats.cycles = maxc;
        g->stats.status = worst;
        if (worst == FAS_OK) g->last_cycles = maxc;
        if (worst == FAS_ERR_NONFINITE) return fail(FAS_ERR_NONFINITE, "a residual norm is not finite");
        if (worst == FAS_NOT_CONVERGED) g_last_error = "some problems did not converge within kmax cycles";
        return worst;
    });
}

int fas_solve_noalloc(int dim, const int64_t n[3], double h, int bc, int dtype, int coarsest, void* stream, double dt,
                      double kappa, const void* kappa_cell, const void* rhs, void* u, double tol, int nu1, int nu2,
                      int kmax, int* cycles_out)
{
    return guarded([&]() -> int {
        return solve_noalloc_impl(dim, n, h, bc, dtype, coarsest, stream, dt, kappa, kappa_cell, rhs, u, tol, nu1, nu2,
                                  kmax, cycles_out);
    });
}

int fas_solve_batched(int nprob, const fas_grid_t* grids, double dt, const fas_kappa_t* kappa, const void* const* rhs,
                      void* const* u, double tol, int nu1, int nu2, int* status_out)
{
    return guarded([&]() -> int {
        return solve_batched_impl(nprob, grids, dt, kappa, rhs, u, tol, nu1, nu2, status_out);
    });
}

int fas_grain_rhs(void* stream, int dtype, int q, int64_t ncells, double dt, double alpha, double beta, double gamma,
                  const void* eta, void* f)
{
    return guarded([&]() -> int {
        if (q < 1 || ncells < 1 || !eta || !f || eta == f) return fail(FAS_ERR_ARG, "bad grain-growth arguments");
        if (dtype != FAS_F64 && dtype != FAS_F32) return fail(FAS_ERR_ARG, "dtype must be FAS_F64 or FAS_F32");
        if (!isfinite(dt) || !isfinite(alpha) || !isfinite(beta) || !isfinite(gamma))
            return fail(FAS_ERR_ARG, "grain-growth coefficients must be finite");
        fas::launch_grain_rhs((hipStream_t)stream, dtype, q, ncells, dt, alpha, beta, gamma, eta, f);
        return FAS_OK;
    });
}

int fas_grain_argmax(void* stream, int q, int64_t ncells, const void* eta, void* label)
{
    return guarded([&]() -> int {
        if (q < 1 || ncells < 1 || !eta || !label) return fail(FAS_ERR_ARG, "bad grain-map arguments");
        fas::launch_grain_argmax((hipStream_t)stream, q, ncells, (const float*)eta, (int*)label);
        return FAS_OK;
    });
}

int fas_get_stats(fas_grid_t g, fas_stats_t* out)
{
    if (!g || !out) return fail(FAS_ERR_ARG, "null argument");
    *out = g->stats;
    return FAS_OK;
}

int fas_get_profile(fas_grid_t g, fas_profile_t* out, int reset)
{
    return guarded([&]() -> int {
        check_grid(g);
        if (!out) return fail(FAS_ERR_ARG, "null argument");
        prof_flush(g);
        *out = g->prof;
        if (reset) memset(&g->prof, 0, sizeof(g->prof));
        return FAS_OK;
    });
}

const char* fas_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
