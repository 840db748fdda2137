// C ABI of the staggered-grid FAS solver and of the first-order projection step
// (include/fas_stag.h): level plan, workspace layout, the V-cycle of Algorithm 1 on each
// staggered variable (Section 4.1) and the step of Scheme 1 (Section 4.2) in both field
// layouts.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <string>

#include "../../include/fas_stag.h"
#include "fas_internal.h"
#include "stag_internal.h"

using fas::Error;
using namespace fas::stag;

struct fas_stag {
    int loc, cell_bc, coarsest, nuc;
    int fused;      // 1: persistent tail for the coarse levels and the correction fused into
                    // the first post-smoothing launch; 0: one kernel per step and level
    int tail_top;   // first level of the persistent tail
    int tail_ou[fas::stag::kTailMaxLevels], tail_of[fas::stag::kTailMaxLevels], tail_ou0[fas::stag::kTailMaxLevels];
    int kx, ky;
    int64_t mx, my;  // cells of the finest level
    double h;
    int L;
    struct Level {
        int nx, ny;       // unknowns
        double* u;        // iterate (levels >= 1; the caller's array on level 0)
        double* ut;       // second buffer of the iterate
        double* u0;       // restricted iterate before the coarse solve (levels >= 1)
        double* f;        // right-hand side (levels >= 1)
        double* r;        // restricted residual of the finer level (levels >= 1, fused path)
    } lev[fas::kMaxLevels];
    double* partials;
    double* norm;
    hipStream_t stream;
    // FAS_OPT_PROFILE: HIP events around the finest level's pre- and post-smoothing launches
    int profile;
    hipEvent_t ev[4];
    bool ev_pending;
    double prof_ms[2];
    int prof_n;
};

struct fas_ns {
    int64_t nx, ny;
    double h, re;
    int layout;
    double* fld[9];
    double* rhs;
    size_t ws_bytes;
    fas_stag_t* su;
    fas_stag_t* sv;
    fas_stag_t* sp;
    hipStream_t stream;
};

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

template <typename F>
int guarded(F&& body)
{
    try {
        return body();
    } catch (const Error& e) {
        fas::set_last_error(e.what());
        return e.code;
    } catch (const std::exception& e) {
        fas::set_last_error(e.what());
        return FAS_ERR_ARG;
    } catch (...) {
        fas::set_last_error("unknown error");
        return FAS_ERR_ARG;
    }
}

// Unknowns of a location on an mx x my cell grid.
void unknowns(int loc, int64_t mx, int64_t my, int64_t& nx, int64_t& ny)
{
    nx = loc == LOC_EDGE_X ? mx - 1 : mx;
    ny = loc == LOC_EDGE_Y ? my - 1 : my;
}

// Number of levels: both axes halve while they stay even and >= coarsest.
int count_levels(int64_t mx, int64_t my, int coarsest)
{
    int L = 1;
    while (mx % 2 == 0 && my % 2 == 0 && mx / 2 >= coarsest && my / 2 >= coarsest && L < fas::kMaxLevels) {
        mx /= 2;
        my /= 2;
        ++L;
    }
    return L;
}

void check_shape(int loc, int64_t mx, int64_t my, int coarsest)
{
    if (loc < LOC_CELL || loc > LOC_EDGE_Y) throw Error(FAS_ERR_ARG, "unknown location");
    if (coarsest < 2) throw Error(FAS_ERR_SHAPE, "coarsest must be >= 2");
    if (mx < 2 * coarsest || my < 2 * coarsest || mx > (1 << 20) || my > (1 << 20) || mx * my > (int64_t)1 << 30)
        throw Error(FAS_ERR_SHAPE, "sizes must be at least 2 * coarsest and at most 2^20 per axis (2^30 cells)");
    const int L = count_levels(mx, my, coarsest);
    const int64_t fx = mx >> (L - 1), fy = my >> (L - 1);
    if ((fx << (L - 1)) != mx || (fy << (L - 1)) != my || std::min(fx, fy) >= 2 * coarsest || std::min(fx, fy) < coarsest)
        throw Error(FAS_ERR_SHAPE, "nx and ny must be coarsest * 2^L times a common factor, L >= 1");
    if (L < 2) throw Error(FAS_ERR_SHAPE, "at least two levels are needed");
}

// Partial sums a norm needs: the residual pass, or the finest sweep launch with the norm.
int partials_count(int loc, int64_t mx, int64_t my)
{
    int64_t nx, ny;
    unknowns(loc, mx, my, nx, ny);
    Lev L{};
    L.nx = (int)nx;
    L.ny = (int)ny;
    return std::max(kNormBlocks, std::max(sweep_blocks(L, 1, SW_CORR | SW_NORM, nullptr),
                                          sweep_blocks(L, 2, SW_CORR | SW_NORM, nullptr)));
}

// Bytes of the workspace of one staggered variable (0 on a bad shape).
size_t stag_bytes(int loc, int64_t mx, int64_t my, int coarsest)
{
    const int L = count_levels(mx, my, coarsest);
    size_t b = 0;
    for (int l = 0; l < L; ++l) {
        int64_t nx, ny;
        unknowns(loc, mx >> l, my >> l, nx, ny);
        const size_t arr = align_up((size_t)(nx * ny) * sizeof(double));
        b += l == 0 ? arr : 5 * arr;
    }
    b += align_up((partials_count(loc, mx, my) + 8) * sizeof(double));
    return b;
}

Lev level_op(const fas_stag& S, int l, double a, double c)
{
    Lev L;
    L.nx = S.lev[l].nx;
    L.ny = S.lev[l].ny;
    L.kx = S.kx;
    L.ky = S.ky;
    L.a = a;
    L.c = c;
    const double h = S.h * (double)(1 << l);
    L.h2 = h * h;
    L.ih2 = 1.0 / L.h2;
    return L;
}

// nu sweeps from buffer cur (alt: the other buffer of the level).  The launches do two sweeps
// each, one when nu is odd; with `want` set, one two-sweep launch becomes two one-sweep
// launches (or a copy follows) so that the result lands in `want`.  corr: FAS correction
// applied as the first launch loads its window; partials: the last launch sums the residual
// norm (its block count goes to norm_blocks).  Returns the buffer that holds the result.
double* sweeps(hipStream_t st, int loc, const Lev& L, const double* f, double* cur, double* alt, int nu, double* want,
               const Coarse* corr = nullptr, double* partials = nullptr, int* norm_blocks = nullptr)
{
    if (nu <= 0) {
        if (want && want != cur) {
            launch_copy(st, cur, want, (int64_t)L.nx * L.ny);
            return want;
        }
        return cur;
    }
    int twos = nu / 2, ones = nu % 2;
    const int count = twos + ones;
    bool copy_after = false;
    if (want) {
        double* lands = count % 2 == 0 ? cur : alt;
        if (lands != want) {
            if (twos > 0) {
                --twos;
                ones += 2;
            } else {
                copy_after = true;
            }
        }
    }
    double* a = cur;
    double* b = alt;
    const int n = twos + ones;
    for (int i = 0; i < n; ++i) {
        const bool last = i == n - 1 && !copy_after;
        SweepIO io{};
        unsigned flags = 0;
        if (i == 0 && corr) {
            io.C = *corr;
            flags |= SW_CORR;
        }
        if (last && partials && (flags & SW_CORR)) {
            io.partials = partials;
            flags |= SW_NORM;
        }
        const int nb = launch_sweep(st, loc, L, i < twos ? 2 : 1, f, a, b, io, flags);
        if (flags & SW_NORM && norm_blocks) *norm_blocks = nb;
        std::swap(a, b);
    }
    if (copy_after) {
        launch_copy(st, a, want, (int64_t)L.nx * L.ny);
        return want;
    }
    return a;
}

int launches(int nu) { return nu / 2 + nu % 2; }

// Pre-smoothing of the fused path: nu >= 1 sweeps from u (ut: the other buffer).  With r set,
// the first launch forms the right-hand side f = r + L u (and writes f); the last restricts
// the smoothed iterate and its residual into level C.  Returns the buffer holding the
// smoothed iterate.
double* pre_fused(hipStream_t st, int loc, const Lev& L, const double* r, double* f, double* u, double* ut, int nu,
                  fas_stag::Level& C)
{
    const int twos = nu / 2, n = twos + nu % 2;
    double* a = u;
    double* b = ut;
    for (int i = 0; i < n; ++i) {
        SweepIO io{};
        unsigned flags = 0;
        const double* fin = f;
        if (i == 0 && r) {
            flags |= SW_RHS;
            io.fout = f;
            fin = r;
        }
        if (i == n - 1) {
            flags |= SW_RES;
            io.uc = C.u;
            io.uc0 = C.u0;
            io.rc = C.r;
            io.ncx = C.nx;
            io.ncy = C.ny;
        }
        launch_sweep(st, loc, L, i < twos ? 2 : 1, fin, a, b, io, flags);
        std::swap(a, b);
    }
    return a;
}

// One V(nu1, nu2) cycle from level l on right-hand side f with the iterate in u (the result
// returns to u).  r: the level's restricted residual when its right-hand side has yet to be
// formed (f = r + L u; fused path, levels >= 1), else null.  Returns the number of residual
// partial sums the last sweep left in S.partials (0: none, the norm needs its own pass).
int vcycle(fas_stag& S, int l, double a, double c, double* f, double* u, int nu1, int nu2, const double* r = nullptr)
{
    const Lev L = level_op(S, l, a, c);
    double* ut = S.lev[l].ut;
    if (S.fused && l == S.tail_top) {
        TailArgs A{};
        A.nlev = S.L - l;
        for (int k = 0; k < A.nlev; ++k) {
            A.op[k] = level_op(S, l + k, a, c);
            A.ou[k] = S.tail_ou[k];
            A.of[k] = S.tail_of[k];
            A.ou0[k] = S.tail_ou0[k];
        }
        A.u = u;
        A.f = f;
        A.r = r;
        A.nu1 = nu1;
        A.nu2 = nu2;
        A.nuc = S.nuc;
        launch_tail(S.stream, S.loc, A);
        return 0;
    }
    if (r && (nu1 == 0 || l == S.L - 1)) {
        launch_form_rhs(S.stream, L, r, u, f);  // no pre-smoothing launch to form it in
        r = nullptr;
    }
    if (l == S.L - 1) {
        sweeps(S.stream, S.loc, L, f, u, ut, S.nuc, u);  // Remark 1: the coarsest level is smoothed
        return 0;
    }
    auto& C = S.lev[l + 1];
    double* cur;
    const bool prof = S.profile && l == 0 && S.fused && nu1 > 0 && nu2 > 0 && !S.ev_pending;
    if (prof) FAS_HIP_CHECK(hipEventRecord(S.ev[0], S.stream));
    if (S.fused && nu1 > 0) {
        cur = pre_fused(S.stream, S.loc, L, r, f, u, ut, nu1, C);
        if (prof) FAS_HIP_CHECK(hipEventRecord(S.ev[1], S.stream));
        vcycle(S, l + 1, a, c, C.f, C.u, nu1, nu2, C.r);
    } else {
        cur = sweeps(S.stream, S.loc, L, f, u, ut, nu1, nullptr);
        launch_restrict(S.stream, S.loc, L, f, cur, C.nx, C.ny, C.u, C.u0, C.f);
        launch_coarse_rhs(S.stream, level_op(S, l + 1, a, c), C.f, C.u);
        vcycle(S, l + 1, a, c, C.f, C.u, nu1, nu2);
    }
    if (S.fused && nu2 > 0) {
        // correction in the first post-smoothing launch, the residual norm (finest level) in
        // the last
        const Coarse corr{C.u, C.u0, C.nx, C.ny};
        int nb = 0;
        if (prof) FAS_HIP_CHECK(hipEventRecord(S.ev[2], S.stream));
        sweeps(S.stream, S.loc, L, f, cur, cur == u ? ut : u, nu2, u, &corr, l == 0 ? S.partials : nullptr, &nb);
        if (prof) {
            FAS_HIP_CHECK(hipEventRecord(S.ev[3], S.stream));
            S.ev_pending = true;
        }
        return nb;
    }
    // the correction goes to the buffer from which nu2 sweeps end in u
    double* dst = launches(nu2) % 2 == 0 ? u : ut;
    launch_correct(S.stream, S.loc, L, C.u, C.u0, C.nx, C.ny, cur, dst);
    sweeps(S.stream, S.loc, L, f, dst, dst == u ? ut : u, nu2, u);
    return 0;
}

// Adds the last cycle's event times (the stream has been synchronised).
void profile_collect(fas_stag& S)
{
    if (!S.ev_pending) return;
    float a = 0.f, b = 0.f;
    FAS_HIP_CHECK(hipEventElapsedTime(&a, S.ev[0], S.ev[1]));
    FAS_HIP_CHECK(hipEventElapsedTime(&b, S.ev[2], S.ev[3]));
    S.prof_ms[0] += a;
    S.prof_ms[1] += b;
    S.prof_n += 1;
    S.ev_pending = false;
}

double read_norm(fas_stag& S)
{
    double s2 = 0.0;
    FAS_HIP_CHECK(hipMemcpyAsync(&s2, S.norm, sizeof(double), hipMemcpyDeviceToHost, S.stream));
    FAS_HIP_CHECK(hipStreamSynchronize(S.stream));
    profile_collect(S);
    return S.h * sqrt(s2);
}

double residual_norm(fas_stag& S, double a, double c, const double* f, const double* u, double* r)
{
    const Lev L = level_op(S, 0, a, c);
    launch_resnorm(S.stream, L, f, u, r, S.partials, S.norm);
    double s2 = 0.0;
    FAS_HIP_CHECK(hipMemcpyAsync(&s2, S.norm, sizeof(double), hipMemcpyDeviceToHost, S.stream));
    FAS_HIP_CHECK(hipStreamSynchronize(S.stream));
    profile_collect(S);
    return S.h * sqrt(s2);
}

void check_pointers(const void* f, const void* u)
{
    if (!f || !u) throw Error(FAS_ERR_ARG, "null array");
    if (f == u) throw Error(FAS_ERR_ARG, "f and w must not alias");
}

int solve(fas_stag& S, double a, double c, const double* f, double* u, double tol, int nu1, int nu2, int kmax,
          int* cycles_out, double* res_out)
{
    if (nu1 < 0 || nu2 < 0 || kmax < 0 || !(tol >= 0.0)) throw Error(FAS_ERR_ARG, "bad nu1, nu2, kmax or tol");
    double res = residual_norm(S, a, c, f, u, nullptr);
    int k = 0;
    while (isfinite(res) && res > tol && k < kmax) {
        const int nb = vcycle(S, 0, a, c, const_cast<double*>(f), u, nu1, nu2);
        ++k;
        if (nb > 0) {
            launch_sum(S.stream, S.partials, nb, S.norm);
            res = read_norm(S);
        } else {
            res = residual_norm(S, a, c, f, u, nullptr);
        }
    }
    if (cycles_out) *cycles_out = k;
    if (res_out) *res_out = res;
    if (!isfinite(res)) throw Error(FAS_ERR_NONFINITE, "a residual norm is not finite");
    if (res > tol) {
        fas::set_last_error("not converged within kmax cycles");
        return FAS_NOT_CONVERGED;
    }
    return FAS_OK;
}

void init_stag(fas_stag& S, int loc, int64_t mx, int64_t my, double h, int cell_bc, int coarsest, char* ws,
               hipStream_t stream)
{
    S.loc = loc;
    S.cell_bc = cell_bc;
    S.coarsest = coarsest;
    S.nuc = 16;
    const int ck = cell_bc == 0 ? K_CN : K_CD;
    S.kx = loc == LOC_CELL ? ck : (loc == LOC_EDGE_X ? K_V : K_CD);
    S.ky = loc == LOC_CELL ? ck : (loc == LOC_EDGE_Y ? K_V : K_CD);
    S.mx = mx;
    S.my = my;
    S.h = h;
    S.L = count_levels(mx, my, coarsest);
    S.stream = stream;
    size_t off = 0;
    for (int l = 0; l < S.L; ++l) {
        int64_t nx, ny;
        unknowns(loc, mx >> l, my >> l, nx, ny);
        auto& V = S.lev[l];
        V.nx = (int)nx;
        V.ny = (int)ny;
        const size_t arr = align_up((size_t)(nx * ny) * sizeof(double));
        V.ut = reinterpret_cast<double*>(ws + off);
        off += arr;
        if (l == 0) {
            V.u = V.u0 = V.f = V.r = nullptr;
            continue;
        }
        V.u = reinterpret_cast<double*>(ws + off);
        V.u0 = reinterpret_cast<double*>(ws + off + arr);
        V.f = reinterpret_cast<double*>(ws + off + 2 * arr);
        V.r = reinterpret_cast<double*>(ws + off + 3 * arr);
        off += 4 * arr;
    }
    S.partials = reinterpret_cast<double*>(ws + off);
    S.norm = S.partials + partials_count(loc, mx, my);
    // persistent tail: the first level from which every level down to the coarsest fits
    S.fused = 1;
    S.tail_top = -1;
    for (int top = 0; top < S.L; ++top) {
        if ((int64_t)S.lev[top].nx * S.lev[top].ny > kTailTopMax || S.L - top > kTailMaxLevels) continue;
        int need = 0;
        for (int l = top; l < S.L; ++l) need += (l == top ? 2 : 3) * S.lev[l].nx * S.lev[l].ny;
        if (need > kTailDoubles) continue;
        int o = 0;
        for (int l = top; l < S.L; ++l) {
            const int n = S.lev[l].nx * S.lev[l].ny, k = l - top;
            S.tail_ou[k] = o;
            S.tail_of[k] = o + n;
            S.tail_ou0[k] = l == top ? -1 : o + 2 * n;
            o += (l == top ? 2 : 3) * n;
        }
        S.tail_top = top;
        break;
    }
}

int set_option(fas_stag& S, int option, double value)
{
    if (option == FAS_OPT_FUSED && (value == 0.0 || value == 1.0)) {
        S.fused = (int)value;
        return FAS_OK;
    }
    if (option == FAS_OPT_PROFILE && (value == 0.0 || value == 1.0)) {
        if (value == 1.0 && !S.profile) {
            if (!S.ev[0])
                for (auto& e : S.ev) FAS_HIP_CHECK(hipEventCreate(&e));
            S.ev_pending = false;
            S.prof_ms[0] = S.prof_ms[1] = 0.0;
            S.prof_n = 0;
        }
        S.profile = (int)value;
        return FAS_OK;
    }
    if (option != FAS_OPT_COARSE_SWEEPS || !(value >= 1.0) || value > 1e6)
        throw Error(FAS_ERR_ARG,
                    "a staggered solver takes FAS_OPT_COARSE_SWEEPS (>= 1), FAS_OPT_FUSED and FAS_OPT_PROFILE (0 or 1)");
    S.nuc = (int)value;
    return FAS_OK;
}

void release_events(fas_stag* s)
{
    if (s && s->ev[0])
        for (auto& e : s->ev) {
            (void)hipEventDestroy(e);
            e = nullptr;
        }
}

}  // namespace

extern "C" {

size_t fas_stag_workspace_size(int loc, int64_t nx, int64_t ny, int coarsest)
{
    try {
        check_shape(loc, nx, ny, coarsest);
    } catch (const Error&) {
        return 0;
    }
    return stag_bytes(loc, nx, ny, coarsest);
}

int fas_stag_create(int loc, int64_t nx, int64_t ny, double h, int cell_bc, int coarsest, void* workspace,
                    size_t workspace_bytes, void* stream, fas_stag_t** out)
{
    return guarded([&] {
        if (!out) throw Error(FAS_ERR_ARG, "out is NULL");
        *out = nullptr;
        check_shape(loc, nx, ny, coarsest);
        if (!(h > 0.0) || (cell_bc != 0 && cell_bc != 1)) throw Error(FAS_ERR_ARG, "bad h or cell_bc");
        if (loc != LOC_CELL && cell_bc != 1) throw Error(FAS_ERR_ARG, "edge locations are Dirichlet (cell_bc = 1)");
        if (!workspace) throw Error(FAS_ERR_ARG, "workspace is NULL");
        if (workspace_bytes < stag_bytes(loc, nx, ny, coarsest))
            throw Error(FAS_ERR_NOMEM, "workspace smaller than fas_stag_workspace_size()");
        fas_stag* S = new fas_stag();
        init_stag(*S, loc, nx, ny, h, cell_bc, coarsest, static_cast<char*>(workspace),
                  static_cast<hipStream_t>(stream));
        *out = S;
        return FAS_OK;
    });
}

int fas_stag_destroy(fas_stag_t* s)
{
    release_events(s);
    delete s;
    return FAS_OK;
}

int fas_stag_profile(fas_stag_t* s, double* pre_us, double* post_us, int* cycles)
{
    return guarded([&] {
        if (!s || !s->profile) throw Error(FAS_ERR_ARG, "null handle or FAS_OPT_PROFILE off");
        FAS_HIP_CHECK(hipStreamSynchronize(s->stream));
        profile_collect(*s);
        const int n = s->prof_n;
        if (pre_us) *pre_us = n ? 1e3 * s->prof_ms[0] / n : 0.0;
        if (post_us) *post_us = n ? 1e3 * s->prof_ms[1] / n : 0.0;
        if (cycles) *cycles = n;
        return FAS_OK;
    });
}

int fas_stag_set(fas_stag_t* s, int option, double value)
{
    return guarded([&] {
        if (!s) throw Error(FAS_ERR_ARG, "null handle");
        return set_option(*s, option, value);
    });
}

int fas_stag_levels(const fas_stag_t* s) { return s ? s->L : 0; }

int fas_stag_solve(fas_stag_t* s, double a, double c, const void* f, void* w, double tol, int nu1, int nu2,
                   int kmax, int* cycles_out, double* res_out)
{
    return guarded([&] {
        if (!s) throw Error(FAS_ERR_ARG, "null handle");
        check_pointers(f, w);
        return solve(*s, a, c, static_cast<const double*>(f), static_cast<double*>(w), tol, nu1, nu2, kmax,
                     cycles_out, res_out);
    });
}

int fas_stag_vcycle(fas_stag_t* s, double a, double c, const void* f, void* w, int nu1, int nu2)
{
    return guarded([&] {
        if (!s) throw Error(FAS_ERR_ARG, "null handle");
        check_pointers(f, w);
        if (nu1 < 0 || nu2 < 0) throw Error(FAS_ERR_ARG, "negative sweep count");
        vcycle(*s, 0, a, c, static_cast<double*>(const_cast<void*>(f)), static_cast<double*>(w), nu1, nu2);
        FAS_HIP_CHECK(hipGetLastError());
        return FAS_OK;
    });
}

int fas_stag_smooth(fas_stag_t* s, double a, double c, const void* f, void* w, int nu)
{
    return guarded([&] {
        if (!s) throw Error(FAS_ERR_ARG, "null handle");
        check_pointers(f, w);
        if (nu < 0) throw Error(FAS_ERR_ARG, "negative sweep count");
        double* u = static_cast<double*>(w);
        sweeps(s->stream, s->loc, level_op(*s, 0, a, c), static_cast<const double*>(f), u, s->lev[0].ut, nu, u);
        FAS_HIP_CHECK(hipGetLastError());
        return FAS_OK;
    });
}

int fas_stag_residual(fas_stag_t* s, double a, double c, const void* f, const void* w, void* r, double* res_out)
{
    return guarded([&] {
        if (!s) throw Error(FAS_ERR_ARG, "null handle");
        check_pointers(f, w);
        if (r == f || r == w) throw Error(FAS_ERR_ARG, "r must not alias f or w");
        const double res = residual_norm(*s, a, c, static_cast<const double*>(f), static_cast<const double*>(w),
                                         static_cast<double*>(r));
        if (res_out) *res_out = res;
        return FAS_OK;
    });
}

// ---- projection step ---------------------------------------------------------------------
int fas_ns_fields(int layout)
{
    return layout == FAS_NS_MEMORY_EFFICIENT ? 6 : (layout == FAS_NS_CLASSICAL ? 9 : 0);
}

size_t fas_ns_workspace_size(int64_t nx, int64_t ny, int coarsest)
{
    try {
        for (int loc = LOC_CELL; loc <= LOC_EDGE_Y; ++loc) check_shape(loc, nx, ny, coarsest);
    } catch (const Error&) {
        return 0;
    }
    size_t b = 0;
    for (int loc = LOC_CELL; loc <= LOC_EDGE_Y; ++loc) b = std::max(b, stag_bytes(loc, nx, ny, coarsest));
    return align_up((size_t)(nx * ny) * sizeof(double)) + b;
}

int fas_ns_create(int64_t nx, int64_t ny, double h, double re, int layout, int coarsest, void* const* fields,
                  void* workspace, size_t workspace_bytes, void* stream, fas_ns_t** out)
{
    return guarded([&] {
        if (!out) throw Error(FAS_ERR_ARG, "out is NULL");
        *out = nullptr;
        const int nf = fas_ns_fields(layout);
        if (!nf) throw Error(FAS_ERR_ARG, "unknown layout");
        for (int loc = LOC_CELL; loc <= LOC_EDGE_Y; ++loc) check_shape(loc, nx, ny, coarsest);
        if (!(h > 0.0) || !(re > 0.0)) throw Error(FAS_ERR_ARG, "h and re must be positive");
        if (!fields || !workspace) throw Error(FAS_ERR_ARG, "null fields or workspace");
        for (int i = 0; i < nf; ++i) {
            if (!fields[i]) throw Error(FAS_ERR_ARG, "null field");
            for (int j = 0; j < i; ++j)
                if (fields[i] == fields[j]) throw Error(FAS_ERR_ARG, "fields must be distinct");
        }
        if (workspace_bytes < fas_ns_workspace_size(nx, ny, coarsest))
            throw Error(FAS_ERR_NOMEM, "workspace smaller than fas_ns_workspace_size()");
        fas_ns* N = new fas_ns();
        N->nx = nx;
        N->ny = ny;
        N->h = h;
        N->re = re;
        N->layout = layout;
        for (int i = 0; i < nf; ++i) N->fld[i] = static_cast<double*>(fields[i]);
        char* ws = static_cast<char*>(workspace);
        N->rhs = reinterpret_cast<double*>(ws);
        char* shared = ws + align_up((size_t)(nx * ny) * sizeof(double));
        N->ws_bytes = fas_ns_workspace_size(nx, ny, coarsest);
        N->stream = static_cast<hipStream_t>(stream);
        // the three solves run one after another on one stream and share the coarse levels
        N->su = new fas_stag();
        N->sv = new fas_stag();
        N->sp = new fas_stag();
        init_stag(*N->su, LOC_EDGE_X, nx, ny, h, 1, coarsest, shared, N->stream);
        init_stag(*N->sv, LOC_EDGE_Y, nx, ny, h, 1, coarsest, shared, N->stream);
        init_stag(*N->sp, LOC_CELL, nx, ny, h, 0, coarsest, shared, N->stream);
        *out = N;
        return FAS_OK;
    });
}

int fas_ns_destroy(fas_ns_t* ns)
{
    if (ns) {
        release_events(ns->su);
        release_events(ns->sv);
        release_events(ns->sp);
        delete ns->su;
        delete ns->sv;
        delete ns->sp;
        delete ns;
    }
    return FAS_OK;
}

int fas_ns_set(fas_ns_t* ns, int option, double value)
{
    return guarded([&] {
        if (!ns) throw Error(FAS_ERR_ARG, "null handle");
        set_option(*ns->su, option, value);
        set_option(*ns->sv, option, value);
        return set_option(*ns->sp, option, value);
    });
}

int fas_ns_step(fas_ns_t* ns, double dt, double lid, int nforce, const void* const* force_u,
                const void* const* force_v, const double* coef, double tol, int nu1, int nu2, int kmax,
                int* cycles_out, double* res_out)
{
    return guarded([&] {
        if (!ns) throw Error(FAS_ERR_ARG, "null handle");
        if (!(dt > 0.0) || !isfinite(lid)) throw Error(FAS_ERR_ARG, "dt must be positive and lid finite");
        if (nforce < 0 || nforce > 4) throw Error(FAS_ERR_ARG, "nforce must be 0..4");
        if (nforce > 0 && (!force_u || !force_v || !coef)) throw Error(FAS_ERR_ARG, "null forcing arrays");
        NsArgs A{};
        A.nx = (int)ns->nx;
        A.ny = (int)ns->ny;
        A.dt = dt;
        A.ih = 1.0 / ns->h;
        A.ih2 = 1.0 / (ns->h * ns->h);
        const double c = dt / ns->re;
        A.lift = (2.0 * c * lid) * A.ih2;
        A.lid = lid;
        A.nforce = nforce;
        for (int k = 0; k < nforce; ++k) {
            if (!force_u[k] || !force_v[k]) throw Error(FAS_ERR_ARG, "null forcing field");
            A.fu[k] = static_cast<const double*>(force_u[k]);
            A.fv[k] = static_cast<const double*>(force_v[k]);
            A.coef[k] = coef[k];
        }
        double** F = ns->fld;
        const bool me = ns->layout == FAS_NS_MEMORY_EFFICIENT;
        // state u^n, v^n, p^n and the solves' targets u~, v~, p~
        double* u = me ? F[0] : F[1];
        double* v = me ? F[2] : F[4];
        double* p = me ? F[4] : F[7];
        double* ut = me ? F[1] : F[2];
        double* vt = me ? F[3] : F[5];
        double* pt = me ? F[5] : F[8];
        hipStream_t st = ns->stream;
        int cyc[3] = {0, 0, 0};
        double res[3] = {0, 0, 0};
        int worst = FAS_OK;
        launch_rhs_u(st, A, u, v, p, ns->rhs);
        worst = std::max(worst, solve(*ns->su, 1.0, c, ns->rhs, ut, tol, nu1, nu2, kmax, &cyc[0], &res[0]));
        launch_rhs_v(st, A, u, v, p, ns->rhs);
        worst = std::max(worst, solve(*ns->sv, 1.0, c, ns->rhs, vt, tol, nu1, nu2, kmax, &cyc[1], &res[1]));
        launch_neg_div(st, A, ut, vt, ns->rhs);
        worst = std::max(worst, solve(*ns->sp, 0.0, dt, ns->rhs, pt, tol, nu1, nu2, kmax, &cyc[2], &res[2]));
        if (me) {
            // u^{n+1} overwrites u^n in U_old (no copy new -> old)
            launch_project(st, A, ut, vt, pt, p, u, v, p);
        } else {
            launch_project(st, A, ut, vt, pt, p, F[0], F[3], F[6]);
            const int64_t nu_ = (ns->nx - 1) * ns->ny, nv_ = ns->nx * (ns->ny - 1), np_ = ns->nx * ns->ny;
            launch_copy(st, F[0], u, nu_);
            launch_copy(st, F[3], v, nv_);
            launch_copy(st, F[6], p, np_);
        }
        FAS_HIP_CHECK(hipGetLastError());
        for (int i = 0; i < 3; ++i) {
            if (cycles_out) cycles_out[i] = cyc[i];
            if (res_out) res_out[i] = res[i];
        }
        if (worst == FAS_NOT_CONVERGED) fas::set_last_error("a solve did not converge within kmax cycles");
        return worst;
    });
}

int fas_ns_memory(const fas_ns_t* ns, size_t* field_bytes, size_t* workspace_bytes)
{
    if (!ns) return FAS_ERR_ARG;
    const size_t nu_ = (ns->nx - 1) * ns->ny, nv_ = ns->nx * (ns->ny - 1), np_ = ns->nx * ns->ny;
    const size_t per = ns->layout == FAS_NS_MEMORY_EFFICIENT ? 2 : 3;
    if (field_bytes) *field_bytes = per * (nu_ + nv_ + np_) * sizeof(double);
    if (workspace_bytes) *workspace_bytes = ns->ws_bytes;
    return FAS_OK;
}

}  // extern "C"
