/*
 * CPU oracle for the matrix-free FAS multigrid V-cycle on cell-centred grids
 * (arXiv 2510.11152, Section 2 and Appendices A-C), written from the paper.
 *
 * TEST INFRASTRUCTURE ONLY: this library exists so that tests, the smoke check and the
 * benchmark's CPU-baseline leg can check and time the GPU library against a plain,
 * obviously correct implementation.  It shares no code with the GPU library.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (oracle/build.py).  No fast-math, no
 * FMA contraction, so each expression rounds exactly as written.
 *
 * Problem (eq. PDE_discret with a time step and a diffusion coefficient): one backward-Euler heat step
 *     u - dt * div(kappa grad u) = f   on a cell-centred grid, spacing h,
 * with homogeneous Neumann (default), Dirichlet (ghost = -adjacent value, the reading
 * that reproduces Tables 2-3) or periodic boundaries.  Layout: x fastest,
 * idx = i + n0*(j + n1*l).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OG_NEUMANN 0
#define OG_DIRICHLET 1
#define OG_PERIODIC 2
#define OG_MAXL 32

typedef struct {
    int dim;       /* 2 or 3 */
    int bc;        /* OG_NEUMANN, OG_DIRICHLET, OG_PERIODIC */
    long n[3];     /* finest cells per axis; n[2] == 1 when dim == 2 */
    double h;      /* finest spacing, equal on every axis (Section 2.1) */
    double dt;     /* time step */
    double kappa;  /* constant diffusivity, used when no cell field is given */
    int coarsest;  /* cells along the shortest axis of the coarsest level */
    int nuc;       /* sweeps on the coarsest level (Remark 1: smoothing, no direct solve) */
    int order;     /* multi-colour set order of a sweep: OG_X (default), OG_U or OG_Z */
    int symmetric; /* 1: every second sweep visits the sets in reverse (1234-4321) */
    double atol;   /* absolute stopping tolerance on ||f - A u||_2 (0: none); Algorithm 1 tests
                      an absolute residual, the relative test is this build's default */
} og_problem;

#define OG_X 0
#define OG_U 1
#define OG_Z 2

/* Set orders of one sweep (Section 2.3 and its figure of the three partitions; Appendix B
 * for 3D).  A set is the cells whose 1-based index along each axis has a fixed parity; it
 * is written as a bit mask, bit a set when the index along axis a (x, y, z) is odd.
 *   X (2D): (o,e) (e,o) (e,e) (o,o)           -- Section 2.3, the paper's sets 1-4
 *   U (2D): (o,o) (e,o) (e,e) (o,e)           -- the U-shaped path through the parity square
 *   Z (2D): (o,o) (o,e) (e,o) (e,e)           -- the Z-shaped (row by row) path
 *   X (3D): (o,e,e) (e,o,e) (e,e,o) (o,o,o) (o,e,o) (e,o,o) (e,e,e) (o,o,e)  -- Appendix B
 *   U (3D): the reflected Gray-code path that extends the 2D U (x flips first)
 *   Z (3D): the lexicographic path that extends the 2D Z (z fastest)
 * The paper draws the 2D partitions only; the 3D U and Z paths are this oracle's reading. */
static const int og_sets2[3][4] = {{1, 2, 0, 3}, {3, 2, 0, 1}, {3, 1, 2, 0}};
static const int og_sets3[3][8] = {{1, 2, 4, 7, 5, 6, 0, 3}, {7, 6, 4, 5, 1, 0, 2, 3}, {7, 3, 5, 1, 6, 2, 4, 0}};

static const int* og_set_order(const og_problem* P)
{
    int o = (P->order >= 0 && P->order <= 2) ? P->order : 0;
    return P->dim == 2 ? og_sets2[o] : og_sets3[o];
}

/* Whether 0-based cell (i,j,l) is in set `mask` (a 1-based odd index is 0-based even). */
static int og_in_set(int dim, int mask, long i, long j, long l)
{
    const long c[3] = {i, j, l};
    for (int a = 0; a < dim; ++a)
        if (((c[a] & 1) == 0) != ((mask >> a) & 1)) return 0;
    return 1;
}

static long og_index(const long m[3], long i, long j, long l) { return i + m[0] * (j + m[1] * l); }

/* Number of coarsenings L: the shortest axis has coarsest * 2^L cells and every axis is
 * divisible by 2^L (Section 2.1: M_0 = M_1/2, h_0 = 2 h_1).  Returns -1 if invalid. */
int og_levels(const og_problem* P)
{
    long nmin = P->n[0];
    for (int a = 1; a < P->dim; ++a)
        if (P->n[a] < nmin) nmin = P->n[a];
    if (P->coarsest < 2 || nmin % P->coarsest) return -1;
    long ratio = nmin / P->coarsest;
    int L = 0;
    while ((1L << L) < ratio) ++L;
    if ((1L << L) != ratio || L < 1 || L >= OG_MAXL) return -1;
    for (int a = 0; a < P->dim; ++a)
        if (P->n[a] % (1L << L)) return -1;
    return L;
}

static void og_level_dims(const og_problem* P, int lev, long m[3])
{
    for (int a = 0; a < 3; ++a) m[a] = (a < P->dim) ? (P->n[a] >> lev) : 1;
}

long og_level_cells(const og_problem* P, int lev)
{
    long m[3];
    og_level_dims(P, lev, m);
    return m[0] * m[1] * m[2];
}

/* k_l = dt*kappa/h_l^2 (constant kappa) or dt/h_l^2 (cell kappa), h_l = h*2^l. */
static double og_kd(const og_problem* P, int lev, int variable)
{
    double hl = P->h * (double)(1L << lev);
    double c = variable ? P->dt : P->dt * P->kappa;
    return c / (hl * hl);
}

/* Neighbour of cell c across its face on axis a (side 0: minus, 1: plus); -1 when the
 * face is on a non-periodic boundary. */
static long og_neighbour(const og_problem* P, const long m[3], const long c[3], int a, int side)
{
    long d[3] = {c[0], c[1], c[2]};
    d[a] += side ? 1 : -1;
    if (d[a] < 0 || d[a] >= m[a]) {
        if (P->bc != OG_PERIODIC) return -1;
        d[a] = (d[a] + m[a]) % m[a];
    }
    return og_index(m, d[0], d[1], d[2]);
}

/* Parity of the 0-based index sum i+j(+l) updated first: the paper's first sets have an
 * odd 1-based sum, and the 0-based sum differs from it by dim. */
static int og_first_parity(const og_problem* P) { return (P->dim + 1) & 1; }

/* Diagonal count for constant kappa: interior faces count 1, a Dirichlet boundary face
 * counts 2 (its ghost value is minus the cell value), a Neumann face counts 0. */
static int og_diag_count(const og_problem* P, int nout)
{
    int nin = 2 * P->dim - nout;
    return nin + (P->bc == OG_DIRICHLET ? 2 * nout : 0);
}

#define REAL double
#define SFX d
#include "fas_oracle_body.h"
#undef REAL
#undef SFX

#define REAL float
#define SFX s
#include "fas_oracle_body.h"
#undef REAL
#undef SFX

/* Mixed precision (the paper is silent): FP64 defect correction
 * around FP32 V-cycles.  Per outer iteration:
 *     r = f - A u (FP64);  rho = ||r||;  stop if rho <= tol*||f|| or rho <= P->atol
 *     r32 = fp32(r);  e = 0;  `inner` FP32 V-cycles on A e = r32
 *     u = u + fp64(e)
 * The residual is not rescaled before the cast: FP32 arithmetic is exact under scaling
 * by a power of two (away from overflow and subnormals), so a power-of-two scale would
 * give the same bits, and FP32's exponent range holds any residual of interest here.
 * kap0 (nullable) is the FP64 cell coefficient; the FP32 cycle uses fp32(kap0).
 * hist (nullable) needs kmax+1 entries: ||r||/||f|| before each correction and at the end.
 * tol = 0 runs exactly kmax corrections.
 * Returns 0 converged, 1 not converged; *outer = corrections applied. */
int og_solve_mixed(const og_problem* P, const double* kap0, const double* f, double* u, double tol, int nu1,
                   int nu2, int inner, int inner_next, int kmax, int* outer, double* hist)
{
    long N = og_level_cells(P, 0);
    if (og_levels(P) < 1) return -1;
    double* r = (double*)calloc((size_t)N, sizeof(double));
    float* r32 = (float*)calloc((size_t)N, sizeof(float));
    float* e = (float*)calloc((size_t)N, sizeof(float));
    float* k32 = kap0 ? (float*)calloc((size_t)N, sizeof(float)) : 0;
    if (k32)
        for (long p = 0; p < N; ++p) k32[p] = (float)kap0[p];
    double nf = norm2_d(N, f);
    int status, it = 0;
    for (;;) {
        og_residual_d(P, 0, kap0, f, u, r);
        double rho = norm2_d(N, r);
        if (hist) hist[it] = nf > 0.0 ? rho / nf : rho;
        if (rho <= tol * nf || rho <= P->atol || rho == 0.0) {
            status = 0;
            break;
        }
        if (it == kmax) {
            status = 1;
            break;
        }
        for (long p = 0; p < N; ++p) {
            r32[p] = (float)r[p];
            e[p] = 0.0f;
        }
        /* inner FP32 cycles: `inner` in the first correction, `inner_next` (if > 0) in the
         * later ones, whose start residual is already small */
        const int cycles = (it == 0 || inner_next <= 0) ? inner : inner_next;
        for (int m = 0; m < cycles; ++m) og_vcycle_s(P, k32, r32, e, nu1, nu2, 0);
        for (long p = 0; p < N; ++p) u[p] = u[p] + (double)e[p];
        ++it;
    }
    if (outer) *outer = it;
    free(r);
    free(r32);
    free(e);
    free(k32);
    return status;
}

/* Gradient of a loss with respect to the cell coefficient through one solve
 * A(kappa) u = b, given the adjoint mu = A^{-T} lambda:  g -= mu^T (dA/dkappa) u, i.e.
 *   g_p -= k * [ sum over interior faces (p,q): dw/dkappa_p * (mu_p - mu_q)(u_p - u_q)
 *               + sum over Dirichlet faces of p: 2 * mu_p * u_p ]
 * with w = 2 kp kq/(kp+kq), dw/dkp = 2 kq^2/(kp+kq)^2 and k = dt/h^2 (finest level).
 * The paper has no adjoint; this is the derivative of the operator defined above. */
void og_kappa_grad_d(const og_problem* P, const double* kap, const double* mu, const double* u, double* g)
{
    long m[3];
    og_level_dims(P, 0, m);
    double k = og_kd(P, 0, 1);
    for (long l = 0; l < m[2]; ++l)
        for (long j = 0; j < m[1]; ++j)
            for (long i = 0; i < m[0]; ++i) {
                long c[3] = {i, j, l};
                long p = og_index(m, i, j, l);
                double t[6] = {0, 0, 0, 0, 0, 0};
                for (int a = 0; a < P->dim; ++a)
                    for (int side = 0; side < 2; ++side) {
                        long q = og_neighbour(P, m, c, a, side);
                        double val;
                        if (q >= 0) {
                            double s = kap[p] + kap[q];
                            double dw = (2.0 * kap[q] * kap[q]) / (s * s);
                            val = dw * ((mu[p] - mu[q]) * (u[p] - u[q]));
                        } else {
                            val = (P->bc == OG_DIRICHLET) ? (2.0 * mu[p]) * u[p] : 0.0;
                        }
                        t[2 * a + side] = val;
                    }
                double S = (t[0] + t[1]) + (t[2] + t[3]);
                if (P->dim == 3) S = S + (t[4] + t[5]);
                g[p] = g[p] - k * S;
            }
}
