/*
 * Oracle body, instantiated once per real type: fas_oracle.c includes this file
 * with REAL = double (suffix d) and REAL = float (suffix s).
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, single-threaded CPU code used to check the
 * GPU library; the product never calls it.
 *
 * Every arithmetic expression below is written as one fixed evaluation tree (the
 * parentheses are the order), compiled with -ffp-contract=off, so that a GPU kernel
 * evaluating the same trees produces the same bits.
 */

#define OG_CAT2(a, b) a##_##b
#define OG_CAT(a, b) OG_CAT2(a, b)
#define F(name) OG_CAT(name, SFX)

/* Harmonic-mean face weight of the face between the cell on its minus side (klo) and
 * the cell on its plus side (khi): 2*klo*khi/(klo+khi).  Variable coefficients are not
 * in the paper; this is the usual cell-centred flux form. */
static REAL F(face_w)(REAL klo, REAL khi)
{
    REAL t = (REAL)2 * klo;
    t = t * khi;
    return t / (klo + khi);
}

/* Gather the 2*dim neighbour values v[] (0 outside a non-periodic domain) and, for a
 * variable coefficient, the face weights w[] of cell p = (i,j,l) on a level of size m.
 * Returns the number of faces that lie on a non-periodic boundary. */
static int F(gather)(const og_problem* P, const long m[3], long i, long j, long l, const REAL* u,
                     const REAL* kap, REAL v[6], REAL w[6])
{
    long c[3] = {i, j, l};
    long p = og_index(m, i, j, l);
    int nout = 0;
    for (int a = 0; a < P->dim; ++a) {
        for (int side = 0; side < 2; ++side) {
            int slot = 2 * a + side;
            long q = og_neighbour(P, m, c, a, side);
            if (q >= 0) {
                v[slot] = u[q];
                if (kap) w[slot] = side ? F(face_w)(kap[p], kap[q]) : F(face_w)(kap[q], kap[p]);
            } else {
                ++nout;
                v[slot] = (REAL)0;
                if (kap) w[slot] = (P->bc == OG_DIRICHLET) ? (REAL)2 * kap[p] : (REAL)0;
            }
        }
    }
    return nout;
}

/* Per-level scalars of the operator (fixed on the host in double, rounded once):
 *   constant kappa: k = dt*kappa/h_l^2, q[W] = 1/(1 + k*W) for the diagonal count W
 *   variable kappa: k = dt/h_l^2                                                     */
static void F(level_coeffs)(const og_problem* P, int lev, int variable, REAL* k, REAL q[16])
{
    double kd = og_kd(P, lev, variable);
    *k = (REAL)kd;
    for (int W = 0; W < 16; ++W) q[W] = (REAL)(1.0 / (1.0 + kd * (double)W));
}

static REAL F(nbsum)(const og_problem* P, const REAL v[6])
{
    REAL S = (v[0] + v[1]) + (v[2] + v[3]);
    if (P->dim == 3) S = S + (v[4] + v[5]);
    return S;
}

static REAL F(wsum)(const og_problem* P, const REAL v[6], const REAL w[6])
{
    REAL S = (w[0] * v[0] + w[1] * v[1]) + (w[2] * v[2] + w[3] * v[3]);
    if (P->dim == 3) S = S + (w[4] * v[4] + w[5] * v[5]);
    return S;
}

static REAL F(wtot)(const og_problem* P, const REAL w[6])
{
    REAL S = (w[0] + w[1]) + (w[2] + w[3]);
    if (P->dim == 3) S = S + (w[4] + w[5]);
    return S;
}

/* (A u)_p for the backward-Euler operator u - dt div(kappa grad u), row scaled by 1
 * (i.e. divided by h^2 relative to the paper's h^2 p - h^2 Lap p form). */
static REAL F(apply_point)(const og_problem* P, const long m[3], long i, long j, long l, const REAL* u,
                           const REAL* kap, REAL k)
{
    REAL v[6], w[6];
    int nout = F(gather)(P, m, i, j, l, u, kap, v, w);
    REAL up = u[og_index(m, i, j, l)];
    if (!kap) {
        REAL S = F(nbsum)(P, v);
        REAL W = (REAL)og_diag_count(P, nout);
        return up + k * (W * up - S);
    }
    REAL Sw = F(wsum)(P, v, w);
    REAL Wt = F(wtot)(P, w);
    return up + k * (Wt * up - Sw);
}

/* One Gauss-Seidel point update: solve row p of A u = f for u_p with the neighbours
 * fixed (the update of eqs. FCGS-1..4 / BWGS-B,W generalised to dt, kappa and BCs). */
static REAL F(gs_point)(const og_problem* P, const long m[3], long i, long j, long l, const REAL* u,
                        const REAL* f, const REAL* kap, REAL k, const REAL q[16])
{
    REAL v[6], w[6];
    int nout = F(gather)(P, m, i, j, l, u, kap, v, w);
    long p = og_index(m, i, j, l);
    if (!kap) {
        REAL S = F(nbsum)(P, v);
        return (f[p] + k * S) * q[og_diag_count(P, nout)];
    }
    REAL Sw = F(wsum)(P, v, w);
    REAL Wt = F(wtot)(P, w);
    return (f[p] + k * Sw) / ((REAL)1 + k * Wt);
}

/* Multi-colour sweeps through the 2^d index-parity sets in the order of P->order: each
 * set in turn, its cells lexicographically (no two cells of a set are neighbours, so
 * their order does not matter); with P->symmetric every second sweep takes the sets in
 * reverse (the 1234-4321 sequence of Section 2.3), and reverse != 0 reverses every
 * sweep once more (the transpose). */
static void F(smooth_sets)(const og_problem* P, int lev, const REAL* kap, const REAL* f, REAL* u, int sweeps,
                           int reverse)
{
    long m[3];
    REAL k, q[16];
    og_level_dims(P, lev, m);
    F(level_coeffs)(P, lev, kap != 0, &k, q);
    const int* order = og_set_order(P);
    const int nsets = 1 << P->dim;
    for (int s = 0; s < sweeps; ++s) {
        int rev = (P->symmetric && (s & 1)) != (reverse != 0);
        for (int t = 0; t < nsets; ++t) {
            int mask = order[rev ? nsets - 1 - t : t];
            for (long l = 0; l < m[2]; ++l)
                for (long j = 0; j < m[1]; ++j)
                    for (long i = 0; i < m[0]; ++i)
                        if (og_in_set(P->dim, mask, i, j, l))
                            u[og_index(m, i, j, l)] = F(gs_point)(P, m, i, j, l, u, f, kap, k, q);
        }
    }
}

/* Smoother S (Section 2.3 and Appendix A/B), X order: one sweep first updates the cells
 * whose 1-based index sum is odd (X-MCGS sets 1-2 in 2D, sets 1-4 in 3D), then the others
 * (sets 3-4 / 5-8), each phase visited lexicographically.  Other set orders, and the
 * symmetric sequence, go through smooth_sets.  With 0-based indices the
 * first phase is the odd-sum cells in 2D and the even-sum cells in 3D.  reverse != 0
 * runs the two phases in the opposite order, the transpose of the forward sweep. */
void F(og_smooth)(const og_problem* P, int lev, const REAL* kap, const REAL* f, REAL* u, int sweeps,
                  int reverse)
{
    long m[3];
    REAL k, q[16];
    if (P->order != OG_X || P->symmetric) {
        F(smooth_sets)(P, lev, kap, f, u, sweeps, reverse);
        return;
    }
    og_level_dims(P, lev, m);
    F(level_coeffs)(P, lev, kap != 0, &k, q);
    for (int s = 0; s < sweeps; ++s) {
        for (int ph = 0; ph < 2; ++ph) {
            int first = og_first_parity(P);
            int parity = (ph == 0) != (reverse != 0) ? first : 1 - first;
            for (long l = 0; l < m[2]; ++l)
                for (long j = 0; j < m[1]; ++j)
                    for (long i = 0; i < m[0]; ++i)
                        if (((i + j + l) & 1) == parity)
                            u[og_index(m, i, j, l)] = F(gs_point)(P, m, i, j, l, u, f, kap, k, q);
        }
    }
}

void F(og_apply)(const og_problem* P, int lev, const REAL* kap, const REAL* u, REAL* Au)
{
    long m[3];
    REAL k, q[16];
    og_level_dims(P, lev, m);
    F(level_coeffs)(P, lev, kap != 0, &k, q);
    for (long l = 0; l < m[2]; ++l)
        for (long j = 0; j < m[1]; ++j)
            for (long i = 0; i < m[0]; ++i) Au[og_index(m, i, j, l)] = F(apply_point)(P, m, i, j, l, u, kap, k);
}

/* Point-wise residual r = f - L(u) (eq. residual). */
void F(og_residual)(const og_problem* P, int lev, const REAL* kap, const REAL* f, const REAL* u, REAL* r)
{
    long m[3];
    REAL k, q[16];
    og_level_dims(P, lev, m);
    F(level_coeffs)(P, lev, kap != 0, &k, q);
    for (long l = 0; l < m[2]; ++l)
        for (long j = 0; j < m[1]; ++j)
            for (long i = 0; i < m[0]; ++i) {
                long p = og_index(m, i, j, l);
                r[p] = f[p] - F(apply_point)(P, m, i, j, l, u, kap, k);
            }
}

/* Restriction R (Appendix C): average of the 2^d fine children, summed pairwise along
 * x first, then y, then z. */
void F(og_restrict)(const og_problem* P, int lev, const REAL* fine, REAL* coarse)
{
    long m[3], mc[3];
    og_level_dims(P, lev, m);
    og_level_dims(P, lev + 1, mc);
    for (long K = 0; K < mc[2]; ++K)
        for (long J = 0; J < mc[1]; ++J)
            for (long I = 0; I < mc[0]; ++I) {
                long i = 2 * I, j = 2 * J;
                if (P->dim == 2) {
                    REAL a = fine[og_index(m, i, j, 0)] + fine[og_index(m, i + 1, j, 0)];
                    REAL b = fine[og_index(m, i, j + 1, 0)] + fine[og_index(m, i + 1, j + 1, 0)];
                    coarse[og_index(mc, I, J, 0)] = (a + b) * (REAL)0.25;
                } else {
                    long l = 2 * K;
                    REAL a = fine[og_index(m, i, j, l)] + fine[og_index(m, i + 1, j, l)];
                    REAL b = fine[og_index(m, i, j + 1, l)] + fine[og_index(m, i + 1, j + 1, l)];
                    REAL c = fine[og_index(m, i, j, l + 1)] + fine[og_index(m, i + 1, j, l + 1)];
                    REAL d = fine[og_index(m, i, j + 1, l + 1)] + fine[og_index(m, i + 1, j + 1, l + 1)];
                    coarse[og_index(mc, I, J, K)] = ((a + b) + (c + d)) * (REAL)0.125;
                }
            }
}

/* Prolongation P (Appendix C, piecewise constant) of the correction c0 = cnew - cold
 * added to the fine grid (Alg. 1, coarse and fine grid correction). */
void F(og_prolong_add)(const og_problem* P, int lev, const REAL* cnew, const REAL* cold, REAL* fine)
{
    long m[3], mc[3];
    og_level_dims(P, lev, m);
    og_level_dims(P, lev + 1, mc);
    for (long l = 0; l < m[2]; ++l)
        for (long j = 0; j < m[1]; ++j)
            for (long i = 0; i < m[0]; ++i) {
                long pc = og_index(mc, i / 2, j / 2, P->dim == 3 ? l / 2 : 0);
                long p = og_index(m, i, j, l);
                fine[p] = fine[p] + (cnew[pc] - cold[pc]);
            }
}

/* ---- level hierarchy for the V-cycle --------------------------------------------- */
typedef struct {
    int L;                 /* index of the coarsest level */
    REAL* u[OG_MAXL];      /* u[0], f[0] belong to the caller */
    REAL* f[OG_MAXL];
    REAL* kap[OG_MAXL];    /* kap[0] belongs to the caller; NULL for constant kappa */
    REAL* r;               /* residual scratch, finest size */
    REAL* t;               /* restricted scratch, level-1 size */
    int own_kap;
} F(og_hier);

static int F(hier_init)(const og_problem* P, const REAL* kap0, F(og_hier)* H)
{
    memset(H, 0, sizeof(*H));
    H->L = og_levels(P);
    if (H->L < 1) return -1;
    for (int lev = 1; lev <= H->L; ++lev) {
        long N = og_level_cells(P, lev);
        H->u[lev] = (REAL*)calloc((size_t)N, sizeof(REAL));
        H->f[lev] = (REAL*)calloc((size_t)N, sizeof(REAL));
        if (kap0) H->kap[lev] = (REAL*)calloc((size_t)N, sizeof(REAL));
    }
    H->r = (REAL*)calloc((size_t)og_level_cells(P, 0), sizeof(REAL));
    H->t = (REAL*)calloc((size_t)og_level_cells(P, 1), sizeof(REAL));
    H->kap[0] = (REAL*)kap0;
    /* Coarse coefficient: kappa_{l+1} = R kappa_l, then harmonic faces on every level. */
    if (kap0)
        for (int lev = 0; lev < H->L; ++lev) F(og_restrict)(P, lev, H->kap[lev], H->kap[lev + 1]);
    return 0;
}

static void F(hier_free)(F(og_hier)* H)
{
    for (int lev = 1; lev <= H->L; ++lev) {
        free(H->u[lev]);
        free(H->f[lev]);
        free(H->kap[lev]);
    }
    free(H->r);
    free(H->t);
}

/* FAS V-cycle (Alg. 1 applied recursively, Remark 2; coarsest level smoothed only,
 * Remark 1).  transposed != 0 gives the transpose of the cycle as a linear map:
 * pre/post sweep counts swapped and every sweep run in reverse phase order. */
static void F(vcycle_rec)(const og_problem* P, F(og_hier)* H, int lev, int nu1, int nu2, int transposed)
{
    REAL* u = H->u[lev];
    REAL* f = H->f[lev];
    const REAL* kap = H->kap[lev];
    if (lev == H->L) {
        F(og_smooth)(P, lev, kap, f, u, P->nuc, transposed);
        return;
    }
    int pre = transposed ? nu2 : nu1;
    int post = transposed ? nu1 : nu2;
    /* pre-smoothing */
    F(og_smooth)(P, lev, kap, f, u, pre, transposed);
    /* r = f - L(u);  p0 = R(p1);  r0 = R(r1);  f0 = r0 + L0(p0) */
    F(og_residual)(P, lev, kap, f, u, H->r);
    F(og_restrict)(P, lev, u, H->u[lev + 1]);
    F(og_restrict)(P, lev, H->r, H->t);
    F(og_apply)(P, lev + 1, H->kap[lev + 1], H->u[lev + 1], H->f[lev + 1]);
    {
        long Nc = og_level_cells(P, lev + 1);
        for (long p = 0; p < Nc; ++p) H->f[lev + 1][p] = H->t[p] + H->f[lev + 1][p];
    }
    /* coarse problem: recursion, or smoothing at the coarsest level */
    F(vcycle_rec)(P, H, lev + 1, nu1, nu2, transposed);
    /* c0 = p0_new - p0_old with p0_old = R(p1) recomputed (p1 unchanged meanwhile);
     * p1 := p1 + P(c0) */
    F(og_restrict)(P, lev, u, H->t);
    F(og_prolong_add)(P, lev, H->u[lev + 1], H->t, u);
    /* post-smoothing */
    F(og_smooth)(P, lev, kap, f, u, post, transposed);
}

static double F(norm2)(long N, const REAL* x)
{
    double s = 0.0;
    for (long p = 0; p < N; ++p) s += (double)x[p] * (double)x[p];
    return sqrt(s);
}

/* One V-cycle on the finest level, u updated in place. */
int F(og_vcycle)(const og_problem* P, const REAL* kap0, const REAL* f, REAL* u, int nu1, int nu2,
                 int transposed)
{
    F(og_hier) H;
    if (F(hier_init)(P, kap0, &H)) return -1;
    H.u[0] = u;
    H.f[0] = (REAL*)f;
    F(vcycle_rec)(P, &H, 0, nu1, nu2, transposed);
    F(hier_free)(&H);
    return 0;
}

/* Solve loop (Alg. 1 outer loop): V-cycles until ||f - L(u)||_2 <= tol*||f||_2 (or, with
 * P->atol > 0, ||f - L(u)||_2 <= P->atol: Algorithm 1's absolute test) or kmax cycles.  hist (nullable, kmax entries) receives ||r||_2/||f||_2 after each cycle.
 * Returns 0 when converged, 1 when kmax was reached, -1 on a bad shape. */
int F(og_solve)(const og_problem* P, const REAL* kap0, const REAL* f, REAL* u, double tol, int nu1, int nu2,
                int kmax, int transposed, int* cycles, double* hist)
{
    F(og_hier) H;
    if (F(hier_init)(P, kap0, &H)) return -1;
    H.u[0] = u;
    H.f[0] = (REAL*)f;
    long N = og_level_cells(P, 0);
    double nf = F(norm2)(N, f);
    int status = 1;
    int k;
    for (k = 1; k <= kmax; ++k) {
        F(vcycle_rec)(P, &H, 0, nu1, nu2, transposed);
        F(og_residual)(P, 0, kap0, f, u, H.r);
        double nr = F(norm2)(N, H.r);
        if (hist) hist[k - 1] = nf > 0.0 ? nr / nf : nr;
        if (nr <= tol * nf || nr <= P->atol || nr == 0.0) {
            status = 0;
            break;
        }
    }
    if (cycles) *cycles = status == 0 ? k : kmax;
    F(hier_free)(&H);
    return status;
}

#undef F
#undef OG_CAT
#undef OG_CAT2
