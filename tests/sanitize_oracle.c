/* Driver for the sanitizer build of the CPU oracle (AddressSanitizer and
 * UndefinedBehaviorSanitizer, compiled by tests/test_oracle_sanitize.py): the oracle's
 * source is included whole, and every entry point runs on small grids of each boundary
 * condition, dimension, precision, coefficient kind and set order.  Any invalid access or
 * undefined operation aborts the run with the sanitizer's report. */
#include "../oracle/fas_oracle.c"

#include <stdio.h>

static unsigned long long g_state = 88172645463325252ull;
static double urand(void)
{
    g_state ^= g_state << 13;
    g_state ^= g_state >> 7;
    g_state ^= g_state << 17;
    return (double)(g_state >> 11) / 9007199254740992.0 * 2.0 - 1.0;
}

static int run(int dim, const long* n, int bc, int coarsest, int order, int symmetric, int cell)
{
    og_problem P;
    memset(&P, 0, sizeof P);
    P.dim = dim;
    P.bc = bc;
    for (int a = 0; a < 3; ++a) P.n[a] = a < dim ? n[a] : 1;
    P.h = 1.0 / (double)n[0];
    P.dt = 0.05;
    P.kappa = 1.3;
    P.coarsest = coarsest;
    P.nuc = 2;
    P.order = order;
    P.symmetric = symmetric;
    long N = og_level_cells(&P, 0);
    double* f = malloc(N * sizeof(double));
    double* u = malloc(N * sizeof(double));
    double* k = malloc(N * sizeof(double));
    double* g = calloc(N, sizeof(double));
    float* f32 = malloc(N * sizeof(float));
    float* u32 = malloc(N * sizeof(float));
    for (long p = 0; p < N; ++p) {
        f[p] = urand();
        u[p] = urand();
        k[p] = 1.0 + 0.5 * urand();
        f32[p] = (float)f[p];
        u32[p] = (float)u[p];
    }
    const double* kap = cell ? k : 0;
    int cycles = 0, rc = 0;
    double hist[64];
    rc |= og_vcycle_d(&P, kap, f, u, 2, 1, 0);
    rc |= og_vcycle_d(&P, kap, f, u, 1, 2, 1);
    rc |= og_solve_d(&P, kap, f, u, 1e-8, 2, 2, 40, 0, &cycles, hist) < 0;
    rc |= og_vcycle_s(&P, 0, f32, u32, 2, 2, 0);
    rc |= og_solve_mixed(&P, kap, f, u, 1e-9, 2, 2, 3, 1, 20, &cycles, hist) < 0;
    if (cell) og_kappa_grad_d(&P, k, f, u, g);
    free(f);
    free(u);
    free(k);
    free(g);
    free(f32);
    free(u32);
    return rc;
}

int main(void)
{
    const long n2[3] = {24, 16, 1}, n3[3] = {8, 12, 16}, sq[3] = {16, 16, 1};
    int bad = 0, cases = 0;
    for (int bc = 0; bc < 3; ++bc)
        for (int cell = 0; cell < 2; ++cell) {
            bad |= run(2, n2, bc, 2, OG_X, 0, cell), ++cases;
            bad |= run(3, n3, bc, 2, OG_X, 0, cell), ++cases;
            for (int order = 0; order < 3; ++order)
                for (int sym = 0; sym < 2; ++sym) {
                    bad |= run(2, sq, bc, 4, order, sym, cell), ++cases;
                    bad |= run(3, n3, bc, 2, order, sym, cell), ++cases;
                }
        }
    printf("sanitized oracle: %d cases, %s\n", cases, bad ? "FAILED" : "ok");
    return bad;
}
