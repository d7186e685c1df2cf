/* Sanitizer driver for the FP64 oracle -- TEST INFRASTRUCTURE.
 *
 * Built by tests/test_oracle_sanitize.py with AddressSanitizer and
 * UndefinedBehaviorSanitizer on the host compiler (gcc), it calls every
 * entry point of the oracle on small grids that reach its edge cases:
 * ragged dims, odd n_phi on the coarsest level, the full sphere's zero-area
 * polar faces, all four maps and both metric methods, every outer iteration
 * (stationary, CG, BiCGStab), the projection step and the ADI line solves
 * with both wall conditions.  Any out-of-bounds access, leak, use after
 * free, signed overflow or misaligned access aborts with a report; the
 * driver prints "oracle sanitize: ok" only after all calls returned.
 *
 * The oracle is included as source so that one translation unit carries
 * both (its structs are not in a header). */
#include "../../oracle/cps_oracle.c"

#include <stdio.h>

static double* field(size_t n, unsigned* s)
{
    double* v = malloc(n * sizeof(double));
    for (size_t i = 0; i < n; ++i) {
        *s = *s * 1664525u + 1013904223u;
        v[i] = (double)(*s >> 8) / 16777216.0 - 0.5;
    }
    return v;
}

static void run(const og_grid* g, int method, unsigned seed)
{
    const int nr = g->n_r, nt = g->n_theta, np = g->n_phi;
    const size_t n = (size_t)nr * nt * np;
    double* G = malloc(9 * n * sizeof(double));
    if (orc_face_metrics(g, nr, nt, np, method, G) != 0) {
        fprintf(stderr, "metrics failed\n");
        exit(1);
    }
    double* x = field(n, &seed);
    double* b = field(n, &seed);
    double* y = malloc(n * sizeof(double));
    orc_apply(nr, nt, np, G, x, y);
    orc_residual(nr, nt, np, G, b, x, y);
    const int ncol = 4;
    for (int c = 0; c < ncol; ++c) orc_gs_pass(nr, nt, np, ncol, c, G, b, x);
    if (n <= 512) {
        double* A = malloc(n * n * sizeof(double));
        orc_dense_matrix(nr, nt, np, G, A);
        free(A);
    }
    if (nr % 2 == 0 && nt % 2 == 0 && np % 2 == 0) {
        const size_t nc = n / 8;
        double* bc = malloc(nc * sizeof(double));
        orc_restrict(nr, nt, np, y, bc);
        orc_prolong_add(nr, nt, np, bc, x);
        free(bc);
    }
    og_mg* m = orc_mg_create(g, method, 0, 0);
    if (!m) {
        fprintf(stderr, "multigrid set-up failed\n");
        exit(1);
    }
    int dims[48], nc2 = 0, it = 0;
    orc_mg_levels(m, dims, &nc2);
    (void)orc_mg_metrics(m, 0);
    double* e = malloc(n * sizeof(double));
    orc_mg_vcycle(m, b, e);
    orc_mg_coarse_solve(m, b, e);
    for (int accel = 0; accel <= 2; ++accel) {
        double rel = 0.0, mean = 0.0, hist[12];
        orc_mg_solve(m, b, e, 1e-9, 12, accel, &it, &rel, hist, &mean);
    }
    free(e);
    orc_mg_destroy(m);
    double* u = field(3 * n, &seed);
    double* out = malloc(3 * n * sizeof(double));
    long long cells[3] = {0, (long long)n / 2, (long long)n - 1};
    orc_divergence(g, nr, nt, np, method, u, (long long)n, NULL, out);
    orc_divergence(g, nr, nt, np, method, u, 3, cells, out);
    orc_correct(g, nr, nt, np, method, x, u, (long long)n, NULL, out);
    orc_correct(g, nr, nt, np, method, x, u, 3, cells, out);
    double C[3];
    (void)orc_face_crow(g, nr, nt, np, method, 1, nr, nt, np - 1, C);
    (void)orc_cell_jdet(g, nr, nt, np, method, nr - 1, nt - 1, np - 1);
    for (int d = 0; d < 3; ++d)
        for (int bc = 0; bc <= 1; ++bc) {
            orc_line_apply(g, nr, nt, np, method, d, 0.7, bc, 0.3, 1 - bc, -0.2, x, y);
            long long line = 1;
            (void)orc_line_solve(g, nr, nt, np, method, d, 0.7, bc, 0.3, 1 - bc, -0.2, b, y, 0,
                                 NULL);
            (void)orc_line_solve(g, nr, nt, np, method, d, 0.7, bc, 0.3, 1 - bc, -0.2, b, y, 1,
                                 &line);
        }
    double X[3], t[9] = {1, 0.1, 0, 0, 1, 0.2, 0.1, 0, 1}, Gm[9];
    orc_map(g, 0.3, 0.6, 0.9, X);
    (void)orc_metric_from_chords(t, Gm);
    free(G); free(x); free(b); free(y); free(u); free(out);
}

int main(void)
{
    const double pi = M_PI;
    const og_grid grids[] = {
        {12, 10, 14, OG_SPHERE, 1.5, 2.5, 0.05, pi - 0.05, 2.0, 0.0, 0.0},
        {8, 6, 10, OG_OBLATE, 1.5, 2.5, 0.0, pi, 0.0, 0.1, 0.0},
        {6, 6, 8, OG_TRIAXIAL, 1.5, 2.5, 0.05, pi - 0.05, 1.0, 0.1, 0.2},
        {8, 12, 16, OG_IDENTITY, 0.0, 1.0, 0.0, 2.0, 0.0, 0.0, 0.0},
        {5, 7, 6, OG_SPHERE, 1.5, 2.5, 0.0, pi, 0.0, 0.0, 0.0},
    };
    unsigned seed = 12345u;
    for (size_t k = 0; k < sizeof grids / sizeof grids[0]; ++k)
        for (int method = 0; method <= 1; ++method) run(&grids[k], method, seed + (unsigned)k);
    int dims[48];
    (void)orc_level_plan(192, 256, 512, 0, dims);
    (void)orc_colour(2, 1, 2, 3);
    printf("oracle sanitize: ok\n");
    return 0;
}
