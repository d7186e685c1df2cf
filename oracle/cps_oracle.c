/*
 * cps_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct FP64 CPU implementation of the
 * pressure-correction Poisson solve of Naskar, Chongsiripinyo, Pal and
 * Jananan, "A generalized curvilinear solver for spherical shell
 * Rayleigh-Benard convection" (arXiv 2305.17875), Sec. 3.1-3.3 and the
 * pressure-correction section, eq. (PC_6).
 *
 * Only the test suite, the package's smoke check and the benchmark's CPU
 * baseline call this file.  The GPU library shares no code with it.
 *
 * Conventions
 *   - Cell arrays are [n_r][n_theta][n_phi] in C order, phi contiguous.
 *     Index a runs along r (paper's eta), b along theta (paper's zeta),
 *     c along phi (paper's xi, periodic).
 *   - Face metrics are stored as G[9][n_r][n_theta][n_phi]; entry 3*d+q of
 *     cell (a,b,c) is G_dq on the LOW face of that cell in direction d
 *     (d = 0 r, 1 theta, 2 phi).  Faces on the r- and theta-walls are zero.
 *   - Every transformed cell has unit side (Sec. 3.1): all derivatives are
 *     per index unit of the level the metrics belong to.
 *
 * Parity pins for this file live in tests/test_oracle_*.py.  Functions
 * whose result has no closed form are pinned through the exact solvers in
 * oracle/direct.py; the V-cycle convergence factor and iteration counts are
 * parity unpinned (the paper reports none).
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* threads the oracle's parallel loops use */
int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* set the threads of the parallel loops (n >= 1); for timing at one thread */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Grid and map (Sec. 2, 3.1; the tanh clustering is eq. (stretching))      */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t n_r, n_theta, n_phi;
    int32_t map;            /* 0 identity box, 1 sphere, 2 oblate, 3 triaxial */
    double r_inner, r_outer;
    double theta0, theta1;
    double radial_stretch;  /* rx2 of eq. (stretching); 0 = uniform spacing */
    double flattening;      /* oblate / triaxial: x1 axis scaled by (1-f)   */
    double skew;            /* triaxial: x2 axis scaled by (1+g)            */
} og_grid;

enum { OG_IDENTITY = 0, OG_SPHERE = 1, OG_OBLATE = 2, OG_TRIAXIAL = 3 };

/* radius at normalised radial coordinate s in [0,1].  eq. (stretching)
 * gives r(j) in [-1/2, 1/2] for j-1 = s * nx2; it is shifted to the shell
 * mid-radius and scaled by the gap d. */
static double og_radius(const og_grid* g, double s)
{
    double d = g->r_outer - g->r_inner;
    if (g->radial_stretch == 0.0) return g->r_inner + d * s;
    double k = g->radial_stretch;
    return 0.5 * (g->r_inner + g->r_outer) + d * tanh(k * (s - 0.5)) / (2.0 * tanh(0.5 * k));
}

/* physical point X of computational coordinates (s_r, s_theta, s_phi); the
 * polar axis is x1 (Sec. 2, definition of delta_in). */
void orc_map(const og_grid* g, double sr, double st, double sp, double X[3])
{
    double r = og_radius(g, sr);
    double th = g->theta0 + st * (g->theta1 - g->theta0);
    double ph = 2.0 * M_PI * sp;
    switch (g->map) {
    case OG_IDENTITY:
        X[0] = r; X[1] = th; X[2] = ph;
        break;
    case OG_SPHERE:
        X[0] = r * cos(th); X[1] = r * sin(th) * cos(ph); X[2] = r * sin(th) * sin(ph);
        break;
    case OG_OBLATE:
        X[0] = (1.0 - g->flattening) * r * cos(th);
        X[1] = r * sin(th) * cos(ph); X[2] = r * sin(th) * sin(ph);
        break;
    default: /* OG_TRIAXIAL */
        X[0] = (1.0 - g->flattening) * r * cos(th);
        X[1] = (1.0 + g->skew) * r * sin(th) * cos(ph);
        X[2] = r * sin(th) * sin(ph);
        break;
    }
}

/* X at fractional index position (ia, ib, ic) of a level with dims n */
static void og_point(const og_grid* g, int nr, int nt, int np, double ia, double ib, double ic,
                     double X[3])
{
    orc_map(g, ia / nr, ib / nt, ic / np, X);
}

/* ------------------------------------------------------------------------ */
/* Face metrics (Sec. 3.2 items 1, 2, 4, 5; eq. (jacobi), (skewness))       */
/* ------------------------------------------------------------------------ */

static void og_cross(const double u[3], const double v[3], double w[3])
{
    w[0] = u[1] * v[2] - u[2] * v[1];
    w[1] = u[2] * v[0] - u[0] * v[2];
    w[2] = u[0] * v[1] - u[1] * v[0];
}

static double og_dot(const double u[3], const double v[3])
{
    return u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
}

/* Given the three columns t[q] = dX/ds_q of the inverse Jacobian at a face,
 * return det and G_dq = |J^-1| (ds_d/dx_k)(ds_q/dx_k).  The rows of the
 * Jacobian (the inverse of the matrix with columns t_q) are the cyclic cross
 * products n_d = t_{d+1} x t_{d+2} divided by det, which is the cofactor
 * inversion of item 4. */
double orc_metric_from_chords(const double t[9], double G[9])
{
    double n[3][3];
    og_cross(&t[3], &t[6], n[0]);
    og_cross(&t[6], &t[0], n[1]);
    og_cross(&t[0], &t[3], n[2]);
    double det = og_dot(&t[0], n[0]);
    for (int d = 0; d < 3; ++d)
        for (int q = 0; q < 3; ++q) G[3 * d + q] = og_dot(n[d], n[q]) / det;
    return det;
}

/* Metrics of every face of a level with dims (nr, nt, np).
 * method 0 (default): chords t_q of the map across the face centre,
 *   t_q = X(f + e_q/2) - X(f - e_q/2), central differences of the map.
 * method 1 (the paper's item 1): the normal derivative is the average over
 *   the face's four vertices of the central difference across vertex planes
 *   (weight 1/8), each tangential derivative is the mean of the face's two
 *   edges along that direction (weight 1/2).
 * Cross entries below 1e-10 sqrt(G_dd G_qq) are set to zero (chords are
 * differences of nearby points, so an orthogonal map shows rounding noise of
 * about 1e-12 relative at 512 cells per direction); wall faces are
 * zero.  Returns 0, or -1 if some interior face has det <= 0. */
/* Chords t[3q .. 3q+2] = dX/ds_q across the LOW d-face of cell (a,b,c) of a
 * level with dims (nr, nt, np), by `method` (see orc_face_metrics).  The
 * face may lie on a wall, including the high walls a = nr and b = nt: the
 * map is evaluated wherever the formula asks. */
static void og_face_chords(const og_grid* g, int nr, int nt, int np, int method, int d, int a,
                           int b, int c, double t[9])
{
    double lo[3] = {a, b, c}; /* vertex at the face's low corner */
    if (method == 0) {
        double f[3] = {a + 0.5, b + 0.5, c + 0.5};
        f[d] -= 0.5;
        for (int q = 0; q < 3; ++q) {
            double p1[3] = {f[0], f[1], f[2]}, p0[3] = {f[0], f[1], f[2]};
            p1[q] += 0.5; p0[q] -= 0.5;
            double X1[3], X0[3];
            og_point(g, nr, nt, np, p1[0], p1[1], p1[2], X1);
            og_point(g, nr, nt, np, p0[0], p0[1], p0[2], X0);
            for (int k = 0; k < 3; ++k) t[3 * q + k] = X1[k] - X0[k];
        }
        return;
    }
    int u = (d + 1) % 3, v = (d + 2) % 3; /* tangential directions */
    /* normal: 1/8 sum over 4 face vertices of X(v+e_d) - X(v-e_d) */
    for (int k = 0; k < 3; ++k) t[3 * d + k] = 0.0;
    for (int iu = 0; iu < 2; ++iu)
        for (int iv = 0; iv < 2; ++iv) {
            double p[3] = {lo[0], lo[1], lo[2]};
            p[u] += iu; p[v] += iv;
            double p1[3] = {p[0], p[1], p[2]}, p0[3] = {p[0], p[1], p[2]};
            p1[d] += 1.0; p0[d] -= 1.0;
            double X1[3], X0[3];
            og_point(g, nr, nt, np, p1[0], p1[1], p1[2], X1);
            og_point(g, nr, nt, np, p0[0], p0[1], p0[2], X0);
            for (int k = 0; k < 3; ++k) t[3 * d + k] += 0.125 * (X1[k] - X0[k]);
        }
    /* tangential q: 1/2 sum over the 2 edges along q */
    for (int s = 0; s < 2; ++s) {
        int q = s == 0 ? u : v, o = s == 0 ? v : u;
        for (int k = 0; k < 3; ++k) t[3 * q + k] = 0.0;
        for (int io = 0; io < 2; ++io) {
            double p0[3] = {lo[0], lo[1], lo[2]};
            p0[o] += io;
            double p1[3] = {p0[0], p0[1], p0[2]};
            p1[q] += 1.0;
            double X1[3], X0[3];
            og_point(g, nr, nt, np, p1[0], p1[1], p1[2], X1);
            og_point(g, nr, nt, np, p0[0], p0[1], p0[2], X0);
            for (int k = 0; k < 3; ++k) t[3 * q + k] += 0.5 * (X1[k] - X0[k]);
        }
    }
}

/* Metrics of every face of a level with dims (nr, nt, np).
 * method 0 (default): chords t_q of the map across the face centre,
 *   t_q = X(f + e_q/2) - X(f - e_q/2), central differences of the map.
 * method 1 (the paper's item 1): the normal derivative is the average over
 *   the face's four vertices of the central difference across vertex planes
 *   (weight 1/8), each tangential derivative is the mean of the face's two
 *   edges along that direction (weight 1/2).
 * Cross entries below 1e-10 sqrt(G_dd G_qq) are set to zero (chords are
 * differences of nearby points, so an orthogonal map shows rounding noise of
 * about 1e-12 relative at 512 cells per direction); wall faces are
 * zero.  Returns 0, or -1 if some interior face has det <= 0. */
int orc_face_metrics(const og_grid* g, int nr, int nt, int np, int method, double* G)
{
    const size_t N = (size_t)nr * nt * np;
    int bad = 0;
#pragma omp parallel for collapse(2) reduction(| : bad)
    for (int a = 0; a < nr; ++a)
        for (int b = 0; b < nt; ++b)
            for (int c = 0; c < np; ++c) {
                size_t id = ((size_t)a * nt + b) * np + c;
                for (int d = 0; d < 3; ++d) {
                    double Gf[9] = {0};
                    int wall = (d == 0 && a == 0) || (d == 1 && b == 0);
                    if (!wall) {
                        double t[9];
                        og_face_chords(g, nr, nt, np, method, d, a, b, c, t);
                        double det = orc_metric_from_chords(t, Gf);
                        if (!(det > 0.0)) bad = 1;
                        for (int p = 0; p < 3; ++p)
                            for (int q = 0; q < 3; ++q)
                                if (p != q &&
                                    fabs(Gf[3 * p + q]) <= 1e-10 * sqrt(fabs(Gf[4 * p] * Gf[4 * q])))
                                    Gf[3 * p + q] = 0.0;
                    }
                    for (int q = 0; q < 3; ++q) G[(size_t)(3 * d + q) * N + id] = Gf[3 * d + q];
                }
            }
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Operator: flux form of d/ds_p [ G_pq d phi / ds_q ]                      */
/* eq. (PC_8) with the nine terms written like eq. (PC_term1)-(PC_term3)    */
/* ------------------------------------------------------------------------ */

typedef struct { int nr, nt, np; } og_dims;

static size_t og_idx(og_dims n, int a, int b, int c)
{
    return ((size_t)a * n.nt + b) * n.np + c;
}

/* value of x at (a,b,c): mirror (clamp) in r and theta, wrap in phi */
static double og_x(og_dims n, const double* x, int a, int b, int c)
{
    if (a < 0) a = 0;
    if (a > n.nr - 1) a = n.nr - 1;
    if (b < 0) b = 0;
    if (b > n.nt - 1) b = n.nt - 1;
    c = ((c % n.np) + n.np) % n.np;
    return x[og_idx(n, a, b, c)];
}

/* Flux F_d through the low face (in direction d) of cell (a,b,c): the cell
 * on the high side of the face is (a,b,c), the one on the low side is
 * (a,b,c) - e_d.  F_d = G_dd (x_hi - x_lo) + sum_{q != d} 1/4 G_dq
 * (x_hi+e_q + x_lo+e_q - x_hi-e_q - x_lo-e_q); zero on r- and theta-walls,
 * including the walls at a = n_r and b = n_theta. */
static double og_flux(og_dims n, const double* G, const double* x, int d, int a, int b, int c)
{
    if (d == 0 && (a == 0 || a == n.nr)) return 0.0;
    if (d == 1 && (b == 0 || b == n.nt)) return 0.0;
    int cw = ((c % n.np) + n.np) % n.np;
    size_t N = (size_t)n.nr * n.nt * n.np;
    size_t id = og_idx(n, a, b, cw);
    int hi[3] = {a, b, c}, lo[3] = {a, b, c};
    lo[d] -= 1;
    double F = G[(size_t)(3 * d + d) * N + id] *
               (og_x(n, x, hi[0], hi[1], hi[2]) - og_x(n, x, lo[0], lo[1], lo[2]));
    for (int q = 0; q < 3; ++q) {
        if (q == d) continue;
        double Gdq = G[(size_t)(3 * d + q) * N + id];
        if (Gdq == 0.0) continue;
        int e[3] = {0, 0, 0};
        e[q] = 1;
        double s = og_x(n, x, hi[0] + e[0], hi[1] + e[1], hi[2] + e[2]) +
                   og_x(n, x, lo[0] + e[0], lo[1] + e[1], lo[2] + e[2]) -
                   og_x(n, x, hi[0] - e[0], hi[1] - e[1], hi[2] - e[2]) -
                   og_x(n, x, lo[0] - e[0], lo[1] - e[1], lo[2] - e[2]);
        F += 0.25 * Gdq * s;
    }
    return F;
}

/* (A x) at one cell: sum over directions of F(high face) - F(low face). */
static double og_apply_cell(og_dims n, const double* G, const double* x, int a, int b, int c)
{
    double s = 0.0;
    s += og_flux(n, G, x, 0, a + 1, b, c) - og_flux(n, G, x, 0, a, b, c);
    s += og_flux(n, G, x, 1, a, b + 1, c) - og_flux(n, G, x, 1, a, b, c);
    s += og_flux(n, G, x, 2, a, b, c + 1) - og_flux(n, G, x, 2, a, b, c);
    return s;
}

/* -sum of the six diagonal face metrics G_dd around the cell */
static double og_diag(og_dims n, const double* G, int a, int b, int c)
{
    size_t N = (size_t)n.nr * n.nt * n.np;
    double s = 0.0;
    s += G[0 * N + og_idx(n, a, b, c)];
    if (a + 1 < n.nr) s += G[0 * N + og_idx(n, a + 1, b, c)];
    s += G[4 * N + og_idx(n, a, b, c)];
    if (b + 1 < n.nt) s += G[4 * N + og_idx(n, a, b + 1, c)];
    s += G[8 * N + og_idx(n, a, b, c)];
    s += G[8 * N + og_idx(n, a, b, (c + 1) % n.np)];
    return -s;
}

void orc_apply(int nr, int nt, int np, const double* G, const double* x, double* y)
{
    og_dims n = {nr, nt, np};
#pragma omp parallel for collapse(2)
    for (int a = 0; a < nr; ++a)
        for (int b = 0; b < nt; ++b)
            for (int c = 0; c < np; ++c) y[og_idx(n, a, b, c)] = og_apply_cell(n, G, x, a, b, c);
}

void orc_residual(int nr, int nt, int np, const double* G, const double* bv, const double* x,
                  double* r)
{
    og_dims n = {nr, nt, np};
#pragma omp parallel for collapse(2)
    for (int a = 0; a < nr; ++a)
        for (int b = 0; b < nt; ++b)
            for (int c = 0; c < np; ++c) {
                size_t id = og_idx(n, a, b, c);
                r[id] = bv[id] - og_apply_cell(n, G, x, a, b, c);
            }
}

/* colour of a cell: two colours (a+b+c) mod 2 for 7-point stencils; four
 * colours from ((a+c) mod 2, (b+c) mod 2) for the 19-point stencil, which
 * separates every pair of cells that share a face or an edge. */
int orc_colour(int ncol, int a, int b, int c)
{
    if (ncol == 2) return (a + b + c) & 1;
    return 2 * ((a + c) & 1) + ((b + c) & 1);
}

/* One Gauss-Seidel pass over the cells of one colour, in place:
 * x_c <- x_c + (b_c - (A x)_c) / D_c with D_c = -(sum of the six G_dd).
 * Cells of one colour never read each other, so the order inside the pass
 * does not matter. */
void orc_gs_pass(int nr, int nt, int np, int ncol, int colour, const double* G, const double* bv,
                 double* x)
{
    og_dims n = {nr, nt, np};
#pragma omp parallel for collapse(2)
    for (int a = 0; a < nr; ++a)
        for (int b = 0; b < nt; ++b)
            for (int c = 0; c < np; ++c) {
                if (orc_colour(ncol, a, b, c) != colour) continue;
                size_t id = og_idx(n, a, b, c);
                double Ax = og_apply_cell(n, G, x, a, b, c);
                x[id] += (bv[id] - Ax) / og_diag(n, G, a, b, c);
            }
}

/* ------------------------------------------------------------------------ */
/* Grid transfers                                                           */
/* ------------------------------------------------------------------------ */

/* 1-D cell-centred linear interpolation weights: fine cell i of a dimension
 * with nc coarse cells takes 3/4 of coarse cell i/2 and 1/4 of its nearer
 * neighbour (i/2 - 1 for even i, i/2 + 1 for odd i).  The neighbour index is
 * clamped at walls and wrapped when periodic. */
static void og_w1(int i, int nc, int periodic, int I[2], double w[2])
{
    int C = i / 2;
    int Nb = (i % 2 == 0) ? C - 1 : C + 1;
    if (periodic) Nb = ((Nb % nc) + nc) % nc;
    else if (Nb < 0) Nb = 0;
    else if (Nb > nc - 1) Nb = nc - 1;
    I[0] = C; w[0] = 0.75;
    I[1] = Nb; w[1] = 0.25;
}

/* x_fine += P e_coarse (trilinear); (nr, nt, np) are the FINE dims. */
void orc_prolong_add(int nr, int nt, int np, const double* e, double* x)
{
    og_dims nf = {nr, nt, np}, ncd = {nr / 2, nt / 2, np / 2};
#pragma omp parallel for collapse(2)
    for (int a = 0; a < nr; ++a)
        for (int b = 0; b < nt; ++b)
            for (int c = 0; c < np; ++c) {
                int Ia[2], Ib[2], Ic[2];
                double wa[2], wb[2], wc[2];
                og_w1(a, ncd.nr, 0, Ia, wa);
                og_w1(b, ncd.nt, 0, Ib, wb);
                og_w1(c, ncd.np, 1, Ic, wc);
                double s = 0.0;
                for (int i = 0; i < 2; ++i)
                    for (int j = 0; j < 2; ++j)
                        for (int k = 0; k < 2; ++k)
                            s += wa[i] * wb[j] * wc[k] * e[og_idx(ncd, Ia[i], Ib[j], Ic[k])];
                x[og_idx(nf, a, b, c)] += s;
            }
}

/* b_coarse = P^T r_fine, written as the transpose: every fine cell scatters
 * its residual to the coarse cells that interpolate to it, with the same
 * weights.  (nr, nt, np) are the FINE dims.  Serial on purpose (scatter). */
void orc_restrict(int nr, int nt, int np, const double* r, double* bc)
{
    og_dims nf = {nr, nt, np}, ncd = {nr / 2, nt / 2, np / 2};
    memset(bc, 0, sizeof(double) * (size_t)ncd.nr * ncd.nt * ncd.np);
    for (int a = 0; a < nr; ++a)
        for (int b = 0; b < nt; ++b)
            for (int c = 0; c < np; ++c) {
                int Ia[2], Ib[2], Ic[2];
                double wa[2], wb[2], wc[2];
                og_w1(a, ncd.nr, 0, Ia, wa);
                og_w1(b, ncd.nt, 0, Ib, wb);
                og_w1(c, ncd.np, 1, Ic, wc);
                double v = r[og_idx(nf, a, b, c)];
                for (int i = 0; i < 2; ++i)
                    for (int j = 0; j < 2; ++j)
                        for (int k = 0; k < 2; ++k)
                            bc[og_idx(ncd, Ia[i], Ib[j], Ic[k])] += wa[i] * wb[j] * wc[k] * v;
            }
}

/* ------------------------------------------------------------------------ */
/* Dense coarse operator and LU                                             */
/* ------------------------------------------------------------------------ */

/* Column j of A is A applied to the j-th unit vector.  A is row-major n x n. */
void orc_dense_matrix(int nr, int nt, int np, const double* G, double* A)
{
    size_t n = (size_t)nr * nt * np;
    double* e = calloc(n, sizeof(double));
    double* y = malloc(n * sizeof(double));
    for (size_t j = 0; j < n; ++j) {
        e[j] = 1.0;
        orc_apply(nr, nt, np, G, e, y);
        e[j] = 0.0;
        for (size_t i = 0; i < n; ++i) A[i * n + j] = y[i];
    }
    free(e);
    free(y);
}

/* LU with partial pivoting, in place, row-major. */
static int og_lu(int n, double* A, int* piv)
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i)
            if (fabs(A[(size_t)i * n + k]) > fabs(A[(size_t)p * n + k])) p = i;
        piv[k] = p;
        if (A[(size_t)p * n + k] == 0.0) return -1;
        if (p != k)
            for (int j = 0; j < n; ++j) {
                double t = A[(size_t)k * n + j];
                A[(size_t)k * n + j] = A[(size_t)p * n + j];
                A[(size_t)p * n + j] = t;
            }
        for (int i = k + 1; i < n; ++i) {
            double l = A[(size_t)i * n + k] / A[(size_t)k * n + k];
            A[(size_t)i * n + k] = l;
            for (int j = k + 1; j < n; ++j) A[(size_t)i * n + j] -= l * A[(size_t)k * n + j];
        }
    }
    return 0;
}

static void og_lu_solve(int n, const double* LU, const int* piv, double* x)
{
    for (int k = 0; k < n; ++k) {
        int p = piv[k];
        if (p != k) { double t = x[k]; x[k] = x[p]; x[p] = t; }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) x[i] -= LU[(size_t)i * n + j] * x[j];
    for (int i = n - 1; i >= 0; --i) {
        for (int j = i + 1; j < n; ++j) x[i] -= LU[(size_t)i * n + j] * x[j];
        x[i] /= LU[(size_t)i * n + i];
    }
}

/* ------------------------------------------------------------------------ */
/* Multigrid: level plan, V(2,2), outer iterations                          */
/* ------------------------------------------------------------------------ */

#define OG_MAXL 16

typedef struct {
    og_grid g;
    int L;
    og_dims d[OG_MAXL];
    double* G[OG_MAXL];
    double *x[OG_MAXL], *b[OG_MAXL], *r[OG_MAXL];
    int ncol;
    double* lu;
    int* piv;
    int nc;
    double alpha;
    int pre, post;
} og_mg;

static size_t og_n(og_dims d) { return (size_t)d.nr * d.nt * d.np; }

/* Level plan: halve every dimension while the level has more than 1024
 * cells, every dimension is even and at least 4, and n_phi stays even on
 * the coarser level (red-black colouring wraps around the periodic phi
 * direction only when n_phi is even).  n_levels > 0 asks for exactly that
 * many levels (-1 if impossible). */
int orc_level_plan(int nr, int nt, int np, int n_levels, int* dims_out /* [16][3] */)
{
    int L = 1;
    dims_out[0] = nr; dims_out[1] = nt; dims_out[2] = np;
    for (;;) {
        int* p = &dims_out[3 * (L - 1)];
        int can = p[0] % 2 == 0 && p[1] % 2 == 0 && p[2] % 4 == 0 && p[0] >= 4 && p[1] >= 4 &&
                  p[2] >= 4;
        long cells = (long)p[0] * p[1] * p[2];
        int want = n_levels > 0 ? L < n_levels : cells > 1024;
        if (!want) break;
        if (!can || L == OG_MAXL) return n_levels > 0 ? -1 : L;
        int* q = &dims_out[3 * L];
        q[0] = p[0] / 2; q[1] = p[1] / 2; q[2] = p[2] / 2;
        ++L;
    }
    return L;
}

void orc_mg_destroy(og_mg* m)
{
    if (!m) return;
    for (int l = 0; l < m->L; ++l) {
        free(m->G[l]); free(m->x[l]); free(m->b[l]); free(m->r[l]);
    }
    free(m->lu);
    free(m->piv);
    free(m);
}

/* Face metrics of a coarse level from those of the fine level below it.
 * The low d-face of coarse cell (A, B, C) is made of the four fine low
 * d-faces at index 2A (d = r), 2B (d = theta) or 2C (d = phi) along d and
 * the two fine indices of each other direction.  A face metric is an area
 * over a normal length (G_dd = |J^-1| |grad s_d|^2 = area^2 / volume per
 * unit index spacing): the coarse face has four times the area and twice
 * the normal length, so G_H = 2 G_h = (1/2) of the sum over the four
 * children, entry by entry (the cross entries scale the same way).  Exact
 * for a uniform box; second order otherwise.  Wall faces stay zero. */
void orc_coarsen_metrics(int nr, int nt, int np, const double* Gf, double* Gc)
{
    og_dims f = {nr, nt, np}, c = {nr / 2, nt / 2, np / 2};
    size_t nf = og_n(f), ncell = og_n(c);
#pragma omp parallel for
    for (long long i = 0; i < (long long)ncell; ++i) {
        int C = (int)(i % c.np), B = (int)((i / c.np) % c.nt), A = (int)(i / ((size_t)c.np * c.nt));
        for (int d = 0; d < 3; ++d)
            for (int q = 0; q < 3; ++q) {
                const double* g = Gf + (size_t)(3 * d + q) * nf;
                double s = 0.0;
                for (int u = 0; u < 2; ++u)
                    for (int v = 0; v < 2; ++v) {
                        int a = 2 * A, b = 2 * B, cc = 2 * C;
                        if (d == 0) { b += u; cc += v; }
                        else if (d == 1) { a += u; cc += v; }
                        else { a += u; b += v; }
                        s += g[og_idx(f, a, b, cc)];
                    }
                Gc[(size_t)(3 * d + q) * ncell + i] = 0.5 * s;
            }
    }
}

/* Shared part of the set-ups: level plan and buffers, every level's metrics
 * through `fill`, the colouring and the coarsest operator's LU.  fill
 * returns nonzero on failure. */
static og_mg* og_mg_build(const og_grid* g, int n_levels, int force_ncol,
                          int (*fill)(og_mg* m, int l, const void* ctx), const void* ctx)
{
    int dims[3 * OG_MAXL];
    int L = orc_level_plan(g->n_r, g->n_theta, g->n_phi, n_levels, dims);
    if (L < 1) return NULL;
    og_mg* m = calloc(1, sizeof(og_mg));
    m->g = *g;
    m->L = L;
    m->pre = 2;
    m->post = 2;
    int ortho = 1;
    for (int l = 0; l < L; ++l) {
        og_dims d = {dims[3 * l], dims[3 * l + 1], dims[3 * l + 2]};
        m->d[l] = d;
        size_t n = og_n(d);
        m->G[l] = malloc(9 * n * sizeof(double));
        m->x[l] = calloc(n, sizeof(double));
        m->b[l] = calloc(n, sizeof(double));
        m->r[l] = calloc(n, sizeof(double));
        if (fill(m, l, ctx) != 0) {
            orc_mg_destroy(m);
            return NULL;
        }
        for (int k = 0; k < 9; ++k) {
            if (k == 0 || k == 4 || k == 8) continue;
            for (size_t i = 0; i < n; ++i)
                if (m->G[l][(size_t)k * n + i] != 0.0) { ortho = 0; break; }
        }
    }
    m->ncol = force_ncol ? force_ncol : (ortho ? 2 : 4);
    /* coarsest operator plus alpha 1 1^T, alpha = mean |diag| / n */
    og_dims dc = m->d[L - 1];
    int nc = (int)og_n(dc);
    m->nc = nc;
    m->lu = malloc((size_t)nc * nc * sizeof(double));
    m->piv = malloc((size_t)nc * sizeof(int));
    orc_dense_matrix(dc.nr, dc.nt, dc.np, m->G[L - 1], m->lu);
    double s = 0.0;
    for (int i = 0; i < nc; ++i) s += fabs(m->lu[(size_t)i * nc + i]);
    m->alpha = s / nc / nc;
    for (size_t i = 0; i < (size_t)nc * nc; ++i) m->lu[i] += m->alpha;
    if (og_lu(nc, m->lu, m->piv) != 0) {
        orc_mg_destroy(m);
        return NULL;
    }
    return m;
}

typedef struct { int method; } og_map_ctx;

static int og_fill_map(og_mg* m, int l, const void* ctx)
{
    const og_map_ctx* c = ctx;
    return orc_face_metrics(&m->g, m->d[l].nr, m->d[l].nt, m->d[l].np, c->method, m->G[l]);
}

/* Every level's metrics from the map at its own index spacing. */
og_mg* orc_mg_create(const og_grid* g, int method, int n_levels, int force_ncol)
{
    og_map_ctx c = {method};
    return og_mg_build(g, n_levels, force_ncol, og_fill_map, &c);
}

/* Level 0 from caller-given face metrics G0 [9][nr][nt][np] (the low r- and
 * theta-wall faces carry no flux: their entries are taken as zero), coarse
 * levels by orc_coarsen_metrics.  orc_mg_create_user returns NULL when an
 * entry is not finite or a diagonal entry is negative. */
static int og_fill_user(og_mg* m, int l, const void* ctx)
{
    og_dims d = m->d[l];
    size_t n = og_n(d);
    if (l > 0) {
        og_dims f = m->d[l - 1];
        orc_coarsen_metrics(f.nr, f.nt, f.np, m->G[l - 1], m->G[l]);
        return 0;
    }
    const double* G0 = ctx;
    for (int k = 0; k < 9; ++k)
        for (size_t i = 0; i < n; ++i) {
            double v = G0[(size_t)k * n + i];
            int b = (int)((i / d.np) % d.nt), a = (int)(i / ((size_t)d.np * d.nt));
            if ((k < 3 && a == 0) || (k >= 3 && k < 6 && b == 0)) v = 0.0; /* wall face */
            if (!isfinite(v) || ((k == 0 || k == 4 || k == 8) && v < 0.0)) return 1;
            m->G[0][(size_t)k * n + i] = v;
        }
    return 0;
}

og_mg* orc_mg_create_user(const double* G0, int nr, int nt, int np, int n_levels, int force_ncol)
{
    og_grid g;
    memset(&g, 0, sizeof g);
    g.n_r = nr; g.n_theta = nt; g.n_phi = np;
    return og_mg_build(&g, n_levels, force_ncol, og_fill_user, G0);
}

int orc_mg_levels(const og_mg* m, int* dims_out, int* ncol)
{
    for (int l = 0; l < m->L; ++l) {
        dims_out[3 * l] = m->d[l].nr;
        dims_out[3 * l + 1] = m->d[l].nt;
        dims_out[3 * l + 2] = m->d[l].np;
    }
    *ncol = m->ncol;
    return m->L;
}

const double* orc_mg_metrics(const og_mg* m, int level) { return m->G[level]; }

/* e = (A_c + alpha 1 1^T)^{-1} (b - mean b) on the coarsest level */
static void og_coarse_solve(og_mg* m, const double* bvec, double* e)
{
    int n = m->nc;
    double mean = 0.0;
    for (int i = 0; i < n; ++i) mean += bvec[i];
    mean /= n;
    for (int i = 0; i < n; ++i) e[i] = bvec[i] - mean;
    og_lu_solve(n, m->lu, m->piv, e);
}

void orc_mg_coarse_solve(og_mg* m, const double* bvec, double* e) { og_coarse_solve(m, bvec, e); }

static void og_smooth(og_mg* m, int l, int sweeps, int reverse)
{
    og_dims d = m->d[l];
    for (int s = 0; s < sweeps; ++s)
        for (int k = 0; k < m->ncol; ++k) {
            int col = reverse ? m->ncol - 1 - k : k;
            orc_gs_pass(d.nr, d.nt, d.np, m->ncol, col, m->G[l], m->b[l], m->x[l]);
        }
}

/* One V(pre,post) cycle on level 0 with right-hand side bvec, in place on x:
 * pre-smooth, residual, restrict, recurse, coarse solve, prolongate and add,
 * post-smooth with the colours in reverse order. */
void orc_mg_vcycle(og_mg* m, const double* bvec, double* x)
{
    size_t n0 = og_n(m->d[0]);
    memcpy(m->b[0], bvec, n0 * sizeof(double));
    memcpy(m->x[0], x, n0 * sizeof(double));
    for (int l = 0; l < m->L - 1; ++l) {
        og_dims d = m->d[l];
        if (l > 0) memset(m->x[l], 0, og_n(d) * sizeof(double));
        og_smooth(m, l, m->pre, 0);
        orc_residual(d.nr, d.nt, d.np, m->G[l], m->b[l], m->x[l], m->r[l]);
        orc_restrict(d.nr, d.nt, d.np, m->r[l], m->b[l + 1]);
    }
    og_coarse_solve(m, m->b[m->L - 1], m->x[m->L - 1]);
    for (int l = m->L - 2; l >= 0; --l) {
        og_dims d = m->d[l];
        orc_prolong_add(d.nr, d.nt, d.np, m->x[l + 1], m->x[l]);
        og_smooth(m, l, m->post, 1);
    }
    memcpy(x, m->x[0], n0 * sizeof(double));
}

static double og_dotv(size_t n, const double* u, const double* v)
{
    double s = 0.0;
    for (size_t i = 0; i < n; ++i) s += u[i] * v[i];
    return s;
}

/* Solve A x = b with sum(x) = 0 (eq. (PC_6) with zero-flux walls).
 * accel 0: x <- V-cycle(x) repeated (Richardson); 1: conjugate gradients
 * preconditioned by one V-cycle from zero; 2: BiCGStab, right-preconditioned
 * by the same V-cycle.  The mean of b is removed first and reported in
 * *mean_removed; x is returned with zero mean.  history[k] = relative
 * residual after iteration k+1 (if history != NULL, at most max_iters).
 * Returns 0 converged, -4 not converged, -5 diverged (non-finite norm). */
int orc_mg_solve(og_mg* m, const double* b_in, double* x, double tol, int max_iters, int accel,
                 int* iters, double* relres, double* history, double* mean_removed)
{
    size_t n = og_n(m->d[0]);
    og_dims d = m->d[0];
    double* bb = malloc(n * sizeof(double));
    double* r = malloc(n * sizeof(double));
    double mean = 0.0;
    for (size_t i = 0; i < n; ++i) mean += b_in[i];
    mean /= (double)n;
    for (size_t i = 0; i < n; ++i) bb[i] = b_in[i] - mean;
    if (mean_removed) *mean_removed = mean;
    memset(x, 0, n * sizeof(double));
    double nb = sqrt(og_dotv(n, bb, bb));
    int it = 0, status = -4;
    double rel = 0.0;
    if (nb == 0.0) {
        *iters = 0; *relres = 0.0;
        free(bb); free(r);
        return 0;
    }
    if (accel == 0) {
        for (it = 1; it <= max_iters; ++it) {
            orc_mg_vcycle(m, bb, x);
            orc_residual(d.nr, d.nt, d.np, m->G[0], bb, x, r);
            rel = sqrt(og_dotv(n, r, r)) / nb;
            if (history) history[it - 1] = rel;
            if (!isfinite(rel)) { status = -5; break; }
            if (rel <= tol) { status = 0; break; }
        }
    } else if (accel == 1) {
        double *z = calloc(n, sizeof(double)), *p = malloc(n * sizeof(double)),
               *q = malloc(n * sizeof(double));
        memcpy(r, bb, n * sizeof(double));
        orc_mg_vcycle(m, r, z);
        memcpy(p, z, n * sizeof(double));
        double rz = og_dotv(n, r, z);
        for (it = 1; it <= max_iters; ++it) {
            orc_apply(d.nr, d.nt, d.np, m->G[0], p, q);
            double al = rz / og_dotv(n, p, q);
            for (size_t i = 0; i < n; ++i) { x[i] += al * p[i]; r[i] -= al * q[i]; }
            rel = sqrt(og_dotv(n, r, r)) / nb;
            if (history) history[it - 1] = rel;
            if (!isfinite(rel)) { status = -5; break; }
            if (rel <= tol) { status = 0; break; }
            memset(z, 0, n * sizeof(double));
            orc_mg_vcycle(m, r, z);
            double rz1 = og_dotv(n, r, z);
            double be = rz1 / rz;
            rz = rz1;
            for (size_t i = 0; i < n; ++i) p[i] = z[i] + be * p[i];
        }
        free(z); free(p); free(q);
    } else {
        double *r0 = malloc(n * sizeof(double)), *p = calloc(n, sizeof(double)),
               *v = calloc(n, sizeof(double)), *ph = calloc(n, sizeof(double)),
               *s = malloc(n * sizeof(double)), *sh = calloc(n, sizeof(double)),
               *t = malloc(n * sizeof(double));
        memcpy(r, bb, n * sizeof(double));
        memcpy(r0, bb, n * sizeof(double));
        double rho = 1.0, al = 1.0, om = 1.0;
        for (it = 1; it <= max_iters; ++it) {
            double rho1 = og_dotv(n, r0, r);
            double be = (rho1 / rho) * (al / om);
            rho = rho1;
            for (size_t i = 0; i < n; ++i) p[i] = r[i] + be * (p[i] - om * v[i]);
            memset(ph, 0, n * sizeof(double));
            orc_mg_vcycle(m, p, ph);
            orc_apply(d.nr, d.nt, d.np, m->G[0], ph, v);
            al = rho / og_dotv(n, r0, v);
            for (size_t i = 0; i < n; ++i) s[i] = r[i] - al * v[i];
            memset(sh, 0, n * sizeof(double));
            orc_mg_vcycle(m, s, sh);
            orc_apply(d.nr, d.nt, d.np, m->G[0], sh, t);
            om = og_dotv(n, t, s) / og_dotv(n, t, t);
            for (size_t i = 0; i < n; ++i) {
                x[i] += al * ph[i] + om * sh[i];
                r[i] = s[i] - om * t[i];
            }
            rel = sqrt(og_dotv(n, r, r)) / nb;
            if (history) history[it - 1] = rel;
            if (!isfinite(rel)) { status = -5; break; }
            if (rel <= tol) { status = 0; break; }
        }
        free(r0); free(p); free(v); free(ph); free(s); free(sh); free(t);
    }
    if (it > max_iters) it = max_iters;
    double mx = 0.0;
    for (size_t i = 0; i < n; ++i) mx += x[i];
    mx /= (double)n;
    for (size_t i = 0; i < n; ++i) x[i] -= mx;
    *iters = it;
    *relres = rel;
    free(bb);
    free(r);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Projection step around the solve: the right-hand side of eq. (PC_6),     */
/* d/ds_j [C_ji u_i], and the velocity correction of eq. (PC_7),            */
/* u_i <- u_i - (1/|J^-1|) d/ds_j [C_ji phi], with phi the solution of      */
/* eq. (PC_6) (phi = h dP).  Flux form on the collocated grid: face values  */
/* are the mean of the two cells sharing the face, as in eq. (PC_term1).    */
/* Velocities are [3][n_r][n_theta][n_phi], Cartesian components.           */
/* ------------------------------------------------------------------------ */

/* Row d of C at the LOW d-face of cell (a,b,c) (eq. (skewness), Sec. 3.2
 * items 4-5): C_dq = |J^-1| ds_d/dx_q, and the rows of |J^-1| J are the
 * cyclic cross products of the chords, n_d = t_{d+1} x t_{d+2}.  Returns
 * |J^-1| at that face (item 2).  a may be n_r, b may be n_theta (the high
 * walls); c wraps. */
double orc_face_crow(const og_grid* g, int nr, int nt, int np, int method, int d, int a, int b,
                     int c, double Crow[3])
{
    double t[9];
    og_face_chords(g, nr, nt, np, method, d, a, b, c, t);
    og_cross(&t[3 * ((d + 1) % 3)], &t[3 * ((d + 2) % 3)], Crow);
    double n0[3];
    og_cross(&t[3], &t[6], n0);
    return og_dot(&t[0], n0);
}

/* |J^-1| at the centre of cell (a,b,c): the mean of the determinants of its
 * six faces (Sec. 3.2 item 3). */
double orc_cell_jdet(const og_grid* g, int nr, int nt, int np, int method, int a, int b, int c)
{
    double C[3], s = 0.0;
    s += orc_face_crow(g, nr, nt, np, method, 0, a, b, c, C);
    s += orc_face_crow(g, nr, nt, np, method, 0, a + 1, b, c, C);
    s += orc_face_crow(g, nr, nt, np, method, 1, a, b, c, C);
    s += orc_face_crow(g, nr, nt, np, method, 1, a, b + 1, c, C);
    s += orc_face_crow(g, nr, nt, np, method, 2, a, b, c, C);
    s += orc_face_crow(g, nr, nt, np, method, 2, a, b, c + 1, C);
    return s / 6.0;
}

/* Contravariant flux U_d = C_dq u_q through the LOW d-face of (a,b,c); u at
 * the face is the mean of the two cells sharing it.  Zero through the r-
 * and theta-walls (no flow through the walls). */
static double og_uflux(const og_grid* g, og_dims n, int method, const double* u, int d, int a,
                       int b, int c)
{
    if (d == 0 && (a == 0 || a == n.nr)) return 0.0;
    if (d == 1 && (b == 0 || b == n.nt)) return 0.0;
    const size_t N = (size_t)n.nr * n.nt * n.np;
    double C[3];
    orc_face_crow(g, n.nr, n.nt, n.np, method, d, a, b, c, C);
    int lo[3] = {a, b, c};
    lo[d] -= 1;
    double U = 0.0;
    for (int q = 0; q < 3; ++q) {
        double uf = 0.5 * (og_x(n, u + q * N, a, b, c) + og_x(n, u + q * N, lo[0], lo[1], lo[2]));
        U += C[q] * uf;
    }
    return U;
}

/* Right-hand side of eq. (PC_6) at `ncell` cells (flat indices `cells`, or
 * every cell when cells is NULL): the sum over directions of the flux
 * through the high face minus the flux through the low face. */
void orc_divergence(const og_grid* g, int nr, int nt, int np, int method, const double* u,
                    long long ncell, const long long* cells, double* out)
{
    og_dims n = {nr, nt, np};
#pragma omp parallel for
    for (long long i = 0; i < ncell; ++i) {
        long long id = cells ? cells[i] : i;
        int c = (int)(id % np), b = (int)((id / np) % nt), a = (int)(id / ((long long)np * nt));
        double s = 0.0;
        s += og_uflux(g, n, method, u, 0, a + 1, b, c) - og_uflux(g, n, method, u, 0, a, b, c);
        s += og_uflux(g, n, method, u, 1, a, b + 1, c) - og_uflux(g, n, method, u, 1, a, b, c);
        s += og_uflux(g, n, method, u, 2, a, b, c + 1) - og_uflux(g, n, method, u, 2, a, b, c);
        out[i] = s;
    }
}

/* eq. (PC_7) at `ncell` cells: out[3 i + q] = u_q - (1/|J^-1|_c) sum_d
 * [C_dq phi]_{low face}^{high face}, phi at a face the mean of the two
 * cells, mirrored (the cell's own value) on the r- and theta-walls, where
 * the metric C is that of the wall face. */
void orc_correct(const og_grid* g, int nr, int nt, int np, int method, const double* phi,
                 const double* u, long long ncell, const long long* cells, double* out)
{
    og_dims n = {nr, nt, np};
    const size_t N = (size_t)nr * nt * np;
#pragma omp parallel for
    for (long long i = 0; i < ncell; ++i) {
        long long id = cells ? cells[i] : i;
        int c = (int)(id % np), b = (int)((id / np) % nt), a = (int)(id / ((long long)np * nt));
        double grad[3] = {0.0, 0.0, 0.0};
        for (int d = 0; d < 3; ++d)
            for (int side = 0; side < 2; ++side) { /* 0: low face, 1: high face */
                int f[3] = {a, b, c};
                f[d] += side;
                int o[3] = {a, b, c}; /* the other cell sharing the face */
                o[d] += side ? 1 : -1;
                double C[3];
                orc_face_crow(g, nr, nt, np, method, d, f[0], f[1], f[2], C);
                double pf = 0.5 * (og_x(n, phi, a, b, c) + og_x(n, phi, o[0], o[1], o[2]));
                for (int q = 0; q < 3; ++q) grad[q] += (side ? 1.0 : -1.0) * C[q] * pf;
            }
        double J = orc_cell_jdet(g, nr, nt, np, method, a, b, c);
        for (int q = 0; q < 3; ++q) out[3 * i + q] = u[q * N + id] - grad[q] / J;
    }
}

/* ------------------------------------------------------------------------ */
/* Implicit line solves of the ADI steps, eq. (solve_2)-(solve_4)           */
/* ------------------------------------------------------------------------ */
/* Along direction d every line of cells solves
 *     |J^-1|_i psi_i - coef [F_{i+1/2} - F_{i-1/2}] = g_i,
 * F = G_dd (psi_hi - psi_lo) on an interior face (the diagonal term of
 * eq. (PC_term1)), |J^-1|_i the cell value of Sec. 3.2 item 3 and G_dd of a
 * face |C_d|^2 / |J^-1|_face from the face's chords.  On an r- or theta-wall
 * face: bc 0, F = 0 (no flux); bc 1, the value v on the wall face:
 * F = 2 G_dd (psi_0 - v) at the low wall, 2 G_dd (v - psi_{n-1}) at the high
 * wall.  phi is periodic.  Lines: d = 0 indexed by (b, c), d = 1 by (a, c),
 * d = 2 by (a, b). */

typedef struct { int type_lo, type_hi; double v_lo, v_hi; } og_line_bc;

/* A face of zero area (the pole faces of a full sphere, theta0 = 0 or
 * theta1 = pi) carries no flux: G_dd = 0 there. */
static double og_face_gdd(const og_grid* g, og_dims n, int method, int d, int a, int b, int c)
{
    double C[3];
    double det = orc_face_crow(g, n.nr, n.nt, n.np, method, d, a, b, c, C);
    return det > 0.0 ? og_dot(C, C) / det : 0.0;
}

/* position of cell i of line `line` along direction d */
static void og_line_cell(og_dims n, int d, long long line, int i, int p[3])
{
    if (d == 0) { p[0] = i; p[1] = (int)(line / n.np); p[2] = (int)(line % n.np); }
    else if (d == 1) { p[0] = (int)(line / n.np); p[1] = i; p[2] = (int)(line % n.np); }
    else { p[0] = (int)(line / n.nt); p[1] = (int)(line % n.nt); p[2] = i; }
}

static int og_line_len(og_dims n, int d) { return d == 0 ? n.nr : (d == 1 ? n.nt : n.np); }

static long long og_line_count(og_dims n, int d)
{
    return d == 0 ? (long long)n.nt * n.np : (d == 1 ? (long long)n.nr * n.np
                                                     : (long long)n.nr * n.nt);
}

/* Coefficients of one line: lo[i] psi_{i-1} + di[i] psi_i + hi[i] psi_{i+1}
 * = g_i + ex[i]; for d = 2, lo[0] couples psi_{n-1} and hi[n-1] psi_0. */
static void og_line_coefs(const og_grid* g, og_dims n, int method, int d, long long line,
                          double coef, const og_line_bc* bc, double* lo, double* di, double* hi,
                          double* ex)
{
    int len = og_line_len(n, d);
    for (int i = 0; i < len; ++i) {
        int p[3];
        og_line_cell(n, d, line, i, p);
        double J = orc_cell_jdet(g, n.nr, n.nt, n.np, method, p[0], p[1], p[2]);
        int q[3] = {p[0], p[1], p[2]};
        q[d] += 1; /* the high face is the low face of the next position */
        double Gl = og_face_gdd(g, n, method, d, p[0], p[1], p[2]);
        double Gh = og_face_gdd(g, n, method, d, q[0], q[1], q[2]);
        lo[i] = -coef * Gl;
        hi[i] = -coef * Gh;
        di[i] = J + coef * (Gl + Gh);
        ex[i] = 0.0;
        if (d < 2 && i == 0) {
            lo[i] = 0.0;
            if (bc->type_lo == 1) { di[i] += coef * Gl; ex[i] += 2.0 * coef * Gl * bc->v_lo; }
            else di[i] -= coef * Gl;
        }
        if (d < 2 && i == len - 1) {
            hi[i] = 0.0;
            if (bc->type_hi == 1) { di[i] += coef * Gh; ex[i] += 2.0 * coef * Gh * bc->v_hi; }
            else di[i] -= coef * Gh;
        }
    }
}

/* out = |J^-1| psi - coef [F]_{low face}^{high face} along direction d, the
 * plain definition with the wall fluxes above (values included). */
void orc_line_apply(const og_grid* g, int nr, int nt, int np, int method, int d, double coef,
                    int bc_lo, double v_lo, int bc_hi, double v_hi, const double* psi,
                    double* out)
{
    og_dims n = {nr, nt, np};
    int len = og_line_len(n, d);
#pragma omp parallel for
    for (long long line = 0; line < og_line_count(n, d); ++line) {
        for (int i = 0; i < len; ++i) {
            int p[3], lo_[3], hi_[3];
            og_line_cell(n, d, line, i, p);
            for (int k = 0; k < 3; ++k) { lo_[k] = p[k]; hi_[k] = p[k]; }
            lo_[d] -= 1;
            hi_[d] += 1;
            double x = psi[og_idx(n, p[0], p[1], p[2])];
            double Fl, Fh;
            double Gl = og_face_gdd(g, n, method, d, p[0], p[1], p[2]);
            double Gh = og_face_gdd(g, n, method, d, hi_[0], hi_[1], hi_[2]);
            if (d < 2 && i == 0) Fl = bc_lo == 1 ? 2.0 * Gl * (x - v_lo) : 0.0;
            else Fl = Gl * (x - og_x(n, psi, lo_[0], lo_[1], lo_[2]));
            if (d < 2 && i == len - 1) Fh = bc_hi == 1 ? 2.0 * Gh * (v_hi - x) : 0.0;
            else Fh = Gh * (og_x(n, psi, hi_[0], hi_[1], hi_[2]) - x);
            double J = orc_cell_jdet(g, nr, nt, np, method, p[0], p[1], p[2]);
            out[og_idx(n, p[0], p[1], p[2])] = J * x - coef * (Fh - Fl);
        }
    }
}

/* Thomas algorithm, eq. (FIBRE_TA1)-(FIBRE_TA2): forward elimination of the
 * sub-diagonal (b'_i = b_i - a_i c_{i-1} / b'_{i-1}, g'_i likewise), then
 * back substitution psi_i = (g'_i - c_i psi_{i+1}) / b'_i.  Uses bp, gp. */
static void og_thomas(int n, const double* a, const double* b, const double* c, const double* r,
                      double* x, double* bp, double* gp)
{
    bp[0] = b[0];
    gp[0] = r[0];
    for (int i = 1; i < n; ++i) {
        double m = a[i] / bp[i - 1];
        bp[i] = b[i] - m * c[i - 1];
        gp[i] = r[i] - m * gp[i - 1];
    }
    x[n - 1] = gp[n - 1] / bp[n - 1];
    for (int i = n - 2; i >= 0; --i) x[i] = (gp[i] - c[i] * x[i + 1]) / bp[i];
}

/* Solve every line along d (see above) for psi; rhs and psi are
 * [n_r][n_theta][n_phi].  Periodic lines (d = 2, length n >= 3): the paper's
 * split of eq. (FIBRE_TAP1)-(FIBRE_TAP8): the first n-1 unknowns solve the
 * open system twice, for g and for the corner column (-a_0 at the first row,
 * -c_{n-2} at the last), the last unknown follows from the closing row, and
 * psi = psi1 + psi2 psi_{n-1}.  `lines` (nullable): solve only the listed
 * line indices (d = 0: b n_phi + c; d = 1: a n_phi + c; d = 2: a n_theta + b),
 * `nline` of them; psi is written on those lines only.  Returns -1 for a
 * periodic line shorter than 3. */
int orc_line_solve(const og_grid* g, int nr, int nt, int np, int method, int d, double coef,
                   int bc_lo, double v_lo, int bc_hi, double v_hi, const double* rhs,
                   double* psi, long long nline, const long long* lines)
{
    og_dims n = {nr, nt, np};
    og_line_bc bc = {bc_lo, bc_hi, v_lo, v_hi};
    int len = og_line_len(n, d);
    if (d == 2 && len < 3) return -1;
#pragma omp parallel
    {
        double* w = (double*)malloc(sizeof(double) * 10 * (size_t)len);
        double *lo = w, *di = w + len, *hi = w + 2 * len, *ex = w + 3 * len, *r = w + 4 * len,
               *x = w + 5 * len, *bp = w + 6 * len, *gp = w + 7 * len, *x2 = w + 8 * len,
               *r2 = w + 9 * len;
        const long long count = lines ? nline : og_line_count(n, d);
#pragma omp for
        for (long long li = 0; li < count; ++li) {
            const long long line = lines ? lines[li] : li;
            og_line_coefs(g, n, method, d, line, coef, &bc, lo, di, hi, ex);
            for (int i = 0; i < len; ++i) {
                int p[3];
                og_line_cell(n, d, line, i, p);
                r[i] = rhs[og_idx(n, p[0], p[1], p[2])] + ex[i];
            }
            if (d < 2) {
                og_thomas(len, lo, di, hi, r, x, bp, gp);
            } else {
                int m = len - 1; /* open system of the first m unknowns */
                og_thomas(m, lo, di, hi, r, x, bp, gp);
                for (int i = 0; i < m; ++i) r2[i] = 0.0;
                r2[0] = -lo[0];
                r2[m - 1] -= hi[m - 1];
                og_thomas(m, lo, di, hi, r2, x2, bp, gp);
                double xl = (r[m] - hi[m] * x[0] - lo[m] * x[m - 1]) /
                            (di[m] + hi[m] * x2[0] + lo[m] * x2[m - 1]);
                for (int i = 0; i < m; ++i) x[i] += x2[i] * xl;
                x[m] = xl;
            }
            for (int i = 0; i < len; ++i) {
                int p[3];
                og_line_cell(n, d, line, i, p);
                psi[og_idx(n, p[0], p[1], p[2])] = x[i];
            }
        }
        free(w);
    }
    return 0;
}
