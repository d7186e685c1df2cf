// project.hpp -- the two steps either side of the pressure-correction solve,
// on the finest grid of a handle.  Included by cps.hip after kernels.hpp.
//
// Right-hand side of eq. (PC_6): the divergence d/ds_j [C_ji u_i] of the
// contravariant flux, with C_ji = |J^-1| ds_j/dx_i (eq. (skewness)) at the
// cell faces (Sec. 3.2 items 4-5).  Velocity correction of eq. (PC_7):
// u_i <- u_i - (1/|J^-1|) d/ds_j [C_ji phi], phi = h dP the solution of
// eq. (PC_6), |J^-1| at a cell the mean of its six face determinants
// (item 3).  Both in flux form on the collocated grid, like the terms of
// eq. (PC_term1): a face value is the mean of the two cells sharing the
// face; no flow through the r- and theta-walls; phi is mirrored there (the
// wall face takes the cell's own value), with the wall face's C.
//
// Velocities are [3][n_r][n_theta][n_phi] (Cartesian components, polar axis
// x1), phi and the right-hand side [n_r][n_theta][n_phi], natural order, one
// thread per cell, phi fastest across a wavefront.
//
// C rows of the LOW d-face of every position (a, b, c), a <= n_r, b <=
// n_theta (the high walls included): Cf[(3d + q) F + (a (n_theta + 1) + b)
// nc + c], F = (n_r + 1)(n_theta + 1) nc, in one of three forms (CSym):
//  - kRotational (sphere, oblate shell: symmetric under rotation about the
//    polar axis): the faces of cell c are those of cell 0 turned by
//    2 pi c / n_phi about x1, so nc = 1 and the kernels rotate the (x2, x3)
//    components;
//  - kInvariant (identity box: phi is a translation): nc = 1, no rotation;
//  - kPerCell (triaxial): nc = n_phi.

namespace cps {

// chord rows of every face position: C row d and |J^-1| of the LOW d-face
// (C_d = t_{d+1} x t_{d+2}, |J^-1| = t_0 . (t_1 x t_2))
__global__ void __launch_bounds__(kBlock) k_crows(MapParams m, int nr, int nt, int np, int nc,
                                                  int method, double* __restrict__ Cf,
                                                  double* __restrict__ Jf)
{
    const long long F = (long long)(nr + 1) * (nt + 1) * nc;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= F) return;
    const int c = (int)(i % nc);
    const long long row = i / nc;
    const int b = (int)(row % (nt + 1)), a = (int)(row / (nt + 1));
    auto cross = [](const double* u, const double* v, double* w) {
        w[0] = u[1] * v[2] - u[2] * v[1];
        w[1] = u[2] * v[0] - u[0] * v[2];
        w[2] = u[0] * v[1] - u[1] * v[0];
    };
    for (int d = 0; d < 3; ++d) {
        double t[3][3], C[3], n0[3];
        face_chords(m, nr, nt, np, method, d, a, b, c, t);
        cross(t[(d + 1) % 3], t[(d + 2) % 3], C);
        cross(t[1], t[2], n0);
        for (int q = 0; q < 3; ++q) Cf[(3 * d + q) * F + i] = C[q];
        Jf[d * F + i] = t[0][0] * n0[0] + t[0][1] * n0[1] + t[0][2] * n0[2];
    }
}

// |J^-1| of every cell (c < nc): the mean of its six face determinants
__global__ void __launch_bounds__(kBlock) k_cell_jdet(int nr, int nt, int nc,
                                                      const double* __restrict__ Jf,
                                                      double* __restrict__ Jc)
{
    const long long n = (long long)nr * nt * nc, F = (long long)(nr + 1) * (nt + 1) * nc;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = (int)(i % nc);
    const long long row = i / nc;
    const int b = (int)(row % nt), a = (int)(row / nt);
    auto fi = [&](int fa, int fb, int fc) { return ((long long)fa * (nt + 1) + fb) * nc + fc; };
    double s = 0.0;
    s += Jf[fi(a, b, c)];
    s += Jf[fi(a + 1, b, c)];
    s += Jf[F + fi(a, b, c)];
    s += Jf[F + fi(a, b + 1, c)];
    s += Jf[2 * F + fi(a, b, c)];
    s += Jf[2 * F + fi(a, b, (c + 1) % nc)];
    Jc[i] = s / 6.0;
}

enum CSym { kPerCell = 0, kInvariant = 1, kRotational = 2 };

struct CRows {
    const double* C;
    long long F;
    int nt1, nc;
    const double* rot; // kRotational: cos, sin of 2 pi c / n_phi for c = 0 .. n_phi
};

// Launch shape of the per-cell kernels: a block is 4 theta rows x 64
// consecutive phi cells marching over a chunk of kProjChunk r-planes (each
// thread keeps its own column's r-neighbours in registers); the linear block
// index is remapped so that each of the 8 XCDs (which receive blocks
// round-robin) takes one contiguous range of (chunk, row group, phi
// segment), sharing the theta-neighbour rows in its own L2.
constexpr int kProjRows = 4;
constexpr int kProjChunk = 8;

struct ProjCol {
    int a0, a1, b, c;
    bool live;
};

__host__ __device__ inline long long proj_blocks(int nr, int nt, int np)
{
    return (long long)((nr + kProjChunk - 1) / kProjChunk) * ((nt + kProjRows - 1) / kProjRows) *
           ((np + 63) / 64);
}

__host__ __device__ inline long long proj_grid(int nr, int nt, int np)
{
    return (proj_blocks(nr, nt, np) + 7) / 8 * 8;
}

__device__ inline ProjCol proj_col(int nr, int nt, int np)
{
    ProjCol p{0, 0, 0, 0, false};
    const long long nb = proj_blocks(nr, nt, np), per = (nb + 7) / 8;
    const long long lb = (long long)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (lb >= nb) return p;
    const int segs = (np + 63) / 64, groups = (nt + kProjRows - 1) / kProjRows;
    const int cs = (int)(lb % segs);
    const long long t = lb / segs;
    const int ch = (int)(t / groups);
    p.a0 = ch * kProjChunk;
    p.a1 = p.a0 + kProjChunk < nr ? p.a0 + kProjChunk : nr;
    // the theta row is one per wavefront: made uniform so that the face
    // tables (one row per (r, theta)) are read with scalar loads
    p.b = __builtin_amdgcn_readfirstlane((int)(t % groups) * kProjRows + (int)(threadIdx.x >> 6));
    p.c = cs * 64 + (int)(threadIdx.x & 63);
    p.live = p.b < nt && p.c < np;
    return p;
}

// C row d of the LOW d-face of position (a, b, c); kRotational: the entry
// of (a, b, 0) turned about x1 by the angle with cosine cs and sine sn
template <int SYM>
__device__ __forceinline__ void crow(const CRows& R, int d, int a, int b, int c, double cs,
                                     double sn, double out[3])
{
    const long long fi = ((long long)a * R.nt1 + b) * R.nc + (SYM == kPerCell ? c : 0);
    const double c0 = R.C[(3 * d) * R.F + fi], c1 = R.C[(3 * d + 1) * R.F + fi],
                 c2 = R.C[(3 * d + 2) * R.F + fi];
    out[0] = c0;
    if (SYM == kRotational) {
        out[1] = c1 * cs - c2 * sn;
        out[2] = c1 * sn + c2 * cs;
    } else {
        out[1] = c1;
        out[2] = c2;
    }
}

// rhs = d/ds_j [C_ji u_i]: per direction, flux through the high face minus
// flux through the low face; a flux is C_d . (mean of the two cells' u).
// A thread marches its (b, c) column over a chunk of planes with u at a - 1,
// a and a + 1 in registers (the load of a + 2 issued before a is computed).
template <int SYM>
__global__ void __launch_bounds__(kBlock) k_divergence(int nr, int nt, int np, CRows R,
                                                       const double* __restrict__ u,
                                                       double* __restrict__ rhs)
{
    const ProjCol col = proj_col(nr, nt, np);
    if (!col.live) return;
    const int b = col.b, c = col.c;
    const long long N = (long long)nr * nt * np, plane = (long long)nt * np;
    const int cm = c == 0 ? np - 1 : c - 1, cp = c == np - 1 ? 0 : c + 1;
    double s0 = 0.0, c0 = 1.0, s1 = 0.0, c1 = 1.0;
    if (SYM == kRotational) {
        c0 = R.rot[2 * c];
        s0 = R.rot[2 * c + 1];
        c1 = R.rot[2 * c + 2];
        s1 = R.rot[2 * c + 3];
    }
    const double* u0 = u;
    const double* u1 = u + N;
    const double* u2 = u + 2 * N;
    const long long col0 = (long long)b * np + c;
    const int lane = (int)(threadIdx.x & 63);
    const bool whole = np <= 64; // the ring is the wavefront's lanes 0 .. np-1
    const int lane_lo = whole ? cm : lane - 1, lane_hi = whole ? cp : lane + 1;
    const bool shfl_lo = whole || lane > 0, shfl_hi = whole || (lane < 63 && c + 1 < np);
    auto load = [&](int a, double v[3]) {
        const long long i = a * plane + col0;
        v[0] = u0[i];
        v[1] = u1[i];
        v[2] = u2[i];
    };
    auto flux = [&](int d, int fa, int fb, int fc, const double hi[3], const double lo[3],
                    double cs, double sn) {
        double C[3];
        crow<SYM>(R, d, fa, fb, fc, cs, sn, C);
        double U = 0.0;
        U += C[0] * (0.5 * (hi[0] + lo[0]));
        U += C[1] * (0.5 * (hi[1] + lo[1]));
        U += C[2] * (0.5 * (hi[2] + lo[2]));
        return U;
    };
    double um[3] = {0.0, 0.0, 0.0}, uc[3], up[3] = {0.0, 0.0, 0.0};
    if (col.a0 > 0) load(col.a0 - 1, um);
    load(col.a0, uc);
    if (col.a0 + 1 < nr) load(col.a0 + 1, up);
    for (int a = col.a0; a < col.a1; ++a) {
        double un[3] = {0.0, 0.0, 0.0};
        if (a + 2 < nr && a + 1 < col.a1) load(a + 2, un);
        const long long i = a * plane + col0;
        double nb[3], v[3];
        const double r_lo = a > 0 ? flux(0, a, b, c, uc, um, c0, s0) : 0.0;
        const double r_hi = a < nr - 1 ? flux(0, a + 1, b, c, up, uc, c0, s0) : 0.0;
        double t_lo = 0.0, t_hi = 0.0;
        if (b > 0) {
            v[0] = u0[i - np]; v[1] = u1[i - np]; v[2] = u2[i - np];
            t_lo = flux(1, a, b, c, uc, v, c0, s0);
        }
        if (b < nt - 1) {
            v[0] = u0[i + np]; v[1] = u1[i + np]; v[2] = u2[i + np];
            t_hi = flux(1, a, b + 1, c, v, uc, c0, s0);
        }
        // phi-neighbours: the adjacent lanes' own values where they hold
        // them (the ring fits the wavefront, or the neighbour is in this
        // 64-cell segment), else loaded
        for (int q = 0; q < 3; ++q) nb[q] = __shfl(uc[q], lane_lo);
        if (!shfl_lo) {
            nb[0] = u0[i - c + cm]; nb[1] = u1[i - c + cm]; nb[2] = u2[i - c + cm];
        }
        const double p_lo = flux(2, a, b, c, uc, nb, c0, s0);
        for (int q = 0; q < 3; ++q) nb[q] = __shfl(uc[q], lane_hi);
        if (!shfl_hi) {
            nb[0] = u0[i - c + cp]; nb[1] = u1[i - c + cp]; nb[2] = u2[i - c + cp];
        }
        const double p_hi = flux(2, a, b, cp, nb, uc, c1, s1);
        double s = 0.0;
        s += r_hi - r_lo;
        s += t_hi - t_lo;
        s += p_hi - p_lo;
        rhs[i] = s;
        for (int q = 0; q < 3; ++q) {
            um[q] = uc[q];
            uc[q] = up[q];
            up[q] = un[q];
        }
    }
}

// The divergence over theta-row pairs (n_theta even): wavefront w of a
// block owns rows b0 = 2 (4 G + w) and b0 + 1 over one 64-cell phi segment
// and marches both columns over a chunk of kProjChunk2 planes.  The theta
// face between its rows is formed once from the two columns in registers,
// so only the rows just outside the pair are loaded: 4 row loads per 2
// cells and plane, against 3 per cell.  Block order as proj_col (each XCD a
// contiguous range).  Every flux is the same expression, on the same values,
// as in k_divergence, and each cell sums its faces in the same order.
constexpr int kProjChunk2 = 8;

struct ProjPair {
    int a0, a1, b0, c;
    bool live;
};

__host__ __device__ inline long long proj2_blocks(int nr, int nt, int np)
{
    return (long long)((nr + kProjChunk2 - 1) / kProjChunk2) *
           ((nt / 2 + kProjRows - 1) / kProjRows) * ((np + 63) / 64);
}

__host__ __device__ inline long long proj2_grid(int nr, int nt, int np)
{
    return (proj2_blocks(nr, nt, np) + 7) / 8 * 8;
}

__device__ inline ProjPair proj_pair(int nr, int nt, int np)
{
    ProjPair p{0, 0, 0, 0, false};
    const long long nb = proj2_blocks(nr, nt, np), per = (nb + 7) / 8;
    const long long lb = (long long)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (lb >= nb) return p;
    const int segs = (np + 63) / 64, groups = (nt / 2 + kProjRows - 1) / kProjRows;
    const int cs = (int)(lb % segs);
    const long long t = lb / segs;
    const int ch = (int)(t / groups);
    p.a0 = ch * kProjChunk2;
    p.a1 = p.a0 + kProjChunk2 < nr ? p.a0 + kProjChunk2 : nr;
    p.b0 = 2 * __builtin_amdgcn_readfirstlane((int)(t % groups) * kProjRows +
                                              (int)(threadIdx.x >> 6));
    p.c = cs * 64 + (int)(threadIdx.x & 63);
    p.live = p.b0 < nt && p.c < np;
    return p;
}

template <int SYM>
__global__ void __launch_bounds__(kBlock) k_divergence2(int nr, int nt, int np, CRows R,
                                                        const double* __restrict__ u,
                                                        double* __restrict__ rhs)
{
    const ProjPair col = proj_pair(nr, nt, np);
    if (!col.live) return;
    const int b0 = col.b0, b1 = b0 + 1, c = col.c;
    const long long N = (long long)nr * nt * np, plane = (long long)nt * np;
    const int cm = c == 0 ? np - 1 : c - 1, cp = c == np - 1 ? 0 : c + 1;
    double s0 = 0.0, c0 = 1.0, s1 = 0.0, c1 = 1.0;
    if (SYM == kRotational) {
        c0 = R.rot[2 * c];
        s0 = R.rot[2 * c + 1];
        c1 = R.rot[2 * c + 2];
        s1 = R.rot[2 * c + 3];
    }
    const double* u0 = u;
    const double* u1 = u + N;
    const double* u2 = u + 2 * N;
    const long long col0 = (long long)b0 * np + c;
    const int lane = (int)(threadIdx.x & 63);
    const bool whole = np <= 64;
    const int lane_lo = whole ? cm : lane - 1, lane_hi = whole ? cp : lane + 1;
    const bool shfl_lo = whole || lane > 0, shfl_hi = whole || (lane < 63 && c + 1 < np);
    // both rows' columns at plane a: v[0..2] row b0, v[3..5] row b1
    auto load = [&](int a, double v[6]) {
        const long long i = a * plane + col0;
        v[0] = u0[i];
        v[1] = u1[i];
        v[2] = u2[i];
        v[3] = u0[i + np];
        v[4] = u1[i + np];
        v[5] = u2[i + np];
    };
    auto flux = [&](int d, int fa, int fb, int fc, const double hi[3], const double lo[3],
                    double cs, double sn) {
        double C[3];
        crow<SYM>(R, d, fa, fb, fc, cs, sn, C);
        double U = 0.0;
        U += C[0] * (0.5 * (hi[0] + lo[0]));
        U += C[1] * (0.5 * (hi[1] + lo[1]));
        U += C[2] * (0.5 * (hi[2] + lo[2]));
        return U;
    };
    // the phi faces and the sum of one cell, given its theta fluxes
    auto cell = [&](int a, int b, long long i, const double uc[3], double r_lo, double r_hi,
                    double t_lo, double t_hi) {
        double nb[3];
        for (int q = 0; q < 3; ++q) nb[q] = __shfl(uc[q], lane_lo);
        if (!shfl_lo) {
            nb[0] = u0[i - c + cm]; nb[1] = u1[i - c + cm]; nb[2] = u2[i - c + cm];
        }
        const double p_lo = flux(2, a, b, c, uc, nb, c0, s0);
        for (int q = 0; q < 3; ++q) nb[q] = __shfl(uc[q], lane_hi);
        if (!shfl_hi) {
            nb[0] = u0[i - c + cp]; nb[1] = u1[i - c + cp]; nb[2] = u2[i - c + cp];
        }
        const double p_hi = flux(2, a, b, cp, nb, uc, c1, s1);
        double s = 0.0;
        s += r_hi - r_lo;
        s += t_hi - t_lo;
        s += p_hi - p_lo;
        rhs[i] = s;
    };
    double um[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, uc[6], up[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (col.a0 > 0) load(col.a0 - 1, um);
    load(col.a0, uc);
    if (col.a0 + 1 < nr) load(col.a0 + 1, up);
    for (int a = col.a0; a < col.a1; ++a) {
        double un[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (a + 2 < nr && a + 1 < col.a1) load(a + 2, un);
        const long long i = a * plane + col0;
        double v[3];
        // rows outside the pair (loading them a plane ahead costs registers:
        // 137 VGPRs, 3 waves per SIMD, 283 against 272 us)
        double t_lo0 = 0.0, t_hi1 = 0.0;
        if (b0 > 0) {
            v[0] = u0[i - np]; v[1] = u1[i - np]; v[2] = u2[i - np];
            t_lo0 = flux(1, a, b0, c, uc, v, c0, s0);
        }
        if (b1 < nt - 1) {
            v[0] = u0[i + 2 * np]; v[1] = u1[i + 2 * np]; v[2] = u2[i + 2 * np];
            t_hi1 = flux(1, a, b1 + 1, c, v, uc + 3, c0, s0);
        }
        // the face between the rows, once for both
        const double t_mid = flux(1, a, b1, c, uc + 3, uc, c0, s0);
        const double r_lo0 = a > 0 ? flux(0, a, b0, c, uc, um, c0, s0) : 0.0;
        const double r_hi0 = a < nr - 1 ? flux(0, a + 1, b0, c, up, uc, c0, s0) : 0.0;
        const double r_lo1 = a > 0 ? flux(0, a, b1, c, uc + 3, um + 3, c0, s0) : 0.0;
        const double r_hi1 = a < nr - 1 ? flux(0, a + 1, b1, c, up + 3, uc + 3, c0, s0) : 0.0;
        cell(a, b0, i, uc, r_lo0, r_hi0, t_lo0, t_mid);
        cell(a, b1, i + np, uc + 3, r_lo1, r_hi1, t_mid, t_hi1);
        for (int q = 0; q < 6; ++q) {
            um[q] = uc[q];
            uc[q] = up[q];
            up[q] = un[q];
        }
    }
}

// u_q <- u_q - (1/|J^-1|) sum over the six faces of +-C_dq (face mean of
// phi); phi is mirrored on the r- and theta-walls.  Marches like
// k_divergence with phi at a - 1, a and a + 1 in registers.
template <int SYM>
__global__ void __launch_bounds__(kBlock) k_correct(int nr, int nt, int np, CRows R,
                                                    const double* __restrict__ Jc,
                                                    const double* __restrict__ phi,
                                                    double* __restrict__ u)
{
    const ProjCol col = proj_col(nr, nt, np);
    if (!col.live) return;
    const int b = col.b, c = col.c;
    const long long N = (long long)nr * nt * np, plane = (long long)nt * np;
    const int cm = c == 0 ? np - 1 : c - 1, cp = c == np - 1 ? 0 : c + 1;
    double s0 = 0.0, c0 = 1.0, s1 = 0.0, c1 = 1.0;
    if (SYM == kRotational) {
        c0 = R.rot[2 * c];
        s0 = R.rot[2 * c + 1];
        c1 = R.rot[2 * c + 2];
        s1 = R.rot[2 * c + 3];
    }
    const long long col0 = (long long)b * np + c;
    double pm = 0.0, pc = phi[col.a0 * plane + col0], pp = 0.0;
    if (col.a0 > 0) pm = phi[(col.a0 - 1) * plane + col0];
    if (col.a0 + 1 < nr) pp = phi[(col.a0 + 1) * plane + col0];
    for (int a = col.a0; a < col.a1; ++a) {
        double pn = 0.0;
        if (a + 2 < nr && a + 1 < col.a1) pn = phi[(a + 2) * plane + col0];
        const long long i = a * plane + col0;
        double g[3] = {0.0, 0.0, 0.0};
        auto face = [&](int d, int fa, int fb, int fc, double po, double sign, double cs,
                        double sn) {
            double C[3];
            crow<SYM>(R, d, fa, fb, fc, cs, sn, C);
            const double pf = 0.5 * (pc + po);
            for (int q = 0; q < 3; ++q) g[q] += sign * C[q] * pf;
        };
        face(0, a, b, c, a > 0 ? pm : pc, -1.0, c0, s0);
        face(0, a + 1, b, c, a < nr - 1 ? pp : pc, 1.0, c0, s0);
        face(1, a, b, c, b > 0 ? phi[i - np] : pc, -1.0, c0, s0);
        face(1, a, b + 1, c, b < nt - 1 ? phi[i + np] : pc, 1.0, c0, s0);
        face(2, a, b, c, phi[i - c + cm], -1.0, c0, s0);
        face(2, a, b, cp, phi[i - c + cp], 1.0, c1, s1);
        const double iJ = 1.0 / Jc[SYM == kPerCell ? i : (long long)a * nt + b];
        for (int q = 0; q < 3; ++q) u[q * N + i] = u[q * N + i] - g[q] * iJ;
        pm = pc;
        pc = pp;
        pp = pn;
    }
}

} // namespace cps
