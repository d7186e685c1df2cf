// lines.hpp -- implicit line solves of the ADI steps, eq. (solve_2)-(solve_4),
// on the finest grid of a handle whose metrics are phi-invariant.  Included
// by cps.hip after project.hpp (it reads the projection step's face tables).
//
// Along direction d every line of cells solves
//     |J^-1|_i psi_i - coef [F_{i+1/2} - F_{i-1/2}] = g_i,
// F = G_dd (psi_hi - psi_lo) on an interior face (the diagonal term of eq.
// (PC_term1)), G_dd of a face = |C_d|^2 / |J^-1|_face from the face's chords,
// |J^-1|_i the cell value (mean of its six face determinants).  r- and
// theta-wall faces: no flux, or the value v on the wall face (F = 2 G_dd
// (psi_0 - v) at the low wall, 2 G_dd (v - psi_{n-1}) at the high wall);
// phi is periodic.  Fields are [n_r][n_theta][n_phi], natural order.
//
//  - r- and theta-lines: the Thomas algorithm (eq. (FIBRE_TA1)-(FIBRE_TA2)).
//    On a phi-invariant map a line's coefficients depend on one index (b for
//    r-lines, a for theta-lines), so k_line_factor runs the elimination of
//    the coefficients once per distinct line; k_line_open then streams the
//    right-hand side down and up every line, one thread per line, lines
//    consecutive in phi across a wavefront, a batch of steps of loads in
//    flight.  psi holds the eliminated right-hand side between the sweeps.
//  - phi-lines: the paper's periodic form (eq. (FIBRE_TAP1)-(FIBRE_TAP8)):
//    the first n - 1 unknowns solve the open system for g and for the corner
//    column, the last follows from the closing row, and psi = psi1 +
//    psi2 psi_{n-1}; one thread per (a, b) line walking its ring.

namespace cps {

struct LineBC {
    int type_lo, type_hi;
    double v_lo, v_hi;
};

constexpr int kLineBatch = 16;

// G_dd of the LOW d-face of position (a, b) of phi-invariant face tables; a
// face of zero area (a pole of a full sphere) carries no flux: 0
__device__ __forceinline__ double face_gdd(const CRows& R, const double* __restrict__ Jf, int d,
                                           int a, int b)
{
    const long long fi = (long long)a * R.nt1 + b;
    const double c0 = R.C[(3 * d) * R.F + fi], c1 = R.C[(3 * d + 1) * R.F + fi],
                 c2 = R.C[(3 * d + 2) * R.F + fi];
    const double J = Jf[d * R.F + fi];
    return J > 0.0 ? (c0 * c0 + c1 * c1 + c2 * c2) / J : 0.0;
}

// Elimination of the distinct open lines along d (0 r: one per b; 1 theta:
// one per a), n cells each: Fm[p n + i] = a_i / b'_{i-1} (0 at i = 0),
// Fi[p n + i] = 1 / b'_i, Fh[p n + i] = c_i; Fx[2p], Fx[2p + 1]: the wall
// terms added to the first and last right-hand side entries.
__global__ void __launch_bounds__(kBlock) k_line_factor(int nr, int nt, int d, double coef,
                                                        LineBC bc, CRows R,
                                                        const double* __restrict__ Jf,
                                                        const double* __restrict__ Jc,
                                                        double* __restrict__ Fm,
                                                        double* __restrict__ Fi,
                                                        double* __restrict__ Fh,
                                                        double* __restrict__ Fx)
{
    const int lines = d == 0 ? nt : nr, n = d == 0 ? nr : nt;
    const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (p >= lines) return;
    double bp = 0.0, hprev = 0.0, ex0 = 0.0, exl = 0.0;
    for (int i = 0; i < n; ++i) {
        const int a = d == 0 ? i : p, b = d == 0 ? p : i;
        const double J = Jc[(long long)a * nt + b];
        const double Gl = face_gdd(R, Jf, d, a, b);
        const double Gh = face_gdd(R, Jf, d, d == 0 ? a + 1 : a, d == 0 ? b : b + 1);
        double lo = -coef * Gl, hi = -coef * Gh, di = J + coef * (Gl + Gh);
        if (i == 0) {
            lo = 0.0;
            if (bc.type_lo == 1) {
                di += coef * Gl;
                ex0 += 2.0 * coef * Gl * bc.v_lo;
            } else {
                di -= coef * Gl;
            }
        }
        if (i == n - 1) {
            hi = 0.0;
            double e = 0.0;
            if (bc.type_hi == 1) {
                di += coef * Gh;
                e = 2.0 * coef * Gh * bc.v_hi;
            } else {
                di -= coef * Gh;
            }
            if (n == 1) ex0 += e;
            else exl = e;
        }
        double m = 0.0;
        if (i == 0) {
            bp = di;
        } else {
            m = lo / bp;
            bp = di - m * hprev;
        }
        Fm[(long long)p * n + i] = m;
        Fi[(long long)p * n + i] = 1.0 / bp;
        Fh[(long long)p * n + i] = hi;
        hprev = hi;
    }
    Fx[2 * p] = ex0;
    Fx[2 * p + 1] = exl;
}

// Tables of the ring transform for rings of n_phi = np cells (nh = np / 2
// complex values): tw[q] = exp(-2 pi i q / nh) for q < nh / 2, twN[k] =
// exp(-2 pi i k / n_phi) and lam[k] = 2 cos(2 pi k / n_phi) - 2 for k <= nh
// (as (re, im) pairs for tw and twN).  Formed on the device, so that a call
// that may not copy from the host can build them too.
__global__ void __launch_bounds__(kBlock) k_ring_tables(int np, double* __restrict__ tw,
                                                        double* __restrict__ twN,
                                                        double* __restrict__ lam)
{
    const int nh = np / 2;
    const int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k < nh / 2) {
        double sn, cs;
        sincos(-2.0 * M_PI * k / nh, &sn, &cs);
        tw[2 * k] = cs;
        tw[2 * k + 1] = sn;
    }
    if (k <= nh) {
        double sn, cs;
        sincos(-2.0 * M_PI * k / np, &sn, &cs);
        twN[2 * k] = cs;
        twN[2 * k + 1] = sn;
        lam[k] = 2.0 * cos(2.0 * M_PI * k / np) - 2.0;
    }
}

// Open lines along d (0 r, 1 theta): one thread per (other index, c).
template <int D>
__global__ void __launch_bounds__(kBlock) k_line_open(int nr, int nt, int np,
                                                      const double* __restrict__ Fm,
                                                      const double* __restrict__ Fi,
                                                      const double* __restrict__ Fh,
                                                      const double* __restrict__ Fx,
                                                      const double* rhs, double* psi)
{
    const int other = D == 0 ? nt : nr, n = D == 0 ? nr : nt;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)other * np) return;
    const int p = (int)(t / np), c = (int)(t - (long long)p * np);
    const long long base = D == 0 ? (long long)p * np + c : (long long)p * nt * np + c;
    const long long stride = D == 0 ? (long long)nt * np : np;
    const double* fm = Fm + (long long)p * n;
    const double* fi = Fi + (long long)p * n;
    const double* fh = Fh + (long long)p * n;
    const double ex0 = Fx[2 * p], exl = Fx[2 * p + 1];
    double gp = 0.0;
    for (int i0 = 0; i0 < n; i0 += kLineBatch) {
        double r[kLineBatch];
#pragma unroll
        for (int k = 0; k < kLineBatch; ++k)
            if (i0 + k < n) r[k] = rhs[base + (i0 + k) * stride];
#pragma unroll
        for (int k = 0; k < kLineBatch; ++k) {
            const int i = i0 + k;
            if (i < n) {
                double v = r[k];
                if (i == 0) v += ex0;
                if (i == n - 1 && n > 1) v += exl;
                gp = i == 0 ? v : v - fm[i] * gp;
                psi[base + i * stride] = gp;
            }
        }
    }
    double x = gp * fi[n - 1];
    psi[base + (long long)(n - 1) * stride] = x;
    for (int i0 = n - 2; i0 >= 0; i0 -= kLineBatch) {
        double g[kLineBatch];
#pragma unroll
        for (int k = 0; k < kLineBatch; ++k)
            if (i0 - k >= 0) g[k] = psi[base + (i0 - k) * stride];
#pragma unroll
        for (int k = 0; k < kLineBatch; ++k) {
            const int i = i0 - k;
            if (i >= 0) {
                x = (g[k] - fh[i] * x) * fi[i];
                psi[base + i * stride] = x;
            }
        }
    }
}

// Periodic phi-lines (n_phi >= 3), one thread per (a, b) line; constant
// coefficients along a line of a phi-invariant map.  S2: the corner-column
// solution, SI: the inverse pivots (scratch of n_r n_theta n_phi words each).
__global__ void __launch_bounds__(kBlock) k_line_periodic(int nr, int nt, int np, double coef,
                                                          CRows R,
                                                          const double* __restrict__ Jf,
                                                          const double* __restrict__ Jc,
                                                          const double* rhs, double* psi,
                                                          double* __restrict__ S2,
                                                          double* __restrict__ SI)
{
    const long long row = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= (long long)nr * nt) return;
    const int a = (int)(row / nt), b = (int)(row - (long long)a * nt);
    const double G = face_gdd(R, Jf, 2, a, b), J = Jc[row];
    const double lo = -coef * G, hi = -coef * G, di = J + coef * (G + G);
    const long long base = row * np;
    const int m = np - 1; // the open system of the first m unknowns
    double bp = 0.0, g1 = 0.0, g2 = 0.0;
    for (int i = 0; i < m; ++i) {
        double r2 = 0.0;
        if (i == 0) r2 = -lo;
        if (i == m - 1) r2 -= hi;
        const double r1 = rhs[base + i];
        if (i == 0) {
            bp = di;
            g1 = r1;
            g2 = r2;
        } else {
            const double mm = lo / bp;
            bp = di - mm * hi;
            g1 = r1 - mm * g1;
            g2 = r2 - mm * g2;
        }
        const double inv = 1.0 / bp;
        psi[base + i] = g1;
        S2[base + i] = g2;
        SI[base + i] = inv;
    }
    double x1 = g1 * SI[base + m - 1], x2 = g2 * SI[base + m - 1];
    const double x1l = x1, x2l = x2; // at i = m - 1
    psi[base + m - 1] = x1;
    S2[base + m - 1] = x2;
    for (int i = m - 2; i >= 0; --i) {
        const double inv = SI[base + i];
        x1 = (psi[base + i] - hi * x1) * inv;
        x2 = (S2[base + i] - hi * x2) * inv;
        psi[base + i] = x1;
        S2[base + i] = x2;
    }
    // closing row: hi couples the first cell (wrap), lo the cell before it
    const double xl = (rhs[base + m] - hi * x1 - lo * x1l) / (di + hi * x2 + lo * x2l);
    for (int i = 0; i < m; ++i) psi[base + i] = psi[base + i] + S2[base + i] * xl;
    psi[base + m] = xl;
}

} // namespace cps

namespace cps {

// Periodic phi-lines with constant coefficients (phi-invariant metrics) are
// circulant: a real Fourier transform along the ring diagonalises them, mode
// m having the symbol |J^-1| - coef G_pp lam_m, lam_m = 2 cos(2 pi m / n_phi)
// - 2.  One wavefront per ring (n_phi / 2 a power of two <= kPlaneLds): the
// ring is read once as n_phi / 2 complex pairs (x_{2j}, x_{2j+1}), transformed
// in LDS (wave_fft), divided mode by mode, transformed back and written once.
struct FftLineLaunch {
    int tpr, rb, threads, rings, blocks;
};

__host__ __device__ inline FftLineLaunch fft_line_launch(int nr, int nt, int np)
{
    FftLineLaunch p;
    const int nh = np / 2;
    p.tpr = nh / 2 < 64 ? nh / 2 : 64;
    // a ring takes nh complex slots of the block's LDS (mode nh aliases slot
    // 0), so a ring of kPlaneLds values still fits a block on its own
    p.rb = kBlock / p.tpr;
    if (p.rb * nh > kPlaneLds) p.rb = kPlaneLds / nh;
    p.threads = p.rb * p.tpr;
    p.rings = nr * nt;
    p.blocks = (p.rings + p.rb - 1) / p.rb;
    return p;
}

template <int NMAX>
__global__ void __launch_bounds__(kBlock) k_line_fft(int nr, int nt, int np, double coef, CRows R,
                                                     const double* __restrict__ Jf,
                                                     const double* __restrict__ Jc,
                                                     const Vec2<double>* __restrict__ tw,
                                                     const Vec2<double>* __restrict__ twN,
                                                     const double* __restrict__ lam,
                                                     const double* rhs, double* psi)
{
    __shared__ Vec2<double> buf[kPlaneLds], twS[kPlaneLds / 2];
    const FftLineLaunch pl = fft_line_launch(nr, nt, np);
    const int nh = np / 2;
    for (int q = (int)threadIdx.x; q < nh / 2; q += pl.threads) twS[q] = tw[q];
    // one ring = nh complex values (the pair of mode m = nh aliases slot 0)
    const int rl = (int)threadIdx.x / pl.tpr, tr = (int)threadIdx.x - rl * pl.tpr;
    const int ring = (int)blockIdx.x * pl.rb + rl;
    const bool live = ring < pl.rings;
    Vec2<double>* A = buf + rl * nh;
    const long long base = (long long)ring * np;
    if (live)
        for (int j0 = tr; j0 < nh; j0 += kLdBatch * pl.tpr) {
            Vec2<double> z[kLdBatch];
#pragma unroll
            for (int u = 0; u < kLdBatch; ++u) {
                const int j = j0 + u * pl.tpr;
                if (j < nh) z[u] = *reinterpret_cast<const Vec2<double>*>(rhs + base + 2 * j);
            }
#pragma unroll
            for (int u = 0; u < kLdBatch; ++u) {
                const int j = j0 + u * pl.tpr;
                if (j < nh) A[j] = z[u];
            }
        }
    __syncthreads(); // twiddles of the block (the ring's values are wave-local)
    if (!live) return;
    const int a = ring / nt, b = ring - a * nt;
    const double G = face_gdd(R, Jf, 2, a, b), J = Jc[ring];
    wave_fft<double, NMAX>(A, nh, tr, pl.tpr, twS, false);
    // Mode pairs (m, nh - m), m <= nh / 2, one lane each: the two slots of
    // the half-length transform give the real modes X_m and X_{nh-m} (X_m =
    // E + twN[m] O, E and O the even and odd parts), each is divided by its
    // symbol, and the inverse recombination writes the same two slots back;
    // no other lane reads them.
    const double dJ = J, cG = coef * G;
    auto real_mode = [&](Vec2<double> zm, Vec2<double> zc, int k) {
        // zm = Z_k, zc = conj(Z_{nh-k})
        Vec2<double> E, O;
        E.x = 0.5 * (zm.x + zc.x);
        E.y = 0.5 * (zm.y + zc.y);
        O.x = 0.5 * (zm.y - zc.y);
        O.y = -0.5 * (zm.x - zc.x);
        const double s = 1.0 / (dJ - cG * lam[k]);
        return (E + cmul(twN[k], O)) * s;
    };
    auto half_seq = [&](Vec2<double> xm, Vec2<double> xc, int k) {
        // xm = Y_k, xc = conj(Y_{nh-k}): the half-length value z_k
        Vec2<double> E, D;
        E.x = 0.5 * (xm.x + xc.x);
        E.y = 0.5 * (xm.y + xc.y);
        D.x = 0.5 * (xm.x - xc.x);
        D.y = 0.5 * (xm.y - xc.y);
        const Vec2<double> O = cmul(conjv(twN[k]), D);
        Vec2<double> z;
        z.x = E.x - O.y;
        z.y = E.y + O.x;
        return z;
    };
    for (int m = tr; m <= nh / 2; m += pl.tpr) {
        const int k = nh - m;
        const Vec2<double> Zm = A[m], Zk = A[k == nh ? 0 : k];
        const Vec2<double> Ym = real_mode(Zm, conjv(Zk), m);
        const Vec2<double> Yk = real_mode(Zk, conjv(Zm), k);
        A[m] = half_seq(Ym, conjv(Yk), m);
        if (k != m && k < nh) A[k] = half_seq(Yk, conjv(Ym), k);
    }
    wave_sync();
    wave_fft<double, NMAX>(A, nh, tr, pl.tpr, twS, true);
    const double sc = 1.0 / nh;
    for (int j = tr; j < nh; j += pl.tpr) {
        Vec2<double> v = A[j];
        v.x *= sc;
        v.y *= sc;
        *reinterpret_cast<Vec2<double>*>(psi + base + 2 * j) = v;
    }
}

} // namespace cps
