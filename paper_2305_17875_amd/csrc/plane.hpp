// plane.hpp -- zebra (r, phi)-plane relaxation for the 7-point operator with
// phi-invariant metrics.  Included by cps.hip after kernels.hpp.
//
// A half-sweep of parity k relaxes every theta row b = k (mod 2): each row's
// (r, phi) plane is solved exactly with the rows of the other parity held
// fixed (their theta fluxes go to the right-hand side), i.e. block
// Gauss-Seidel with the theta rows as blocks.  On a plane the metrics do not
// depend on phi, so the periodic phi coupling is diagonalised by a Fourier
// transform along phi and every azimuthal mode m leaves a tridiagonal system
// in r (the Thomas algorithm):
//
//   grl_a X_{a-1} + (-(grl_a + grh_a + gtl_a + gth_a) + gpp_a lam_m) X_a
//     + grh_a X_{a+1} = R_a,       lam_m = 2 cos(2 pi m / n_phi) - 2,
//
// R = FFT_phi(b - gtl x_{b-1} - gth x_{b+1}).  Three launches per half-sweep:
//  - k_plane_fwd: right-hand side of each (r, row) ring and its real Fourier
//    transform.  A ring of n_phi reals is the complex sequence
//    z_j = x_{2j} + i x_{2j+1}, exactly the two parity planes of the split
//    layout; a Stockham radix-4 transform of length n_phi/2 in LDS and the
//    usual even/odd recombination give the n_phi/2 + 1 modes.  The lanes of
//    a ring lie in one wavefront, so the stages need no block barrier;
//  - k_plane_tri: forward elimination and back substitution down and up the
//    r-line of every (row, mode), real and imaginary parts on two lanes.  The
//    inverse pivots depend on the operator only and are computed once per
//    set-up (k_plane_factor); a pass streams the spectra and the pivots with
//    a batch of r-steps in flight per lane;
//  - k_plane_inv: the inverse transform back into the rows.
// Spectra and pivots are laid out [a][row][mode], so the r-line solves read
// and write consecutive modes across a wavefront.
//
// CROSS: the r-theta cross metrics of an axisymmetric map with cross terms
// (the oblate shell; G_r.phi = G_theta.phi = 0, so phi still decouples).  The
// theta-face cross terms couple a row's own r-neighbours, and where a theta
// wall mirrors row b -/+ 1 onto row b the r-face cross terms do too: the
// r-line stays tridiagonal (not symmetric) with phi-invariant coefficients
// (plane_row).  The cross terms that reach rows b -/+ 1 go to the
// right-hand side.

namespace cps {

template <typename T>
__device__ __forceinline__ Vec2<T> cmul(Vec2<T> a, Vec2<T> b)
{
    Vec2<T> r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}

template <typename T>
__device__ __forceinline__ Vec2<T> conjv(Vec2<T> a)
{
    a.y = -a.y;
    return a;
}

constexpr int kPlaneLds = 1024; // complex values per LDS buffer (rings x length)
constexpr int kTriBlock = 64;
constexpr int kTriBatch = 8;   // r-steps whose loads a lane issues together
constexpr int kLdBatch = 4;    // ring positions whose loads a lane issues together
constexpr int kSmallRing = 256; // ring-size class of the paper-scale shell

// Orders the LDS accesses of the lanes of one wavefront (no block barrier).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// In-place Stockham transform of length n (a power of 2, <= kPlaneLds) of
// one ring held at A, tpr lanes of one wavefront per ring: a radix-2 stage
// when log2 n is odd, then radix-4 stages.  A stage reads all of its inputs
// into registers before any lane writes, so one buffer serves; the lanes of
// a ring are one wavefront, so the stages need no block barrier.  tw[q] =
// exp(-2 pi i q / n) for q < n / 2 (in LDS); inverse: conjugate twiddles and
// rotations, no scaling.  NMAX bounds n (the register staging of a stage
// is sized for it: kernels are built for rings up to 256 and up to
// kPlaneLds).
//
// A radix-4 stage of span Ls merges the four length-Ls transforms at block
// offsets q n / 4 (q = 0..3, the residues q of the index mod 4 Ls / Ls) into
// one of length 4 Ls: y_{j + p Ls} = sum_q (-i)^{pq} W^{qj} X_q[j],
// W = exp(-2 pi i / (4 Ls)); W^{qj} = tw[q j n / (4 Ls)], and for an index
// past n / 2, tw[s] = -tw[s - n / 2].
template <typename T, int NMAX>
__device__ void wave_fft(Vec2<T>* A, int n, int tr, int tpr, const Vec2<T>* tw, bool inverse)
{
    // butterflies per lane of a radix-2 and a radix-4 stage
    constexpr int kB2 = NMAX / 128 > 0 ? NMAX / 128 : 1, kB4 = NMAX / 256 > 0 ? NMAX / 256 : 1;
    int Ls = 1;
    if (__builtin_ctz(n) & 1) {
        Vec2<T> u[kB2], v[kB2];
#pragma unroll
        for (int i = 0; i < kB2; ++i) {
            const int t = tr + i * tpr;
            if (t < n / 2) {
                u[i] = A[t];
                v[i] = A[t + n / 2];
            }
        }
        wave_sync();
#pragma unroll
        for (int i = 0; i < kB2; ++i) {
            const int t = tr + i * tpr;
            if (t < n / 2) {
                A[2 * t] = u[i] + v[i];
                A[2 * t + 1] = u[i] - v[i];
            }
        }
        wave_sync();
        Ls = 2;
    }
    for (; Ls < n; Ls *= 4) {
        const int stride = n / (4 * Ls);
        Vec2<T> c[kB4][4];
#pragma unroll
        for (int i = 0; i < kB4; ++i) {
            const int t = tr + i * tpr;
            if (t < n / 4) {
                const int j = t & (Ls - 1), k = t / Ls;
#pragma unroll
                for (int q = 0; q < 4; ++q) c[i][q] = A[k * Ls + j + q * (n / 4)];
            }
        }
        wave_sync();
#pragma unroll
        for (int i = 0; i < kB4; ++i) {
            const int t = tr + i * tpr;
            if (t < n / 4) {
                const int j = t & (Ls - 1), k = t / Ls;
                const int s1 = j * stride, s3 = 3 * j * stride;
                Vec2<T> w1 = tw[s1], w2 = tw[2 * s1];
                Vec2<T> w3 = s3 < n / 2 ? tw[s3] : -tw[s3 - n / 2];
                if (inverse) {
                    w1.y = -w1.y;
                    w2.y = -w2.y;
                    w3.y = -w3.y;
                }
                const Vec2<T> c0 = c[i][0], c1 = cmul(w1, c[i][1]), c2 = cmul(w2, c[i][2]),
                              c3 = cmul(w3, c[i][3]);
                const Vec2<T> s02 = c0 + c2, d02 = c0 - c2, s13 = c1 + c3, d13 = c1 - c3;
                Vec2<T> rot; // -i d13 (forward), +i d13 (inverse)
                rot.x = inverse ? -d13.y : d13.y;
                rot.y = inverse ? d13.x : -d13.x;
                Vec2<T>* o = A + 4 * k * Ls + j;
                o[0] = s02 + s13;
                o[Ls] = d02 + rot;
                o[2 * Ls] = s02 - s13;
                o[3 * Ls] = d02 - rot;
            }
        }
        wave_sync();
    }
}

struct PlaneLaunch {
    int tpr, rb, threads, rows, rings, blocks;
};

// rows of parity k; lanes per ring (a power of two <= 64, so a ring never
// straddles wavefronts), rings per block (<= 256 lanes, <= kPlaneLds values;
// rb > 0 asks for at most that many: the autotuner's choice)
__host__ __device__ inline PlaneLaunch plane_launch(const Geo& g, int parity, int rb = 0)
{
    PlaneLaunch p;
    p.rows = (g.nt - parity + 1) / 2;
    p.tpr = g.nh / 2 < 64 ? g.nh / 2 : 64;
    p.rb = kBlock / p.tpr;
    if (p.rb * g.nh > kPlaneLds) p.rb = kPlaneLds / g.nh;
    if (rb > 0 && rb < p.rb) p.rb = rb;
    p.threads = p.rb * p.tpr;
    p.rings = g.nr * p.rows;
    p.blocks = (p.rings + p.rb - 1) / p.rb;
    return p;
}

// offset of parity k's pivots in a level's table
__host__ __device__ inline long long plane_pivot_offset(const Geo& g, int parity)
{
    return parity ? (long long)g.nr * ((g.nt + 1) / 2) * (g.nh + 1) : 0;
}

// Right-hand sides of the rings of parity k and their real transforms:
// S[(a rows + bi)(nh + 1) + m], m = 0..nh.
// The r-line of row b at a: sub x_{a-1} + (dia + G_pp lam_m) x_a + sup x_{a+1},
// with walls (zero metrics on wall faces, mirrored reads) included.
template <typename T, bool CROSS>
__device__ __forceinline__ void plane_row(const Geo& g, const T* __restrict__ G, long long gk,
                                          int a, int b, T& sub, T& dia, T& sup)
{
    const long long ci = (long long)a * g.nt + b;
    const T grl = G[ci];
    const T grh = a < g.nr - 1 ? G[ci + g.nt] : T(0);
    const T gtl = G[4 * gk + ci];
    const T gth = b < g.nt - 1 ? G[4 * gk + ci + 1] : T(0);
    sub = grl;
    sup = grh;
    dia = -(grl + grh + gtl + gth);
    if (CROSS) {
        // r-face cross terms whose row b -/+ 1 the theta walls mirror onto b
        const T qrl = T(0.25) * G[gk + ci];
        const T qrh = a < g.nr - 1 ? T(0.25) * G[gk + ci + g.nt] : T(0);
        if (b == g.nt - 1) {
            sup += qrh;
            dia += qrh - qrl;
            sub -= qrl;
        }
        if (b == 0) {
            sup -= qrh;
            dia += qrl - qrh;
            sub += qrl;
        }
        // theta-face cross terms on this row: (qth - qtl)(x_{a+1} - x_{a-1})
        const T qtl = T(0.25) * G[3 * gk + ci];
        const T qth = b < g.nt - 1 ? T(0.25) * G[3 * gk + ci + 1] : T(0);
        const T s = qth - qtl;
        if (a < g.nr - 1) sup += s;
        else dia += s;
        if (a > 0) sub -= s;
        else dia -= s;
    }
}

// Bodies take the logical block index (the batched form maps its blocks to
// problems); buf and twS are the block's LDS.
template <typename T, int NMAX, bool CROSS = false>
__device__ __forceinline__ void d_plane_fwd(unsigned blk, Vec2<T>* buf, Vec2<T>* twS, Geo g,
                                            const T* __restrict__ G, long long gk,
                                            const T* __restrict__ bv, const T* __restrict__ x,
                                            int parity, const Vec2<T>* __restrict__ tw,
                                            const Vec2<T>* __restrict__ twN,
                                            Vec2<T>* __restrict__ S, int rb = 0)
{
    const PlaneLaunch pl = plane_launch(g, parity, rb);
    const int nh = g.nh;
    for (int q = (int)threadIdx.x; q < nh / 2; q += pl.threads) twS[q] = tw[q];
    const int rl = (int)threadIdx.x / pl.tpr, tr = (int)threadIdx.x - rl * pl.tpr;
    const int ring = (int)blk * pl.rb + rl;
    // threads past the block's rings (a batched launch of a fixed block
    // size) only take part in the barrier
    const bool live = rl < pl.rb && ring < pl.rings;
    const int a = live ? ring / pl.rows : 0, bi = live ? ring - a * pl.rows : 0;
    const int b = 2 * bi + parity;
    Vec2<T>* A = buf + rl * nh;
    if (live && CROSS) {
        // b + sum over rows b -/+ 1 at a - 1, a, a + 1 (mirrored in r) of
        // coefficient x value: the theta-face metrics and both faces' cross
        // terms (a mirrored position carries a zero metric or folds onto a)
        const long long ci = (long long)a * g.nt + b;
        const bool lo = b > 0, hi = b < g.nt - 1;
        const T gtl = G[4 * gk + ci], gth = hi ? G[4 * gk + ci + 1] : T(0);
        const T qrl = T(0.25) * G[gk + ci];
        const T qrh = a < g.nr - 1 ? T(0.25) * G[gk + ci + g.nt] : T(0);
        const T qtl = T(0.25) * G[3 * gk + ci], qth = hi ? T(0.25) * G[3 * gk + ci + 1] : T(0);
        const T ch0 = -gth - qrh + qrl, chp = -qrh - qth, chm = qrl + qth;
        const T cl0 = -gtl + qrh - qrl, clp = qrh + qtl, clm = -qrl - qtl;
        const long long base = (long long)a * g.rowlen + (long long)b * nh;
        const long long dp = a < g.nr - 1 ? g.rowlen : 0, dm = a > 0 ? g.rowlen : 0;
        for (int j = tr; j < nh; j += pl.tpr) {
            Vec2<T> z;
            z.x = ld_once(bv + base + j);
            z.y = ld_once(bv + g.P + base + j);
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const bool on = side ? hi : lo;
                if (!on) continue;
                const long long r0 = base + (side ? nh : -nh) + j;
                const T c0 = side ? ch0 : cl0, cp = side ? chp : clp, cm = side ? chm : clm;
                z.x += c0 * x[r0] + cp * x[r0 + dp] + cm * x[r0 - dm];
                z.y += c0 * x[g.P + r0] + cp * x[g.P + r0 + dp] + cm * x[g.P + r0 - dm];
            }
            A[j] = z;
        }
    } else if (live) {
        const long long ci = (long long)a * g.nt + b;
        const T gtl = G[4 * gk + ci];
        const T gth = b < g.nt - 1 ? G[4 * gk + ci + 1] : T(0);
        const long long base = (long long)a * g.rowlen + (long long)b * nh;
        const bool lo = b > 0, hi = b < g.nt - 1;
        for (int j0 = tr; j0 < nh; j0 += kLdBatch * pl.tpr) {
            // the loads of a batch are all issued before any is used
            T e[kLdBatch], o[kLdBatch], el[kLdBatch], ol[kLdBatch], eh[kLdBatch], oh[kLdBatch];
#pragma unroll
            for (int u = 0; u < kLdBatch; ++u) {
                const int j = j0 + u * pl.tpr;
                if (j < nh) {
                    e[u] = ld_once(bv + base + j);
                    o[u] = ld_once(bv + g.P + base + j);
                    el[u] = lo ? x[base - nh + j] : T(0);
                    ol[u] = lo ? x[g.P + base - nh + j] : T(0);
                    eh[u] = hi ? x[base + nh + j] : T(0);
                    oh[u] = hi ? x[g.P + base + nh + j] : T(0);
                }
            }
#pragma unroll
            for (int u = 0; u < kLdBatch; ++u) {
                const int j = j0 + u * pl.tpr;
                if (j < nh) {
                    Vec2<T> z;
                    z.x = e[u];
                    z.y = o[u];
                    if (lo) {
                        z.x -= gtl * el[u];
                        z.y -= gtl * ol[u];
                    }
                    if (hi) {
                        z.x -= gth * eh[u];
                        z.y -= gth * oh[u];
                    }
                    A[j] = z;
                }
            }
        }
    }
    __syncthreads(); // twiddles of the block (the ring's values are wave-local)
    if (!live) return;
    wave_fft<T, NMAX>(A, nh, tr, pl.tpr, twS, false);
    const Vec2<T>* Z = A;
    Vec2<T>* out = S + (long long)ring * (nh + 1);
    for (int m0 = tr; m0 <= nh; m0 += kLdBatch * pl.tpr) {
        Vec2<T> w[kLdBatch];
#pragma unroll
        for (int u = 0; u < kLdBatch; ++u) {
            const int m = m0 + u * pl.tpr;
            if (m <= nh) w[u] = twN[m];
        }
#pragma unroll
        for (int u = 0; u < kLdBatch; ++u) {
            const int m = m0 + u * pl.tpr;
            if (m <= nh) {
                const Vec2<T> zm = Z[m == nh ? 0 : m];
                const Vec2<T> zc = conjv(Z[m == 0 ? 0 : nh - m]);
                // even part E = (zm + zc) / 2, odd part O = (zm - zc) / (2i)
                Vec2<T> E, O;
                E.x = T(0.5) * (zm.x + zc.x);
                E.y = T(0.5) * (zm.y + zc.y);
                O.x = T(0.5) * (zm.y - zc.y);
                O.y = -T(0.5) * (zm.x - zc.x);
                out[m] = E + cmul(w[u], O);
            }
        }
    }
}

template <typename T, int NMAX, bool CROSS>
__global__ void __launch_bounds__(kBlock) k_plane_fwd(Geo g, const T* __restrict__ G, long long gk,
                                                      const T* __restrict__ bv,
                                                      const T* __restrict__ x, int parity,
                                                      const Vec2<T>* __restrict__ tw,
                                                      const Vec2<T>* __restrict__ twN,
                                                      Vec2<T>* __restrict__ S, int rb)
{
    __shared__ Vec2<T> buf[kPlaneLds], twS[kPlaneLds / 2];
    d_plane_fwd<T, NMAX, CROSS>(blockIdx.x, buf, twS, g, G, gk, bv, x, parity, tw, twN, S, rb);
}

// Inverse pivots of the Thomas elimination of every (row, mode) r-line of
// parity k: P[(a rows + bi)(nh + 1) + m] = 1 / (diag - grl c_{a-1}),
// c_a = grh_a P_a.  One thread per (row, mode); set-up only.
template <typename T, bool CROSS>
__global__ void __launch_bounds__(kBlock) k_plane_factor(Geo g, const T* __restrict__ G,
                                                         long long gk, int parity,
                                                         const T* __restrict__ lam,
                                                         T* __restrict__ P)
{
    const int rows = (g.nt - parity + 1) / 2;
    const int nm = g.nh + 1;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)rows * nm) return;
    const int bi = (int)(t / nm), m = (int)(t - (long long)bi * nm);
    const int b = 2 * bi + parity;
    const T lm = lam[m];
    const long long stride = (long long)rows * nm;
    T c = T(0);
    for (int a = 0; a < g.nr; ++a) {
        const long long ci = (long long)a * g.nt + b;
        T sub, dia, sup;
        plane_row<T, CROSS>(g, G, gk, a, b, sub, dia, sup);
        const T diag = dia + G[8 * gk + ci] * lm;
        const T inv = T(1) / (diag - sub * c);
        P[a * stride + t] = inv;
        c = sup * inv;
    }
}

// Thomas algorithm along r for every (row, mode) of parity k, in place in
// the spectra S (read as reals: lane 2u + q takes component q of system u),
// with the inverse pivots P of k_plane_factor; TB r-steps of loads in
// flight per lane.
template <typename T, bool CROSS = false, int TB = kTriBatch>
__device__ __forceinline__ void d_plane_tri(long long u, Geo g, const T* __restrict__ G,
                                            long long gk, int parity, const T* __restrict__ P,
                                            T* __restrict__ S)
{
    const int rows = (g.nt - parity + 1) / 2;
    const int nm = g.nh + 1, nr = g.nr, nt = g.nt;
    const long long sys = (long long)rows * nm; // one r-plane of spectra
    if (u >= 2 * sys) return;
    const long long t = u >> 1;
    const int q = (int)(u & 1);
    const int b = 2 * (int)(t / nm) + parity;
    T d = T(0);
    for (int a0 = 0; a0 < nr; a0 += TB) {
        T r[TB], p[TB], gl[TB];
#pragma unroll
        for (int k = 0; k < TB; ++k) {
            const int a = a0 + k;
            if (a < nr) {
                const long long o = a * sys + t;
                r[k] = S[2 * o + q];
                p[k] = P[o];
                if (CROSS) {
                    T dia, sup;
                    plane_row<T, true>(g, G, gk, a, b, gl[k], dia, sup);
                } else {
                    gl[k] = G[(long long)a * nt + b];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < TB; ++k) {
            const int a = a0 + k;
            if (a < nr) {
                d = (r[k] - gl[k] * d) * p[k];
                S[2 * (a * sys + t) + q] = d;
            }
        }
    }
    T xn = d; // X at a = nr - 1
    for (int a0 = nr - 2; a0 >= 0; a0 -= TB) {
        T s[TB], p[TB], gh[TB];
#pragma unroll
        for (int k = 0; k < TB; ++k) {
            const int a = a0 - k;
            if (a >= 0) {
                const long long o = a * sys + t;
                s[k] = S[2 * o + q];
                p[k] = P[o];
                if (CROSS) {
                    T sub, dia;
                    plane_row<T, true>(g, G, gk, a, b, sub, dia, gh[k]);
                } else {
                    gh[k] = G[(long long)(a + 1) * nt + b];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < TB; ++k) {
            const int a = a0 - k;
            if (a >= 0) {
                const T c = gh[k] * p[k];
                xn = s[k] - c * xn;
                S[2 * (a * sys + t) + q] = xn;
            }
        }
    }
}

template <typename T, bool CROSS, int TB>
__global__ void __launch_bounds__(kTriBlock) k_plane_tri(Geo g, const T* __restrict__ G,
                                                         long long gk, int parity,
                                                         const T* __restrict__ P,
                                                         T* __restrict__ S)
{
    d_plane_tri<T, CROSS, TB>((long long)blockIdx.x * blockDim.x + threadIdx.x, g, G, gk, parity,
                              P, S);
}

// r-steps in flight per lane of the elimination: the candidates the
// autotuner times (the same arithmetic in the same order for each)
__host__ __device__ inline int tri_batch_of(int tb) { return tb == 4 || tb == 16 ? tb : kTriBatch; }


// Inverse transforms of the solved spectra into the rows of parity k.
template <typename T, int NMAX>
__device__ __forceinline__ void d_plane_inv(unsigned blk, Vec2<T>* buf, Vec2<T>* twS, Geo g,
                                            int parity, const Vec2<T>* __restrict__ tw,
                                            const Vec2<T>* __restrict__ twN,
                                            const Vec2<T>* __restrict__ S, T* __restrict__ x,
                                            int rb = 0)
{
    const PlaneLaunch pl = plane_launch(g, parity, rb);
    const int nh = g.nh;
    for (int q = (int)threadIdx.x; q < nh / 2; q += pl.threads) twS[q] = tw[q];
    const int rl = (int)threadIdx.x / pl.tpr, tr = (int)threadIdx.x - rl * pl.tpr;
    const int ring = (int)blk * pl.rb + rl;
    const bool live = rl < pl.rb && ring < pl.rings;
    Vec2<T>* A = buf + rl * nh;
    if (live) {
        const Vec2<T>* X = S + (long long)ring * (nh + 1);
        for (int m0 = tr; m0 < nh; m0 += kLdBatch * pl.tpr) {
            Vec2<T> xm[kLdBatch], xc[kLdBatch], w[kLdBatch];
#pragma unroll
            for (int u = 0; u < kLdBatch; ++u) {
                const int m = m0 + u * pl.tpr;
                if (m < nh) {
                    xm[u] = X[m];
                    xc[u] = conjv(X[nh - m]);
                    w[u] = conjv(twN[m]);
                }
            }
#pragma unroll
            for (int u = 0; u < kLdBatch; ++u) {
                const int m = m0 + u * pl.tpr;
                if (m < nh) {
                    // E = (xm + xc) / 2, O = (xm - xc) conj(twN[m]) / 2, Z = E + i O
                    Vec2<T> E, D;
                    E.x = T(0.5) * (xm[u].x + xc[u].x);
                    E.y = T(0.5) * (xm[u].y + xc[u].y);
                    D.x = T(0.5) * (xm[u].x - xc[u].x);
                    D.y = T(0.5) * (xm[u].y - xc[u].y);
                    const Vec2<T> O = cmul(w[u], D);
                    Vec2<T> z;
                    z.x = E.x - O.y;
                    z.y = E.y + O.x;
                    A[m] = z;
                }
            }
        }
    }
    __syncthreads(); // twiddles of the block (the ring's values are wave-local)
    if (!live) return;
    wave_fft<T, NMAX>(A, nh, tr, pl.tpr, twS, true);
    const Vec2<T>* z = A;
    const int a = ring / pl.rows, bi = ring - a * pl.rows;
    const int b = 2 * bi + parity;
    const long long base = (long long)a * g.rowlen + (long long)b * nh;
    const T s = T(1) / T(nh);
    for (int j = tr; j < nh; j += pl.tpr) {
        const Vec2<T> v = z[j];
        x[base + j] = v.x * s;
        x[g.P + base + j] = v.y * s;
    }
}

template <typename T, int NMAX>
__global__ void __launch_bounds__(kBlock) k_plane_inv(Geo g, int parity,
                                                      const Vec2<T>* __restrict__ tw,
                                                      const Vec2<T>* __restrict__ twN,
                                                      const Vec2<T>* __restrict__ S,
                                                      T* __restrict__ x, int rb)
{
    __shared__ Vec2<T> buf[kPlaneLds], twS[kPlaneLds / 2];
    d_plane_inv<T, NMAX>(blockIdx.x, buf, twS, g, parity, tw, twN, S, x, rb);
}

} // namespace cps
