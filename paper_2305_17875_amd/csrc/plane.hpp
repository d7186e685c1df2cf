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
//    layout; a Stockham radix-2 transform of length n_phi/2 in LDS and the
//    usual even/odd recombination give the n_phi/2 + 1 modes;
//  - k_plane_tri: one thread per (row, mode) runs the Thomas algorithm down
//    and up the r-line, keeping the elimination factors in a scratch array;
//  - k_plane_inv: the inverse transform back into the rows.
// Spectra are laid out [a][row][mode], so the r-line solves read and write
// consecutive modes across a wavefront.

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

// Stockham radix-2 transform of length n (a power of 2) of the ring held at
// A + ring * n, tpr threads per ring; the result is in the returned buffer.
// tw[q] = exp(-2 pi i q / n) for q < n / 2; inverse: conjugate twiddles, no
// scaling.  Every thread of the block must call it (it holds the barriers).
template <typename T>
__device__ Vec2<T>* lds_fft(Vec2<T>* A, Vec2<T>* B, int n, int ring, int tr, int tpr,
                            const Vec2<T>* __restrict__ tw, bool inverse)
{
    for (int Ls = 1; Ls < n; Ls <<= 1) {
        const int stride = n / (2 * Ls);
        for (int t = tr; t < n / 2; t += tpr) {
            const int j = t & (Ls - 1), k = t / Ls;
            Vec2<T> w = tw[j * stride];
            if (inverse) w.y = -w.y;
            const Vec2<T> a = A[ring * n + k * Ls + j];
            const Vec2<T> wb = cmul(w, A[ring * n + k * Ls + j + n / 2]);
            B[ring * n + 2 * k * Ls + j] = a + wb;
            B[ring * n + 2 * k * Ls + j + Ls] = a - wb;
        }
        __syncthreads();
        Vec2<T>* s = A;
        A = B;
        B = s;
    }
    return A;
}

struct PlaneLaunch {
    int tpr, rb, rows, rings, blocks;
};

// rows of parity k; threads per ring and rings per 256-thread block
__host__ __device__ inline PlaneLaunch plane_launch(const Geo& g, int parity)
{
    PlaneLaunch p;
    p.rows = (g.nt - parity + 1) / 2;
    p.tpr = g.nh / 2 < kBlock ? g.nh / 2 : kBlock;
    p.rb = kBlock / p.tpr;
    p.rings = g.nr * p.rows;
    p.blocks = (p.rings + p.rb - 1) / p.rb;
    return p;
}

// Right-hand sides of the rings of parity k and their real transforms:
// S[(a rows + bi)(nh + 1) + m], m = 0..nh.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_plane_fwd(Geo g, const T* __restrict__ G, long long gk,
                                                      const T* __restrict__ bv,
                                                      const T* __restrict__ x, int parity,
                                                      const Vec2<T>* __restrict__ tw,
                                                      const Vec2<T>* __restrict__ twN,
                                                      Vec2<T>* __restrict__ S)
{
    __shared__ Vec2<T> bufA[kPlaneLds], bufB[kPlaneLds];
    const PlaneLaunch pl = plane_launch(g, parity);
    const int nh = g.nh;
    const int rl = (int)threadIdx.x / pl.tpr, tr = (int)threadIdx.x - rl * pl.tpr;
    const int ring = (int)blockIdx.x * pl.rb + rl;
    const bool live = ring < pl.rings;
    const int a = live ? ring / pl.rows : 0, bi = live ? ring - a * pl.rows : 0;
    const int b = 2 * bi + parity;
    if (live) {
        const long long ci = (long long)a * g.nt + b;
        const T gtl = G[4 * gk + ci];
        const T gth = b < g.nt - 1 ? G[4 * gk + ci + 1] : T(0);
        const long long base = (long long)a * g.rowlen + (long long)b * nh;
        for (int j = tr; j < nh; j += pl.tpr) {
            Vec2<T> z;
            z.x = bv[base + j];
            z.y = bv[g.P + base + j];
            if (b > 0) {
                z.x -= gtl * x[base - nh + j];
                z.y -= gtl * x[g.P + base - nh + j];
            }
            if (b < g.nt - 1) {
                z.x -= gth * x[base + nh + j];
                z.y -= gth * x[g.P + base + nh + j];
            }
            bufA[rl * nh + j] = z;
        }
    } else {
        for (int j = tr; j < nh; j += pl.tpr) bufA[rl * nh + j] = Vec2<T>{T(0), T(0)};
    }
    __syncthreads();
    const Vec2<T>* Z = lds_fft<T>(bufA, bufB, nh, rl, tr, pl.tpr, tw, false);
    if (!live) return;
    Vec2<T>* out = S + (long long)ring * (nh + 1);
    for (int m = tr; m <= nh; m += pl.tpr) {
        const Vec2<T> zm = Z[rl * nh + (m == nh ? 0 : m)];
        const Vec2<T> zc = conjv(Z[rl * nh + (m == 0 ? 0 : nh - m)]);
        // even part E = (zm + zc) / 2, odd part O = (zm - zc) / (2i)
        Vec2<T> E, O;
        E.x = T(0.5) * (zm.x + zc.x);
        E.y = T(0.5) * (zm.y + zc.y);
        O.x = T(0.5) * (zm.y - zc.y);
        O.y = -T(0.5) * (zm.x - zc.x);
        out[m] = E + cmul(twN[m], O);
    }
}

// Thomas algorithm along r for every (row, mode) of parity k, in place in S;
// cp: scratch for the elimination factors (same indexing as S).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_plane_tri(Geo g, const T* __restrict__ G, long long gk,
                                                      int parity, const T* __restrict__ lam,
                                                      Vec2<T>* __restrict__ S,
                                                      T* __restrict__ cp)
{
    const int rows = (g.nt - parity + 1) / 2;
    const int nm = g.nh + 1;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)rows * nm) return;
    const int bi = (int)(t / nm), m = (int)(t - (long long)bi * nm);
    const int b = 2 * bi + parity;
    const T lm = lam[m];
    const long long stride = (long long)rows * nm; // one r-plane of spectra
    T c = T(0);
    Vec2<T> d{T(0), T(0)};
    for (int a = 0; a < g.nr; ++a) {
        const long long ci = (long long)a * g.nt + b;
        const T grl = G[ci];
        const T grh = a < g.nr - 1 ? G[ci + g.nt] : T(0);
        const T gtl = G[4 * gk + ci];
        const T gth = b < g.nt - 1 ? G[4 * gk + ci + 1] : T(0);
        const T diag = -(grl + grh + gtl + gth) + G[8 * gk + ci] * lm;
        const T inv = T(1) / (diag - grl * c);
        const long long o = (long long)a * stride + t;
        const Vec2<T> r = S[o];
        d.x = (r.x - grl * d.x) * inv;
        d.y = (r.y - grl * d.y) * inv;
        c = grh * inv;
        S[o] = d;
        cp[o] = c;
    }
    Vec2<T> xn = d; // X at a = nr - 1
    for (int a = g.nr - 2; a >= 0; --a) {
        const long long o = (long long)a * stride + t;
        const Vec2<T> da = S[o];
        const T ca = cp[o];
        xn.x = da.x - ca * xn.x;
        xn.y = da.y - ca * xn.y;
        S[o] = xn;
    }
}

// Inverse transforms of the solved spectra into the rows of parity k.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_plane_inv(Geo g, int parity,
                                                      const Vec2<T>* __restrict__ tw,
                                                      const Vec2<T>* __restrict__ twN,
                                                      const Vec2<T>* __restrict__ S,
                                                      T* __restrict__ x)
{
    __shared__ Vec2<T> bufA[kPlaneLds], bufB[kPlaneLds];
    const PlaneLaunch pl = plane_launch(g, parity);
    const int nh = g.nh;
    const int rl = (int)threadIdx.x / pl.tpr, tr = (int)threadIdx.x - rl * pl.tpr;
    const int ring = (int)blockIdx.x * pl.rb + rl;
    const bool live = ring < pl.rings;
    if (live) {
        const Vec2<T>* X = S + (long long)ring * (nh + 1);
        for (int m = tr; m < nh; m += pl.tpr) {
            const Vec2<T> xm = X[m];
            const Vec2<T> xc = conjv(X[nh - m]);
            // E = (xm + xc) / 2, O = (xm - xc) conj(twN[m]) / 2, Z = E + i O
            Vec2<T> E, D;
            E.x = T(0.5) * (xm.x + xc.x);
            E.y = T(0.5) * (xm.y + xc.y);
            D.x = T(0.5) * (xm.x - xc.x);
            D.y = T(0.5) * (xm.y - xc.y);
            const Vec2<T> O = cmul(conjv(twN[m]), D);
            Vec2<T> z;
            z.x = E.x - O.y;
            z.y = E.y + O.x;
            bufA[rl * nh + m] = z;
        }
    } else {
        for (int m = tr; m < nh; m += pl.tpr) bufA[rl * nh + m] = Vec2<T>{T(0), T(0)};
    }
    __syncthreads();
    const Vec2<T>* z = lds_fft<T>(bufA, bufB, nh, rl, tr, pl.tpr, tw, true);
    if (!live) return;
    const int a = ring / pl.rows, bi = ring - a * pl.rows;
    const int b = 2 * bi + parity;
    const long long base = (long long)a * g.rowlen + (long long)b * nh;
    const T s = T(1) / T(nh);
    for (int j = tr; j < nh; j += pl.tpr) {
        const Vec2<T> v = z[rl * nh + j];
        x[base + j] = v.x * s;
        x[g.P + base + j] = v.y * s;
    }
}

} // namespace cps
