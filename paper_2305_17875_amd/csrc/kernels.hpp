// kernels.hpp -- gfx950 kernels of the shell pressure-Poisson multigrid.
//
// Every kernel is a template over the value type T (double or float), the
// stencil shape MODE and the metric storage AXI:
//   MODE_ORTHO   all cross metrics vanish: 7-point stencil, 3 arrays
//                (G_rr, G_tt, G_pp);
//   MODE_RT      only G_rt and G_tr cross terms (every map that is invariant
//                under rotation about the polar axis): 11 points;
//   MODE_FULL    all nine metrics: the 19-point stencil of eq. (PC_8).
//   AXI          metrics independent of phi, stored once per (r, theta).
// Metrics are [9][n_r][n_theta][nc] with nc = 1 (AXI) or n_phi; entry 3d+q
// of a cell is G_dq on the cell's low face in direction d (Sec. 3.2), zero on
// the low r- and theta-walls; the high walls are implicit zeros.
//
// Fields are [n_r][n_theta][n_phi], phi contiguous; one thread per cell (or
// per cell of one colour) with consecutive threads along phi, so every load
// of a wavefront is one contiguous run.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cps {

enum { MODE_ORTHO = 0, MODE_RT = 1, MODE_FULL = 2 };

constexpr int kBlock = 256;

template <typename T>
struct Level {
    int nr, nt, np;
    const T* G;   // [9][nr][nt][nc]
    long long gk; // nr * nt * nc
};

__device__ __forceinline__ int clampi(int v, int hi) { return v < 0 ? 0 : (v > hi ? hi : v); }

// Reads field values of the 3x3x3 block around (a, b, c), mirrored in r and
// theta and wrapped in phi.
template <typename T>
struct Field {
    const T* x;
    __device__ __forceinline__ T operator()(long long i) const { return x[i]; }
};

// The indicator of one cell: used to assemble matrix rows from the stencil.
template <typename T>
struct Delta {
    long long j;
    __device__ __forceinline__ T operator()(long long i) const { return i == j ? T(1) : T(0); }
};

template <typename T, int MODE, bool AXI>
__device__ __forceinline__ T coef(const Level<T>& L, int k, int a, int b, int c)
{
    long long i = AXI ? (long long)a * L.nt + b : ((long long)a * L.nt + b) * L.np + c;
    return L.G[k * L.gk + i];
}

// (A x) at cell (a, b, c) as the sum over directions of (flux through the
// high face) - (flux through the low face), and D = -(sum of the six G_dd).
// The flux through a face in direction d is
//   G_dd (x_hi - x_lo) + sum_{q != d} G_dq/4 (x_hi+q + x_lo+q - x_hi-q - x_lo-q),
// eq. (PC_term1)-(PC_term3) generalised to all nine terms.
template <typename T, int MODE, bool AXI, typename Acc>
__device__ __forceinline__ T apply_cell(const Level<T>& L, const Acc& X, int a, int b, int c,
                                        T& D)
{
    const int nr = L.nr, nt = L.nt, np = L.np;
    const long long st = np, sr = (long long)nt * np;
    const int cm = c == 0 ? np - 1 : c - 1;
    const int cp = c == np - 1 ? 0 : c + 1;
    const bool rhi = a < nr - 1, thi = b < nt - 1;
    // diagonal metrics of the six faces
    const T grl = coef<T, MODE, AXI>(L, 0, a, b, c);
    const T grh = rhi ? coef<T, MODE, AXI>(L, 0, a + 1, b, c) : T(0);
    const T gtl = coef<T, MODE, AXI>(L, 4, a, b, c);
    const T gth = thi ? coef<T, MODE, AXI>(L, 4, a, b + 1, c) : T(0);
    const T gpl = coef<T, MODE, AXI>(L, 8, a, b, c);
    const T gph = coef<T, MODE, AXI>(L, 8, a, b, cp);
    D = -(grl + grh + gtl + gth + gpl + gph);
    // offsets of the neighbour planes, mirrored at the walls
    const long long ra = a > 0 ? -sr : 0, rb = rhi ? sr : 0;
    const long long ta = b > 0 ? -st : 0, tb = thi ? st : 0;
    const long long base = (long long)a * sr + (long long)b * st;
    const long long pa = cm - c, pb = cp - c;
    const long long i0 = base + c;
    const T x0 = X(i0);
    const T xrm = X(i0 + ra), xrp = X(i0 + rb);
    const T xtm = X(i0 + ta), xtp = X(i0 + tb);
    const T xpm = X(i0 + pa), xpp = X(i0 + pb);
    T s = grh * (xrp - x0) - grl * (x0 - xrm) + gth * (xtp - x0) - gtl * (x0 - xtm) +
          gph * (xpp - x0) - gpl * (x0 - xpm);
    if constexpr (MODE != MODE_ORTHO) {
        // r-theta edges
        const T xrmtm = X(i0 + ra + ta), xrmtp = X(i0 + ra + tb);
        const T xrptm = X(i0 + rb + ta), xrptp = X(i0 + rb + tb);
        const T q = T(0.25);
        const T grt_l = coef<T, MODE, AXI>(L, 1, a, b, c);
        const T grt_h = rhi ? coef<T, MODE, AXI>(L, 1, a + 1, b, c) : T(0);
        const T gtr_l = coef<T, MODE, AXI>(L, 3, a, b, c);
        const T gtr_h = thi ? coef<T, MODE, AXI>(L, 3, a, b + 1, c) : T(0);
        // r-flux cross terms (q = theta)
        s += q * grt_h * (xrptp + xtp - xrptm - xtm) - q * grt_l * (xtp + xrmtp - xtm - xrmtm);
        // theta-flux cross terms (q = r)
        s += q * gtr_h * (xrptp + xrp - xrmtp - xrm) - q * gtr_l * (xrp + xrptm - xrm - xrmtm);
        if constexpr (MODE == MODE_FULL) {
            const T xrmpm = X(i0 + ra + pa), xrmpp = X(i0 + ra + pb);
            const T xrppm = X(i0 + rb + pa), xrppp = X(i0 + rb + pb);
            const T xtmpm = X(i0 + ta + pa), xtmpp = X(i0 + ta + pb);
            const T xtppm = X(i0 + tb + pa), xtppp = X(i0 + tb + pb);
            const T grp_l = coef<T, MODE, AXI>(L, 2, a, b, c);
            const T grp_h = rhi ? coef<T, MODE, AXI>(L, 2, a + 1, b, c) : T(0);
            const T gtp_l = coef<T, MODE, AXI>(L, 5, a, b, c);
            const T gtp_h = thi ? coef<T, MODE, AXI>(L, 5, a, b + 1, c) : T(0);
            const T gpr_l = coef<T, MODE, AXI>(L, 6, a, b, c);
            const T gpr_h = coef<T, MODE, AXI>(L, 6, a, b, cp);
            const T gpt_l = coef<T, MODE, AXI>(L, 7, a, b, c);
            const T gpt_h = coef<T, MODE, AXI>(L, 7, a, b, cp);
            // r-flux, q = phi
            s += q * grp_h * (xrppp + xpp - xrppm - xpm) - q * grp_l * (xpp + xrmpp - xpm - xrmpm);
            // theta-flux, q = phi
            s += q * gtp_h * (xtppp + xpp - xtppm - xpm) - q * gtp_l * (xpp + xtmpp - xpm - xtmpm);
            // phi-flux, q = r
            s += q * gpr_h * (xrppp + xrp - xrmpp - xrm) - q * gpr_l * (xrp + xrppm - xrm - xrmpm);
            // phi-flux, q = theta
            s += q * gpt_h * (xtppp + xtp - xtmpp - xtm) - q * gpt_l * (xtp + xtppm - xtm - xtmpm);
        }
    }
    return s;
}

// ---------------------------------------------------------------------------
// Reductions: wave64 shuffles, then LDS across the block; fixed order.
// ---------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// Sum over the block; the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v)
{
    __shared__ double sh[kBlock / 64];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
    __syncthreads();
    return t;
}

// out[slot] = sum of partial[0..n) in a fixed order (one block).
__global__ void __launch_bounds__(kBlock) k_reduce(const double* __restrict__ partial, long long n,
                                                   double* __restrict__ out)
{
    double s = 0.0;
    for (long long i = threadIdx.x; i < n; i += blockDim.x) s += partial[i];
    s = block_sum(s);
    if (threadIdx.x == 0) *out = s;
}

// ---------------------------------------------------------------------------
// Operator kernels
// ---------------------------------------------------------------------------

// y = A x over all cells.
template <typename T, int MODE, bool AXI>
__global__ void __launch_bounds__(kBlock) k_apply(Level<T> L, const T* __restrict__ x,
                                                  T* __restrict__ y, double* __restrict__ partial,
                                                  const T* __restrict__ dotv)
{
    const long long n = (long long)L.nr * L.nt * L.np;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (i < n) {
        const int c = (int)(i % L.np);
        const long long row = i / L.np;
        const int b = (int)(row % L.nt), a = (int)(row / L.nt);
        T D;
        const T v = apply_cell<T, MODE, AXI>(L, Field<T>{x}, a, b, c, D);
        y[i] = v;
        if (dotv) acc = (double)v * (double)dotv[i];
    }
    if (partial) {
        acc = block_sum(acc);
        if (threadIdx.x == 0) partial[blockIdx.x] = acc;
    }
}

// r = b - A x, and per-block partial sums of r^2.
template <typename T, int MODE, bool AXI>
__global__ void __launch_bounds__(kBlock) k_residual(Level<T> L, const T* __restrict__ bv,
                                                     const T* __restrict__ x, T* __restrict__ r,
                                                     double* __restrict__ partial)
{
    const long long n = (long long)L.nr * L.nt * L.np;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (i < n) {
        const int c = (int)(i % L.np);
        const long long row = i / L.np;
        const int b = (int)(row % L.nt), a = (int)(row / L.nt);
        T D;
        const T v = bv[i] - apply_cell<T, MODE, AXI>(L, Field<T>{x}, a, b, c, D);
        r[i] = v;
        acc = (double)v * (double)v;
    }
    if (partial) {
        acc = block_sum(acc);
        if (threadIdx.x == 0) partial[blockIdx.x] = acc;
    }
}

// One Gauss-Seidel pass over the cells of one colour, in place:
// x_c += (b_c - (A x)_c) / D_c.  Two colours: (a+b+c) mod 2.  Four colours:
// k = 2((a+c) mod 2) + ((b+c) mod 2).  Cells of one colour never read one
// another, so all threads of the pass update concurrently.  Needs even dims.
template <typename T, int MODE, bool AXI>
__global__ void __launch_bounds__(kBlock) k_gs(Level<T> L, const T* __restrict__ bv,
                                               T* __restrict__ x, int colour, int ncol)
{
    const int np2 = L.np >> 1;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int a, b, c;
    if (ncol == 2) {
        if (i >= (long long)L.nr * L.nt * np2) return;
        const int ch = (int)(i % np2);
        const long long row = i / np2;
        b = (int)(row % L.nt);
        a = (int)(row / L.nt);
        c = 2 * ch + ((colour + a + b) & 1);
    } else {
        const int nt2 = L.nt >> 1;
        if (i >= (long long)L.nr * nt2 * np2) return;
        const int ch = (int)(i % np2);
        const long long row = i / np2;
        const int bh = (int)(row % nt2);
        a = (int)(row / nt2);
        const int k1 = colour >> 1, k0 = colour & 1;
        b = 2 * bh + ((a + k0 + k1) & 1);
        c = 2 * ch + ((k1 + a) & 1);
    }
    T D;
    const T Ax = apply_cell<T, MODE, AXI>(L, Field<T>{x}, a, b, c, D);
    const long long id = ((long long)a * L.nt + b) * L.np + c;
    x[id] += (bv[id] - Ax) / D;
}

// ---------------------------------------------------------------------------
// Grid transfers (cell-centred, coarsening by 2 in every direction)
// ---------------------------------------------------------------------------

// bc = P^T r, gathered: coarse index I takes fine 2I-1, 2I, 2I+1, 2I+2 with
// weights 1/4, 3/4, 3/4, 1/4 per direction; fine indices past a wall fold
// onto the wall cell, phi wraps.  (nr, nt, np) are the fine dims.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_restrict(int nr, int nt, int np,
                                                     const T* __restrict__ r,
                                                     T* __restrict__ bc)
{
    const int mr = nr >> 1, mt = nt >> 1, mp = np >> 1;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)mr * mt * mp) return;
    const int K = (int)(i % mp);
    const long long row = i / mp;
    const int J = (int)(row % mt), I = (int)(row / mt);
    const T w[4] = {T(0.25), T(0.75), T(0.75), T(0.25)};
    int ia[4], ib[4], ic[4];
    for (int o = 0; o < 4; ++o) {
        ia[o] = clampi(2 * I - 1 + o, nr - 1);
        ib[o] = clampi(2 * J - 1 + o, nt - 1);
        int cc = 2 * K - 1 + o;
        ic[o] = cc < 0 ? cc + np : (cc >= np ? cc - np : cc);
    }
    T s = T(0);
    for (int p = 0; p < 4; ++p)
        for (int q = 0; q < 4; ++q) {
            const T* rowp = r + ((long long)ia[p] * nt + ib[q]) * np;
            T t = w[0] * rowp[ic[0]] + w[1] * rowp[ic[1]] + w[2] * rowp[ic[2]] + w[3] * rowp[ic[3]];
            s += w[p] * w[q] * t;
        }
    bc[i] = s;
}

// x += P e: fine cell i in a direction takes 3/4 of coarse i/2 and 1/4 of
// coarse i/2 - 1 (even i) or i/2 + 1 (odd i), mirrored at walls, wrapped in
// phi; trilinear = the product of the three.  (nr, nt, np) are fine dims.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_prolong(int nr, int nt, int np,
                                                    const T* __restrict__ e,
                                                    T* __restrict__ x)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)nr * nt * np) return;
    const int c = (int)(i % np);
    const long long row = i / np;
    const int b = (int)(row % nt), a = (int)(row / nt);
    const int mr = nr >> 1, mt = nt >> 1, mp = np >> 1;
    const int A0 = a >> 1, B0 = b >> 1, C0 = c >> 1;
    const int A1 = clampi((a & 1) ? A0 + 1 : A0 - 1, mr - 1);
    const int B1 = clampi((b & 1) ? B0 + 1 : B0 - 1, mt - 1);
    int C1 = (c & 1) ? C0 + 1 : C0 - 1;
    C1 = C1 < 0 ? C1 + mp : (C1 >= mp ? C1 - mp : C1);
    const T w0 = T(0.75), w1 = T(0.25);
    auto E = [&](int p, int q, int s) { return e[((long long)p * mt + q) * mp + s]; };
    const T v0 = w0 * (w0 * E(A0, B0, C0) + w1 * E(A0, B0, C1)) +
                 w1 * (w0 * E(A0, B1, C0) + w1 * E(A0, B1, C1));
    const T v1 = w0 * (w0 * E(A1, B0, C0) + w1 * E(A1, B0, C1)) +
                 w1 * (w0 * E(A1, B1, C0) + w1 * E(A1, B1, C1));
    x[i] += w0 * v0 + w1 * v1;
}

// ---------------------------------------------------------------------------
// Coarsest level: e = Ainv (b - mean b), Ainv row-major FP64.  One wave per
// row, lanes striding over the columns; every block recomputes the mean.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kBlock) k_coarse_gemv(int n, const double* __restrict__ Ainv,
                                                        const T* __restrict__ bv,
                                                        T* __restrict__ e)
{
    __shared__ double smean;
    double s = 0.0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) s += (double)bv[j];
    s = block_sum(s);
    if (threadIdx.x == 0) smean = s / n;
    __syncthreads();
    const double m = smean;
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (row >= n) return;
    const double* Ar = Ainv + (long long)row * n;
    double acc = 0.0;
    for (int j = lane; j < n; j += 64) acc += Ar[j] * ((double)bv[j] - m);
    acc = wave_sum(acc);
    if (lane == 0) e[row] = (T)acc;
}

// ---------------------------------------------------------------------------
// Vector kernels
// ---------------------------------------------------------------------------

// partial sums of u.v (or of u alone when v == nullptr)
template <typename T, typename U>
__global__ void __launch_bounds__(kBlock) k_dot(long long n, const T* __restrict__ u,
                                                const U* __restrict__ v,
                                                double* __restrict__ partial)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (i < n) acc = v ? (double)u[i] * (double)v[i] : (double)u[i];
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// y = x - (*sum)/n  (mean removal; *sum is a device scalar)
__global__ void __launch_bounds__(kBlock) k_sub_mean(long long n, const double* __restrict__ x,
                                                     const double* __restrict__ sum,
                                                     double* __restrict__ y)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = x[i] - *sum / (double)n;
}

// y = (U) (x * s) with s = sc[slot] or 1 / sc[slot] (a device scalar)
template <typename T, typename U>
__global__ void __launch_bounds__(kBlock) k_cast(long long n, const T* __restrict__ x,
                                                 U* __restrict__ y, const double* __restrict__ sc,
                                                 int slot, int invert)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const double s = invert ? 1.0 / sc[slot] : sc[slot];
    if (i < n) y[i] = (U)((double)x[i] * s);
}

// x[i] = v
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fill(long long n, T* __restrict__ x, T v)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

// y[i] = x[i]
template <typename T>
__global__ void __launch_bounds__(kBlock) k_copy(long long n, const T* __restrict__ x,
                                                 T* __restrict__ y)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = x[i];
}

// x += s * (double) e   (iterative-refinement update, s a device scalar
// holding the norm the residual was divided by)
template <typename U>
__global__ void __launch_bounds__(kBlock) k_ir_update(long long n, double* __restrict__ x,
                                                      const U* __restrict__ e,
                                                      const double* __restrict__ s)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] += *s * (double)e[i];
}

// Scalar recurrences of the Krylov solvers, evaluated by one thread on
// device scalars (sc[] slots) so that no host round trip is needed.
enum {
    S_BB = 0, S_RR, S_RZ, S_RZ_OLD, S_PQ, S_ZQ, S_ALPHA, S_BETA, S_OMEGA, S_RHO, S_RHO_OLD,
    S_TS, S_TT, S_R0V, S_SUM, S_SCALE, S_COUNT
};

// CG / flexible CG: alpha = rz / pq
__global__ void k_cg_alpha(double* sc) { sc[S_ALPHA] = sc[S_RZ] / sc[S_PQ]; }
// beta = rz_new / rz_old (CG) or -alpha zq / rz_old (flexible, Polak-Ribiere)
__global__ void k_cg_beta(double* sc, int flexible)
{
    sc[S_BETA] = flexible ? -sc[S_ALPHA] * sc[S_ZQ] / sc[S_RZ_OLD] : sc[S_RZ] / sc[S_RZ_OLD];
}
__global__ void k_bicg_beta(double* sc)
{
    sc[S_BETA] = (sc[S_RHO] / sc[S_RHO_OLD]) * (sc[S_ALPHA] / sc[S_OMEGA]);
}
__global__ void k_bicg_alpha(double* sc) { sc[S_ALPHA] = sc[S_RHO] / sc[S_R0V]; }
__global__ void k_bicg_omega(double* sc) { sc[S_OMEGA] = sc[S_TS] / sc[S_TT]; }
__global__ void k_copy_scalar(double* sc, int dst, int src) { sc[dst] = sc[src]; }
__global__ void k_set_scalar(double* sc, int dst, double v) { sc[dst] = v; }
// sc[S_SCALE] = sqrt(sc[src])
__global__ void k_sqrt_scalar(double* sc, int dst, int src) { sc[dst] = sqrt(sc[src]); }

// x += alpha p ; r -= alpha q ; partial sums of r^2   (CG step)
__global__ void __launch_bounds__(kBlock) k_cg_step(long long n, const double* __restrict__ sc,
                                                    double* __restrict__ x,
                                                    double* __restrict__ r,
                                                    const double* __restrict__ p,
                                                    const double* __restrict__ q,
                                                    double* __restrict__ partial)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const double al = sc[S_ALPHA];
    double acc = 0.0;
    if (i < n) {
        x[i] += al * p[i];
        const double v = r[i] - al * q[i];
        r[i] = v;
        acc = v * v;
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// p = z + beta p
__global__ void __launch_bounds__(kBlock) k_cg_dir(long long n, const double* __restrict__ sc,
                                                   const double* __restrict__ z,
                                                   double* __restrict__ p)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = z[i] + sc[S_BETA] * p[i];
}

// BiCGStab: p = r + beta (p - omega v)
__global__ void __launch_bounds__(kBlock) k_bicg_dir(long long n, const double* __restrict__ sc,
                                                     const double* __restrict__ r,
                                                     const double* __restrict__ v,
                                                     double* __restrict__ p)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = r[i] + sc[S_BETA] * (p[i] - sc[S_OMEGA] * v[i]);
}

// BiCGStab: s = r - alpha v (into s)
__global__ void __launch_bounds__(kBlock) k_bicg_s(long long n, const double* __restrict__ sc,
                                                   const double* __restrict__ r,
                                                   const double* __restrict__ v,
                                                   double* __restrict__ s)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) s[i] = r[i] - sc[S_ALPHA] * v[i];
}

// BiCGStab: x += alpha ph + omega sh ; r = s - omega t ; partial r^2
__global__ void __launch_bounds__(kBlock) k_bicg_step(long long n, const double* __restrict__ sc,
                                                      double* __restrict__ x,
                                                      double* __restrict__ r,
                                                      const double* __restrict__ ph,
                                                      const double* __restrict__ sh,
                                                      const double* __restrict__ s,
                                                      const double* __restrict__ t,
                                                      double* __restrict__ partial)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (i < n) {
        x[i] += sc[S_ALPHA] * ph[i] + sc[S_OMEGA] * sh[i];
        const double v = s[i] - sc[S_OMEGA] * t[i];
        r[i] = v;
        acc = v * v;
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// ---------------------------------------------------------------------------
// Setup: face metrics from the map (Sec. 3.2), per level, on the device
// ---------------------------------------------------------------------------

struct MapParams {
    int map;
    double r_inner, r_outer, theta0, theta1, stretch, flattening, skew;
};

__device__ inline void map_point(const MapParams& m, double sr, double st, double sp, double X[3])
{
    const double d = m.r_outer - m.r_inner;
    double r;
    if (m.stretch == 0.0)
        r = m.r_inner + d * sr;
    else
        r = 0.5 * (m.r_inner + m.r_outer) + d * tanh(m.stretch * (sr - 0.5)) / (2.0 * tanh(0.5 * m.stretch));
    const double th = m.theta0 + st * (m.theta1 - m.theta0);
    const double ph = 6.283185307179586476925 * sp;
    if (m.map == 0) {
        X[0] = r; X[1] = th; X[2] = ph;
        return;
    }
    double sth, cth, sph, cph;
    sincos(th, &sth, &cth);
    sincos(ph, &sph, &cph);
    const double f = m.map >= 2 ? m.flattening : 0.0;
    const double g = m.map == 3 ? m.skew : 0.0;
    X[0] = (1.0 - f) * r * cth;
    X[1] = (1.0 + g) * r * sth * cph;
    X[2] = r * sth * sph;
}

// Face metrics of one level.  One thread per (a, b, c) (c = 0 only when the
// metrics are phi-invariant), three faces each.  method 0: chords of the map
// across the face centre; method 1: the paper's vertex averages.  flags[blk]
// gets bit 0 for a face with det <= 0, bit 1 for a non-zero r-theta cross
// metric, bit 2 for a non-zero cross metric involving phi.
__global__ void __launch_bounds__(kBlock) k_metrics(MapParams m, int nr, int nt, int np, int nc,
                                                    int method, double* __restrict__ G,
                                                    int* __restrict__ flags)
{
    __shared__ int sflag;
    if (threadIdx.x == 0) sflag = 0;
    __syncthreads();
    const long long n = (long long)nr * nt * nc;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int fl = 0;
    if (i < n) {
        const int c = (int)(i % nc);
        const long long row = i / nc;
        const int b = (int)(row % nt), a = (int)(row / nt);
        auto P = [&](double ia, double ib, double ic, double X[3]) {
            map_point(m, ia / nr, ib / nt, ic / np, X);
        };
        for (int d = 0; d < 3; ++d) {
            double Gd[3] = {0.0, 0.0, 0.0};
            const bool wall = (d == 0 && a == 0) || (d == 1 && b == 0);
            if (!wall) {
                double t[3][3];
                const double lo[3] = {(double)a, (double)b, (double)c};
                if (method == 0) {
                    double f[3] = {a + 0.5, b + 0.5, c + 0.5};
                    f[d] -= 0.5;
                    for (int q = 0; q < 3; ++q) {
                        double p1[3] = {f[0], f[1], f[2]}, p0[3] = {f[0], f[1], f[2]};
                        p1[q] += 0.5;
                        p0[q] -= 0.5;
                        double X1[3], X0[3];
                        P(p1[0], p1[1], p1[2], X1);
                        P(p0[0], p0[1], p0[2], X0);
                        for (int k = 0; k < 3; ++k) t[q][k] = X1[k] - X0[k];
                    }
                } else {
                    const int u = (d + 1) % 3, v = (d + 2) % 3;
                    for (int k = 0; k < 3; ++k) t[d][k] = t[u][k] = t[v][k] = 0.0;
                    for (int iu = 0; iu < 2; ++iu)
                        for (int iv = 0; iv < 2; ++iv) {
                            double p1[3] = {lo[0], lo[1], lo[2]};
                            p1[u] += iu;
                            p1[v] += iv;
                            double p0[3] = {p1[0], p1[1], p1[2]};
                            p1[d] += 1.0;
                            p0[d] -= 1.0;
                            double X1[3], X0[3];
                            P(p1[0], p1[1], p1[2], X1);
                            P(p0[0], p0[1], p0[2], X0);
                            for (int k = 0; k < 3; ++k) t[d][k] += 0.125 * (X1[k] - X0[k]);
                        }
                    for (int s = 0; s < 2; ++s) {
                        const int q = s == 0 ? u : v, o = s == 0 ? v : u;
                        for (int io = 0; io < 2; ++io) {
                            double p0[3] = {lo[0], lo[1], lo[2]};
                            p0[o] += io;
                            double p1[3] = {p0[0], p0[1], p0[2]};
                            p1[q] += 1.0;
                            double X1[3], X0[3];
                            P(p1[0], p1[1], p1[2], X1);
                            P(p0[0], p0[1], p0[2], X0);
                            for (int k = 0; k < 3; ++k) t[q][k] += 0.5 * (X1[k] - X0[k]);
                        }
                    }
                }
                // rows of the Jacobian: cyclic cross products over det
                double nv[3][3];
                for (int e = 0; e < 3; ++e) {
                    const double* u1 = t[(e + 1) % 3];
                    const double* u2 = t[(e + 2) % 3];
                    nv[e][0] = u1[1] * u2[2] - u1[2] * u2[1];
                    nv[e][1] = u1[2] * u2[0] - u1[0] * u2[2];
                    nv[e][2] = u1[0] * u2[1] - u1[1] * u2[0];
                }
                const double det = t[0][0] * nv[0][0] + t[0][1] * nv[0][1] + t[0][2] * nv[0][2];
                if (!(det > 0.0)) fl |= 1;
                double nn[3];
                for (int q = 0; q < 3; ++q)
                    nn[q] = nv[q][0] * nv[q][0] + nv[q][1] * nv[q][1] + nv[q][2] * nv[q][2];
                for (int q = 0; q < 3; ++q) {
                    double v = (nv[d][0] * nv[q][0] + nv[d][1] * nv[q][1] + nv[d][2] * nv[q][2]) / det;
                    if (q != d && fabs(v) <= 1e-13 * sqrt(fabs(nn[d] * nn[q])) / fabs(det)) v = 0.0;
                    Gd[q] = v;
                }
                for (int q = 0; q < 3; ++q)
                    if (q != d && Gd[q] != 0.0) fl |= (d == 2 || q == 2) ? 4 : 2;
            }
            for (int q = 0; q < 3; ++q) G[(long long)(3 * d + q) * n + i] = Gd[q];
        }
    }
    if (fl) atomicOr(&sflag, fl);
    __syncthreads();
    if (threadIdx.x == 0) flags[blockIdx.x] = sflag;
}

// Float copy of an FP64 array.
__global__ void __launch_bounds__(kBlock) k_to_f32(long long n, const double* __restrict__ a,
                                                   float* __restrict__ b)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

// Expand stored metrics to [9][nr][nt][np] (for inspection).
__global__ void __launch_bounds__(kBlock) k_expand_metrics(int nr, int nt, int np, int nc,
                                                           const double* __restrict__ G,
                                                           double* __restrict__ out)
{
    const long long n = (long long)nr * nt * np;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = (int)(i % np);
    const long long row = i / np;
    const long long src = row * nc + (nc == 1 ? 0 : c);
    const long long gk = (long long)nr * nt * nc;
    for (int k = 0; k < 9; ++k) out[k * n + i] = G[k * gk + src];
}

// Dense coarsest operator: row i gets A[i][j] = (A delta_j)_i for every
// cell j of the 3x3x3 block around cell i (mirrored / wrapped; a cell
// reached twice is evaluated once).  A must be zeroed first.
template <int MODE, bool AXI>
__global__ void __launch_bounds__(kBlock) k_dense_rows(Level<double> L, double* __restrict__ A)
{
    const long long n = (long long)L.nr * L.nt * L.np;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * 27) return;
    const long long i = t / 27;
    const int s = (int)(t % 27);
    const int c = (int)(i % L.np);
    const long long row = i / L.np;
    const int b = (int)(row % L.nt), a = (int)(row / L.nt);
    auto nb = [&](int k) {
        const int da = k / 9 - 1, db = (k / 3) % 3 - 1, dc = k % 3 - 1;
        const int aa = clampi(a + da, L.nr - 1), bb = clampi(b + db, L.nt - 1);
        int cc = c + dc;
        cc = cc < 0 ? cc + L.np : (cc >= L.np ? cc - L.np : cc);
        return ((long long)aa * L.nt + bb) * L.np + cc;
    };
    const long long j = nb(s);
    for (int k = 0; k < s; ++k)
        if (nb(k) == j) return;
    double D;
    A[i * n + j] = apply_cell<double, MODE, AXI>(L, Delta<double>{j}, a, b, c, D);
}

// alpha = mean |diag| / n, added to every entry (A + alpha 1 1^T); also
// writes the identity into the right half of the augmented [A | I] buffer.
__global__ void __launch_bounds__(kBlock) k_augment(int n, const double* __restrict__ A,
                                                    double* __restrict__ M)
{
    __shared__ double salpha;
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += fabs(A[(long long)i * n + i]);
    s = block_sum(s);
    if (threadIdx.x == 0) salpha = s / n / n;
    __syncthreads();
    const double al = salpha;
    const long long tot = (long long)n * 2 * n;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < tot;
         t += (long long)gridDim.x * blockDim.x) {
        const long long i = t / (2 * n), j = t % (2 * n);
        M[t] = j < n ? A[i * n + j] + al : (j - n == i ? 1.0 : 0.0);
    }
}

// One Gauss-Jordan step on the augmented n x 2n matrix, out of place.
// Partial pivoting: the pivot of column k is the not-yet-used row with the
// largest |entry| (lowest index on ties); used_at[i] = step at which row i
// became a pivot (INT_MAX if not yet).  Every block finds the pivot itself.
__global__ void __launch_bounds__(kBlock) k_gj_step(int n, int k, const double* __restrict__ src,
                                                    double* __restrict__ dst,
                                                    int* __restrict__ used_at,
                                                    int* __restrict__ piv,
                                                    int* __restrict__ fail)
{
    __shared__ double sv[kBlock];
    __shared__ int si[kBlock];
    const long long w = 2LL * n;
    double best = -1.0;
    int bi = -1;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        if (used_at[i] < k) continue;
        const double v = fabs(src[i * w + k]);
        if (v > best) { best = v; bi = i; }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            const double v2 = sv[threadIdx.x + o];
            const int i2 = si[threadIdx.x + o];
            if (v2 > sv[threadIdx.x] || (v2 == sv[threadIdx.x] && i2 >= 0 &&
                                         (si[threadIdx.x] < 0 || i2 < si[threadIdx.x]))) {
                sv[threadIdx.x] = v2;
                si[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    const int p = si[0];
    if (p < 0 || sv[0] == 0.0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *fail = 1;
        return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        used_at[p] = k;
        piv[k] = p;
    }
    const double inv = 1.0 / src[p * w + k];
    const long long tot = (long long)n * w;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < tot;
         t += (long long)gridDim.x * blockDim.x) {
        const long long i = t / w, j = t % w;
        const double pj = src[p * w + j] * inv;
        dst[t] = i == p ? pj : src[t] - src[i * w + k] * pj;
    }
}

// Ainv row k = right half of row piv[k].
__global__ void __launch_bounds__(kBlock) k_gj_extract(int n, const double* __restrict__ M,
                                                       const int* __restrict__ piv,
                                                       double* __restrict__ Ainv)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)n * n) return;
    const long long k = t / n, j = t % n;
    Ainv[t] = M[(long long)piv[k] * 2 * n + n + j];
}

} // namespace cps
