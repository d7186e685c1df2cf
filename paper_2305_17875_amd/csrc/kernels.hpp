// kernels.hpp -- gfx950 kernels of the shell pressure-Poisson multigrid.
//
// Every stencil kernel is a template over the value type T (double or
// float), the stencil shape MODE and the metric storage AXI:
//   MODE_ORTHO   all cross metrics vanish: 7-point stencil (G_rr, G_tt, G_pp);
//   MODE_RT      only the G_rt and G_tr cross terms (maps invariant under
//                rotation about the polar axis): 11-point stencil;
//   MODE_FULL    all nine metrics: the 19-point stencil of eq. (PC_8).
//   AXI          metrics independent of phi, stored once per (r, theta).
//
// Field layout ("phi-parity split"): a level vector is [2][n_r][n_theta][nh]
// with nh = n_phi / 2; cell (a, b, c) lives in plane s = c mod 2 at index
// j = c / 2.  A colour pass then reads only the planes of the other colours
// and writes only its own, so no cache line carries cells it does not need.
// Metrics are [9][n_r][n_theta] (AXI) or [9][2][n_r][n_theta][nh]; entry
// 3d+q of a cell is G_dq on the cell's low face in direction d (Sec. 3.2),
// zero on the low r- and theta-walls; the high walls are implicit zeros.
//
// Launch shape: 1-D grids of 256-thread blocks.  A block's logical index is
// remapped so that each of the 8 XCDs (which receive blocks round-robin)
// works on one contiguous range of r-planes and keeps its neighbours in its
// own L2.  Within a plane, consecutive threads take consecutive (theta, j)
// positions, so each wavefront touches contiguous runs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cps {

enum { MODE_ORTHO = 0, MODE_RT = 1, MODE_FULL = 2 };

// device scalar slots of the Krylov solvers (sc[])
enum {
    S_BB = 0, S_RR, S_RZ, S_RZ_OLD, S_PQ, S_ZQ, S_ALPHA, S_BETA, S_OMEGA, S_RHO, S_RHO_OLD,
    S_TS, S_TT, S_R0V, S_SUM, S_SCALE, S_ALPHA_OLD, S_COUNT
};

constexpr int kBlock = 256;

// geometry of one level in the parity-split layout
struct Geo {
    int nr, nt, np, nh; // nh = np / 2
    int rowlen;         // nt * nh: cells of one parity in one r-plane
    long long P;        // nr * nt * nh: one parity plane
};

inline Geo make_geo(int nr, int nt, int np)
{
    Geo g;
    g.nr = nr;
    g.nt = nt;
    g.np = np;
    g.nh = np / 2;
    g.rowlen = nt * g.nh;
    g.P = (long long)nr * g.rowlen;
    return g;
}

template <typename T>
struct Level {
    Geo g;
    const T* G;   // metrics, see above
    long long gk; // stride between the nine metric arrays
};

__device__ __forceinline__ int clampi(int v, int hi) { return v < 0 ? 0 : (v > hi ? hi : v); }

// Streaming accesses: values read once or written once by a pass carry the
// non-temporal hint, so that the L2 of an XCD keeps the stencil field whose
// rows neighbouring wavefronts read again.
template <typename T>
__device__ __forceinline__ T ld_once(const T* p) { return __builtin_nontemporal_load(p); }
template <typename T>
__device__ __forceinline__ void st_once(T* p, T v) { __builtin_nontemporal_store(v, p); }


__device__ __forceinline__ long long split_index(const Geo& g, int a, int b, int c)
{
    return (long long)(c & 1) * g.P + ((long long)a * g.nt + b) * g.nh + (c >> 1);
}

// Logical block index with XCD-contiguous ranges: hardware block B runs on
// XCD B mod 8; XCD x gets the logical range [x q + min(x, r), ...) where
// q, r = divmod(number of blocks, 8).
__device__ __forceinline__ unsigned xcd_block()
{
    const unsigned B = blockIdx.x, T = gridDim.x;
    const unsigned x = B & 7u, k = B >> 3, q = T >> 3, r = T & 7u;
    return x * q + (x < r ? x : r) + k;
}

// The block a kernel body works as: logical index L of G blocks of one
// problem's launch.  A single-problem launch takes its XCD-remapped block
// index; a batched launch takes (problem, L, G) from a work table.
struct Blk {
    unsigned L, G;
};

__device__ __forceinline__ Blk self_blk() { return Blk{xcd_block(), gridDim.x}; }

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

// (A x) at cell (a, b, c = 2j + s) as the sum over directions of (flux
// through the high face) - (flux through the low face), and
// D = -(sum of the six G_dd).  The flux through a face in direction d is
//   G_dd (x_hi - x_lo) + sum_{q != d} G_dq/4 (x_hi+q + x_lo+q - x_hi-q - x_lo-q),
// eq. (PC_term1)-(PC_term3) generalised to all nine terms; reads that leave
// the domain in r or theta mirror onto the wall cell, phi wraps.
// OFFDIAG: return instead S = (A x)_c - D x_c, the sum over the neighbours
// (including a wall-mirrored read of the cell itself in a cross term), so a
// Gauss-Seidel update x_c = (b_c - S) / D never loads the old x_c.  The flux
// form (differences first) is kept for residuals, whose value is small next
// to D x_c near convergence.
template <typename T, int MODE, bool AXI, bool OFFDIAG = false, typename Acc>
__device__ __forceinline__ T apply_cell(const Geo& g, const T* __restrict__ G, long long gk,
                                        const Acc& X, int a, int b, int s, int j, T& D)
{
    const int nh = g.nh;
    const long long sr = g.rowlen, st = nh;
    const long long row = (long long)a * sr + (long long)b * nh;
    const long long i0 = s * g.P + row + j;
    // phi neighbours c+1 and c-1 live in the other plane
    long long ipp, ipm;
    if (s == 0) {
        ipp = g.P + row + j;
        ipm = g.P + row + (j == 0 ? nh - 1 : j - 1);
    } else {
        ipp = row + (j == nh - 1 ? 0 : j + 1);
        ipm = row + j;
    }
    const long long pa = ipm - i0, pb = ipp - i0;
    const bool rhi = a < g.nr - 1, thi = b < g.nt - 1;
    // metric indices of the low faces and of the three high faces
    long long ci, cr, ct, cp;
    if (AXI) {
        ci = (long long)a * g.nt + b;
        cr = ci + g.nt;
        ct = ci + 1;
        cp = ci;
    } else {
        ci = i0;
        cr = i0 + sr;
        ct = i0 + st;
        cp = ipp;
    }
    const T grl = G[ci];
    const T grh = rhi ? G[cr] : T(0);
    const T gtl = G[4 * gk + ci];
    const T gth = thi ? G[4 * gk + ct] : T(0);
    const T gpl = G[8 * gk + ci];
    const T gph = G[8 * gk + cp];
    D = -(grl + grh + gtl + gth + gpl + gph);
    const long long ra = a > 0 ? -sr : 0, rb = rhi ? sr : 0;
    const long long ta = b > 0 ? -st : 0, tb = thi ? st : 0;
    const T xrm = X(i0 + ra), xrp = X(i0 + rb);
    const T xtm = X(i0 + ta), xtp = X(i0 + tb);
    const T xpm = X(i0 + pa), xpp = X(i0 + pb);
    T acc;
    if constexpr (OFFDIAG) {
        acc = grh * xrp + grl * xrm + gth * xtp + gtl * xtm + gph * xpp + gpl * xpm;
    } else {
        const T x0 = X(i0);
        acc = grh * (xrp - x0) - grl * (x0 - xrm) + gth * (xtp - x0) - gtl * (x0 - xtm) +
              gph * (xpp - x0) - gpl * (x0 - xpm);
    }
    if constexpr (MODE != MODE_ORTHO) {
        const T q = T(0.25);
        const T xrmtm = X(i0 + ra + ta), xrmtp = X(i0 + ra + tb);
        const T xrptm = X(i0 + rb + ta), xrptp = X(i0 + rb + tb);
        const T grt_l = G[gk + ci];
        const T grt_h = rhi ? G[gk + cr] : T(0);
        const T gtr_l = G[3 * gk + ci];
        const T gtr_h = thi ? G[3 * gk + ct] : T(0);
        // r-flux, q = theta
        acc += q * grt_h * (xrptp + xtp - xrptm - xtm) - q * grt_l * (xtp + xrmtp - xtm - xrmtm);
        // theta-flux, q = r
        acc += q * gtr_h * (xrptp + xrp - xrmtp - xrm) - q * gtr_l * (xrp + xrptm - xrm - xrmtm);
        if constexpr (MODE == MODE_FULL) {
            const T xrmpm = X(i0 + ra + pa), xrmpp = X(i0 + ra + pb);
            const T xrppm = X(i0 + rb + pa), xrppp = X(i0 + rb + pb);
            const T xtmpm = X(i0 + ta + pa), xtmpp = X(i0 + ta + pb);
            const T xtppm = X(i0 + tb + pa), xtppp = X(i0 + tb + pb);
            const T grp_l = G[2 * gk + ci];
            const T grp_h = rhi ? G[2 * gk + cr] : T(0);
            const T gtp_l = G[5 * gk + ci];
            const T gtp_h = thi ? G[5 * gk + ct] : T(0);
            const T gpr_l = G[6 * gk + ci], gpr_h = G[6 * gk + cp];
            const T gpt_l = G[7 * gk + ci], gpt_h = G[7 * gk + cp];
            // r-flux, q = phi
            acc += q * grp_h * (xrppp + xpp - xrppm - xpm) - q * grp_l * (xpp + xrmpp - xpm - xrmpm);
            // theta-flux, q = phi
            acc += q * gtp_h * (xtppp + xpp - xtppm - xpm) - q * gtp_l * (xpp + xtmpp - xpm - xtmpm);
            // phi-flux, q = r
            acc += q * gpr_h * (xrppp + xrp - xrmpp - xrm) - q * gpr_l * (xrp + xrppm - xrm - xrmpm);
            // phi-flux, q = theta
            acc += q * gpt_h * (xtppp + xtp - xtmpp - xtm) - q * gpt_l * (xtp + xtppm - xtm - xtmpm);
        }
    }
    return acc;
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

// The sum of partial[0..n) in a fixed order, valid in thread 0 (one block;
// four independent accumulators per thread keep several loads in flight).
__device__ __forceinline__ double d_reduce_sum(const double* __restrict__ partial, long long n)
{
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    long long i = threadIdx.x;
    for (; i + 3 * kBlock < n; i += 4 * kBlock) {
        s0 += partial[i];
        s1 += partial[i + kBlock];
        s2 += partial[i + 2 * kBlock];
        s3 += partial[i + 3 * kBlock];
    }
    for (; i < n; i += kBlock) s0 += partial[i];
    return block_sum((s0 + s1) + (s2 + s3));
}

// *out = sum of partial[0..n)
__device__ __forceinline__ void d_reduce(Blk bk, const double* __restrict__ partial, long long n,
                                                   double* __restrict__ out)
{
    const double s = d_reduce_sum(partial, n);
    if (threadIdx.x == 0) *out = s;
}

// host != nullptr: the sum is also stored there (coherent pinned host
// memory, read by the host once the stream is synchronised), in place of a
// copy after the launch
__global__ void __launch_bounds__(kBlock) k_reduce(const double* __restrict__ partial, long long n,
                                                   double* __restrict__ out,
                                                   double* __restrict__ host)
{
    const double s = d_reduce_sum(partial, n);
    if (threadIdx.x == 0) {
        *out = s;
        if (host) *host = s;
    }
}

// Blocks of the stencil kernels walk a contiguous range of "units" (256
// consecutive positions of one r-plane): unit u covers plane a = u / bpa,
// positions m = (u mod bpa) * 256 + thread.  Grids are capped (kMaxGrid), so
// a block takes several units in order and each kernel leaves at most
// kMaxGrid partial sums.
constexpr int kMaxGrid = 4096;

template <typename F>
__device__ __forceinline__ void for_units(Blk bk, int rowlen, int bpa, long long nunits, F&& f)
{
    const long long L = bk.L, G = bk.G;
    const unsigned u0 = (unsigned)(nunits * L / G), u1 = (unsigned)(nunits * (L + 1) / G);
    for (unsigned u = u0; u < u1; ++u) {
        const unsigned a = u / (unsigned)bpa;
        const int m = (int)(u - a * (unsigned)bpa) * kBlock + (int)threadIdx.x;
        if (m < rowlen) f((int)a, m);
    }
}

// Row (theta index) of plane position m.  UROW: n_phi / 2 is a multiple of
// 64, so no wavefront straddles two rows; the row is then made
// wave-uniform, which turns the per-row metric loads of phi-invariant maps
// into scalar loads.
template <bool UROW>
__device__ __forceinline__ int row_of(int m, int nh)
{
    int b = m / nh;
    if constexpr (UROW) b = __builtin_amdgcn_readfirstlane(b);
    return b;
}

// ---------------------------------------------------------------------------
// Operator kernels.  One thread per (a, b, j): both parities of the pair.
// LTAG only tells the finest level (0) from the others (1) so that profiles
// can separate them; the code is the same.
// ---------------------------------------------------------------------------

// y = A x; with dotv, per-block partial sums of y . dotv
template <typename T, int MODE, bool AXI, bool UROW, int LTAG>
__device__ __forceinline__ void d_apply(Blk bk, Geo g, const T* __restrict__ G, long long gk,
                                                  int bpa, const T* __restrict__ x,
                                                  T* __restrict__ y, double* __restrict__ partial,
                                                  const T* __restrict__ dotv)
{
    double acc = 0.0;
    for_units(bk, g.rowlen, bpa, (long long)g.nr * bpa, [&](int a, int m) {
        const int b = row_of<UROW>(m, g.nh), j = m - b * g.nh;
        const long long i0 = (long long)a * g.rowlen + m;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            T D;
            const T v = apply_cell<T, MODE, AXI>(g, G, gk, Field<T>{x}, a, b, s, j, D);
            y[i0 + s * g.P] = v;
            if (dotv) acc += (double)v * (double)dotv[i0 + s * g.P];
        }
    });
    if (partial) {
        acc = block_sum(acc);
        if (threadIdx.x == 0) partial[bk.L] = acc;
    }
}

template <typename T, int MODE, bool AXI, bool UROW, int LTAG>
__global__ void __launch_bounds__(kBlock) k_apply(Geo g, const T* __restrict__ G, long long gk,
                                                  int bpa, const T* __restrict__ x,
                                                  T* __restrict__ y, double* __restrict__ partial,
                                                  const T* __restrict__ dotv)
{
    d_apply<T, MODE, AXI, UROW, LTAG>(self_blk(), g, G, gk, bpa, x, y, partial, dotv);
}

// r = b - A x; with partial, per-block partial sums of r^2
template <typename T, int MODE, bool AXI, bool UROW, int LTAG>
__device__ __forceinline__ void d_residual(Blk bk, Geo g, const T* __restrict__ G, long long gk,
                                                     int bpa, const T* __restrict__ bv,
                                                     const T* __restrict__ x, T* __restrict__ r,
                                                     double* __restrict__ partial)
{
    double acc = 0.0;
    for_units(bk, g.rowlen, bpa, (long long)g.nr * bpa, [&](int a, int m) {
        const int b = row_of<UROW>(m, g.nh), j = m - b * g.nh;
        const long long i0 = (long long)a * g.rowlen + m;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            T D;
            const long long i = i0 + s * g.P;
            const T v = bv[i] - apply_cell<T, MODE, AXI>(g, G, gk, Field<T>{x}, a, b, s, j, D);
            r[i] = v;
            acc += (double)v * (double)v;
        }
    });
    if (partial) {
        acc = block_sum(acc);
        if (threadIdx.x == 0) partial[bk.L] = acc;
    }
}

template <typename T, int MODE, bool AXI, bool UROW, int LTAG>
__global__ void __launch_bounds__(kBlock) k_residual(Geo g, const T* __restrict__ G, long long gk,
                                                     int bpa, const T* __restrict__ bv,
                                                     const T* __restrict__ x, T* __restrict__ r,
                                                     double* __restrict__ partial)
{
    d_residual<T, MODE, AXI, UROW, LTAG>(self_blk(), g, G, gk, bpa, bv, x, r, partial);
}

// One Gauss-Seidel pass over the cells of one colour, in place:
// x_c = (b_c - S_c) / D_c with S_c the neighbour sum of (A x)_c (the same
// value as x_c + (b_c - (A x)_c) / D_c).  Two colours: (a+b+c) mod 2; four
// colours: k = 2((a+c) mod 2) + ((b+c) mod 2).  Cells of one colour never
// read one another, so all threads of the pass update concurrently.
// Two colours: one thread per (a, b, j), the cell of the colour is in plane
// (k + a + b) mod 2.  Four colours: the colour occupies every other theta
// row (b = (k0 + k1 + a) mod 2 + 2 bh) in plane (k1 + a) mod 2.
// zero != 0 (two colours only): first pass from a zero iterate, the other
// colour is neither read nor needed.
template <typename T, int MODE, bool AXI, bool UROW, int LTAG>
__device__ __forceinline__ void d_gs(Blk bk, Geo g, const T* __restrict__ G, long long gk,
                                               int bpa, const T* __restrict__ bv,
                                               T* __restrict__ x, int colour, int ncol, int zero)
{
    const int rowlen = ncol == 2 ? g.rowlen : g.rowlen / 2;
    for_units(bk, rowlen, bpa, (long long)g.nr * bpa, [&](int a, int m) {
        const int bb = row_of<UROW>(m, g.nh), j = m - bb * g.nh;
        int b, s;
        if (ncol == 2) {
            b = bb;
            s = (colour + a + b) & 1;
        } else {
            const int k1 = colour >> 1, k0 = colour & 1;
            b = 2 * bb + ((k0 + k1 + a) & 1);
            s = (k1 + a) & 1;
        }
        T D;
        const T S = zero ? apply_cell<T, MODE, AXI, true>(g, G, gk, Delta<T>{-1}, a, b, s, j, D)
                         : apply_cell<T, MODE, AXI, true>(g, G, gk, Field<T>{x}, a, b, s, j, D);
        const long long id = s * g.P + ((long long)a * g.nt + b) * g.nh + j;
        x[id] = (bv[id] - S) / D;
    });
}

template <typename T, int MODE, bool AXI, bool UROW, int LTAG>
__global__ void __launch_bounds__(kBlock) k_gs(Geo g, const T* __restrict__ G, long long gk,
                                               int bpa, const T* __restrict__ bv,
                                               T* __restrict__ x, int colour, int ncol, int zero)
{
    d_gs<T, MODE, AXI, UROW, LTAG>(self_blk(), g, G, gk, bpa, bv, x, colour, ncol, zero);
}

// ---------------------------------------------------------------------------
// Marching (2.5-D) kernels for the 7-point stencil with phi-invariant
// metrics.  A block owns 256 consecutive positions (theta row, j) of a plane
// and walks r over a chunk of planes; each thread keeps the values of its
// own column at a-1, a, a+1 in registers, so every r-neighbour is read from
// memory once.  theta and phi neighbours come from the plane being swept by
// all blocks of the chunk at the same time (L2 hits).  With blocks laid out
// chunk-major and XCD-contiguous, each XCD sweeps its own chunk.
// Launch: grid = bpa * nchunks, chunk of `ch` planes.  Neighbour values
// past a wall are replaced by the cell's own value: they are multiplied by
// a zero wall metric.
// ---------------------------------------------------------------------------

struct March {
    int unit, a0, a1, m, b, j;
};

template <bool UROW>
__device__ __forceinline__ bool march_pos(Blk bk, const Geo& g, int bpa, int ch, March& p)
{
    const int L = (int)bk.L;
    const int chunk = L / bpa;
    p.unit = L - chunk * bpa;
    p.m = p.unit * kBlock + (int)threadIdx.x;
    p.a0 = chunk * ch;
    p.a1 = min(g.nr, p.a0 + ch);
    if (p.m >= g.rowlen || p.a0 >= g.nr) return false;
    p.b = row_of<UROW>(p.m, g.nh);
    p.j = p.m - p.b * g.nh;
    return true;
}

// Planes a marching thread loads ahead: the loads of kAhead planes are
// issued together before any of them is used, so each wavefront keeps
// several memory requests in flight (one plane at a time leaves the kernels
// bound by memory latency, not bandwidth).
// The colour pass loads 5 values per plane, the two-cell residual and
// product kernels 10: they go 2 planes ahead to stay at high occupancy.
constexpr int kAhead = 4;
constexpr int kAhead2 = 2;

// Red-black Gauss-Seidel pass (colour k): at plane a the cell of column
// (b, j) with colour k sits in plane p = (k + a + b) mod 2 and its black
// neighbours are: the column's own cells at a-1, a+1 (plane p) and at a
// (plane 1-p), the cells at (a, b+-1) in plane p, and one phi neighbour in
// plane 1-p of the adjacent column.  A pass writes only cells of colour k
// and reads only the other colour, so loads may run ahead of the stores.
// zero != 0: first pass from a zero iterate (the other colour is taken as 0
// and not read; it need not be initialised), x = b / D.

template <typename T, int AHEAD>
__device__ __forceinline__ void gs_march_body(const Geo& g, const T* __restrict__ G, long long gk,
                                              const March& p, const T* __restrict__ bv,
                                              T* __restrict__ x, int colour, int zero, double& acc)
{
    const int b = p.b;
    const bool thi = b < g.nt - 1;
    // metrics of the column at plane a: D and the five face values
    auto diag = [&](int a, T& grl, T& grh, T& gtl, T& gth, T& gpp) {
        const long long ci = (long long)a * g.nt + b;
        grl = G[ci];
        grh = a < g.nr - 1 ? G[ci + g.nt] : T(0);
        gtl = G[4 * gk + ci];
        gth = thi ? G[4 * gk + ci + 1] : T(0);
        gpp = G[8 * gk + ci];
    };
    if (zero) {
        for (int a = p.a0; a < p.a1; a += AHEAD) {
            T bb[AHEAD];
#pragma unroll
            for (int u = 0; u < AHEAD; ++u)
                if (a + u < p.a1)
                    bb[u] = bv[((colour + a + u + b) & 1) * g.P + (long long)(a + u) * g.rowlen + p.m];
#pragma unroll
            for (int u = 0; u < AHEAD; ++u)
                if (a + u < p.a1) {
                    T grl, grh, gtl, gth, gpp;
                    diag(a + u, grl, grh, gtl, gth, gpp);
                    const T D = -(grl + grh + gtl + gth + T(2) * gpp);
                    x[((colour + a + u + b) & 1) * g.P + (long long)(a + u) * g.rowlen + p.m] =
                        bb[u] / D;
                }
        }
        return;
    }
    const long long sr = g.rowlen;
    const int nh = g.nh, j = p.j;
    const bool tlo = b > 0;
    // the other-colour cell of this column at plane a
    auto other = [&](int a) -> T {
        if (a < 0 || a >= g.nr) return T(0);
        const int q = (colour + a + b + 1) & 1;
        return x[q * g.P + (long long)a * sr + p.m];
    };
    T om = other(p.a0 - 1), o0 = other(p.a0);
    const int jn0 = j == 0 ? nh - 1 : j - 1, jn1 = j == nh - 1 ? 0 : j + 1;
    for (int a = p.a0; a < p.a1; a += AHEAD) {
        T op[AHEAD], tm[AHEAD], tp[AHEAD], on[AHEAD], bb[AHEAD];
#pragma unroll
        for (int u = 0; u < AHEAD; ++u) {
            const int aa = a + u;
            if (aa < p.a1) {
                const int s = (colour + aa + b) & 1;
                const long long base = (long long)aa * sr + p.m; // (a, b, j) within a plane
                const T* xs = x + s * g.P;
                op[u] = other(aa + 1);
                tm[u] = tlo ? xs[base - nh] : T(0);
                tp[u] = thi ? xs[base + nh] : T(0);
                // phi: plane 1-s holds c-1 and c+1; o0 is the one at index j
                on[u] = x[(1 - s) * g.P + base - j + (s == 0 ? jn0 : jn1)];
                bb[u] = bv[s * g.P + base];
            }
        }
#pragma unroll
        for (int u = 0; u < AHEAD; ++u) {
            const int aa = a + u;
            if (aa < p.a1) {
                T grl, grh, gtl, gth, gpp;
                diag(aa, grl, grh, gtl, gth, gpp);
                const T D = -(grl + grh + gtl + gth + gpp + gpp);
                const T S = grh * op[u] + grl * om + gth * tp[u] + gtl * tm[u] + gpp * (o0 + on[u]);
                const int s = (colour + aa + b) & 1;
                const T xn = (bb[u] - S) / D;
                x[s * g.P + (long long)aa * sr + p.m] = xn;
                acc += (double)bb[u] * (double)xn;
                om = o0;
                o0 = op[u];
            }
        }
    }
}

// dot != nullptr (non-zero passes): per-block partial sums of b_c x_c over
// the cells the pass updates, with their new values.  The last two passes
// of a sweep update every cell once more and leave it final, so their sums
// give b . x for the smoothed iterate without another pass over memory.
template <typename T, bool UROW, int LTAG, int AHEAD = kAhead>
__device__ __forceinline__ void d_gs_march(Blk bk, Geo g, const T* __restrict__ G, long long gk,
                                                     int bpa, int ch, const T* __restrict__ bv,
                                                     T* __restrict__ x, int colour, int zero,
                                                     double* __restrict__ dot = nullptr)
{
    March p;
    double acc = 0.0;
    if (march_pos<UROW>(bk, g, bpa, ch, p)) gs_march_body<T, AHEAD>(g, G, gk, p, bv, x, colour, zero, acc);
    if (dot) {
        acc = block_sum(acc);
        if (threadIdx.x == 0) dot[bk.L] = acc;
    }
}

template <typename T, bool UROW, int LTAG, int ZERO>
__global__ void __launch_bounds__(kBlock) k_gs_march(Geo g, const T* __restrict__ G, long long gk,
                                                     int bpa, int ch, const T* __restrict__ bv,
                                                     T* __restrict__ x, int colour,
                                                     double* __restrict__ dot)
{
    d_gs_march<T, UROW, LTAG>(self_blk(), g, G, gk, bpa, ch, bv, x, colour, ZERO, dot);
}


// Values a marching thread needs at plane a for the two cells (a, b, 2j)
// and (a, b, 2j+1) besides the column at a-1 and a: the column at a+1, the
// theta neighbours of both cells and their phi neighbours in the other
// plane.  A read past an r- or theta-wall takes the cell itself (its flux
// difference is then 0 and the zero wall metric multiplies it).
template <typename T>
struct Nb2 {
    T up, vp, utm, utp, vtm, vtp, vjm, ujp;
};

template <typename T>
__device__ __forceinline__ void march_load2(const Geo& g, const T* __restrict__ x, int a, int b,
                                            int j, long long base, Nb2<T>& n)
{
    const int nh = g.nh;
    const long long ab = a < g.nr - 1 ? base + g.rowlen : base;
    const long long tl = b > 0 ? base - nh : base, th = b < g.nt - 1 ? base + nh : base;
    n.up = x[ab];
    n.vp = x[g.P + ab];
    n.utm = x[tl];
    n.utp = x[th];
    n.vtm = x[g.P + tl];
    n.vtp = x[g.P + th];
    // plane 0 cell c = 2j: phi neighbours c-1 = (1, j-1), c+1 = (1, j);
    // plane 1 cell c = 2j+1: c-1 = (0, j), c+1 = (0, j+1)
    n.vjm = x[g.P + base - j + (j == 0 ? nh - 1 : j - 1)];
    n.ujp = x[base - j + (j == nh - 1 ? 0 : j + 1)];
}

// Flux-form (A x) of the two cells given the column values at a-1, a
// (u = plane 0, v = plane 1) and the neighbours n.
template <typename T>
__device__ __forceinline__ void march_apply2(const Geo& g, const T* __restrict__ G, long long gk,
                                             int a, int b, T um, T u0, T vm, T v0, const Nb2<T>& n,
                                             T& y0, T& y1)
{
    const long long ci = (long long)a * g.nt + b;
    const T grl = G[ci];
    const T grh = a < g.nr - 1 ? G[ci + g.nt] : T(0);
    const T gtl = G[4 * gk + ci];
    const T gth = b < g.nt - 1 ? G[4 * gk + ci + 1] : T(0);
    const T gpp = G[8 * gk + ci];
    y0 = grh * (n.up - u0) - grl * (u0 - um) + gth * (n.utp - u0) - gtl * (u0 - n.utm) +
         gpp * (v0 - u0) - gpp * (u0 - n.vjm);
    y1 = grh * (n.vp - v0) - grl * (v0 - vm) + gth * (n.vtp - v0) - gtl * (v0 - n.vtm) +
         gpp * (n.ujp - v0) - gpp * (v0 - u0);
}

// First column values of a marching thread: (um, u0, vm, v0) at a0-1, a0,
// with the cell itself past the low r-wall.
template <typename T>
__device__ __forceinline__ void march_start(const Geo& g, const T* __restrict__ x, const March& p,
                                            T& um, T& u0, T& vm, T& v0)
{
    const long long base = (long long)p.a0 * g.rowlen + p.m;
    const long long bm = p.a0 > 0 ? base - g.rowlen : base;
    u0 = x[base];
    v0 = x[g.P + base];
    um = x[bm];
    vm = x[g.P + bm];
}

// r = b - A x (and partial sums of r^2), marching.
template <typename T, bool UROW, int LTAG>
__device__ __forceinline__ void d_residual_march(Blk bk, Geo g, const T* __restrict__ G,
                                                           long long gk, int bpa, int ch,
                                                           const T* __restrict__ bv,
                                                           const T* __restrict__ x,
                                                           T* __restrict__ r,
                                                           double* __restrict__ partial)
{
    March p;
    double acc = 0.0;
    if (march_pos<UROW>(bk, g, bpa, ch, p)) {
        T um, u0, vm, v0;
        march_start<T>(g, x, p, um, u0, vm, v0);
        for (int a = p.a0; a < p.a1; a += kAhead2) {
            Nb2<T> nb[kAhead2];
            T b0[kAhead2], b1[kAhead2];
#pragma unroll
            for (int u = 0; u < kAhead2; ++u)
                if (a + u < p.a1) {
                    const long long base = (long long)(a + u) * g.rowlen + p.m;
                    march_load2<T>(g, x, a + u, p.b, p.j, base, nb[u]);
                    b0[u] = bv[base];
                    b1[u] = bv[g.P + base];
                }
#pragma unroll
            for (int u = 0; u < kAhead2; ++u)
                if (a + u < p.a1) {
                    const long long base = (long long)(a + u) * g.rowlen + p.m;
                    T y0, y1;
                    march_apply2<T>(g, G, gk, a + u, p.b, um, u0, vm, v0, nb[u], y0, y1);
                    const T r0 = b0[u] - y0, r1 = b1[u] - y1;
                    r[base] = r0;
                    r[g.P + base] = r1;
                    acc += (double)r0 * (double)r0 + (double)r1 * (double)r1;
                    um = u0; u0 = nb[u].up; vm = v0; v0 = nb[u].vp;
                }
        }
    }
    if (partial) {
        acc = block_sum(acc);
        if (threadIdx.x == 0) partial[bk.L] = acc;
    }
}

template <typename T, bool UROW, int LTAG>
__global__ void __launch_bounds__(kBlock) k_residual_march(Geo g, const T* __restrict__ G,
                                                           long long gk, int bpa, int ch,
                                                           const T* __restrict__ bv,
                                                           const T* __restrict__ x,
                                                           T* __restrict__ r,
                                                           double* __restrict__ partial)
{
    d_residual_march<T, UROW, LTAG>(self_blk(), g, G, gk, bpa, ch, bv, x, r, partial);
}

// y = A x (and partial sums of y . dotv), marching.
template <typename T, bool UROW, int LTAG>
__device__ __forceinline__ void d_apply_march(Blk bk, Geo g, const T* __restrict__ G,
                                                        long long gk, int bpa, int ch,
                                                        const T* __restrict__ x,
                                                        T* __restrict__ y,
                                                        double* __restrict__ partial,
                                                        const T* __restrict__ dotv)
{
    March p;
    double acc = 0.0;
    if (march_pos<UROW>(bk, g, bpa, ch, p)) {
        T um, u0, vm, v0;
        march_start<T>(g, x, p, um, u0, vm, v0);
        for (int a = p.a0; a < p.a1; a += kAhead2) {
            Nb2<T> nb[kAhead2];
            T d0[kAhead2], d1[kAhead2];
#pragma unroll
            for (int u = 0; u < kAhead2; ++u)
                if (a + u < p.a1) {
                    const long long base = (long long)(a + u) * g.rowlen + p.m;
                    march_load2<T>(g, x, a + u, p.b, p.j, base, nb[u]);
                    if (dotv) {
                        d0[u] = dotv[base];
                        d1[u] = dotv[g.P + base];
                    }
                }
#pragma unroll
            for (int u = 0; u < kAhead2; ++u)
                if (a + u < p.a1) {
                    const long long base = (long long)(a + u) * g.rowlen + p.m;
                    T y0, y1;
                    march_apply2<T>(g, G, gk, a + u, p.b, um, u0, vm, v0, nb[u], y0, y1);
                    y[base] = y0;
                    y[g.P + base] = y1;
                    if (dotv) acc += (double)y0 * (double)d0[u] + (double)y1 * (double)d1[u];
                    um = u0; u0 = nb[u].up; vm = v0; v0 = nb[u].vp;
                }
        }
    }
    if (partial) {
        acc = block_sum(acc);
        if (threadIdx.x == 0) partial[bk.L] = acc;
    }
}

template <typename T, bool UROW, int LTAG>
__global__ void __launch_bounds__(kBlock) k_apply_march(Geo g, const T* __restrict__ G,
                                                        long long gk, int bpa, int ch,
                                                        const T* __restrict__ x,
                                                        T* __restrict__ y,
                                                        double* __restrict__ partial,
                                                        const T* __restrict__ dotv)
{
    d_apply_march<T, UROW, LTAG>(self_blk(), g, G, gk, bpa, ch, x, y, partial, dotv);
}

// ---------------------------------------------------------------------------
// Row-pair marching kernels (7-point, phi-invariant metrics; levels whose
// n_phi / 2 is a multiple of 64 and whose n_theta is even).  A thread owns
// the columns (b0 = 2 bp, j) and (b1 = b0 + 1, j) and marches over a chunk
// of r-planes like the kernels above.  The theta neighbour between its two
// rows is the other row's value, already in registers, and a wavefront
// covers 64 consecutive j of one row pair, so phi neighbours are the
// adjacent lanes' values (lane shuffles; with n_phi / 2 = 64 the wavefront
// is the whole ring).  Besides the streamed column values only the rows
// just outside the pair and, for longer rings, the phi neighbours past the
// wavefront's ends are loaded.  Launch: grid = bpa * nchunks with bpa
// blocks over the (n_theta / 2) * (n_phi / 2) row-pair positions.
// ---------------------------------------------------------------------------

__host__ __device__ inline bool row_pairs(const Geo& g) { return g.nh % 64 == 0 && g.nt % 2 == 0; }

struct March2 {
    int a0, a1, b0, j, lane;
    long long r0; // offset of (b0, j) within a plane
    bool ring;    // the wavefront holds the whole phi ring of its rows
};

// A block is kPairs adjacent row pairs x one 64-wide segment of phi (one
// wavefront per pair), so the rows just outside a pair are mostly the
// neighbouring wavefronts' own rows, read on the same CU at about the same
// time.  Units of a plane: cdiv(n_theta / 2, kPairs) pair groups x
// (n_phi / 128) segments.
constexpr int kPairs = kBlock / 64;

__device__ __forceinline__ bool march2_pos(Blk bk, const Geo& g, int bpa, int ch, March2& p)
{
    const int L = (int)bk.L;
    const int chunk = L / bpa;
    const int unit = L - chunk * bpa;
    const int segs = g.nh >> 6;
    const int pg = unit / segs, seg = unit - pg * segs;
    const int bp = pg * kPairs + __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    p.a0 = chunk * ch;
    p.a1 = min(g.nr, p.a0 + ch);
    p.b0 = p.j = p.lane = 0; // defined for the wavefronts that drop out too
    p.r0 = 0;
    p.ring = false;
    // pairs past the last one: whole wavefronts drop out
    if (bp >= (g.nt >> 1) || p.a0 >= g.nr) return false;
    p.b0 = 2 * bp;
    p.lane = (int)threadIdx.x & 63;
    p.j = seg * 64 + p.lane;
    p.r0 = (long long)p.b0 * g.nh + p.j;
    p.ring = g.nh == 64;
    return true;
}

// Red-black colour pass over row pairs (stencil and colouring of
// d_gs_march).  At plane a the cells of colour k of row b sit in plane
// s_b = (k + a + b) mod 2 and the other colour of the column in 1 - s_b; for
// the two rows s_b1 = 1 - s_b0, so each row's theta neighbour across the
// pair is the other row's column value.  zero != 0: first pass from a zero
// iterate, x = b / D.
template <typename T, int AHEAD>
__device__ __forceinline__ void gs_march2_body(const Geo& g, const T* __restrict__ G, long long gk,
                                               const March2& p, bool live,
                                               const T* __restrict__ bv, T* __restrict__ x,
                                               int colour, int zero, double& acc)
{
    // full FP64 passes: the other-colour values of the rows next to a pair
    // (its theta neighbours) are the adjacent wavefronts' own column values;
    // they come through LDS (double-buffered, one barrier per AHEAD planes)
    // and only the block's outermost rows are read from memory.  Every
    // wavefront of a block with planes stays in the loop for the barriers.
    // FP32 passes read those rows themselves: with half the bytes per plane
    // the barrier costs more than the loads it saves (38.5 against 37.1 us).
    constexpr bool kLds = sizeof(T) == 8;
    __shared__ T sh[kLds ? 2 : 1][AHEAD][kPairs][2][64];
    if (p.a0 >= g.nr || (zero && !live)) return; // block-uniform / no barriers
    const int w = (int)threadIdx.x >> 6;
    const long long sr = g.rowlen, r0 = p.r0, r1 = p.r0 + g.nh;
    const int b0 = p.b0, b1 = b0 + 1, nh = g.nh, j = p.j, lane = p.lane;
    const bool tlo = b0 > 0, thi = b1 < g.nt - 1;
    // metrics of rows b0, b1 at plane a
    auto metrics = [&](int a, T* m0, T* m1) {
        const long long ci = (long long)a * g.nt + b0;
        const bool rh = a < g.nr - 1;
        m0[0] = G[ci];
        m0[1] = rh ? G[ci + g.nt] : T(0);
        m0[2] = G[4 * gk + ci];
        m0[3] = G[4 * gk + ci + 1];
        m0[4] = G[8 * gk + ci];
        m1[0] = G[ci + 1];
        m1[1] = rh ? G[ci + 1 + g.nt] : T(0);
        m1[2] = G[4 * gk + ci + 1];
        m1[3] = thi ? G[4 * gk + ci + 2] : T(0);
        m1[4] = G[8 * gk + ci + 1];
    };
    if (zero) {
        for (int a = p.a0; a < p.a1; a += AHEAD) {
            T q0[AHEAD], q1[AHEAD];
#pragma unroll
            for (int u = 0; u < AHEAD; ++u)
                if (a + u < p.a1) {
                    const int s0 = (colour + a + u + b0) & 1;
                    const long long base = (long long)(a + u) * sr;
                    q0[u] = bv[s0 * g.P + base + r0];
                    q1[u] = bv[(1 - s0) * g.P + base + r1];
                }
#pragma unroll
            for (int u = 0; u < AHEAD; ++u)
                if (a + u < p.a1) {
                    const int s0 = (colour + a + u + b0) & 1;
                    const long long base = (long long)(a + u) * sr;
                    T m0[5], m1[5];
                    metrics(a + u, m0, m1);
                    const T D0 = -(m0[0] + m0[1] + m0[2] + m0[3] + T(2) * m0[4]);
                    const T D1 = -(m1[0] + m1[1] + m1[2] + m1[3] + T(2) * m1[4]);
                    x[s0 * g.P + base + r0] = q0[u] / D0;
                    x[(1 - s0) * g.P + base + r1] = q1[u] / D1;
                }
        }
        return;
    }
    const int jlo = j == 0 ? nh - 1 : j - 1, jhi = j == nh - 1 ? 0 : j + 1;
    // the other-colour cell of row b's column at plane a (0 past the r-walls)
    auto col = [&](int a, int b, long long r) -> T {
        if (a < 0 || a >= g.nr) return T(0);
        return x[((colour + a + b + 1) & 1) * g.P + (long long)a * sr + r];
    };
    // a row whose updated cells are in plane s needs the other colour at
    // j - 1 (s = 0) or j + 1 (s = 1): loaded at the wavefront's ends
    auto edge = [&](int s) { return !p.ring && (s == 0 ? lane == 0 : lane == 63); };
    T m0 = T(0), c0 = T(0), m1 = T(0), c1 = T(0);
    if (live) {
        m0 = col(p.a0 - 1, b0, r0);
        c0 = col(p.a0, b0, r0);
        m1 = col(p.a0 - 1, b1, r1);
        c1 = col(p.a0, b1, r1);
    }
    for (int a = p.a0, buf = 0; a < p.a1; a += AHEAD, buf ^= 1) {
        T p0[AHEAD], p1[AHEAD], q0[AHEAD], q1[AHEAD], tm0[AHEAD], tp1[AHEAD], e0[AHEAD], e1[AHEAD];
        if (live) {
#pragma unroll
            for (int u = 0; u < AHEAD; ++u) {
                const int aa = a + u;
                if (aa < p.a1) {
                    const int s0 = (colour + aa + b0) & 1, s1 = 1 - s0;
                    const long long base = (long long)aa * sr;
                    p0[u] = col(aa + 1, b0, r0);
                    p1[u] = col(aa + 1, b1, r1);
                    q0[u] = ld_once(bv + s0 * g.P + base + r0);
                    q1[u] = ld_once(bv + s1 * g.P + base + r1);
                    tm0[u] = ((!kLds || w == 0) && tlo) ? x[s0 * g.P + base + r0 - nh] : T(0);
                    tp1[u] = ((!kLds || w == kPairs - 1) && thi) ? x[s1 * g.P + base + r1 + nh]
                                                                   : T(0);
                    e0[u] = edge(s0) ? x[s1 * g.P + base + r0 - j + (s0 == 0 ? jlo : jhi)] : T(0);
                    e1[u] = edge(s1) ? x[s0 * g.P + base + r1 - j + (s1 == 0 ? jlo : jhi)] : T(0);
                }
            }
            // this pair's other-colour values at planes a .. a + AHEAD - 1:
            // row b0's is the theta neighbour of the pair below's row b1,
            // row b1's that of the pair above's row b0
            if constexpr (kLds) {
#pragma unroll
                for (int u = 0; u < AHEAD; ++u) {
                    sh[buf][u][w][0][lane] = u == 0 ? c0 : p0[u - 1];
                    sh[buf][u][w][1][lane] = u == 0 ? c1 : p1[u - 1];
                }
            }
        }
        if constexpr (kLds) __syncthreads();
        if (!live) continue;
        // a neighbour row exists only where its pair (and wavefront) does
        if constexpr (kLds) {
#pragma unroll
            for (int u = 0; u < AHEAD; ++u) {
                if (w > 0 && tlo) tm0[u] = sh[buf][u][w - 1][1][lane];
                if (w < kPairs - 1 && thi) tp1[u] = sh[buf][u][w + 1][0][lane];
            }
        }
#pragma unroll
        for (int u = 0; u < AHEAD; ++u) {
            const int aa = a + u;
            if (aa < p.a1) {
                const int s0 = (colour + aa + b0) & 1, s1 = 1 - s0;
                const T n0 = __shfl(c0, s0 == 0 ? lane - 1 : lane + 1);
                const T n1 = __shfl(c1, s1 == 0 ? lane - 1 : lane + 1);
                const T on0 = edge(s0) ? e0[u] : n0;
                const T on1 = edge(s1) ? e1[u] : n1;
                T g0[5], g1[5];
                metrics(aa, g0, g1);
                // g[]: r low, r high, theta low, theta high, phi (both faces)
                const T D0 = -(g0[0] + g0[1] + g0[2] + g0[3] + g0[4] + g0[4]);
                const T D1 = -(g1[0] + g1[1] + g1[2] + g1[3] + g1[4] + g1[4]);
                const T S0 = g0[1] * p0[u] + g0[0] * m0 + g0[3] * c1 + g0[2] * tm0[u] +
                             g0[4] * (c0 + on0);
                const T S1 = g1[1] * p1[u] + g1[0] * m1 + g1[3] * tp1[u] + g1[2] * c0 +
                             g1[4] * (c1 + on1);
                const long long base = (long long)aa * sr;
                const T x0n = (q0[u] - S0) / D0, x1n = (q1[u] - S1) / D1;
                st_once(x + s0 * g.P + base + r0, x0n);
                st_once(x + s1 * g.P + base + r1, x1n);
                acc += (double)q0[u] * (double)x0n + (double)q1[u] * (double)x1n;
                m0 = c0;
                c0 = p0[u];
                m1 = c1;
                c1 = p1[u];
            }
        }
    }
}

// dot: as for d_gs_march.
template <typename T, int LTAG, int AHEAD = 2>
__device__ __forceinline__ void d_gs_march2(Blk bk, Geo g, const T* __restrict__ G, long long gk,
                                                      int bpa, int ch, const T* __restrict__ bv,
                                                      T* __restrict__ x, int colour, int zero,
                                                      double* __restrict__ dot = nullptr)
{
    March2 p;
    double acc = 0.0;
    const bool live = march2_pos(bk, g, bpa, ch, p);
    gs_march2_body<T, AHEAD>(g, G, gk, p, live, bv, x, colour, zero, acc);
    if (dot) {
        acc = block_sum(acc);
        if (threadIdx.x == 0) dot[bk.L] = acc;
    }
}

// ZERO: the zero-iterate first pass, a kernel of its own so that profiles
// keep it apart from the full passes.
template <typename T, int LTAG, int ZERO>
__global__ void __launch_bounds__(kBlock) k_gs_march2(Geo g, const T* __restrict__ G, long long gk,
                                                      int bpa, int ch, const T* __restrict__ bv,
                                                      T* __restrict__ x, int colour,
                                                      double* __restrict__ dot)
{
    d_gs_march2<T, LTAG>(self_blk(), g, G, gk, bpa, ch, bv, x, colour, ZERO, dot);
}

// Column values of a row-pair thread at one plane: u = plane 0, v = plane 1
// of rows b0 (suffix 0) and b1 (suffix 1).
template <typename T>
struct Col4 {
    T u0, v0, u1, v1;
};

// Values a row-pair thread loads at plane a for (A x) of its four cells:
// the columns at a+1 (the cell itself past the high r-wall), the theta
// neighbours outside the pair (the cell itself past a theta-wall) and the
// phi neighbours past the wavefront's ends (only lanes 0 and 63 of long
// rings read them).
template <typename T>
struct Nb4 {
    Col4<T> up;
    T utm0, vtm0, utp1, vtp1;
    T vjm0, vjm1, ujp0, ujp1;
};

// Element access of the field a row-pair stencil kernel reads: a plain
// array, or the search direction p = z + beta p_old formed where it is read.
template <typename T>
struct Plain {
    const T* __restrict__ x;
    __device__ __forceinline__ T operator()(long long i) const { return x[i]; }
};
// Where two paths must form bit-identical values (a single solve and the
// batched form), the products that feed a sum are written as explicit fmas
// and a product that must round on its own goes through mul_t: whether the
// compiler contracts a * b + c otherwise depends on the surrounding code.
__device__ __forceinline__ double fma_t(double a, double b, double c)
{
    return __builtin_fma(a, b, c);
}
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <typename T>
__device__ __forceinline__ T mul_t(T a, T b)
{
#pragma clang fp contract(off)
    return a * b;
}

// The search direction p = z + beta p_old is one fma wherever it is formed
// (here, in d_cg_dir and in the batched form), so all paths round alike.
template <typename T>
struct Dir {
    const T* __restrict__ z;
    const T* __restrict__ p;
    T beta;
    __device__ __forceinline__ T operator()(long long i) const
    {
        return __builtin_fma(beta, p[i], z[i]);
    }
    // the same from p_old[i] already in a register
    __device__ __forceinline__ T from(T pold, long long i) const
    {
        return __builtin_fma(beta, pold, z[i]);
    }
};
// The same with z the FP32 correction of the mixed form, cast as k_cast_dots
// casts it (z = (double) e * s, rounded before the direction is formed).
struct DirCast {
    const float* __restrict__ e;
    double s;
    const double* __restrict__ p;
    double beta;
    __device__ __forceinline__ double operator()(long long i) const
    {
        return __builtin_fma(beta, p[i], mul_t((double)e[i], s));
    }
    __device__ __forceinline__ double from(double pold, long long i) const
    {
        return __builtin_fma(beta, pold, mul_t((double)e[i], s));
    }
};

// below / above: load the theta row below / above the pair (a caller that
// has them from the adjacent wavefronts passes false); up == false: the
// column at a + 1 is the caller's.
template <typename T, typename X>
__device__ __forceinline__ void march2_load(const Geo& g, const X& x, const March2& p, int a,
                                            Nb4<T>& n, bool below = true, bool above = true,
                                            bool up = true)
{
    const int nh = g.nh, j = p.j;
    const long long base = (long long)a * g.rowlen + p.r0;
    const long long ab = a < g.nr - 1 ? base + g.rowlen : base;
    if (up) {
        n.up.u0 = x(ab);
        n.up.v0 = x(g.P + ab);
        n.up.u1 = x(ab + nh);
        n.up.v1 = x(g.P + ab + nh);
    }
    if (below) {
        const long long tl = p.b0 > 0 ? base - nh : base;
        n.utm0 = x(tl);
        n.vtm0 = x(g.P + tl);
    }
    if (above) {
        const long long th = p.b0 + 1 < g.nt - 1 ? base + 2 * nh : base + nh;
        n.utp1 = x(th);
        n.vtp1 = x(g.P + th);
    }
    if (!p.ring && p.lane == 0) {
        const long long jm = base - j + (j == 0 ? nh - 1 : j - 1);
        n.vjm0 = x(g.P + jm);
        n.vjm1 = x(g.P + jm + nh);
    }
    if (!p.ring && p.lane == 63) {
        const long long jp = base - j + (j == nh - 1 ? 0 : j + 1);
        n.ujp0 = x(jp);
        n.ujp1 = x(jp + nh);
    }
}

// Flux-form (A x) of one plane-0 cell (phi index 2j) of a row: its column
// values at a-1 (um), a (u), a+1 (up), its theta neighbours below (utm) and
// above (utp), and its phi neighbours v (plane 1, j) and vjm (plane 1, j-1);
// metrics r low/high (grl, grh), theta low/high (gtl, gth), phi (gpp).  The
// sum is an explicit fma chain, so every kernel that forms it rounds alike.
template <typename T>
__device__ __forceinline__ T cell_apply_e(T grl, T grh, T gtl, T gth, T gpp, T um, T u, T up,
                                          T utm, T utp, T v, T vjm)
{
    T s = mul_t(grh, up - u);
    s = fma_t(-grl, u - um, s);
    s = fma_t(gth, utp - u, s);
    s = fma_t(-gtl, u - utm, s);
    s = fma_t(gpp, v - u, s);
    return fma_t(-gpp, u - vjm, s);
}
// The same for a plane-1 cell (phi index 2j + 1): its phi neighbours are
// ujp (plane 0, j + 1) and u (plane 0, j).
template <typename T>
__device__ __forceinline__ T cell_apply_o(T grl, T grh, T gtl, T gth, T gpp, T vm, T v, T vp,
                                          T vtm, T vtp, T ujp, T u)
{
    T s = mul_t(grh, vp - v);
    s = fma_t(-grl, v - vm, s);
    s = fma_t(gth, vtp - v, s);
    s = fma_t(-gtl, v - vtm, s);
    s = fma_t(gpp, ujp - v, s);
    return fma_t(-gpp, v - u, s);
}

// Flux-form (A x) of one row's two cells (plane 0 cell 2j, plane 1 cell
// 2j+1) from the row's column values at a-1 (um, vm), a (u, v), a+1 (up,
// vp), its theta neighbours below (utm, vtm) and above (utp, vtp), and the
// phi neighbours vjm (plane 1, j-1) and ujp (plane 0, j+1); the sums are
// those of march_apply2.
template <typename T>
__device__ __forceinline__ void row_apply(const T* __restrict__ G, long long gk, long long ci,
                                          bool rh, bool th, long long nt, T um, T u, T up, T vm,
                                          T v, T vp, T utm, T utp, T vtm, T vtp, T vjm, T ujp,
                                          T& y0, T& y1)
{
    const T grl = G[ci];
    const T grh = rh ? G[ci + nt] : T(0);
    const T gtl = G[4 * gk + ci];
    const T gth = th ? G[4 * gk + ci + 1] : T(0);
    const T gpp = G[8 * gk + ci];
    y0 = cell_apply_e(grl, grh, gtl, gth, gpp, um, u, up, utm, utp, v, vjm);
    y1 = cell_apply_o(grl, grh, gtl, gth, gpp, vm, v, vp, vtm, vtp, ujp, u);
}

// (A x) of the four cells of a row-pair thread at plane a.
template <typename T>
__device__ __forceinline__ void march2_apply(const Geo& g, const T* __restrict__ G, long long gk,
                                             const March2& p, int a, const Col4<T>& cm,
                                             const Col4<T>& c, const Nb4<T>& n, T y[4])
{
    const int lane = p.lane;
    // phi neighbours inside the wavefront come from the adjacent lanes (the
    // shuffles run on every lane; the ends of a long ring take the loads)
    const T sv0 = __shfl(c.v0, lane - 1), sv1 = __shfl(c.v1, lane - 1);
    const T su0 = __shfl(c.u0, lane + 1), su1 = __shfl(c.u1, lane + 1);
    const T vjm0 = p.ring || lane > 0 ? sv0 : n.vjm0;
    const T vjm1 = p.ring || lane > 0 ? sv1 : n.vjm1;
    const T ujp0 = p.ring || lane < 63 ? su0 : n.ujp0;
    const T ujp1 = p.ring || lane < 63 ? su1 : n.ujp1;
    const long long ci = (long long)a * g.nt + p.b0;
    const bool rh = a < g.nr - 1;
    // row b0: theta below from memory (the cell itself at the wall), above = row b1
    row_apply<T>(G, gk, ci, rh, true, g.nt, cm.u0, c.u0, n.up.u0, cm.v0, c.v0, n.up.v0,
                 p.b0 > 0 ? n.utm0 : c.u0, c.u1, p.b0 > 0 ? n.vtm0 : c.v0, c.v1, vjm0, ujp0,
                 y[0], y[1]);
    // row b1: theta below = row b0, above from memory
    const bool thi = p.b0 + 1 < g.nt - 1;
    row_apply<T>(G, gk, ci + 1, rh, thi, g.nt, cm.u1, c.u1, n.up.u1, cm.v1, c.v1, n.up.v1, c.u0,
                 thi ? n.utp1 : c.u1, c.v0, thi ? n.vtp1 : c.v1, vjm1, ujp1, y[2], y[3]);
}

template <typename T, typename X>
__device__ __forceinline__ void march2_start(const Geo& g, const X& x, const March2& p,
                                             Col4<T>& cm, Col4<T>& c)
{
    const long long base = (long long)p.a0 * g.rowlen + p.r0;
    const long long bm = p.a0 > 0 ? base - g.rowlen : base;
    c.u0 = x(base);
    c.v0 = x(g.P + base);
    c.u1 = x(base + g.nh);
    c.v1 = x(g.P + base + g.nh);
    cm.u0 = x(bm);
    cm.v0 = x(g.P + bm);
    cm.u1 = x(bm + g.nh);
    cm.v1 = x(g.P + bm + g.nh);
}

// r = b - A x (and partial sums of r^2) over row pairs.
// red != 0: the residual after a red-black smoothing whose last pass was
// the black one (colour 1).  Each black cell's update made its own equation
// hold with its red neighbours as they stand, and none has changed since, so
// its residual is zero (in exact arithmetic; rounding leaves ~1e-16 of b).
// Only the red cells (colour 0: plane (a + b) mod 2 of row b at plane a) are
// formed: b is read and r written there only, and r's black entries are
// left as they are -- the restriction (red != 0) never reads them.  No norm.
template <typename T, int LTAG, int AHEAD = 1>
__device__ __forceinline__ void d_residual_march2(Blk bk, Geo g, const T* __restrict__ G,
                                                            long long gk, int bpa, int ch,
                                                            const T* __restrict__ bv,
                                                            const T* __restrict__ x,
                                                            T* __restrict__ r,
                                                            double* __restrict__ partial,
                                                            int red = 0)
{
    March2 p;
    double acc = 0.0;
    if (march2_pos(bk, g, bpa, ch, p)) {
        Col4<T> cm, c;
        march2_start<T>(g, Plain<T>{x}, p, cm, c);
        const long long o[4] = {0, g.P, g.nh, g.P + g.nh}; // u0, v0, u1, v1
        for (int a = p.a0; a < p.a1; a += AHEAD) {
            Nb4<T> nb[AHEAD];
            T bb[AHEAD][4];
            // the red cells of the pair at plane a: (u0, v1) for even a,
            // (v0, u1) for odd a (row b0 is even)
            auto is_red = [&](int k, int aa) { return (((k == 1 || k == 2) ? 1 : 0) ^ (aa & 1)) == 0; };
#pragma unroll
            for (int u = 0; u < AHEAD; ++u)
                if (a + u < p.a1) {
                    march2_load<T>(g, Plain<T>{x}, p, a + u, nb[u]);
                    const long long base = (long long)(a + u) * g.rowlen + p.r0;
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if (!red || is_red(k, a + u)) bb[u][k] = ld_once(bv + base + o[k]);
                }
#pragma unroll
            for (int u = 0; u < AHEAD; ++u)
                if (a + u < p.a1) {
                    T y[4];
                    march2_apply<T>(g, G, gk, p, a + u, cm, c, nb[u], y);
                    const long long base = (long long)(a + u) * g.rowlen + p.r0;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        if (red && !is_red(k, a + u)) continue;
                        const T rk = bb[u][k] - y[k];
                        st_once(r + base + o[k], rk);
                        acc += (double)rk * (double)rk;
                    }
                    cm = c;
                    c = nb[u].up;
                }
        }
    }
    if (partial) {
        acc = block_sum(acc);
        if (threadIdx.x == 0) partial[bk.L] = acc;
    }
}

template <typename T, int LTAG>
__global__ void __launch_bounds__(kBlock) k_residual_march2(Geo g, const T* __restrict__ G,
                                                            long long gk, int bpa, int ch,
                                                            const T* __restrict__ bv,
                                                            const T* __restrict__ x,
                                                            T* __restrict__ r,
                                                            double* __restrict__ partial,
                                                            int red)
{
    d_residual_march2<T, LTAG>(self_blk(), g, G, gk, bpa, ch, bv, x, r, partial, red);
}

// y = A x (and partial sums of y . dotv) over row pairs.
template <typename T, int LTAG, int AHEAD = 1>
__device__ __forceinline__ void d_apply_march2(Blk bk, Geo g, const T* __restrict__ G,
                                                         long long gk, int bpa, int ch,
                                                         const T* __restrict__ x,
                                                         T* __restrict__ y,
                                                         double* __restrict__ partial,
                                                         const T* __restrict__ dotv)
{
    March2 p;
    double acc = 0.0;
    if (march2_pos(bk, g, bpa, ch, p)) {
        Col4<T> cm, c;
        march2_start<T>(g, Plain<T>{x}, p, cm, c);
        const long long o[4] = {0, g.P, g.nh, g.P + g.nh};
        for (int a = p.a0; a < p.a1; a += AHEAD) {
            Nb4<T> nb[AHEAD];
            T dv[AHEAD][4];
#pragma unroll
            for (int u = 0; u < AHEAD; ++u)
                if (a + u < p.a1) {
                    march2_load<T>(g, Plain<T>{x}, p, a + u, nb[u]);
                    if (dotv) {
                        const long long base = (long long)(a + u) * g.rowlen + p.r0;
#pragma unroll
                        for (int k = 0; k < 4; ++k) dv[u][k] = dotv[base + o[k]];
                    }
                }
#pragma unroll
            for (int u = 0; u < AHEAD; ++u)
                if (a + u < p.a1) {
                    T yk[4];
                    march2_apply<T>(g, G, gk, p, a + u, cm, c, nb[u], yk);
                    const long long base = (long long)(a + u) * g.rowlen + p.r0;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        st_once(y + base + o[k], yk[k]);
                        if (dotv) acc = __builtin_fma((double)yk[k], (double)dv[u][k], acc);
                    }
                    cm = c;
                    c = nb[u].up;
                }
        }
    }
    if (partial) {
        acc = block_sum(acc);
        if (threadIdx.x == 0) partial[bk.L] = acc;
    }
}

template <typename T, int LTAG>
__global__ void __launch_bounds__(kBlock) k_apply_march2(Geo g, const T* __restrict__ G,
                                                         long long gk, int bpa, int ch,
                                                         const T* __restrict__ x,
                                                         T* __restrict__ y,
                                                         double* __restrict__ partial,
                                                         const T* __restrict__ dotv)
{
    d_apply_march2<T, LTAG>(self_blk(), g, G, gk, bpa, ch, x, y, partial, dotv);
}

// Conjugate-gradient direction and product in one pass over row pairs:
// p = z + beta p_old (beta: a device scalar) is formed wherever it is read,
// written for the thread's own cells, and q = A p with partial sums of
// p . q (q is stored unless null: a step that forms q again from p needs
// none).  p must not alias p_old (other threads still read p_old).
// The theta rows just outside a pair are the adjacent wavefronts' own rows:
// each wavefront hands its plane-a values to its neighbours through LDS
// (double-buffered by plane, one barrier per plane), so only the block's
// outermost rows are formed from memory.  Reading both z and p_old at every
// neighbour instead doubles the L2 traffic of the stencil rows, and half of
// it then misses.
// X: the field p is formed from (Dir, or DirCast in the mixed form).
// XU (compile-time, so a launch without updates carries none of their
// registers): 0, the iterate is not touched; 1, also the previous step's
// pending update of the iterate, xs += alpha p_old on the thread's own
// cells (one fma, as in d_cg_step), so the step itself need not stream x
// and p -- p_old of plane a + 1 is loaded once, forms the direction there
// (X.from) and makes that plane's update; 2, the iterate also owes the
// update of the step before, xs += alpha2 p_{k-2} first, with p_{k-2} read
// from pnew's buffer before this kernel overwrites it (the same two
// roundings as two passes), so the iterate is streamed every other
// iteration only.
template <typename T, int LTAG, int XU, typename X_>
__device__ __forceinline__ void d_apply_dir_march2(Blk bk, Geo g, const T* __restrict__ G,
                                                             long long gk, int bpa, int ch,
                                                             const X_ X, T* __restrict__ pnew,
                                                             T* __restrict__ q,
                                                             double* __restrict__ partial,
                                                             T* __restrict__ xs = nullptr,
                                                             const T* __restrict__ pold = nullptr,
                                                             T alpha = T(0), T alpha2 = T(0))
{
    constexpr bool kX = XU > 0, two = XU == 2;
    __shared__ T sh[2][kPairs][4][64];
    March2 p;
    double acc = 0.0;
    const bool live = march2_pos(bk, g, bpa, ch, p);
    // the chunk of planes is the block's: wavefronts past the last pair stay
    // in the loop for its barriers (a neighbour's row is read only where the
    // pair exists, i.e. its wavefront is live)
    if (p.a0 < g.nr) {
        const int w = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
        const long long o[4] = {0, g.P, g.nh, g.P + g.nh};
        Col4<T> cm, c;
        if (live) march2_start<T>(g, X, p, cm, c);
        // the pending update of the chunk's first plane; each later plane's
        // comes with the loads that form its direction (p_old read once)
        if (kX && live) {
            const long long b0 = (long long)p.a0 * g.rowlen + p.r0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                T xv = ld_once(xs + b0 + o[k]);
                if constexpr (two) xv = __builtin_fma(alpha2, pnew[b0 + o[k]], xv);
                st_once(xs + b0 + o[k], __builtin_fma(alpha, pold[b0 + o[k]], xv));
            }
        }
        for (int a = p.a0, buf = 0; a < p.a1; ++a, buf ^= 1) {
            Nb4<T> nb;
            const long long base = (long long)a * g.rowlen + p.r0;
            const long long ab = a < g.nr - 1 ? base + g.rowlen : base;
            const bool upd = kX && a + 1 < p.a1; // plane a + 1 is the chunk's
            T xo[4], po[4], p2[4];
            if (live) {
                sh[buf][w][0][lane] = c.u0;
                sh[buf][w][1][lane] = c.v0;
                sh[buf][w][2][lane] = c.u1;
                sh[buf][w][3][lane] = c.v1;
                march2_load<T>(g, X, p, a, nb, w == 0, w == kPairs - 1, !kX);
                if constexpr (kX) { // the direction at a + 1 from p_old held for the update
#pragma unroll
                    for (int k = 0; k < 4; ++k) po[k] = pold[ab + o[k]];
                    nb.up.u0 = X.from(po[0], ab + o[0]);
                    nb.up.v0 = X.from(po[1], ab + o[1]);
                    nb.up.u1 = X.from(po[2], ab + o[2]);
                    nb.up.v1 = X.from(po[3], ab + o[3]);
                    if (upd) {
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            xo[k] = ld_once(xs + ab + o[k]);
                            if constexpr (two) p2[k] = pnew[ab + o[k]]; // before it is overwritten
                        }
                    }
                }
            }
            __syncthreads();
            if (!live) continue;
            if (w > 0) {
                nb.utm0 = sh[buf][w - 1][2][lane];
                nb.vtm0 = sh[buf][w - 1][3][lane];
            }
            if (w < kPairs - 1) {
                nb.utp1 = sh[buf][w + 1][0][lane];
                nb.vtp1 = sh[buf][w + 1][1][lane];
            }
            T yk[4];
            march2_apply<T>(g, G, gk, p, a, cm, c, nb, yk);
            const T own[4] = {c.u0, c.v0, c.u1, c.v1};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                st_once(pnew + base + o[k], own[k]);
                if (q) st_once(q + base + o[k], yk[k]);
                acc = __builtin_fma((double)yk[k], (double)own[k], acc);
                if (upd) {
                    T xv = xo[k];
                    if constexpr (two) xv = __builtin_fma(alpha2, p2[k], xv);
                    st_once(xs + ab + o[k], __builtin_fma(alpha, po[k], xv));
                }
            }
            cm = c;
            c = nb.up;
        }
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[bk.L] = acc;
}

template <typename T, int LTAG, int XU>
__global__ void __launch_bounds__(kBlock) k_apply_dir_march2(Geo g, const T* __restrict__ G,
                                                             long long gk, int bpa, int ch,
                                                             const T* __restrict__ z,
                                                             const T* __restrict__ pold,
                                                             const double* __restrict__ beta,
                                                             T* __restrict__ pnew,
                                                             T* __restrict__ q,
                                                             double* __restrict__ partial,
                                                             T* __restrict__ xs,
                                                             const double* __restrict__ sc)
{
    d_apply_dir_march2<T, LTAG, XU>(self_blk(), g, G, gk, bpa, ch, Dir<T>{z, pold, (T)*beta},
                                    pnew, q, partial, xs, pold,
                                    XU > 0 ? (T)sc[S_ALPHA] : T(0),
                                    XU == 2 ? (T)sc[S_ALPHA_OLD] : T(0));
}

// The same in the mixed form: z = (double) e * sc[S_SCALE] from the FP32
// correction e of the V-cycle, formed where it is read (z is not stored).
template <int XU>
__global__ void __launch_bounds__(kBlock) k_apply_dircast_march2(Geo g,
                                                                 const double* __restrict__ G,
                                                                 long long gk, int bpa, int ch,
                                                                 const float* __restrict__ e,
                                                                 const double* __restrict__ sc,
                                                                 int scale_slot, int beta_slot,
                                                                 const double* __restrict__ pold,
                                                                 double* __restrict__ pnew,
                                                                 double* __restrict__ q,
                                                                 double* __restrict__ partial,
                                                                 double* __restrict__ xs)
{
    d_apply_dir_march2<double, 0, XU>(self_blk(), g, G, gk, bpa, ch,
                                      DirCast{e, sc[scale_slot], pold, sc[beta_slot]}, pnew, q,
                                      partial, xs, pold, XU > 0 ? sc[S_ALPHA] : 0.0,
                                      XU == 2 ? sc[S_ALPHA_OLD] : 0.0);
}

// ---------------------------------------------------------------------------
// Grid transfers (cell-centred, coarsening by 2 in every direction)
// ---------------------------------------------------------------------------

// Both transfers are separable products of 1-D cell-centred linear
// interpolation (P) and its transpose (R = P^T): fine cell i takes 3/4 of
// coarse i/2 and 1/4 of coarse i/2 - 1 (even i) or i/2 + 1 (odd i), indices
// mirrored at walls and wrapped in phi; coarse I gathers fine 2I-1, 2I,
// 2I+1, 2I+2 with weights 1/4, 3/4, 3/4, 1/4 (a fine index past a wall folds
// onto the wall cell).  One thread per coarse column (J, jc), i.e. the
// coarse cells K = 2 jc and 2 jc + 1, marching over a chunk of coarse
// planes: the theta-phi part for one plane is formed once and used by every
// r position that needs it.  Launch: grid = bpa * nchunks over the coarse
// plane positions, `ch` coarse planes per chunk.

// Two consecutive values of one parity plane (16 B for FP64, 8 B for FP32):
// fine phi indices 2jc, 2jc+1 of a coarse column's cells.  Level vectors
// are separate device allocations and every offset used is even, so the
// accesses are aligned.
template <typename T>
using Vec2 = T __attribute__((ext_vector_type(2)));

struct CoarseCol {
    int I0, I1, m, J, jc;
};

__device__ __forceinline__ bool coarse_col(Blk bk, const Geo& c, int bpa, int ch, CoarseCol& p)
{
    const int L = (int)bk.L;
    const int chunk = L / bpa;
    p.m = (L - chunk * bpa) * kBlock + (int)threadIdx.x;
    p.I0 = chunk * ch;
    p.I1 = min(c.nr, p.I0 + ch);
    if (p.m >= c.rowlen || p.I0 >= c.nr) return false;
    p.J = p.m / c.nh;
    p.jc = p.m - p.J * c.nh;
    return true;
}

// bc = R r (full weighting; interior rows sum to 8).  red != 0: r is the
// red-only residual of d_residual_march2 (zero on the black cells, whose
// entries hold stale values): of each fine row only its red parity plane,
// (plane + row) mod 2, is read, the other taken as zero.
template <typename T>
__device__ __forceinline__ void d_restrict(Blk bk, Geo f, Geo c, int bpa, int ch,
                                                     const T* __restrict__ r,
                                                     T* __restrict__ bc, int red = 0)
{
    CoarseCol p;
    if (!coarse_col(bk, c, bpa, ch, p)) return;
    const T w0 = T(0.25), w1 = T(0.75);
    long long rowo[4];
    for (int q = 0; q < 4; ++q) rowo[q] = (long long)clampi(2 * p.J - 1 + q, f.nt - 1) * f.nh;
    // fine phi positions 4jc-1 .. 4jc+4: 4jc .. 4jc+3 are the pairs at index
    // 2jc, 2jc+1 of both planes (one 2-vector each); 4jc-1 is plane 1 index
    // 2jc-1 and 4jc+4 plane 0 index 2jc+2 (wrapped in phi)
    const long long cv = 2 * p.jc;
    const long long cm = f.P + (p.jc == 0 ? f.nh - 1 : cv - 1);
    const long long cp = p.jc == c.nh - 1 ? 0 : cv + 2;
    const T wq[4] = {w0, w1, w1, w0};
    // the outer phi values 4jc-1 and 4jc+4 are the adjacent threads' pairs
    // (jc-1's last odd value, jc+1's first even one): taken from the
    // adjacent lanes where those hold the same row, else loaded
    const int lane = (int)(threadIdx.x & 63);
    const bool lo_lane = lane > 0 && p.jc > 0;
    const bool hi_lane = lane < 63 && p.jc < c.nh - 1;
    // theta-phi restriction of fine plane a for K = 2jc (s0) and 2jc+1 (s1)
    auto plane = [&](int a, T& s0, T& s1) {
        const int ac = clampi(a, f.nr - 1);
        const T* ra = r + (long long)ac * f.rowlen;
        Vec2<T> e[4], o[4];
        T v0[4], v5[4];
        const Vec2<T> zero2{T(0), T(0)};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const T* rr = ra + rowo[q];
            // red: the row's red cells are in plane (ac + row) mod 2
            const int sp = (ac + (int)(rowo[q] / f.nh)) & 1;
            e[q] = !red || sp == 0 ? *reinterpret_cast<const Vec2<T>*>(rr + cv) : zero2;
            o[q] = !red || sp == 1 ? *reinterpret_cast<const Vec2<T>*>(rr + f.P + cv) : zero2;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int sp = (ac + (int)(rowo[q] / f.nh)) & 1;
            v0[q] = __shfl(o[q].y, lane - 1);
            v5[q] = __shfl(e[q].x, lane + 1);
            if (!lo_lane) v0[q] = !red || sp == 1 ? ra[rowo[q] + cm] : T(0);
            if (!hi_lane) v5[q] = !red || sp == 0 ? ra[rowo[q] + cp] : T(0);
        }
        s0 = T(0);
        s1 = T(0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const T v1 = e[q].x, v2 = o[q].x, v3 = e[q].y, v4 = o[q].y;
            s0 += wq[q] * (w0 * v0[q] + w1 * v1 + w1 * v2 + w0 * v3);
            s1 += wq[q] * (w0 * v2 + w1 * v3 + w1 * v4 + w0 * v5[q]);
        }
    };
    T pa0, pa1, pb0, pb1;
    plane(2 * p.I0 - 1, pa0, pa1);
    plane(2 * p.I0, pb0, pb1);
    for (int I = p.I0; I < p.I1; ++I) {
        T qa0, qa1, qb0, qb1;
        plane(2 * I + 1, qa0, qa1);
        plane(2 * I + 2, qb0, qb1);
        const long long o = (long long)I * c.rowlen + p.m;
        bc[o] = w0 * pa0 + w1 * pb0 + w1 * qa0 + w0 * qb0;
        bc[c.P + o] = w0 * pa1 + w1 * pb1 + w1 * qa1 + w0 * qb1;
        pa0 = qa0; pa1 = qa1; pb0 = qb0; pb1 = qb1;
    }
}

// The restriction with the theta rows shared through LDS, for coarse levels
// whose rows are whole wavefronts (n_phi / 2 of the coarse level a multiple
// of 64) and whose theta count is a multiple of 4.  A block is 4 coarse rows
// x one 64-wide phi segment (the 256 positions of a block of d_restrict,
// regrouped): wavefront w owns coarse row J = 4G + w and loads only its own
// fine rows 2J and 2J + 1.  Each forms the phi restriction of those rows
// (weights 1, 3, 3, 1 over fine phi 4jc - 1 .. 4jc + 4, the outer two from
// the adjacent lanes) and hands it to the neighbouring wavefronts through
// LDS: row 2J - 1 is wavefront w - 1's second row, 2J + 2 wavefront w + 1's
// first; the block's first and last wavefronts form their outer row
// themselves (mirrored at the theta walls).  Half the loads of d_restrict.
// LDS double-buffered by fine plane: one barrier per plane.
//
// The marching over fine planes is latency-bound unless loads run ahead of
// the barriers: the raw values of two planes are held in registers, and the
// loads of a plane are issued as soon as its buffer is consumed, two planes
// before it is restricted.
//
// RED (d_residual_march2's red residual): of each fine row only its red
// parity plane, (plane + row) mod 2, is read -- one 2-vector and one outer
// phi value per row -- and the black values enter as zeros.
template <typename T>
struct RestrictLds {
    Vec2<T> v[2][4][2][64];
};

__host__ __device__ inline bool restrict_rows(const Geo& c)
{
    return c.nh % 64 == 0 && c.nt % 4 == 0;
}

// raw values of one fine row at one plane: the 2-vectors of both parity
// planes at the thread's phi pair and the outer phi values (m: plane 1 at
// 4jc - 1, p: plane 0 at 4jc + 4; loaded only by the lanes without a
// neighbour holding them)
template <typename T, int RED>
struct RestrictRaw {
    Vec2<T> e, o;
    T m, p;
};
// red only: the red parity plane's 2-vector and its one outer value
template <typename T>
struct RestrictRaw<T, 1> {
    Vec2<T> v;
    T edge;
};

template <typename T, int RED>
__device__ __forceinline__ void d_restrict2(Blk bk, Geo f, Geo c, int bpa, int ch,
                                            const T* __restrict__ r, T* __restrict__ bc,
                                            RestrictLds<T>& sh)
{
    const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
    const int segs = c.nh >> 6;
    const int L = (int)bk.L;
    const int chunk = L / bpa, lb = L - chunk * bpa;
    const int G = lb / segs, seg = lb - G * segs;
    const int J = 4 * G + w, jc = seg * 64 + lane;
    const int I0 = chunk * ch, I1 = min(c.nr, I0 + ch);
    if (I0 >= c.nr) return; // whole block: no barrier is skipped by part of it
    const T w0 = T(0.25), w1 = T(0.75);
    const T wq[4] = {w0, w1, w1, w0};
    const long long cv = 2 * jc;
    const long long cm = f.P + (jc == 0 ? f.nh - 1 : cv - 1);
    const long long cp = jc == c.nh - 1 ? 0 : cv + 2;
    const bool lo_lane = lane > 0 && jc > 0;
    const bool hi_lane = lane < 63 && jc < c.nh - 1;
    // the wavefront's rows: 2J, 2J + 1 and (first and last wavefront) the
    // outer row, mirrored at the theta walls
    const bool outer = w == 0 || w == 3;
    const int rows[3] = {2 * J, 2 * J + 1,
                         clampi(w == 0 ? 2 * J - 1 : 2 * J + 2, f.nt - 1)};
    using Raw = RestrictRaw<T, RED>;
    auto load = [&](int a, Raw (&q)[3]) {
        const int ac = clampi(a, f.nr - 1);
        const T* ra = r + (long long)ac * f.rowlen;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (k == 2 && !outer) continue;
            const T* rr = ra + (long long)rows[k] * f.nh;
            if constexpr (RED) {
                const int sp = (ac + rows[k]) & 1;
                q[k].v = *reinterpret_cast<const Vec2<T>*>(rr + (sp ? f.P : 0) + cv);
                q[k].edge = (sp ? !lo_lane : !hi_lane) ? rr[sp ? cm : cp] : T(0);
            } else {
                q[k].e = *reinterpret_cast<const Vec2<T>*>(rr + cv);
                q[k].o = *reinterpret_cast<const Vec2<T>*>(rr + f.P + cv);
                q[k].m = !lo_lane ? rr[cm] : T(0);
                q[k].p = !hi_lane ? rr[cp] : T(0);
            }
        }
    };
    // phi restriction of one row's raw values, for K = 2jc (q0) and 2jc + 1
    // (q1); fine phi 4jc - 1 .. 4jc + 4 are v0 .. v5
    auto phi = [&](int ac, int row, const Raw& q, T& q0, T& q1) {
        if constexpr (RED) {
            if (((ac + row) & 1) == 0) { // red in plane 0: v1, v3, v5
                T v5 = __shfl(q.v.x, lane + 1);
                if (!hi_lane) v5 = q.edge;
                q0 = w1 * q.v.x + w0 * q.v.y;
                q1 = w1 * q.v.y + w0 * v5;
            } else { // red in plane 1: v0, v2, v4
                T v0 = __shfl(q.v.y, lane - 1);
                if (!lo_lane) v0 = q.edge;
                q0 = w0 * v0 + w1 * q.v.x;
                q1 = w0 * q.v.x + w1 * q.v.y;
            }
        } else {
            T v0 = __shfl(q.o.y, lane - 1);
            T v5 = __shfl(q.e.x, lane + 1);
            if (!lo_lane) v0 = q.m;
            if (!hi_lane) v5 = q.p;
            const T v1 = q.e.x, v2 = q.o.x, v3 = q.e.y, v4 = q.o.y;
            q0 = w0 * v0 + w1 * v1 + w1 * v2 + w0 * v3;
            q1 = w0 * v2 + w1 * v3 + w1 * v4 + w0 * v5;
        }
    };
    int buf = 0;
    // theta-phi restriction of fine plane a from its raw values
    auto plane = [&](int a, const Raw (&q)[3], T& s0, T& s1) {
        const int ac = clampi(a, f.nr - 1);
        T p0[4], p1[4]; // fine rows 2J - 1 .. 2J + 2
        phi(ac, rows[0], q[0], p0[1], p1[1]);
        phi(ac, rows[1], q[1], p0[2], p1[2]);
        if (w == 0) phi(ac, rows[2], q[2], p0[0], p1[0]);
        if (w == 3) phi(ac, rows[2], q[2], p0[3], p1[3]);
        Vec2<T> own0, own1;
        own0.x = p0[1];
        own0.y = p1[1];
        own1.x = p0[2];
        own1.y = p1[2];
        sh.v[buf][w][0][lane] = own0;
        sh.v[buf][w][1][lane] = own1;
        __syncthreads();
        if (w > 0) {
            const Vec2<T> v = sh.v[buf][w - 1][1][lane];
            p0[0] = v.x;
            p1[0] = v.y;
        }
        if (w < 3) {
            const Vec2<T> v = sh.v[buf][w + 1][0][lane];
            p0[3] = v.x;
            p1[3] = v.y;
        }
        buf ^= 1;
        s0 = T(0);
        s1 = T(0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            s0 += wq[q] * p0[q];
            s1 += wq[q] * p1[q];
        }
    };
    // coarse plane I takes fine planes 2I - 1 .. 2I + 2 (weights 1, 3, 3, 1);
    // A holds the odd fine planes, B the even ones
    Raw A[3], B[3];
    load(2 * I0 - 1, A);
    load(2 * I0, B);
    T pa0, pa1, pb0, pb1;
    plane(2 * I0 - 1, A, pa0, pa1);
    load(2 * I0 + 1, A);
    plane(2 * I0, B, pb0, pb1);
    load(2 * I0 + 2, B);
    const int m = J * c.nh + jc;
    for (int I = I0; I < I1; ++I) {
        T qa0, qa1, qb0, qb1;
        plane(2 * I + 1, A, qa0, qa1);
        if (I + 1 < I1) load(2 * I + 3, A);
        plane(2 * I + 2, B, qb0, qb1);
        if (I + 1 < I1) load(2 * I + 4, B);
        const long long o = (long long)I * c.rowlen + m;
        bc[o] = w0 * pa0 + w1 * pb0 + w1 * qa0 + w0 * qb0;
        bc[c.P + o] = w0 * pa1 + w1 * pb1 + w1 * qa1 + w0 * qb1;
        pa0 = qa0; pa1 = qa1; pb0 = qb0; pb1 = qb1;
    }
}

// Either restriction, chosen by the coarse level's shape (the same choice in
// the single and the batched form; any chunk gives the same bits).
template <typename T>
__device__ __forceinline__ void d_restrict_any(Blk bk, Geo f, Geo c, int bpa, int ch,
                                               const T* __restrict__ r, T* __restrict__ bc,
                                               RestrictLds<T>& sh, int red)
{
    if (!restrict_rows(c)) d_restrict<T>(bk, f, c, bpa, ch, r, bc, red);
    else if (red) d_restrict2<T, 1>(bk, f, c, bpa, ch, r, bc, sh);
    else d_restrict2<T, 0>(bk, f, c, bpa, ch, r, bc, sh);
}

// the single solve launches each body as a kernel of its own (its registers
// are then its own)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_restrict(Geo f, Geo c, int bpa, int ch,
                                                     const T* __restrict__ r,
                                                     T* __restrict__ bc, int red)
{
    d_restrict<T>(self_blk(), f, c, bpa, ch, r, bc, red);
}

template <typename T, int RED>
__global__ void __launch_bounds__(kBlock) k_restrict_rows(Geo f, Geo c, int bpa, int ch,
                                                          const T* __restrict__ r,
                                                          T* __restrict__ bc)
{
    __shared__ RestrictLds<T> sh;
    d_restrict2<T, RED>(self_blk(), f, c, bpa, ch, r, bc, sh);
}

// ---------------------------------------------------------------------------
// Red residual and restriction in one pass: the V-cycle's transfer on a
// row-pair level after point red-black pre-smoothing (whose last pass was the
// black one, so only the red residual is formed, as d_residual_march2 does
// with red != 0).  bc = P^T r with r = b - A x on the red cells and 0 on the
// black ones; r never goes through memory, which saves writing it and
// reading it back (two fields of half a level's cells).
//
// A block is rr_rows(SEGS) coarse theta rows x the whole phi ring
// (SEGS = coarse n_phi / 128 segments of 64 coarse phi pairs) x a chunk of
// ch coarse planes.  Each wavefront owns one fine row of one segment: the
// 2 * rows fine rows of the block's coarse rows and the two outer rows the
// theta restriction also reads (first - 1 and last + 1, clamped at the
// theta walls as d_restrict2 clamps them), i.e. 2 * rows + 2 wavefronts a
// segment; lane j holds fine phi pairs cv = 2 jc, 2 jc + 1 (jc = 64 s + j)
// of each parity plane.  At each fine plane a a wavefront forms the red
// residual of its row with the sums of cell_apply_e / cell_apply_o (theta
// neighbours loaded, phi neighbours from the adjacent lanes and past the
// wavefront's ends loaded) and stores it in LDS; after one barrier the
// first `rows` wavefronts of each segment restrict fine rows 2J - 1 ..
// 2J + 2 of their coarse row J in phi (the value past a segment's end from
// the adjacent segment) and theta, with the weights and sums of
// d_restrict2<T, 1>, and coarse plane I combines fine planes 2I - 1 ..
// 2I + 2 (clamped at the r walls) as there.  A wavefront's loads of the next
// planes are issued once its residual is formed, before the barrier.
__host__ __device__ constexpr int rr_rows(int segs) { return segs == 1 ? 4 : 2; }
__host__ __device__ constexpr int rr_waves(int segs) { return (2 * rr_rows(segs) + 2) * segs; }

// The ring segments of the fused transfer from level f to c, or 0 where it
// does not apply (then the residual and the restriction run apart).
__host__ __device__ inline int resrestrict_segs(const Geo& f, const Geo& c)
{
    if (!row_pairs(f) || f.nr != 2 * c.nr || f.nt != 2 * c.nt || f.nh != 2 * c.nh) return 0;
    const int segs = c.nh / 64;
    if (c.nh % 64 != 0 || (segs != 1 && segs != 2)) return 0;
    return c.nt % rr_rows(segs) == 0 ? segs : 0;
}

template <typename T, int SEGS>
struct ResRestrictLds {
    Vec2<T> v[2][SEGS][2 * rr_rows(SEGS) + 2][64]; // [buffer][segment][fine row slot][lane]
};

template <typename T, int SEGS>
__device__ __forceinline__ void d_resrestrict(Blk bk, Geo f, const T* __restrict__ G, long long gk,
                                              Geo c, int bpa, int ch, const T* __restrict__ bv,
                                              const T* __restrict__ x, T* __restrict__ bc,
                                              ResRestrictLds<T, SEGS>& sh)
{
    constexpr int ROWS = rr_rows(SEGS), W = 2 * ROWS + 2;
    const int lane = (int)(threadIdx.x & 63), wv = (int)(threadIdx.x >> 6);
    const int s = wv / W, wr = wv - s * W;
    const int L = (int)bk.L;
    const int chunk = L / bpa, Gi = L - chunk * bpa;
    const int I0 = chunk * ch, I1 = min(c.nr, I0 + ch);
    if (I0 >= c.nr) return; // whole block: no barrier is skipped by part of it
    const int jc = s * 64 + lane, cv = 2 * jc;
    const int nh = f.nh, nt = f.nt;
    const long long sr = f.rowlen, P = f.P;
    // this wavefront's fine row (slot wr of the block's rows) and its theta
    // neighbours (the row itself past a wall)
    const int b = clampi(2 * ROWS * Gi - 1 + wr, nt - 1);
    const int bl = b > 0 ? b - 1 : b, bh = b < nt - 1 ? b + 1 : b;
    const int cm = jc == 0 ? nh - 1 : cv - 1;   // plane 1, the phi pair below
    const int cp = jc == c.nh - 1 ? 0 : cv + 2; // plane 0, the phi pair above
    struct RX {
        Vec2<T> e, o;
    };
    struct RB {
        Vec2<T> bb, tl, th;
        T edge;
    };
    // every address: a wavefront-uniform row pointer + the lane's phi index
    auto ld2 = [&](const T* row, int i) { return *reinterpret_cast<const Vec2<T>*>(row + i); };
    auto load_x = [&](int a) {
        const T* p = x + (long long)clampi(a, f.nr - 1) * sr + (long long)b * nh;
        RX v;
        v.e = ld2(p, cv);
        v.o = ld2(p + P, cv);
        return v;
    };
    // b on the red cells, the theta neighbours at the red parity, and the
    // phi value past the wavefront's end (lane 0: plane 1 below; lane 63:
    // plane 0 above)
    auto load_b = [&](int a) {
        a = clampi(a, f.nr - 1);
        const int sp = (a + b) & 1;
        const long long pl = (long long)a * sr + sp * P;
        RB v;
        v.bb = ld2(bv + pl + (long long)b * nh, cv);
        v.tl = ld2(x + pl + (long long)bl * nh, cv);
        v.th = ld2(x + pl + (long long)bh * nh, cv);
        const T* row = x + (long long)a * sr + (long long)b * nh;
        v.edge = T(0);
        if (sp == 0 && lane == 0) v.edge = (row + P)[cm];
        if (sp == 1 && lane == 63) v.edge = row[cp];
        return v;
    };
    const int a_first = max(2 * I0 - 1, 0), a_last = min(2 * I1, f.nr - 1);
    const bool dup_lo = 2 * I0 - 1 < 0, dup_hi = 2 * I1 > f.nr - 1;
    Vec2<T> Xm; // plane a - 1 at the red parity of plane a
    RX Xc, Xn;
    RB Bc;
    {
        const RX m = load_x(a_first - 1);
        Xm = ((a_first + b) & 1) ? m.o : m.e;
        Xc = load_x(a_first);
        Xn = load_x(a_first + 1);
        Bc = load_b(a_first);
    }
    const T w0 = T(0.25), w1 = T(0.75);
    const T wq[4] = {w0, w1, w1, w0};
    // restricting wavefronts: the last three fine planes' sums (nominal
    // planes, the clamped wall planes counted twice); coarse plane I is
    // written when fine plane 2I + 2 arrives
    const bool emit = wr < ROWS;
    const int J = ROWS * Gi + wr;
    T win0[3] = {T(0), T(0), T(0)}, win1[3] = {T(0), T(0), T(0)};
    int knom = 0;
    auto consume = [&](T s0, T s1) {
        if (knom >= 3 && (knom & 1)) {
            const int I = I0 + (knom - 3) / 2;
            T* o = bc + (long long)I * c.rowlen + (long long)J * c.nh;
            o[jc] = w0 * win0[0] + w1 * win0[1] + w1 * win0[2] + w0 * s0;
            (o + c.P)[jc] = w0 * win1[0] + w1 * win1[1] + w1 * win1[2] + w0 * s1;
        }
        win0[0] = win0[1];
        win0[1] = win0[2];
        win0[2] = s0;
        win1[0] = win1[1];
        win1[1] = win1[2];
        win1[2] = s1;
        ++knom;
    };
    for (int a = a_first, buf = 0; a <= a_last; ++a, buf ^= 1) {
        // red residual of the row at plane a
        {
            const int sp = (a + b) & 1;
            const Vec2<T> xs = sp ? Xc.o : Xc.e; // the red cells
            const Vec2<T> xb = sp ? Xc.e : Xc.o; // the row's black cells
            const Vec2<T> xp = sp ? Xn.o : Xn.e;
            const Vec2<T> tl = b > 0 ? Bc.tl : xs, th = b < nt - 1 ? Bc.th : xs;
            const long long ci = (long long)a * nt + b;
            const T grl = G[ci];
            const T grh = a < f.nr - 1 ? G[ci + nt] : T(0);
            const T gtl = G[4 * gk + ci];
            const T gth = b < nt - 1 ? G[4 * gk + ci + 1] : T(0);
            const T gpp = G[8 * gk + ci];
            Vec2<T> y;
            if (sp == 0) { // red in plane 0: phi neighbours in plane 1 at j - 1, j
                const T sv = __shfl(xb.y, lane - 1);
                const T vjm = lane > 0 ? sv : Bc.edge;
                y.x = cell_apply_e(grl, grh, gtl, gth, gpp, Xm.x, xs.x, xp.x, tl.x, th.x, xb.x, vjm);
                y.y = cell_apply_e(grl, grh, gtl, gth, gpp, Xm.y, xs.y, xp.y, tl.y, th.y, xb.y, xb.x);
            } else { // red in plane 1: phi neighbours in plane 0 at j, j + 1
                const T su = __shfl(xb.x, lane + 1);
                const T ujp = lane < 63 ? su : Bc.edge;
                y.x = cell_apply_o(grl, grh, gtl, gth, gpp, Xm.x, xs.x, xp.x, tl.x, th.x, xb.y, xb.x);
                y.y = cell_apply_o(grl, grh, gtl, gth, gpp, Xm.y, xs.y, xp.y, tl.y, th.y, ujp, xb.y);
            }
            Vec2<T> r;
            r.x = Bc.bb.x - y.x;
            r.y = Bc.bb.y - y.y;
            sh.v[buf][s][wr][lane] = r;
        }
        // the next planes' loads fly over the barrier and the restriction
        Xm = ((a + 1 + b) & 1) ? Xc.o : Xc.e;
        Xc = Xn;
        Xn = load_x(a + 2);
        Bc = load_b(a + 1);
        __syncthreads();
        if (emit) { // phi and theta restriction of fine rows 2J - 1 .. 2J + 2
            T p0[4], p1[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int sl = 2 * wr + q;
                const int fr = clampi(2 * ROWS * Gi - 1 + sl, nt - 1);
                const Vec2<T> v = sh.v[buf][s][sl][lane];
                if (((a + fr) & 1) == 0) { // red in plane 0: v1, v3, v5
                    const T v5 = lane < 63 ? sh.v[buf][s][sl][lane + 1].x
                                           : sh.v[buf][(s + 1) % SEGS][sl][0].x;
                    p0[q] = w1 * v.x + w0 * v.y;
                    p1[q] = w1 * v.y + w0 * v5;
                } else { // red in plane 1: v0, v2, v4
                    const T v0 = lane > 0 ? sh.v[buf][s][sl][lane - 1].y
                                          : sh.v[buf][(s + SEGS - 1) % SEGS][sl][63].y;
                    p0[q] = w0 * v0 + w1 * v.x;
                    p1[q] = w0 * v.x + w1 * v.y;
                }
            }
            T s0 = T(0), s1 = T(0);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                s0 += wq[q] * p0[q];
                s1 += wq[q] * p1[q];
            }
            consume(s0, s1);
            if ((a == 0 && dup_lo) || (a == f.nr - 1 && dup_hi)) consume(s0, s1);
        }
    }
}

template <typename T, int SEGS>
__global__ void __launch_bounds__(64 * rr_waves(SEGS))
    k_resrestrict(Geo f, const T* __restrict__ G, long long gk, Geo c, int bpa, int ch,
                  const T* __restrict__ bv, const T* __restrict__ x, T* __restrict__ bc)
{
    __shared__ ResRestrictLds<T, SEGS> sh;
    d_resrestrict<T, SEGS>(self_blk(), f, G, gk, c, bpa, ch, bv, x, bc, sh);
}

// x += P e (trilinear); the thread writes fine rows 2J, 2J+1 and fine phi
// 4jc .. 4jc+3 on the two fine planes of every coarse plane of its chunk.
// RED: only the red cells (colour 0) are corrected -- read and written.  A
// red-black post-smoothing starts with the black pass, which reads only red
// values and overwrites every black cell, so the black cells' correction is
// never read; it is not made (half the fine level's bytes).
template <typename T, int RED = 0>
__device__ __forceinline__ void d_prolong(Blk bk, Geo f, Geo c, int bpa, int ch,
                                                    const T* __restrict__ e,
                                                    T* __restrict__ x)
{
    CoarseCol p;
    if (!coarse_col(bk, c, bpa, ch, p)) return;
    const T w0 = T(0.75), w1 = T(0.25);
    long long crow[3]; // coarse rows J-1, J, J+1 (mirrored)
    for (int q = 0; q < 3; ++q) crow[q] = (long long)clampi(p.J - 1 + q, c.nt - 1) * c.nh;
    long long ck[4]; // coarse K = 2jc-1 .. 2jc+2 (plane + index)
    for (int o = 0; o < 4; ++o) {
        int K = 2 * p.jc - 1 + o;
        K = K < 0 ? K + c.np : (K >= c.np ? K - c.np : K);
        ck[o] = (long long)(K & 1) * c.P + (K >> 1);
    }
    // theta-phi interpolation of coarse plane I onto the thread's 2 x 4
    // fine (row, phi) positions: out[row][t], fine phi = 4jc + t
    auto plane = [&](int I, T out[2][4]) {
        const T* ea = e + (long long)clampi(I, c.nr - 1) * c.rowlen;
        T th[2][4];
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const T em = ea[crow[0] + ck[o]], e0 = ea[crow[1] + ck[o]], ep = ea[crow[2] + ck[o]];
            th[0][o] = w0 * e0 + w1 * em;
            th[1][o] = w0 * e0 + w1 * ep;
        }
#pragma unroll
        for (int rr = 0; rr < 2; ++rr) {
            // fine 4jc, 4jc+1 come from K = 2jc (o = 1); 4jc+2, 4jc+3 from 2jc+1 (o = 2)
            out[rr][0] = w0 * th[rr][1] + w1 * th[rr][0];
            out[rr][1] = w0 * th[rr][1] + w1 * th[rr][2];
            out[rr][2] = w0 * th[rr][2] + w1 * th[rr][1];
            out[rr][3] = w0 * th[rr][2] + w1 * th[rr][3];
        }
    };
    T tm[2][4], t0[2][4], tp[2][4];
    plane(p.I0 - 1, tm);
    plane(p.I0, t0);
    // fine phi 4jc + t sits in plane t & 1 at index 2jc + (t >> 1): per fine
    // row and plane the thread owns the 2-vector at index 2jc (t = s, s + 2)
    long long fo[2][2];
    for (int rr = 0; rr < 2; ++rr)
        for (int sp = 0; sp < 2; ++sp)
            fo[rr][sp] = (long long)sp * f.P + (long long)(2 * p.J + rr) * f.nh + 2 * p.jc;
    // the red cells of fine row 2J + rr sit in plane (a + rr) mod 2 at fine
    // plane a: sp == rr on the even plane 2I, sp != rr on the odd one
    for (int I = p.I0; I < p.I1; ++I) {
        plane(I + 1, tp);
        T* x0 = x + (long long)(2 * I) * f.rowlen;
        T* x1 = x0 + f.rowlen;
        Vec2<T> y0[2][2], y1[2][2];
#pragma unroll
        for (int rr = 0; rr < 2; ++rr)
#pragma unroll
            for (int sp = 0; sp < 2; ++sp) {
                if (!RED || sp == rr) y0[rr][sp] = *reinterpret_cast<const Vec2<T>*>(x0 + fo[rr][sp]);
                if (!RED || sp != rr) y1[rr][sp] = *reinterpret_cast<const Vec2<T>*>(x1 + fo[rr][sp]);
            }
#pragma unroll
        for (int rr = 0; rr < 2; ++rr)
#pragma unroll
            for (int sp = 0; sp < 2; ++sp) {
                if (!RED || sp == rr) {
                    y0[rr][sp].x += w0 * t0[rr][sp] + w1 * tm[rr][sp];
                    y0[rr][sp].y += w0 * t0[rr][sp + 2] + w1 * tm[rr][sp + 2];
                    *reinterpret_cast<Vec2<T>*>(x0 + fo[rr][sp]) = y0[rr][sp];
                }
                if (!RED || sp != rr) {
                    y1[rr][sp].x += w0 * t0[rr][sp] + w1 * tp[rr][sp];
                    y1[rr][sp].y += w0 * t0[rr][sp + 2] + w1 * tp[rr][sp + 2];
                    *reinterpret_cast<Vec2<T>*>(x1 + fo[rr][sp]) = y1[rr][sp];
                }
            }
#pragma unroll
        for (int rr = 0; rr < 2; ++rr)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                tm[rr][t] = t0[rr][t];
                t0[rr][t] = tp[rr][t];
            }
    }
}

template <typename T, int RED>
__global__ void __launch_bounds__(kBlock) k_prolong(Geo f, Geo c, int bpa, int ch,
                                                    const T* __restrict__ e,
                                                    T* __restrict__ x)
{
    d_prolong<T, RED>(self_blk(), f, c, bpa, ch, e, x);
}

// Natural [r][theta][phi] <-> parity-split order.  y_split = x_nat - *mean
// (mean may be null), and the inverse.
template <typename T, typename U>
__device__ __forceinline__ void d_to_split(Blk bk, Geo g, const T* __restrict__ x,
                                                     U* __restrict__ y, const double* __restrict__ sum)
{
    const long long n = 2 * g.P;
    const long long i = (long long)bk.L * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double sub = sum ? *sum / (double)n : 0.0;
    const long long row = i / g.np;
    const int c = (int)(i - row * g.np);
    y[(c & 1) * g.P + row * g.nh + (c >> 1)] = (U)((double)x[i] - sub);
}

template <typename T, typename U>
__global__ void __launch_bounds__(kBlock) k_to_split(Geo g, const T* __restrict__ x,
                                                     U* __restrict__ y, const double* __restrict__ sum)
{
    d_to_split<T, U>(self_blk(), g, x, y, sum);
}

template <typename T, typename U>
__device__ __forceinline__ void d_from_split(Blk bk, Geo g, const T* __restrict__ x,
                                                       U* __restrict__ y, const double* __restrict__ sum)
{
    const long long n = 2 * g.P;
    const long long i = (long long)bk.L * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double sub = sum ? *sum / (double)n : 0.0;
    const long long row = i / g.np;
    const int c = (int)(i - row * g.np);
    y[i] = (U)((double)x[(c & 1) * g.P + row * g.nh + (c >> 1)] - sub);
}

template <typename T, typename U>
__global__ void __launch_bounds__(kBlock) k_from_split(Geo g, const T* __restrict__ x,
                                                       U* __restrict__ y, const double* __restrict__ sum)
{
    d_from_split<T, U>(self_blk(), g, x, y, sum);
}

// ---------------------------------------------------------------------------
// Coarsest level: e = Ainv (b - mean b), Ainv row-major FP64 (rows and
// columns in the parity-split order of the level).  One wave per row, lanes
// striding over the columns; every block recomputes the mean.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void d_coarse_gemv(Blk bk, int n, const double* __restrict__ Ainv,
                                                        const T* __restrict__ bv,
                                                        T* __restrict__ e)
{
    __shared__ double smean;
    double s = 0.0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) s += (double)bv[j];
    s = block_sum(s);
    if (threadIdx.x == 0) smean = s / n;
    __syncthreads();
    const double mu = smean;
    const int lane = threadIdx.x & 63;
    const int row = bk.L * (kBlock / 64) + (threadIdx.x >> 6);
    if (row >= n) return;
    const double* Ar = Ainv + (long long)row * n;
    // four accumulators: each lane's loads of a row go out together instead
    // of one after another on a single dependent sum
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int j = lane;
    for (; j + 192 < n; j += 256) {
        a0 += Ar[j] * ((double)bv[j] - mu);
        a1 += Ar[j + 64] * ((double)bv[j + 64] - mu);
        a2 += Ar[j + 128] * ((double)bv[j + 128] - mu);
        a3 += Ar[j + 192] * ((double)bv[j + 192] - mu);
    }
    for (; j < n; j += 64) a0 += Ar[j] * ((double)bv[j] - mu);
    double acc = (a0 + a1) + (a2 + a3);
    acc = wave_sum(acc);
    if (lane == 0) e[row] = (T)acc;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_coarse_gemv(int n, const double* __restrict__ Ainv,
                                                        const T* __restrict__ bv,
                                                        T* __restrict__ e)
{
    d_coarse_gemv<T>(self_blk(), n, Ainv, bv, e);
}

// ---------------------------------------------------------------------------
// Vector kernels
// ---------------------------------------------------------------------------

// Reducing vector kernels walk the vector with a grid stride (grids are
// capped at kMaxGrid blocks), one partial sum per block.

// partial sums of u.v (or of u alone when v == nullptr)
template <typename T, typename U>
__device__ __forceinline__ void d_dot(Blk bk, long long n, const T* __restrict__ u,
                                                const U* __restrict__ v,
                                                double* __restrict__ partial)
{
    double acc = 0.0;
    const long long stride = (long long)bk.G * blockDim.x;
    for (long long i = (long long)bk.L * blockDim.x + threadIdx.x; i < n; i += stride)
        acc = v ? __builtin_fma((double)u[i], (double)v[i], acc) : acc + (double)u[i];
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[bk.L] = acc;
}

template <typename T, typename U>
__global__ void __launch_bounds__(kBlock) k_dot(long long n, const T* __restrict__ u,
                                                const U* __restrict__ v,
                                                double* __restrict__ partial)
{
    d_dot<T, U>(self_blk(), n, u, v, partial);
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
__device__ __forceinline__ void d_cast(Blk bk, long long n, const T* __restrict__ x,
                                                 U* __restrict__ y, const double* __restrict__ sc,
                                                 int slot, int invert)
{
    const long long i = (long long)bk.L * blockDim.x + threadIdx.x;
    const double s = invert ? 1.0 / sc[slot] : sc[slot];
    if (i < n) y[i] = (U)((double)x[i] * s);
}

template <typename T, typename U>
__global__ void __launch_bounds__(kBlock) k_cast(long long n, const T* __restrict__ x,
                                                 U* __restrict__ y, const double* __restrict__ sc,
                                                 int slot, int invert)
{
    d_cast<T, U>(self_blk(), n, x, y, sc, slot, invert);
}

// z = (double) x * sc[slot] (the cast of k_cast) with per-block partial
// sums of r . z and, when q is given, of q . z, in one grid-stride pass;
// z == nullptr: the sums only (z is formed again where it is read).
__global__ void __launch_bounds__(kBlock) k_cast_dots(long long n, const float* __restrict__ x,
                                                      double* __restrict__ z,
                                                      const double* __restrict__ sc, int slot,
                                                      const double* __restrict__ r,
                                                      const double* __restrict__ q,
                                                      double* __restrict__ prz,
                                                      double* __restrict__ pzq)
{
    const Blk bk = self_blk();
    const double s = sc[slot];
    double arz = 0.0, azq = 0.0;
    const long long stride = (long long)bk.G * blockDim.x;
    for (long long i = (long long)bk.L * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double v = mul_t((double)x[i], s);
        if (z) z[i] = v;
        arz = __builtin_fma(r[i], v, arz);
        if (q) azq = __builtin_fma(q[i], v, azq);
    }
    arz = block_sum(arz);
    if (threadIdx.x == 0) prz[bk.L] = arz;
    if (q) {
        azq = block_sum(azq);
        if (threadIdx.x == 0) pzq[bk.L] = azq;
    }
}

// x[i] = v
template <typename T>
__device__ __forceinline__ void d_fill(Blk bk, long long n, T* __restrict__ x, T v)
{
    const long long i = (long long)bk.L * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_fill(long long n, T* __restrict__ x, T v)
{
    d_fill<T>(self_blk(), n, x, v);
}

// y[i] = x[i]
template <typename T>
__device__ __forceinline__ void d_copy(Blk bk, long long n, const T* __restrict__ x,
                                                 T* __restrict__ y)
{
    const long long i = (long long)bk.L * blockDim.x + threadIdx.x;
    if (i < n) y[i] = x[i];
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_copy(long long n, const T* __restrict__ x,
                                                 T* __restrict__ y)
{
    d_copy<T>(self_blk(), n, x, y);
}

// x += s * (double) e   (iterative-refinement update, s a device scalar
// holding the norm the residual was divided by)
template <typename U>
__device__ __forceinline__ void d_ir_update(Blk bk, long long n, double* __restrict__ x,
                                                      const U* __restrict__ e,
                                                      const double* __restrict__ s)
{
    const long long i = (long long)bk.L * blockDim.x + threadIdx.x;
    if (i < n) x[i] += *s * (double)e[i];
}

template <typename U>
__global__ void __launch_bounds__(kBlock) k_ir_update(long long n, double* __restrict__ x,
                                                      const U* __restrict__ e,
                                                      const double* __restrict__ s)
{
    d_ir_update<U>(self_blk(), n, x, e, s);
}

// Scalar recurrences of the Krylov solvers are evaluated by one thread on
// device scalars (the sc[] slots declared at the top) so that no host round trip is
// needed.

// CG / flexible CG, in the launch of the reduction they follow:
// sc[slot] = sum of partial[0..n), and thread 0 does the scalar updates:
// RED_SHIFT_RZ keeps the old r.z in S_RZ_OLD before the store, then
// RED_BETA (beta = rz_new / rz_old), RED_FBETA (flexible, Polak-Ribiere:
// beta = -alpha zq / rz_old) or RED_ALPHA (alpha = rz / pq; with
// RED_SHIFT_ALPHA the old alpha is kept in S_ALPHA_OLD first).
enum { RED_SHIFT_RZ = 1, RED_BETA = 2, RED_FBETA = 4, RED_ALPHA = 8, RED_SHIFT_ALPHA = 16 };
__global__ void __launch_bounds__(kBlock) k_reduce_cg(const double* __restrict__ partial,
                                                      long long n, double* __restrict__ sc,
                                                      int slot, int ops)
{
    const double s = d_reduce_sum(partial, n);
    if (threadIdx.x != 0) return;
    if (ops & RED_SHIFT_RZ) sc[S_RZ_OLD] = sc[S_RZ];
    sc[slot] = s;
    if (ops & RED_BETA) sc[S_BETA] = sc[S_RZ] / sc[S_RZ_OLD];
    if (ops & RED_FBETA) sc[S_BETA] = -sc[S_ALPHA] * sc[S_ZQ] / sc[S_RZ_OLD];
    if (ops & RED_SHIFT_ALPHA) sc[S_ALPHA_OLD] = sc[S_ALPHA];
    if (ops & RED_ALPHA) sc[S_ALPHA] = sc[S_RZ] / sc[S_PQ];
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
__device__ __forceinline__ void d_cg_step(Blk bk, long long n, const double* __restrict__ sc,
                                                    double* __restrict__ x,
                                                    double* __restrict__ r,
                                                    const double* __restrict__ p,
                                                    const double* __restrict__ q,
                                                    double* __restrict__ partial,
                                                    float* __restrict__ r32 = nullptr)
{
    const double al = sc[S_ALPHA];
    // r32: also the FP32 right-hand side of the next mixed-form V-cycle,
    // (float)(r / scale) as k_cast forms it
    const double inv = r32 ? 1.0 / sc[S_SCALE] : 0.0;
    double acc = 0.0;
    const long long stride = (long long)bk.G * blockDim.x;
    for (long long i = (long long)bk.L * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (x) x[i] = __builtin_fma(al, p[i], x[i]);
        const double v = __builtin_fma(-al, q[i], r[i]);
        r[i] = v;
        if (r32) r32[i] = (float)(v * inv);
        acc = __builtin_fma(v, v, acc);
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[bk.L] = acc;
}

__global__ void __launch_bounds__(kBlock) k_cg_step(long long n, const double* __restrict__ sc,
                                                    double* __restrict__ x,
                                                    double* __restrict__ r,
                                                    const double* __restrict__ p,
                                                    const double* __restrict__ q,
                                                    double* __restrict__ partial,
                                                    float* __restrict__ r32)
{
    d_cg_step(self_blk(), n, sc, x, r, p, q, partial, r32);
}

// The FP64 CG step on a row-pair level (the iterate's update is carried by
// the direction kernel), which also makes the next V-cycle's first pass.
// q is not read from memory: q = A p is formed again from the stored
// direction p (march2_apply on the same values with the same sums as the
// direction kernel's product, so q has the same bits), and the direction
// kernel need not store it.  r -= alpha q with partial sums of r^2, and
// z = r / D on the red cells (colour 0: plane (a + b) mod 2 of row b at
// plane a) with D and the division of the zero-iterate colour pass (the
// same values).  The theta rows just outside a pair come from the adjacent
// wavefronts through LDS, as in the direction kernel.
__global__ void __launch_bounds__(kBlock) k_cg_step_z(Geo g, const double* __restrict__ G,
                                                       long long gk, int bpa, int ch,
                                                       const double* __restrict__ sc,
                                                       const double* __restrict__ pd,
                                                       double* __restrict__ r,
                                                       double* __restrict__ z,
                                                       double* __restrict__ partial)
{
    __shared__ double sh[2][kPairs][4][64];
    const Blk bk = self_blk();
    March2 p;
    double acc = 0.0;
    const bool live = march2_pos(bk, g, bpa, ch, p);
    if (p.a0 < g.nr) { // every wavefront of the block stays for the barriers
        const double al = sc[S_ALPHA];
        const int w = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
        const long long o[4] = {0, g.P, g.nh, g.P + g.nh}; // u0, v0, u1, v1
        const Plain<double> X{pd};
        Col4<double> cm, c;
        if (live) march2_start<double>(g, X, p, cm, c);
        for (int a = p.a0, buf = 0; a < p.a1; ++a, buf ^= 1) {
            Nb4<double> nb;
            const long long base = (long long)a * g.rowlen + p.r0;
            double rv[4];
            if (live) {
                sh[buf][w][0][lane] = c.u0;
                sh[buf][w][1][lane] = c.v0;
                sh[buf][w][2][lane] = c.u1;
                sh[buf][w][3][lane] = c.v1;
                march2_load<double>(g, X, p, a, nb, w == 0, w == kPairs - 1);
#pragma unroll
                for (int k = 0; k < 4; ++k) rv[k] = ld_once(r + base + o[k]);
            }
            __syncthreads();
            if (!live) continue;
            if (w > 0) {
                nb.utm0 = sh[buf][w - 1][2][lane];
                nb.vtm0 = sh[buf][w - 1][3][lane];
            }
            if (w < kPairs - 1) {
                nb.utp1 = sh[buf][w + 1][0][lane];
                nb.vtp1 = sh[buf][w + 1][1][lane];
            }
            double y[4];
            march2_apply<double>(g, G, gk, p, a, cm, c, nb, y);
            // D of rows b0 and b1 at plane a, as the zero-iterate pass forms it
            const long long ci = (long long)a * g.nt + p.b0;
            const bool rh = a < g.nr - 1, thi = p.b0 + 1 < g.nt - 1;
            const double D0 = -(G[ci] + (rh ? G[ci + g.nt] : 0.0) + G[4 * gk + ci] +
                                G[4 * gk + ci + 1] + 2.0 * G[8 * gk + ci]);
            const double D1 = -(G[ci + 1] + (rh ? G[ci + 1 + g.nt] : 0.0) + G[4 * gk + ci + 1] +
                                (thi ? G[4 * gk + ci + 2] : 0.0) + 2.0 * G[8 * gk + ci + 1]);
            // red: u0 and v1 at even a, v0 and u1 at odd a (b0 is even)
            const bool even = (a & 1) == 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const double v = __builtin_fma(-al, y[k], rv[k]);
                st_once(r + base + o[k], v);
                acc = __builtin_fma(v, v, acc);
                const bool red = (k == 0 || k == 3) == even;
                if (red) st_once(z + base + o[k], v / (k < 2 ? D0 : D1));
            }
            cm = c;
            c = nb.up;
        }
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[bk.L] = acc;
}

// x += alpha p: the update the last step of a solve leaves pending when the
// direction kernel carries the iterate's updates
__global__ void __launch_bounds__(kBlock) k_cg_x(long long n, const double* __restrict__ sc,
                                                 const double* __restrict__ p,
                                                 double* __restrict__ x, int slot)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = __builtin_fma(sc[slot], p[i], x[i]);
}

// r = b - y with y = A x: the residual of the iterate itself (the Krylov
// recurrences update r without forming it)
__device__ __forceinline__ void d_sub(Blk bk, long long n, const double* __restrict__ b,
                                      const double* __restrict__ y, double* __restrict__ r)
{
    const long long i = (long long)bk.L * blockDim.x + threadIdx.x;
    if (i < n) r[i] = b[i] - y[i];
}

__global__ void __launch_bounds__(kBlock) k_sub(long long n, const double* __restrict__ b,
                                                const double* __restrict__ y,
                                                double* __restrict__ r)
{
    d_sub(self_blk(), n, b, y, r);
}

// p = z + beta p
__device__ __forceinline__ void d_cg_dir(Blk bk, long long n, const double* __restrict__ sc,
                                                   const double* __restrict__ z,
                                                   double* __restrict__ p)
{
    const long long i = (long long)bk.L * blockDim.x + threadIdx.x;
    if (i < n) p[i] = __builtin_fma(sc[S_BETA], p[i], z[i]);
}

__global__ void __launch_bounds__(kBlock) k_cg_dir(long long n, const double* __restrict__ sc,
                                                   const double* __restrict__ z,
                                                   double* __restrict__ p)
{
    d_cg_dir(self_blk(), n, sc, z, p);
}

// BiCGStab: p = r + beta (p - omega v)
__device__ __forceinline__ void d_bicg_dir(Blk bk, long long n, const double* __restrict__ sc,
                                                     const double* __restrict__ r,
                                                     const double* __restrict__ v,
                                                     double* __restrict__ p)
{
    const long long i = (long long)bk.L * blockDim.x + threadIdx.x;
    if (i < n) p[i] = r[i] + sc[S_BETA] * (p[i] - sc[S_OMEGA] * v[i]);
}

__global__ void __launch_bounds__(kBlock) k_bicg_dir(long long n, const double* __restrict__ sc,
                                                     const double* __restrict__ r,
                                                     const double* __restrict__ v,
                                                     double* __restrict__ p)
{
    d_bicg_dir(self_blk(), n, sc, r, v, p);
}

// BiCGStab: s = r - alpha v (into s)
__device__ __forceinline__ void d_bicg_s(Blk bk, long long n, const double* __restrict__ sc,
                                                   const double* __restrict__ r,
                                                   const double* __restrict__ v,
                                                   double* __restrict__ s)
{
    const long long i = (long long)bk.L * blockDim.x + threadIdx.x;
    if (i < n) s[i] = r[i] - sc[S_ALPHA] * v[i];
}

__global__ void __launch_bounds__(kBlock) k_bicg_s(long long n, const double* __restrict__ sc,
                                                   const double* __restrict__ r,
                                                   const double* __restrict__ v,
                                                   double* __restrict__ s)
{
    d_bicg_s(self_blk(), n, sc, r, v, s);
}

// BiCGStab: x += alpha ph + omega sh ; r = s - omega t ; partial r^2
__device__ __forceinline__ void d_bicg_step(Blk bk, long long n, const double* __restrict__ sc,
                                                      double* __restrict__ x,
                                                      double* __restrict__ r,
                                                      const double* __restrict__ ph,
                                                      const double* __restrict__ sh,
                                                      const double* __restrict__ s,
                                                      const double* __restrict__ t,
                                                      double* __restrict__ partial)
{
    double acc = 0.0;
    const long long stride = (long long)bk.G * blockDim.x;
    for (long long i = (long long)bk.L * blockDim.x + threadIdx.x; i < n; i += stride) {
        x[i] += sc[S_ALPHA] * ph[i] + sc[S_OMEGA] * sh[i];
        const double v = s[i] - sc[S_OMEGA] * t[i];
        r[i] = v;
        acc += v * v;
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[bk.L] = acc;
}

__global__ void __launch_bounds__(kBlock) k_bicg_step(long long n, const double* __restrict__ sc,
                                                      double* __restrict__ x,
                                                      double* __restrict__ r,
                                                      const double* __restrict__ ph,
                                                      const double* __restrict__ sh,
                                                      const double* __restrict__ s,
                                                      const double* __restrict__ t,
                                                      double* __restrict__ partial)
{
    d_bicg_step(self_blk(), n, sc, x, r, ph, sh, s, t, partial);
}

// ---------------------------------------------------------------------------
// Launch shapes, shared by host and device so that a batched launch gives
// each problem exactly the blocks (and reduction order) of its own launch.
// ---------------------------------------------------------------------------

constexpr int kMaxLevels = 16;

__host__ __device__ inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

struct MarchShape {
    int bpa, ch, grid;
};

// Marching launch over the planes of g: bpa blocks per plane, chunks of ch
// planes; ch <= 0 picks chunks that give about 2048 blocks (one resident
// wave of 8 blocks per CU).
__host__ __device__ inline MarchShape chunked(const Geo& g, int bpa, int ch, int target = 2048)
{
    if (ch <= 0) {
        int nchunks = cdiv(target, bpa);
        nchunks = nchunks < 1 ? 1 : (nchunks > g.nr ? g.nr : nchunks);
        ch = cdiv(g.nr, nchunks);
    }
    if (ch > g.nr) ch = g.nr;
    return MarchShape{bpa, ch, bpa * cdiv(g.nr, ch)};
}
__host__ __device__ inline MarchShape march_shape(const Geo& g, int ch = 0)
{
    return chunked(g, cdiv(g.rowlen, kBlock), ch);
}
// The restriction's launch: on whole-wavefront coarse levels about 1024
// blocks (6 coarse planes a block on the paper-scale shell's finest
// restriction: a probe over 2 .. 12 put it fastest), else march_shape.
__host__ __device__ inline MarchShape restrict_shape(const Geo& c)
{
    return restrict_rows(c) ? chunked(c, cdiv(c.rowlen, kBlock), 0, 1024) : march_shape(c);
}
// The fused red residual and restriction: c.nt / rr_rows blocks per chunk
// of coarse planes, chunks for about one block per CU in FP64 (a block of 10
// or 12 wavefronts at ~108 VGPRs has a CU to itself) and two in FP32 (~72
// VGPRs), at least two coarse planes a chunk (a block re-reads two fine
// planes of x at each chunk end).
template <typename T>
__host__ __device__ inline MarchShape resrestrict_shape(const Geo& c, int segs, int ch = 0)
{
    const int bpa = c.nt / rr_rows(segs);
    MarchShape ms = chunked(c, bpa, ch, sizeof(T) == 8 ? 256 : 512);
    if (ch <= 0 && ms.ch < 2 && c.nr >= 2) ms = chunked(c, bpa, 2);
    return ms;
}

// Row-pair kernels: bpa blocks over the (n_theta / 2) * (n_phi / 2)
// positions of a plane.  stencil_shape: the marching launch a level uses.
__host__ __device__ inline MarchShape march2_shape(const Geo& g, int ch = 0, int target = 2048)
{
    return chunked(g, cdiv(g.nt / 2, kPairs) * (g.nh / 64), ch, target);
}
__host__ __device__ inline MarchShape stencil_shape(const Geo& g, int ch = 0)
{
    return row_pairs(g) ? march2_shape(g, ch) : march_shape(g, ch);
}
// The colour pass's launch: on row-pair levels the automatic chunk aims at
// about 1024 blocks (twice the planes per block of the other kernels, which
// halves the r-halo planes a block reads again); FP32 passes whose chunk
// would be 8 planes or more take 4-plane chunks instead (more, shorter
// blocks: the FP32 pass's registers leave room for 7 blocks a CU; the
// autotuner's choice on the paper-scale shell).  The chunk does not change
// a pass's values, but it does change the order of the partial sums of the
// FP64 passes that also form b . x.  Elsewhere as stencil_shape.
template <typename T>
__host__ __device__ inline MarchShape gs_shape(const Geo& g, int ch)
{
    if (!row_pairs(g)) return march_shape(g, ch);
    const MarchShape ms = march2_shape(g, ch, 1024);
    if (ch <= 0 && sizeof(T) == 4 && ms.ch >= 8) return march2_shape(g, 4, 1024);
    return ms;
}

// blocks per plane of the generic colour pass and of generic stencil kernels
__host__ __device__ inline int gs_bpa(const Geo& g, int ncol)
{
    return cdiv(ncol == 2 ? g.rowlen : g.rowlen / 2, kBlock);
}
__host__ __device__ inline int capped_grid(long long blocks)
{
    return blocks < kMaxGrid ? (int)blocks : kMaxGrid;
}

// ---------------------------------------------------------------------------
// Batched launches.  A work table lists, for every block of the launch, the
// problem it serves and its logical index L among the G blocks that the
// problem's own launch would have; the block then runs the same kernel body
// on that problem's data, read from a per-problem descriptor.  Blocks of
// problems marked inactive (converged) return at once.
// ---------------------------------------------------------------------------

struct BItem {
    int prob;
    unsigned L, G;
};

// finest-level FP64 vectors of a problem, by id
enum VecId {
    V_X = 0, V_B0, V_R, V_Z, V_P, V_Q, V_R0, V_V, V_S, V_T, V_PH, V_SH, V_RHS, V_OUT, V_COUNT
};

template <typename T>
struct LDesc {
    Geo g;
    const T* G;
    long long gk;
    T *x, *b, *r;
    int gs_ch; // marching chunk of the colour pass (autotuned)
    // plane smoother (null without it): ring transform tables, the r-line
    // inverse pivots of both parities, the spectra scratch of one parity
    const Vec2<T>* ptw;
    const Vec2<T>* ptwN;
    const T* plam;
    const T* ppiv;
    Vec2<T>* pS;
    int prb; // rings per block of the transforms (autotuned)
    // small levels of the point smoother (tile.hpp): the post-smoothed
    // iterate goes to xt
    int tile;
    T* xt;
};

template <typename T>
struct PDesc {
    int L, nc, ncol, pad;
    const double* Ainv;
    const double* G64; // finest-level FP64 metrics
    long long gk64;
    long long parts_apply, parts_vec; // partial sums left by apply / vector reductions
    double* vec[V_COUNT];
    double* sc;
    double* partial;
    LDesc<T> lv[kMaxLevels];
};

#define CPS_BATCH_BLOCK                                                                    \
    const BItem it = items[blockIdx.x];                                                    \
    if (!active[it.prob]) return;                                                          \
    const Blk bk{it.L, it.G};

template <typename T>
__global__ void __launch_bounds__(kBlock) kb_gs_march(const BItem* __restrict__ items,
                                                      const int* __restrict__ active,
                                                      const PDesc<T>* __restrict__ pd, int level,
                                                      int colour, int zero)
{
    CPS_BATCH_BLOCK
    const LDesc<T>& d = pd[it.prob].lv[level];
    const MarchShape ms = gs_shape<T>(d.g, d.gs_ch);
    if (row_pairs(d.g))
        d_gs_march2<T, 1>(bk, d.g, d.G, d.gk, ms.bpa, ms.ch, d.b, d.x, colour, zero);
    else if (d.g.nh % 64 == 0)
        d_gs_march<T, true, 1>(bk, d.g, d.G, d.gk, ms.bpa, ms.ch, d.b, d.x, colour, zero);
    else
        d_gs_march<T, false, 1>(bk, d.g, d.G, d.gk, ms.bpa, ms.ch, d.b, d.x, colour, zero);
}

template <typename T, int MODE, bool AXI>
__global__ void __launch_bounds__(kBlock) kb_gs(const BItem* __restrict__ items,
                                                const int* __restrict__ active,
                                                const PDesc<T>* __restrict__ pd, int level,
                                                int colour, int zero)
{
    CPS_BATCH_BLOCK
    const PDesc<T>& P = pd[it.prob];
    const LDesc<T>& d = P.lv[level];
    const int bpa = gs_bpa(d.g, P.ncol);
    if (d.g.nh % 64 == 0)
        d_gs<T, MODE, AXI, true, 1>(bk, d.g, d.G, d.gk, bpa, d.b, d.x, colour, P.ncol, zero);
    else
        d_gs<T, MODE, AXI, false, 1>(bk, d.g, d.G, d.gk, bpa, d.b, d.x, colour, P.ncol, zero);
}

// r = b - A x on a level (no norm), marching (7-point, phi-invariant) or generic
// red: the group smooths red-black (not by planes): on row-pair levels the
// red-only residual, as the single solve forms it
template <typename T, int MODE, bool AXI>
__global__ void __launch_bounds__(kBlock) kb_residual(const BItem* __restrict__ items,
                                                      const int* __restrict__ active,
                                                      const PDesc<T>* __restrict__ pd, int level,
                                                      int red)
{
    CPS_BATCH_BLOCK
    const LDesc<T>& d = pd[it.prob].lv[level];
    const bool u = d.g.nh % 64 == 0;
    if constexpr (MODE == MODE_ORTHO && AXI) {
        const MarchShape ms = stencil_shape(d.g);
        if (row_pairs(d.g)) d_residual_march2<T, 1>(bk, d.g, d.G, d.gk, ms.bpa, ms.ch, d.b, d.x, d.r, nullptr, red);
        else if (u) d_residual_march<T, true, 1>(bk, d.g, d.G, d.gk, ms.bpa, ms.ch, d.b, d.x, d.r, nullptr);
        else d_residual_march<T, false, 1>(bk, d.g, d.G, d.gk, ms.bpa, ms.ch, d.b, d.x, d.r, nullptr);
    } else {
        const int bpa = cdiv(d.g.rowlen, kBlock);
        if (u) d_residual<T, MODE, AXI, true, 1>(bk, d.g, d.G, d.gk, bpa, d.b, d.x, d.r, nullptr);
        else d_residual<T, MODE, AXI, false, 1>(bk, d.g, d.G, d.gk, bpa, d.b, d.x, d.r, nullptr);
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) kb_restrict(const BItem* __restrict__ items,
                                                      const int* __restrict__ active,
                                                      const PDesc<T>* __restrict__ pd, int level,
                                                      int red)
{
    CPS_BATCH_BLOCK
    __shared__ RestrictLds<T> sh;
    const PDesc<T>& P = pd[it.prob];
    const MarchShape ms = march_shape(P.lv[level + 1].g);
    d_restrict_any<T>(bk, P.lv[level].g, P.lv[level + 1].g, ms.bpa, ms.ch, P.lv[level].r,
                      P.lv[level + 1].b, sh, red && row_pairs(P.lv[level].g));
}

// the fused red residual and restriction of one problem's level (SEGS as
// resrestrict_segs gives it; the block size is 64 * rr_waves(SEGS))
template <typename T, int SEGS>
__global__ void __launch_bounds__(64 * rr_waves(SEGS))
    kb_resrestrict(const BItem* __restrict__ items, const int* __restrict__ active,
                   const PDesc<T>* __restrict__ pd, int level)
{
    CPS_BATCH_BLOCK
    __shared__ ResRestrictLds<T, SEGS> sh;
    const PDesc<T>& P = pd[it.prob];
    const LDesc<T>& d = P.lv[level];
    const Geo c = P.lv[level + 1].g;
    const MarchShape ms = resrestrict_shape<T>(c, SEGS);
    d_resrestrict<T, SEGS>(bk, d.g, d.G, d.gk, c, ms.bpa, ms.ch, d.b, d.x, P.lv[level + 1].b, sh);
}

// red: only the red cells are corrected (a red-black post-smoothing follows)
template <typename T, int RED>
__global__ void __launch_bounds__(kBlock) kb_prolong(const BItem* __restrict__ items,
                                                     const int* __restrict__ active,
                                                     const PDesc<T>* __restrict__ pd, int level)
{
    CPS_BATCH_BLOCK
    const PDesc<T>& P = pd[it.prob];
    const MarchShape ms = march_shape(P.lv[level + 1].g);
    const LDesc<T>& c = P.lv[level + 1];
    d_prolong<T, RED>(bk, P.lv[level].g, c.g, ms.bpa, ms.ch, c.tile ? c.xt : c.x, P.lv[level].x);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) kb_fill_level(const BItem* __restrict__ items,
                                                        const int* __restrict__ active,
                                                        const PDesc<T>* __restrict__ pd, int level)
{
    CPS_BATCH_BLOCK
    const LDesc<T>& d = pd[it.prob].lv[level];
    d_fill<T>(bk, 2 * d.g.P, d.x, T(0));
}

// coarsest level of each problem (its own level count)
template <typename T>
__global__ void __launch_bounds__(kBlock) kb_coarse(const BItem* __restrict__ items,
                                                    const int* __restrict__ active,
                                                    const PDesc<T>* __restrict__ pd)
{
    CPS_BATCH_BLOCK
    const PDesc<T>& P = pd[it.prob];
    const LDesc<T>& d = P.lv[P.L - 1];
    d_coarse_gemv<T>(bk, P.nc, P.Ainv, d.b, d.x);
}

// finest-level vector in (FP64) -> level-0 b of the V-cycle / level-0 x -> out
template <typename T>
__global__ void __launch_bounds__(kBlock) kb_cast_in(const BItem* __restrict__ items,
                                                     const int* __restrict__ active,
                                                     const PDesc<T>* __restrict__ pd, int in)
{
    CPS_BATCH_BLOCK
    const PDesc<T>& P = pd[it.prob];
    d_cast<double, T>(bk, 2 * P.lv[0].g.P, P.vec[in], P.lv[0].b, P.sc, S_SCALE, 1);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) kb_cast_out(const BItem* __restrict__ items,
                                                      const int* __restrict__ active,
                                                      const PDesc<T>* __restrict__ pd, int out)
{
    CPS_BATCH_BLOCK
    const PDesc<T>& P = pd[it.prob];
    d_cast<T, double>(bk, 2 * P.lv[0].g.P, P.lv[0].x, P.vec[out], P.sc, S_SCALE, 0);
}

// y = A x at the finest level in FP64, with partial sums of y . vec[dot]
template <typename T, int MODE, bool AXI>
__global__ void __launch_bounds__(kBlock) kb_apply64(const BItem* __restrict__ items,
                                                     const int* __restrict__ active,
                                                     const PDesc<T>* __restrict__ pd, int in,
                                                     int out, int dot)
{
    CPS_BATCH_BLOCK
    const PDesc<T>& P = pd[it.prob];
    const Geo& g = P.lv[0].g;
    const bool u = g.nh % 64 == 0;
    const double* dv = dot >= 0 ? P.vec[dot] : nullptr;
    if constexpr (MODE == MODE_ORTHO && AXI) {
        const MarchShape ms = stencil_shape(g);
        if (row_pairs(g)) d_apply_march2<double, 0>(bk, g, P.G64, P.gk64, ms.bpa, ms.ch, P.vec[in], P.vec[out], P.partial, dv);
        else if (u) d_apply_march<double, true, 0>(bk, g, P.G64, P.gk64, ms.bpa, ms.ch, P.vec[in], P.vec[out], P.partial, dv);
        else d_apply_march<double, false, 0>(bk, g, P.G64, P.gk64, ms.bpa, ms.ch, P.vec[in], P.vec[out], P.partial, dv);
    } else {
        const int bpa = cdiv(g.rowlen, kBlock);
        if (u) d_apply<double, MODE, AXI, true, 0>(bk, g, P.G64, P.gk64, bpa, P.vec[in], P.vec[out], P.partial, dv);
        else d_apply<double, MODE, AXI, false, 0>(bk, g, P.G64, P.gk64, bpa, P.vec[in], P.vec[out], P.partial, dv);
    }
}

// partial sums of vec[u] . vec[v] (v < 0: of vec[u])
template <typename T>
__global__ void __launch_bounds__(kBlock) kb_dot(const BItem* __restrict__ items,
                                                 const int* __restrict__ active,
                                                 const PDesc<T>* __restrict__ pd, int u, int v)
{
    CPS_BATCH_BLOCK
    const PDesc<T>& P = pd[it.prob];
    d_dot<double, double>(bk, 2 * P.lv[0].g.P, P.vec[u], v >= 0 ? P.vec[v] : nullptr, P.partial);
}

// sc[slot] = sum of the problem's partial sums (one block per problem);
// apply != 0: the partials of kb_apply64, else of a vector reduction
template <typename T>
__global__ void __launch_bounds__(kBlock) kb_reduce(const int* __restrict__ active,
                                                    const PDesc<T>* __restrict__ pd, int apply,
                                                    int slot)
{
    if (!active[blockIdx.x]) return;
    const PDesc<T>& P = pd[blockIdx.x];
    d_reduce(Blk{0, 1}, P.partial, apply ? P.parts_apply : P.parts_vec, P.sc + slot);
}

enum { SOP_CG_ALPHA = 0, SOP_CG_BETA, SOP_FCG_BETA, SOP_BICG_BETA, SOP_BICG_ALPHA, SOP_BICG_OMEGA,
       SOP_COPY, SOP_SQRT, SOP_SET };

// scalar recurrences, one thread per problem (the formulas of k_reduce_cg's
// updates and of k_bicg_*)
template <typename T>
__global__ void kb_scalar(const int* __restrict__ active, const PDesc<T>* __restrict__ pd, int nprob,
                          int op, int dst, int src, double value)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nprob || !active[p]) return;
    double* sc = pd[p].sc;
    switch (op) {
    case SOP_CG_ALPHA: sc[S_ALPHA] = sc[S_RZ] / sc[S_PQ]; break;
    case SOP_CG_BETA: sc[S_BETA] = sc[S_RZ] / sc[S_RZ_OLD]; break;
    case SOP_FCG_BETA: sc[S_BETA] = -sc[S_ALPHA] * sc[S_ZQ] / sc[S_RZ_OLD]; break;
    case SOP_BICG_BETA: sc[S_BETA] = (sc[S_RHO] / sc[S_RHO_OLD]) * (sc[S_ALPHA] / sc[S_OMEGA]); break;
    case SOP_BICG_ALPHA: sc[S_ALPHA] = sc[S_RHO] / sc[S_R0V]; break;
    case SOP_BICG_OMEGA: sc[S_OMEGA] = sc[S_TS] / sc[S_TT]; break;
    case SOP_COPY: sc[dst] = sc[src]; break;
    case SOP_SQRT: sc[dst] = sqrt(sc[src]); break;
    default: sc[dst] = value; break;
    }
}

// out[p] = sc[slot] of problem p (all problems, active or not)
template <typename T>
__global__ void kb_gather(const PDesc<T>* __restrict__ pd, int nprob, int slot, double* __restrict__ out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nprob) out[p] = pd[p].sc[slot];
}

// element-wise finest-level operations
enum { EOP_FILL = 0, EOP_COPY, EOP_CG_DIR, EOP_BICG_DIR, EOP_BICG_S, EOP_TO_SPLIT, EOP_FROM_SPLIT,
       EOP_SUB };

template <typename T>
__global__ void __launch_bounds__(kBlock) kb_elem(const BItem* __restrict__ items,
                                                  const int* __restrict__ active,
                                                  const PDesc<T>* __restrict__ pd, int op, int a,
                                                  int b, int c)
{
    CPS_BATCH_BLOCK
    const PDesc<T>& P = pd[it.prob];
    const Geo& g = P.lv[0].g;
    const long long n = 2 * g.P;
    switch (op) {
    case EOP_FILL: d_fill<double>(bk, n, P.vec[a], 0.0); break;
    case EOP_COPY: d_copy<double>(bk, n, P.vec[a], P.vec[b]); break;
    case EOP_CG_DIR: d_cg_dir(bk, n, P.sc, P.vec[a], P.vec[b]); break;
    case EOP_BICG_DIR: d_bicg_dir(bk, n, P.sc, P.vec[a], P.vec[b], P.vec[c]); break;
    case EOP_BICG_S: d_bicg_s(bk, n, P.sc, P.vec[a], P.vec[b], P.vec[c]); break;
    case EOP_TO_SPLIT: d_to_split<double, double>(bk, g, P.vec[a], P.vec[b], c >= 0 ? P.sc + c : nullptr); break;
    case EOP_SUB: d_sub(bk, n, P.vec[a], P.vec[b], P.vec[c]); break;
    default: d_from_split<double, double>(bk, g, P.vec[a], P.vec[b], c >= 0 ? P.sc + c : nullptr); break;
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) kb_cg_step(const BItem* __restrict__ items,
                                                     const int* __restrict__ active,
                                                     const PDesc<T>* __restrict__ pd)
{
    CPS_BATCH_BLOCK
    const PDesc<T>& P = pd[it.prob];
    d_cg_step(bk, 2 * P.lv[0].g.P, P.sc, P.vec[V_X], P.vec[V_R], P.vec[V_P], P.vec[V_Q], P.partial);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) kb_bicg_step(const BItem* __restrict__ items,
                                                       const int* __restrict__ active,
                                                       const PDesc<T>* __restrict__ pd)
{
    CPS_BATCH_BLOCK
    const PDesc<T>& P = pd[it.prob];
    d_bicg_step(bk, 2 * P.lv[0].g.P, P.sc, P.vec[V_X], P.vec[V_R], P.vec[V_PH], P.vec[V_SH],
                P.vec[V_S], P.vec[V_T], P.partial);
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

// Chords t[q] = dX/ds_q across the LOW d-face of cell (a, b, c) of a level
// with dims (nr, nt, np).  method 0: chords of the map across the face
// centre; method 1: the paper's vertex averages (the normal derivative is
// the mean over the face's four vertices of the difference across vertex
// planes, weight 1/8; each tangential derivative the mean of the face's two
// edges along it).  The face may lie on a wall, the high walls included.
__device__ inline void face_chords(const MapParams& m, int nr, int nt, int np, int method, int d,
                                   int a, int b, int c, double t[3][3])
{
    auto P = [&](double ia, double ib, double ic, double X[3]) {
        map_point(m, ia / nr, ib / nt, ic / np, X);
    };
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
        return;
    }
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

// Face metrics of one level.  One thread per (a, b, c) (c = 0 only when the
// metrics are phi-invariant), three faces each, chords by face_chords.
// flags[blk] gets bit 0 for a face with det <= 0, bit 1 for a non-zero
// r-theta cross metric, bit 2 for a non-zero cross metric involving phi.
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
        for (int d = 0; d < 3; ++d) {
            double Gd[3] = {0.0, 0.0, 0.0};
            const bool wall = (d == 0 && a == 0) || (d == 1 && b == 0);
            if (!wall) {
                double t[3][3];
                face_chords(m, nr, nt, np, method, d, a, b, c, t);
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
                    if (q != d && fabs(v) <= 1e-10 * sqrt(fabs(nn[d] * nn[q])) / fabs(det)) v = 0.0;
                    Gd[q] = v;
                }
                for (int q = 0; q < 3; ++q)
                    if (q != d && Gd[q] != 0.0) fl |= (d == 2 || q == 2) ? 4 : 2;
            }
            // phi-invariant metrics: one entry per (r, theta); otherwise the
            // parity-split layout of the level's fields
            const long long oi = nc == 1 ? i
                                         : (long long)(c & 1) * (n / 2) +
                                               ((long long)a * nt + b) * (np / 2) + (c >> 1);
            for (int q = 0; q < 3; ++q) G[(long long)(3 * d + q) * n + oi] = Gd[q];
        }
    }
    if (fl) atomicOr(&sflag, fl);
    __syncthreads();
    if (threadIdx.x == 0) flags[blockIdx.x] = sflag;
}

// Caller-supplied face metrics of the finest level, natural layout
// [9][nr][nt][np] (entry 3d+q: G_dq on the cell's low d-face), checked and
// classified in place: the low r- and theta-wall faces carry no flux (their
// entries are set to 0); flags bit 1: an entry is not finite or a diagonal
// entry is negative; 2: r-theta cross entries; 4: cross entries with phi;
// 8: some entry differs from the one at c = 0 of its (r, theta) row by more
// than 1e-12 of the face's diagonal entry (the metrics are not
// phi-invariant; within that, the c = 0 values serve the whole ring, as
// rounding in the caller's own trigonometry leaves ~1e-14 differences on a
// map symmetric about the polar axis).  Per-block flags as k_metrics.
__global__ void __launch_bounds__(kBlock) k_user_metrics(int nr, int nt, int np,
                                                         double* __restrict__ U,
                                                         int* __restrict__ flags)
{
    __shared__ int sflag;
    if (threadIdx.x == 0) sflag = 0;
    __syncthreads();
    const long long n = (long long)nr * nt * np;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int fl = 0;
    if (i < n) {
        const int c = (int)(i % np);
        const long long row = i / np;
        const int b = (int)(row % nt), a = (int)(row / nt);
        for (int k = 0; k < 9; ++k) {
            const int d = k / 3, q = k % 3;
            if ((d == 0 && a == 0) || (d == 1 && b == 0)) { // wall face: no flux
                U[k * n + i] = 0.0;
                continue;
            }
            const double v = U[k * n + i];
            if (!isfinite(v) || (d == q && v < 0.0)) fl |= 1;
            if (d != q && v != 0.0) fl |= (d == 2 || q == 2) ? 4 : 2;
            if (c > 0) {
                const long long dd = (long long)(4 * d) * n;
                const double tol = 1e-12 * fmax(fabs(U[dd + i]), fabs(U[dd + row * np]));
                if (!(fabs(v - U[k * n + row * np]) <= tol)) fl |= 8;
            }
        }
    }
    if (fl) atomicOr(&sflag, fl);
    __syncthreads();
    if (threadIdx.x == 0) flags[blockIdx.x] = sflag;
}

// Natural-layout metrics [9][nr][nt][np] into a level's storage: one entry
// per (r, theta) when phi-invariant (nc == 1: the c = 0 entry), else the
// parity-split layout of the level's fields (as k_metrics writes them).
__global__ void __launch_bounds__(kBlock) k_store_metrics(int nr, int nt, int np, int nc,
                                                          const double* __restrict__ U,
                                                          double* __restrict__ G)
{
    const long long n = (long long)nr * nt * np, gk = (long long)nr * nt * nc;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= gk) return;
    const int c = (int)(i % nc);
    const long long row = i / nc;
    const long long oi = nc == 1 ? i : (long long)(c & 1) * (gk / 2) + row * (np / 2) + (c >> 1);
    for (int k = 0; k < 9; ++k) G[k * gk + oi] = U[k * n + row * np + c];
}

// Face metrics of the next coarser level, natural layout: the low d-face of
// coarse cell (A, B, C) is made of the four fine low d-faces at index 2A,
// 2B or 2C along d and the two fine indices of each other direction; a
// face metric is an area over a normal length, so the coarse face (four
// times the area, twice the length) takes half the sum of the four.
__global__ void __launch_bounds__(kBlock) k_coarsen_metrics(int nr, int nt, int np,
                                                            const double* __restrict__ Uf,
                                                            double* __restrict__ Uc)
{
    const int cr = nr / 2, ct = nt / 2, cp = np / 2;
    const long long nf = (long long)nr * nt * np, ncl = (long long)cr * ct * cp;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ncl) return;
    const int C = (int)(i % cp);
    const long long row = i / cp;
    const int B = (int)(row % ct), A = (int)(row / ct);
    for (int k = 0; k < 9; ++k) {
        const int d = k / 3;
        double s = 0.0;
        for (int u = 0; u < 2; ++u)
            for (int v = 0; v < 2; ++v) {
                const int a = 2 * A + (d == 0 ? 0 : u);
                const int b = 2 * B + (d == 1 ? 0 : (d == 0 ? u : v));
                const int c = 2 * C + (d == 2 ? 0 : v);
                s += Uf[k * nf + ((long long)a * nt + b) * np + c];
            }
        Uc[k * ncl + i] = 0.5 * s;
    }
}

// Float copy of an FP64 array.
__global__ void __launch_bounds__(kBlock) k_to_f32(long long n, const double* __restrict__ a,
                                                   float* __restrict__ b)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

// Expand stored metrics to natural [9][nr][nt][np] (for inspection).
__global__ void __launch_bounds__(kBlock) k_expand_metrics(Geo g, int axi,
                                                           const double* __restrict__ G,
                                                           double* __restrict__ out)
{
    const long long n = 2 * g.P;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const long long row = i / g.np;
    const int c = (int)(i - row * g.np);
    const long long src = axi ? row : (c & 1) * g.P + row * g.nh + (c >> 1);
    const long long gk = axi ? (long long)g.nr * g.nt : n;
    for (int k = 0; k < 9; ++k) out[k * n + i] = G[k * gk + src];
}

// Dense coarsest operator in parity-split order: row i (cell (a, b, c)) gets
// A[i][j] = (A delta_j)_i for every cell j of the 3x3x3 block around it
// (mirrored / wrapped; a cell reached twice is evaluated once).  A must be
// zeroed first.
template <int MODE, bool AXI>
__global__ void __launch_bounds__(kBlock) k_dense_rows(Level<double> L, double* __restrict__ A)
{
    const Geo& g = L.g;
    const long long n = 2 * g.P;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * 27) return;
    const long long nat = t / 27;
    const int k = (int)(t - nat * 27);
    const long long rowi = nat / g.np;
    const int c = (int)(nat - rowi * g.np);
    const int b = (int)(rowi % g.nt), a = (int)(rowi / g.nt);
    auto nb = [&](int q) {
        const int da = q / 9 - 1, db = (q / 3) % 3 - 1, dc = q % 3 - 1;
        const int aa = clampi(a + da, g.nr - 1), bb = clampi(b + db, g.nt - 1);
        int cc = c + dc;
        cc = cc < 0 ? cc + g.np : (cc >= g.np ? cc - g.np : cc);
        return split_index(g, aa, bb, cc);
    };
    const long long j = nb(k);
    for (int q = 0; q < k; ++q)
        if (nb(q) == j) return;
    double D;
    const long long i = split_index(g, a, b, c);
    A[i * n + j] = apply_cell<double, MODE, AXI>(g, L.G, L.gk, Delta<double>{j}, a, b, c & 1, c >> 1, D);
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

// Blocked Gauss-Jordan inversion of the augmented n x 2n matrix [A | I]
// with partial pivoting, in place.  Columns are taken in panels of KB.
// The pivot of column c is the not-yet-used row with the largest |entry|
// (lowest index on ties); used_at[i] = column at which row i became a pivot
// (INT_MAX before).  For a panel:
//  - k_gj_panel (one block of kGJThreads, R rows per thread, the rows' panel
//    entries in registers) runs the KB pivot steps on the panel's own
//    columns and, alongside, on KB probe columns E, where probe u is the
//    unit vector of the pivot row of step u (untouched by the steps before
//    it, so it is set when that step starts).  Afterwards any column x of the
//    rest transforms as x' = (x off the panel's pivot rows) + E x[pivots].
//  - k_gj_pivrows copies the panel's pivot rows aside (Xp) before the update.
//  - k_gj_update applies that rank-KB update to the columns past the panel.
// KB = 16 / R keeps a thread's registers to 2 R KB values (n <= 1024 R).
constexpr int kGJ = 16;          // row stride of E
constexpr int kGJThreads = 1024;

template <int R, int KB>
__global__ void __launch_bounds__(kGJThreads) k_gj_panel(int n, int c0, double* __restrict__ M,
                                                         double* __restrict__ E,
                                                         int* __restrict__ used_at,
                                                         int* __restrict__ piv,
                                                         int* __restrict__ fail)
{
    // per-wave candidates and the broadcast pivot row, alternating between
    // steps so that one barrier separates writers from readers
    __shared__ double sv[2][kGJThreads / 64];
    __shared__ int si[2][kGJThreads / 64];
    __shared__ double prow[2][KB], erow[2][KB];
    const long long w = 2LL * n;
    const int kb = min(KB, n - c0);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    double pv[R][KB], ev[R][KB];
    int used[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = threadIdx.x + r * kGJThreads;
        used[r] = i < n ? used_at[i] : 0; // rows past n never qualify
#pragma unroll
        for (int q = 0; q < KB; ++q) {
            pv[r][q] = (i < n && q < kb) ? M[i * w + c0 + q] : 0.0;
            ev[r][q] = 0.0;
        }
    }
    // entry t of a row's panel values, by selects over compile-time indices:
    // the steps run as a loop (a quarter of the unrolled code), and a
    // register array indexed at run time would live in scratch memory
    auto at = [](const double (&a)[KB], int t) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < KB; ++q) v = q == t ? a[q] : v;
        return v;
    };
#pragma unroll 1
    for (int t = 0; t < kb; ++t) {
        const int c = c0 + t;
        double best = -1.0;
        int bi = -1;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = threadIdx.x + r * kGJThreads;
            const double v = fabs(at(pv[r], t));
            if (used[r] >= c && v > best) { best = v; bi = i; }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double v2 = __shfl_down(best, o);
            const int i2 = __shfl_down(bi, o);
            if (v2 > best || (v2 == best && i2 >= 0 && (bi < 0 || i2 < bi))) { best = v2; bi = i2; }
        }
        const int h = t & 1;
        if (lane == 0) { sv[h][wid] = best; si[h][wid] = bi; }
        __syncthreads();
        // every thread combines the wavefronts' candidates itself (unrolled:
        // the LDS reads issue together instead of one latency per wavefront)
        double bb = sv[h][0];
        int p = si[h][0];
#pragma unroll
        for (int q = 1; q < kGJThreads / 64; ++q) {
            const double v2 = sv[h][q];
            const int i2 = si[h][q];
            if (v2 > bb || (v2 == bb && i2 >= 0 && (p < 0 || i2 < p))) { bb = v2; p = i2; }
        }
        if (p < 0 || bb == 0.0) {
            if (threadIdx.x == 0) *fail = 1;
            return; // uniform: every thread reached the same decision
        }
        // the owner of the pivot row broadcasts it, scaled
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (threadIdx.x + r * kGJThreads == p) {
                used[r] = c;
                used_at[p] = c;
                piv[c] = p;
#pragma unroll
                for (int q = 0; q < KB; ++q)
                    if (q == t) ev[r][q] = 1.0;
                const double inv = 1.0 / at(pv[r], t);
#pragma unroll
                for (int q = 0; q < KB; ++q) {
                    prow[h][q] = q >= t ? pv[r][q] * inv : 0.0;
                    erow[h][q] = ev[r][q] * inv;
                }
            }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = threadIdx.x + r * kGJThreads;
            if (i == p) {
#pragma unroll
                for (int q = 0; q < KB; ++q) {
                    if (q >= t) pv[r][q] = prow[h][q];
                    ev[r][q] = erow[h][q];
                }
            } else {
                const double m = at(pv[r], t);
#pragma unroll
                for (int q = 0; q < KB; ++q) {
                    if (q >= t) pv[r][q] -= m * prow[h][q];
                    ev[r][q] -= m * erow[h][q];
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = threadIdx.x + r * kGJThreads;
        if (i >= n) continue;
#pragma unroll
        for (int q = 0; q < KB; ++q) {
            if (q < kb) M[i * w + c0 + q] = pv[r][q];
            E[(long long)i * kGJ + q] = ev[r][q];
        }
    }
}

// The panel's pivot rows, copied aside before the update of the other
// columns (which overwrites them); only the columns past the panel are read
// from the copy.  Many blocks: in the one-block panel kernel this copy took
// a fifth of its time.
__global__ void __launch_bounds__(kBlock) k_gj_pivrows(int n, int c0, int kb,
                                                       const double* __restrict__ M,
                                                       const int* __restrict__ piv,
                                                       double* __restrict__ Xp)
{
    const long long w = 2LL * n;
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (long long)kb * w) return;
    const int u = (int)(q / w);
    const long long col = q - (long long)u * w;
    Xp[q] = M[(long long)piv[c0 + u] * w + col];
}

// x' = (x off the pivot rows) + E x[pivots] for the columns past the panel.
// A wavefront takes one row and 64 columns; the row's E entries are
// wave-uniform, the pivot rows come from the copy Xp (L2-resident).
__global__ void __launch_bounds__(kBlock) k_gj_update(int n, int c0, int kb, double* __restrict__ M,
                                                      const double* __restrict__ E,
                                                      const double* __restrict__ Xp,
                                                      const int* __restrict__ used_at)
{
    const long long w = 2LL * n;
    const long long cstart = c0 + kb;
    const int ctiles = (int)((w - cstart + 63) / 64);
    const int tile = (int)(blockIdx.x % ctiles), rg = (int)(blockIdx.x / ctiles);
    const int i = rg * (kBlock / 64) + __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const long long col = cstart + (long long)tile * 64 + (threadIdx.x & 63);
    if (i >= n || col >= w) return;
    const int ua = used_at[i];
    double acc = (ua >= c0 && ua < c0 + kb) ? 0.0 : M[i * w + col];
    for (int u = 0; u < kb; ++u) acc += E[(long long)i * kGJ + u] * Xp[(long long)u * w + col];
    M[i * w + col] = acc;
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
