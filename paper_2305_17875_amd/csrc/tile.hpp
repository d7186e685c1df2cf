// tile.hpp -- the V-cycle's small levels in two launches each.  Included by
// cps.hip after kernels.hpp.
//
// On a small level (a few hundred thousand cells or fewer) every kernel of
// the cycle is short and its launch dominates: 11 launches a level (4
// pre-smoothing passes, residual, restriction, prolongation, 4
// post-smoothing passes).  Here the cycle's work on such a level is two
// launches, each block owning one 8 x 8 x 8 tile of cells and working in LDS:
//  - pre: red-black Gauss-Seidel from a zero iterate (colours 0, 1, 0, 1),
//    the residual of the smoothed iterate, and its full-weighting
//    restriction onto the tile's 4 x 4 x 4 coarse cells;
//  - post: the trilinear prolongation of the coarse correction added to the
//    iterate, then the colours 1, 0, 1, 0.
// Same operator, smoother, transfers and wall treatment as the per-kernel
// path (7-point stencil with phi-invariant metrics, Sec. on the multigrid
// solver): the results agree with it to rounding.  The sums are formed in
// another order, so the bits differ; the single and batched forms share
// these bodies, so they agree with each other bit for bit.
//
// A pass on a tile needs the other colour one cell beyond the cells it
// updates, so the tile is loaded with a halo and the passes shrink the
// region they update by one cell each: pre loads a halo of 5 (the zero pass
// reads no neighbour; three more passes; the residual one cell beyond the
// tile; its neighbours one beyond that), post a halo of 4.  Halo cells are
// recomputed by every tile that loads them and written only by their own
// tile; post reads the iterate of one buffer and writes another, so no
// block reads a cell another block has already overwritten.  Cells past the
// r- and theta-walls are zero in LDS and meet a zero wall metric; phi
// wraps.
//
// Pre ends on the black pass, so the black residual is zero (to rounding):
// only the red residual is formed and restricted, as on the row-pair
// levels of the per-kernel path.

namespace cps {

constexpr int kTile = 8;            // owned cells per dimension
constexpr int kTileThreads = 1024;  // threads per tile block
constexpr int kPreHalo = 5, kPostHalo = 4;
constexpr int kPreR = kTile + 2 * kPreHalo;   // 18
constexpr int kPostR = kTile + 2 * kPostHalo; // 16
constexpr int kResR = kTile + 2;              // residual box: the tile +- 1
constexpr int kCoarseR = kTile / 2 + 6;       // coarse correction box of post

// A level takes the tile path when it is small enough that its launches
// dominate and its rings split into whole tiles (the finest level only in
// cycles from a zero iterate; its Krylov dot products then come from a
// separate reduction).  A tile block
// takes 8-12 us (its phases are LDS-latency bound); on the paper-scale
// shell the 24 x 32 x 64 and 12 x 16 x 32 levels gain (pre + post 21 and
// 17 us against 46 and 38 us of per-kernel launches), the 48 x 64 x 128
// level does not (768 tiles at one 117 KB block per CU: 61 against 52 us).
// FP32 tiles take half the LDS (58 KB pre, 43 KB post), two blocks share a
// CU, and the 48 x 64 x 128 level runs in two rounds instead of three.
constexpr long long kTileMaxCells = 1LL << 16;
constexpr long long kTileMaxCells32 = 1LL << 19;

__host__ __device__ inline long long tile_max_cells(bool fp32)
{
    return fp32 ? kTileMaxCells32 : kTileMaxCells;
}

__host__ __device__ inline bool tile_fits(const Geo& g, bool fp32 = false)
{
    return g.np % kTile == 0 && g.nr % 2 == 0 && g.nt % 2 == 0 &&
           (long long)g.nr * g.nt * g.np <= tile_max_cells(fp32);
}

__host__ __device__ inline int tile_count(const Geo& g)
{
    return cdiv(g.nr, kTile) * cdiv(g.nt, kTile) * (g.np / kTile);
}

__device__ __forceinline__ void tile_origin(const Geo& g, int t, int& A0, int& B0, int& C0)
{
    const int nc = g.np / kTile, nb = cdiv(g.nt, kTile);
    C0 = (t % nc) * kTile;
    t /= nc;
    B0 = (t % nb) * kTile;
    A0 = (t / nb) * kTile;
}

// offset of cell (a, b, c) in the parity-split layout
__device__ __forceinline__ long long tile_at(const Geo& g, int a, int b, int c)
{
    return (long long)(c & 1) * g.P + (long long)a * g.rowlen + (long long)b * g.nh + (c >> 1);
}

__device__ __forceinline__ int wrapi(int c, int n)
{
    c %= n;
    return c < 0 ? c + n : c;
}

// metrics of row (a, b): the five face values and 1 / D (D: minus the sum
// of all six; a product in the passes, not a division on their dependent
// chain)
template <typename T>
__device__ __forceinline__ void tile_metrics(const Geo& g, const T* __restrict__ G, long long gk,
                                             int a, int b, T m[6])
{
    const long long ci = (long long)a * g.nt + b;
    m[0] = G[ci];                                  // r low
    m[1] = a < g.nr - 1 ? G[ci + g.nt] : T(0);     // r high
    m[2] = G[4 * gk + ci];                         // theta low
    m[3] = b < g.nt - 1 ? G[4 * gk + ci + 1] : T(0); // theta high
    m[4] = G[8 * gk + ci];                         // phi (both faces)
    m[5] = T(1) / -(m[0] + m[1] + m[2] + m[3] + m[4] + m[4]);
}

template <typename T>
struct TilePreLds {
    T x[kPreR * kPreR * kPreR];
    T b[kPreR * kPreR * kPreR]; // right-hand side; then the restriction's partial sums
    T m[kPreR * kPreR][6];
    T r[kResR * kResR * kResR];
};

template <typename T>
struct TilePostLds {
    T x[kPostR * kPostR * kPostR];
    T b[kPostR * kPostR * kPostR];
    T m[kPostR * kPostR][6];
    T e[kCoarseR * kCoarseR * kCoarseR];
};

// One colour pass over the region box [s, R - s)^3 (clipped to the domain in
// r and theta) of a tile's LDS copy with origin (ra, rb, rc): each cell of
// the colour takes x = (b - S) / D from its six neighbours.  zero: the
// first pass from a zero iterate, x = b / D, reads no neighbour (so s may
// be 0: the region's outer layer has none in LDS).  Cells past the walls
// keep metrics 0 and are never updated.
template <typename T, int R>
__device__ __forceinline__ void tile_pass(const Geo& g, int ra, int rb, int rc, int s, int col,
                                          bool zero, T* __restrict__ x, const T* __restrict__ bl,
                                          const T (*__restrict__ m)[6])
{
    const int a_lo = max(s, -ra), a_hi = min(R - s, g.nr - ra);
    const int b_lo = max(s, -rb), b_hi = min(R - s, g.nt - rb);
    const int na = a_hi - a_lo, nb = b_hi - b_lo, nh = (R - 2 * s) / 2;
    const int cells = na * nb * nh;
    for (int i = (int)threadIdx.x; i < cells; i += (int)blockDim.x) {
        const int t = i % nh, rowi = i / nh;
        const int bb = b_lo + rowi % nb, aa = a_lo + rowi / nb;
        const int cc = s + 2 * t + ((col + ra + aa + rb + bb + rc + s) & 1);
        const int k = (aa * R + bb) * R + cc;
        const T* mm = m[aa * R + bb];
        if (zero) {
            x[k] = bl[k] * mm[5];
            continue;
        }
        const T S = mm[1] * x[k + R * R] + mm[0] * x[k - R * R] + mm[3] * x[k + R] +
                    mm[2] * x[k - R] + mm[4] * (x[k - 1] + x[k + 1]);
        x[k] = (bl[k] - S) * mm[5];
    }
}

// Pre: bc (the tile's coarse cells) = R r, r = b - A x, x = 2 red-black
// sweeps from zero of A x = b; x is written on the tile's cells.
template <typename T>
__device__ __forceinline__ void d_vpre_tile(Blk bk, Geo f, const T* __restrict__ G, long long gk,
                                            const T* __restrict__ bv, T* __restrict__ x,
                                            Geo c, T* __restrict__ bc, TilePreLds<T>& sh)
{
    constexpr int R = kPreR, H = kPreHalo;
    if ((int)bk.L >= tile_count(f)) return; // whole block
    int A0, B0, C0;
    tile_origin(f, (int)bk.L, A0, B0, C0);
    const int ra = A0 - H, rb = B0 - H, rc = C0 - H;
    const int tid = (int)threadIdx.x, nt = (int)blockDim.x;
    // every load of a thread goes out before any is stored (a loop that
    // stores each value before the next load waits on every one in turn)
    constexpr int NL = (R * R * R + kTileThreads - 1) / kTileThreads;
    T v[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int i = tid + k * kTileThreads;
        const int cc = i % R, bb = (i / R) % R, aa = i / (R * R);
        const int a = ra + aa, b = rb + bb;
        v[k] = T(0);
        if (i < R * R * R && a >= 0 && a < f.nr && b >= 0 && b < f.nt)
            v[k] = bv[tile_at(f, a, b, wrapi(rc + cc, f.np))];
    }
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int i = tid + k * kTileThreads;
        if (i < R * R * R) {
            sh.b[i] = v[k];
            sh.x[i] = T(0);
        }
    }
    for (int i = tid; i < R * R; i += nt) {
        const int a = ra + i / R, b = rb + i % R;
        if (a >= 0 && a < f.nr && b >= 0 && b < f.nt) tile_metrics(f, G, gk, a, b, sh.m[i]);
        else
            for (int q = 0; q < 6; ++q) sh.m[i][q] = T(0);
    }
    __syncthreads();
    // colours 0, 1, 0, 1; the first from zero reads no neighbour (shrink 0)
    for (int k = 0; k < 4; ++k) {
        tile_pass<T, R>(f, ra, rb, rc, k, k & 1, k == 0, sh.x, sh.b, sh.m);
        __syncthreads();
    }
    // the tile's cells of x
    for (int i = tid; i < kTile * kTile * kTile; i += nt) {
        const int cc = i % kTile, bb = (i / kTile) % kTile, aa = i / (kTile * kTile);
        const int a = A0 + aa, b = B0 + bb;
        if (a < f.nr && b < f.nt)
            x[tile_at(f, a, b, C0 + cc)] = sh.x[((aa + H) * R + bb + H) * R + cc + H];
    }
    // red residual on the tile +- 1 (black cells and cells past the walls 0)
    constexpr int Q = kResR;
    for (int i = tid; i < Q * Q * Q; i += nt) {
        const int qc = i % Q, qb = (i / Q) % Q, qa = i / (Q * Q);
        const int aa = qa + H - 1, bb = qb + H - 1, cc = qc + H - 1;
        const int a = ra + aa, b = rb + bb;
        T rv = T(0);
        if (a >= 0 && a < f.nr && b >= 0 && b < f.nt && ((a + b + rc + cc) & 1) == 0) {
            const int k = (aa * R + bb) * R + cc;
            const T* mm = sh.m[aa * R + bb];
            const T u = sh.x[k];
            const T y = mm[1] * (sh.x[k + R * R] - u) - mm[0] * (u - sh.x[k - R * R]) +
                        mm[3] * (sh.x[k + R] - u) - mm[2] * (u - sh.x[k - R]) +
                        mm[4] * (sh.x[k + 1] - u) - mm[4] * (u - sh.x[k - 1]);
            rv = sh.b[k] - y;
        }
        sh.r[i] = rv;
    }
    __syncthreads();
    // full weighting onto the coarse cells I = A0/2 .. +3 (weights 1 3 3 1
    // over fine 2I-1 .. 2I+2 in each direction, rows and planes clamped at
    // the walls, phi wrapped), phi first, then theta, then r
    const T w0 = T(0.25), w1 = T(0.75);
    const T w[4] = {w0, w1, w1, w0};
    constexpr int K4 = kTile / 2;
    T* pphi = sh.b;                 // [Q][Q][K4]: phi sums of the residual box rows
    T* pth = sh.b + Q * Q * K4;     // [Q][K4][K4]: then theta
    for (int i = tid; i < Q * Q * K4; i += nt) {
        const int kk = i % K4, row = i / K4;
        const T* rr = sh.r + row * Q + 2 * kk; // fine c = C0 + 2kk - 1 .. +2 at box 2kk .. 2kk+3
        T s = T(0);
        for (int t = 0; t < 4; ++t) s += w[t] * rr[t];
        pphi[i] = s;
    }
    __syncthreads();
    for (int i = tid; i < Q * K4 * K4; i += nt) {
        const int kk = i % K4, jj = (i / K4) % K4, qa = i / (K4 * K4);
        const int J = B0 / 2 + jj;
        T s = T(0);
        for (int q = 0; q < 4; ++q) {
            const int b = clampi(2 * J - 1 + q, f.nt - 1); // fine row, mirrored at the walls
            s += w[q] * pphi[(qa * Q + (b - B0 + 1)) * K4 + kk];
        }
        pth[i] = s;
    }
    __syncthreads();
    for (int i = tid; i < K4 * K4 * K4; i += nt) {
        const int kk = i % K4, jj = (i / K4) % K4, ii = i / (K4 * K4);
        const int I = A0 / 2 + ii, J = B0 / 2 + jj, K = C0 / 2 + kk;
        if (I >= c.nr || J >= c.nt) continue;
        T s = T(0);
        for (int p = 0; p < 4; ++p) {
            const int a = clampi(2 * I - 1 + p, f.nr - 1);
            s += w[p] * pth[((a - A0 + 1) * K4 + jj) * K4 + kk];
        }
        bc[tile_at(c, I, J, K)] = s;
    }
}

// Post: xo = 2 red-black sweeps (colours 1, 0, 1, 0) of A x = b from
// xi + P e on the tile's cells.
template <typename T>
__device__ __forceinline__ void d_vpost_tile(Blk bk, Geo f, const T* __restrict__ G, long long gk,
                                             const T* __restrict__ bv, const T* __restrict__ xi,
                                             T* __restrict__ xo, Geo c, const T* __restrict__ e,
                                             TilePostLds<T>& sh)
{
    constexpr int R = kPostR, H = kPostHalo, E = kCoarseR;
    if ((int)bk.L >= tile_count(f)) return; // whole block
    int A0, B0, C0;
    tile_origin(f, (int)bk.L, A0, B0, C0);
    const int ra = A0 - H, rb = B0 - H, rc = C0 - H;
    // coarse box: I = A0/2 - 3 .. A0/2 + 6 (rows and planes clamped, phi wrapped)
    const int ea = A0 / 2 - 3, eb = B0 / 2 - 3, ec = C0 / 2 - 3;
    const int tid = (int)threadIdx.x, nt = (int)blockDim.x;
    // loads before stores, as in pre
    constexpr int NE = (E * E * E + kTileThreads - 1) / kTileThreads;
    constexpr int NX = (R * R * R + kTileThreads - 1) / kTileThreads;
    T ev[NE], xv[NX], bw[NX];
#pragma unroll
    for (int k = 0; k < NE; ++k) {
        const int i = tid + k * kTileThreads;
        const int kc = i % E, kb = (i / E) % E, ka = i / (E * E);
        ev[k] = i < E * E * E ? e[tile_at(c, clampi(ea + ka, c.nr - 1), clampi(eb + kb, c.nt - 1),
                                           wrapi(ec + kc, c.np))]
                              : T(0);
    }
#pragma unroll
    for (int k = 0; k < NX; ++k) {
        const int i = tid + k * kTileThreads;
        const int cc = i % R, bb = (i / R) % R, aa = i / (R * R);
        const int a = ra + aa, b = rb + bb;
        xv[k] = T(0);
        bw[k] = T(0);
        if (i < R * R * R && a >= 0 && a < f.nr && b >= 0 && b < f.nt) {
            const long long o = tile_at(f, a, b, wrapi(rc + cc, f.np));
            xv[k] = xi[o];
            bw[k] = bv[o];
        }
    }
#pragma unroll
    for (int k = 0; k < NE; ++k) {
        const int i = tid + k * kTileThreads;
        if (i < E * E * E) sh.e[i] = ev[k];
    }
    for (int i = tid; i < R * R; i += nt) {
        const int a = ra + i / R, b = rb + i % R;
        if (a >= 0 && a < f.nr && b >= 0 && b < f.nt) tile_metrics(f, G, gk, a, b, sh.m[i]);
        else
            for (int q = 0; q < 6; ++q) sh.m[i][q] = T(0);
    }
    __syncthreads();
    const T w0 = T(0.75), w1 = T(0.25);
#pragma unroll
    for (int k = 0; k < NX; ++k) {
        const int i = tid + k * kTileThreads;
        if (i >= R * R * R) continue;
        const int cc = i % R, bb = (i / R) % R, aa = i / (R * R);
        const int a = ra + aa, b = rb + bb, cg = rc + cc;
        T xn = T(0);
        if (a >= 0 && a < f.nr && b >= 0 && b < f.nt) {
            // fine 2I takes 3/4 of coarse I and 1/4 of I - 1, fine 2I + 1 of
            // I and I + 1, in each direction: theta, then phi, then r
            const int I = a >> 1, J = b >> 1, K = cg >> 1; // cg may be negative: floor
            const int ka = I - ea, kb = J - eb, kc = K - ec;
            const int da = (a & 1) ? 1 : -1, db = (b & 1) ? 1 : -1, dc = (cg & 1) ? 1 : -1;
            T tr[2];
            for (int pa = 0; pa < 2; ++pa) {
                const int ia = ka + (pa ? da : 0);
                T tp[2];
                for (int pc = 0; pc < 2; ++pc) {
                    const int ic = kc + (pc ? dc : 0);
                    const T* ee = sh.e + ia * E * E + ic;
                    tp[pc] = w0 * ee[kb * E] + w1 * ee[(kb + db) * E];
                }
                tr[pa] = w0 * tp[0] + w1 * tp[1];
            }
            xn = xv[k] + (w0 * tr[0] + w1 * tr[1]);
        }
        sh.x[i] = xn;
        sh.b[i] = bw[k];
    }
    __syncthreads();
    // colours 1, 0, 1, 0, each on a region one cell smaller
    for (int k = 0; k < 4; ++k) {
        tile_pass<T, R>(f, ra, rb, rc, k + 1, 1 - (k & 1), false, sh.x, sh.b, sh.m);
        __syncthreads();
    }
    for (int i = tid; i < kTile * kTile * kTile; i += nt) {
        const int cc = i % kTile, bb = (i / kTile) % kTile, aa = i / (kTile * kTile);
        const int a = A0 + aa, b = B0 + bb;
        if (a < f.nr && b < f.nt)
            xo[tile_at(f, a, b, C0 + cc)] = sh.x[((aa + H) * R + bb + H) * R + cc + H];
    }
}

template <typename T>
__global__ void __launch_bounds__(kTileThreads) k_vpre_tile(Geo f, const T* __restrict__ G,
                                                            long long gk, const T* __restrict__ bv,
                                                            T* __restrict__ x, Geo c,
                                                            T* __restrict__ bc)
{
    __shared__ TilePreLds<T> sh;
    d_vpre_tile<T>(self_blk(), f, G, gk, bv, x, c, bc, sh);
}

template <typename T>
__global__ void __launch_bounds__(kTileThreads) k_vpost_tile(Geo f, const T* __restrict__ G,
                                                             long long gk,
                                                             const T* __restrict__ bv,
                                                             const T* __restrict__ xi,
                                                             T* __restrict__ xo, Geo c,
                                                             const T* __restrict__ e)
{
    __shared__ TilePostLds<T> sh;
    d_vpost_tile<T>(self_blk(), f, G, gk, bv, xi, xo, c, e, sh);
}

// Batched forms: one block per (problem, tile) of the work table.
template <typename T>
__global__ void __launch_bounds__(kTileThreads) kb_vpre_tile(const BItem* __restrict__ items,
                                                             const int* __restrict__ active,
                                                             const PDesc<T>* __restrict__ pd,
                                                             int level)
{
    CPS_BATCH_BLOCK
    __shared__ TilePreLds<T> sh;
    const LDesc<T>& d = pd[it.prob].lv[level];
    const LDesc<T>& c = pd[it.prob].lv[level + 1];
    // as vcycle(): the finest level's pre-smoothed iterate goes to xt
    d_vpre_tile<T>(bk, d.g, d.G, d.gk, d.b, level == 0 ? d.xt : d.x, c.g, c.b, sh);
}

template <typename T>
__global__ void __launch_bounds__(kTileThreads) kb_vpost_tile(const BItem* __restrict__ items,
                                                              const int* __restrict__ active,
                                                              const PDesc<T>* __restrict__ pd,
                                                              int level)
{
    CPS_BATCH_BLOCK
    __shared__ TilePostLds<T> sh;
    const LDesc<T>& d = pd[it.prob].lv[level];
    const LDesc<T>& c = pd[it.prob].lv[level + 1];
    // the finest level reads xt and writes x; the others read x, write xt
    d_vpost_tile<T>(bk, d.g, d.G, d.gk, d.b, level == 0 ? d.xt : d.x, level == 0 ? d.x : d.xt,
                    c.g, c.tile ? c.xt : c.x, sh);
}

} // namespace cps
