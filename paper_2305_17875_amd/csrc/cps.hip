// cps.hip -- hierarchy, V-cycle, outer iterations and the C ABI.
//
// The library solves eq. (PC_6) of the shell solver (pressure correction)
// by geometric multigrid on the transformed grid: face metrics computed on
// the device for every level (Sec. 3.2), the flux-form operator of eq.
// (PC_8), colour Gauss-Seidel smoothing, full-weighting restriction,
// trilinear prolongation, a dense exact coarsest solve, V(2,2) cycles, and an
// outer stationary or Krylov iteration, in FP64 or with FP32 V-cycles inside
// FP64 refinement.
#include "cps.h"
#include "kernels.hpp"
#include "plane.hpp"
#include "project.hpp"
#include "lines.hpp"
#include "tile.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>
#include <map>
#include <mutex>
#include <shared_mutex>
#include <condition_variable>
#include <deque>
#include <memory>
#include <thread>

using namespace cps;

namespace {

thread_local std::string g_err;

struct Fail {
    cps_status st;
};

[[noreturn]] void fail(cps_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
[[noreturn]] void fail(cps_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    throw Fail{st};
}

#define HIPC(call)                                                                         \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            fail(e_ == hipErrorOutOfMemory ? CPS_E_OOM : CPS_E_HIP, "%s: %s (%s:%d)", #call, \
                 hipGetErrorString(e_), __FILE__, __LINE__);                               \
    } while (0)

#define LAUNCH_CHECK() HIPC(hipGetLastError())

constexpr long long kMaxCoarse = 4096;

inline unsigned nblk(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }
// capped grid of a stencil launch over nr planes of bpa blocks each
inline unsigned grid_of(int nr, int bpa) { return (unsigned)std::min<long long>((long long)nr * bpa, kMaxGrid); }
// capped grid of a grid-stride vector launch
inline unsigned vgrid(long long n) { return std::min<unsigned>(nblk(n), kMaxGrid); }

template <int M>
using IM = std::integral_constant<int, M>;
template <bool B>
using BA = std::integral_constant<bool, B>;

// Calls f(MODE, AXI, UROW, LTAG) as integral constants for a level: the
// stencil shape, phi-invariant metrics, wave-uniform rows (n_phi / 2 a
// multiple of 64) and the finest-level tag.
template <typename F>
void dispatch4(int mode, bool axi, bool urow, int ltag, F&& f)
{
    auto rest = [&](auto M, auto A) {
        if (urow) {
            if (ltag == 0) f(M, A, BA<true>{}, IM<0>{});
            else f(M, A, BA<true>{}, IM<1>{});
        } else {
            if (ltag == 0) f(M, A, BA<false>{}, IM<0>{});
            else f(M, A, BA<false>{}, IM<1>{});
        }
    };
    if (axi) {
        if (mode == MODE_ORTHO) rest(IM<MODE_ORTHO>{}, BA<true>{});
        else if (mode == MODE_RT) rest(IM<MODE_RT>{}, BA<true>{});
        else rest(IM<MODE_FULL>{}, BA<true>{});
    } else {
        if (mode == MODE_ORTHO) rest(IM<MODE_ORTHO>{}, BA<false>{});
        else if (mode == MODE_RT) rest(IM<MODE_RT>{}, BA<false>{});
        else rest(IM<MODE_FULL>{}, BA<false>{});
    }
}

template <typename F>
void dispatch(int mode, bool axi, F&& f)
{
    if (axi) {
        if (mode == MODE_ORTHO) f(IM<MODE_ORTHO>{}, BA<true>{});
        else if (mode == MODE_RT) f(IM<MODE_RT>{}, BA<true>{});
        else f(IM<MODE_FULL>{}, BA<true>{});
    } else {
        if (mode == MODE_ORTHO) f(IM<MODE_ORTHO>{}, BA<false>{});
        else if (mode == MODE_RT) f(IM<MODE_RT>{}, BA<false>{});
        else f(IM<MODE_FULL>{}, BA<false>{});
    }
}

// Graph capture and memory management exclude each other, process-wide.
// Freeing device memory synchronises the device, and a device-wide (or
// null-stream) synchronisation while another thread's stream is being
// captured invalidates that capture: with several service workers (or a
// service beside other handles), one worker building or dropping a
// hierarchy would break another's capture of its iteration bodies.
// Captures take the lock shared (they may overlap each other: each is on
// its own non-blocking stream); device and pinned host allocations, frees
// and synchronous null-stream uploads take it exclusively.
std::shared_mutex g_capture_mu;
using MemLock = std::unique_lock<std::shared_mutex>;

// A synchronous upload of set-up tables (pageable host memory).
void upload(void* dst, const void* src, size_t bytes)
{
    MemLock lk(g_capture_mu);
    HIPC(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
}

// Owning device buffer (freed on destruction; not copyable).
template <typename T>
struct Buf {
    T* p = nullptr;
    size_t n = 0;
    Buf() = default;
    Buf(const Buf&) = delete;
    Buf& operator=(const Buf&) = delete;
    ~Buf() { release(); }
    void alloc(size_t count)
    {
        MemLock lk(g_capture_mu);
        if (p) HIPC(hipFree(p));
        p = nullptr;
        n = count;
        if (count) HIPC(hipMalloc(&p, count * sizeof(T)));
    }
    void release()
    {
        if (!p) return;
        MemLock lk(g_capture_mu);
        (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
};

struct LevelMem {
    int nr = 0, nt = 0, np = 0, nc = 0;
    long long n = 0, gk = 0;
    Geo geo{};
    Buf<double> G64;
    Buf<float> G32;
    Buf<double> x64, b64, r64;
    Buf<float> x32, b32, r32;
    // small levels of the point smoother (tile.hpp): the V-cycle's work on
    // the level is two launches; the post-smoothed iterate goes to xt
    bool tile = false;
    Buf<double> xt64;
    Buf<float> xt32;
    int gs_ch = 0; // marching chunk of the colour pass (0 = default; autotuned)
    // plane smoother's launch shapes (0 = default; autotuned): rings per
    // block of the transforms, r-steps in flight per lane of the elimination
    int plane_rb = 0, plane_tb = 0;
    // plane smoother: twiddles exp(-2 pi i q / nh) (q < nh/2), exp(-2 pi i m /
    // n_phi) (m <= nh) as (re, im) pairs, and the symbols 2 cos(2 pi m/n_phi) - 2
    Buf<double> tw64, twN64, lam64;
    Buf<float> tw32, twN32, lam32;
    // inverse pivots of the r-line eliminations of both parities (plane.hpp)
    Buf<double> pv64;
    Buf<float> pv32;
};

} // namespace

struct cps_handle {
    cps_grid grid{};
    cps_metrics met{};
    cps_opts opts{};
    hipStream_t stream = nullptr;
    // coarsest-inverse scratch (augmented matrix, dense operator, panel
    // buffers, pivots); kept between set-ups when keep_gj
    Buf<double> gjA, gjM, gjE, gjXp;
    Buf<int> gjUsed, gjPiv, gjBad;
    bool keep_gj = false;
    int L = 0;
    LevelMem lv[kMaxLevels];
    int mode = MODE_ORTHO;
    bool axi = true;
    int ncol = 2;
    int nc = 0;
    Buf<double> Ainv;
    Buf<double> partial;
    Buf<double> sc; // device scalars (S_* slots)
    double* hsc = nullptr; // pinned host mirror
    // level-0 FP64 work vectors
    Buf<double> x0, b0, r, z, pd, q, r0, v, s, t, ph, sh;
    // plane smoother scratch: the spectra of one parity
    Buf<double> ps64;
    Buf<float> ps32;
    // projection step (finest grid, built on first use): C rows and
    // determinants of the faces, cell |J^-1|, the divergence right-hand side
    Buf<double> pC, pJf, pJc, prhs, prot;
    // ADI line solves (built on first use): elimination tables of the
    // distinct open r- and theta-lines with the (coef, walls) they were built
    // for, the periodic lines' scratch, and the ring transform's tables
    Buf<double> plf[2], pls, plam;
    Buf<double> ptw, ptwN;
    bool lf_valid[2] = {false, false};
    double lf_coef[2] = {0.0, 0.0};
    LineBC lf_bc[2] = {};
    bool cm_valid = false;
    // captured outer-iteration bodies (G_* keys), replayed by run_body
    hipGraphExec_t gexec[4] = {};
    // optional HIP-event timing of the finest-level kernels, per class
    bool prof = false;
    uint32_t prof_mask = ~0u; // kernel classes recorded while prof is on
    std::vector<hipEvent_t> ev[CPS_KERNEL_CLASSES];
    size_t ev_used[CPS_KERNEL_CLASSES] = {};
    int64_t ev_launches[CPS_KERNEL_CLASSES] = {}; // launches the recorded spans cover
};

namespace {

template <typename T>
Level<T> view(const cps_handle* h, int l);

template <>
Level<double> view<double>(const cps_handle* h, int l)
{
    const LevelMem& m = h->lv[l];
    return Level<double>{m.geo, m.G64.p, m.gk};
}

template <>
Level<float> view<float>(const cps_handle* h, int l)
{
    const LevelMem& m = h->lv[l];
    return Level<float>{m.geo, m.G32.p, m.gk};
}

template <typename T>
T* xl(cps_handle* h, int l);
template <>
double* xl<double>(cps_handle* h, int l) { return h->lv[l].x64.p; }
template <>
float* xl<float>(cps_handle* h, int l) { return h->lv[l].x32.p; }
template <typename T>
T* bl(cps_handle* h, int l);
template <>
double* bl<double>(cps_handle* h, int l) { return h->lv[l].b64.p; }
template <>
float* bl<float>(cps_handle* h, int l) { return h->lv[l].b32.p; }
template <typename T>
T* rl(cps_handle* h, int l);
template <>
double* rl<double>(cps_handle* h, int l) { return h->lv[l].r64.p; }
template <>
float* rl<float>(cps_handle* h, int l) { return h->lv[l].r32.p; }
template <typename T>
T* xtl(cps_handle* h, int l);
template <>
double* xtl<double>(cps_handle* h, int l) { return h->lv[l].xt64.p; }
template <>
float* xtl<float>(cps_handle* h, int l) { return h->lv[l].xt32.p; }
// where level l's iterate is after its post-smoothing (l > 0)
template <typename T>
T* xfin(cps_handle* h, int l)
{
    return h->lv[l].tile ? xtl<T>(h, l) : xl<T>(h, l);
}

// Brackets one finest-level launch of kernel class k with two events on the
// handle's stream (no-op unless profiling is enabled).
// One event pair around `count` consecutive launches of class k on the
// finest level (k < 0: not recorded).
struct ProfScope {
    cps_handle* h;
    int k;
    hipEvent_t stop = nullptr;
    ProfScope(cps_handle* hh, int kk, int level, int count = 1) : h(hh), k(kk)
    {
        if (!h->prof || level != 0 || k < 0 || count < 1 || !((h->prof_mask >> k) & 1u)) return;
        h->ev_launches[k] += count;
        auto& v = h->ev[k];
        size_t& u = h->ev_used[k];
        while (v.size() < u + 2) {
            hipEvent_t e;
            HIPC(hipEventCreate(&e));
            v.push_back(e);
        }
        HIPC(hipEventRecord(v[u], h->stream));
        stop = v[u + 1];
        u += 2;
    }
    ~ProfScope() noexcept(false)
    {
        if (stop) HIPC(hipEventRecord(stop, h->stream));
    }
};

// ---------------------------------------------------------------------------
// kernel launchers
// ---------------------------------------------------------------------------

template <typename T>
void fill(cps_handle* h, T* x, long long n, T v)
{
    k_fill<T><<<nblk(n), kBlock, 0, h->stream>>>(n, x, v);
    LAUNCH_CHECK();
}

// marching kernels serve the 7-point stencil with phi-invariant metrics
inline bool marching(const cps_handle* h) { return h->mode == MODE_ORTHO && h->axi; }

// One colour pass; zero: the iterate is zero before this pass (two colours
// only), so the other colour is not read and need not be initialised.
// dot (marching levels only): per-block partial sums of b . x over the
// updated cells, written at dot[0 .. grid); returns the number written.
template <typename T>
long long gs_pass(cps_handle* h, int l, int colour, const T* b, T* x, bool zero = false,
                  double* dot = nullptr, bool grouped = false)
{
    const Level<T> L = view<T>(h, l);
    const int rowlen = h->ncol == 2 ? L.g.rowlen : L.g.rowlen / 2;
    const int bpa = (int)nblk(rowlen);
    const int z = zero ? 1 : 0;
    // the zero-iterate first pass moves fewer bytes: not in the GS class;
    // grouped: timed with its neighbours by the caller
    ProfScope ps(h, zero || grouped ? -1 : CPS_KERNEL_GS, l);
    if (marching(h)) {
        const MarchShape ms = gs_shape<T>(L.g, h->lv[l].gs_ch);
        if (row_pairs(L.g)) {
            auto launch = [&](auto T_, auto Z) {
                k_gs_march2<T, decltype(T_)::value, decltype(Z)::value>
                    <<<ms.grid, kBlock, 0, h->stream>>>(L.g, L.G, L.gk, ms.bpa, ms.ch, b, x, colour,
                                                        dot);
            };
            if (l == 0) zero ? launch(IM<0>{}, IM<1>{}) : launch(IM<0>{}, IM<0>{});
            else zero ? launch(IM<1>{}, IM<1>{}) : launch(IM<1>{}, IM<0>{});
            LAUNCH_CHECK();
            return dot ? ms.grid : 0;
        }
        auto launch = [&](auto U, auto T_, auto Z) {
            k_gs_march<T, decltype(U)::value, decltype(T_)::value, decltype(Z)::value>
                <<<ms.grid, kBlock, 0, h->stream>>>(L.g, L.G, L.gk, ms.bpa, ms.ch, b, x, colour,
                                                    dot);
        };
        const bool u = L.g.nh % 64 == 0;
        auto by_zero = [&](auto U, auto T_) {
            zero ? launch(U, T_, IM<1>{}) : launch(U, T_, IM<0>{});
        };
        if (l == 0) u ? by_zero(BA<true>{}, IM<0>{}) : by_zero(BA<false>{}, IM<0>{});
        else u ? by_zero(BA<true>{}, IM<1>{}) : by_zero(BA<false>{}, IM<1>{});
        LAUNCH_CHECK();
        return dot ? ms.grid : 0;
    }
    if (dot) fail(CPS_E_INVALID, "internal: fused dot on a non-marching level");
    dispatch4(h->mode, h->axi, L.g.nh % 64 == 0, l == 0 ? 0 : 1, [&](auto M, auto A, auto U, auto T_) {
        k_gs<T, decltype(M)::value, decltype(A)::value, decltype(U)::value, decltype(T_)::value>
            <<<grid_of(L.g.nr, bpa), kBlock, 0, h->stream>>>(L.g, L.G, L.gk, bpa, b, x, colour,
                                                             h->ncol, z);
    });
    LAUNCH_CHECK();
    return 0;
}

// One zebra half-sweep of the plane smoother on level l: the theta rows of
// the given parity, each (r, phi) plane solved exactly (plane.hpp).
template <typename T>
struct PlaneBufs;
template <>
struct PlaneBufs<double> {
    static const double* tw(const LevelMem& m) { return m.tw64.p; }
    static const double* twN(const LevelMem& m) { return m.twN64.p; }
    static const double* lam(const LevelMem& m) { return m.lam64.p; }
    static const double* piv(const LevelMem& m) { return m.pv64.p; }
    static double* S(cps_handle* h) { return h->ps64.p; }
};
template <>
struct PlaneBufs<float> {
    static const float* tw(const LevelMem& m) { return m.tw32.p; }
    static const float* twN(const LevelMem& m) { return m.twN32.p; }
    static const float* lam(const LevelMem& m) { return m.lam32.p; }
    static const float* piv(const LevelMem& m) { return m.pv32.p; }
    static float* S(cps_handle* h) { return h->ps32.p; }
};

// The plane smoother's operator classes: phi-invariant metrics (an
// axisymmetric map) with no cross terms, or with the r-theta ones only.
bool plane_class_ok(const cps_handle* h)
{
    return h->axi && (h->mode == MODE_ORTHO || h->mode == MODE_RT);
}

template <typename T, bool CROSS>
void plane_half_sweep_t(cps_handle* h, int l, int parity, const T* b, T* x)
{
    using PB = PlaneBufs<T>;
    const Level<T> L = view<T>(h, l);
    const LevelMem& m = h->lv[l];
    if (!PB::tw(m) || !PB::S(h) || !PB::piv(m))
        fail(CPS_E_INVALID, "internal: plane smoother not set up");
    const int rb = m.plane_rb;
    const PlaneLaunch pl = plane_launch(L.g, parity, rb);
    const auto* tw = reinterpret_cast<const Vec2<T>*>(PB::tw(m));
    const auto* twN = reinterpret_cast<const Vec2<T>*>(PB::twN(m));
    auto* S = reinterpret_cast<Vec2<T>*>(PB::S(h));
    ProfScope ps(h, CPS_KERNEL_GS, l);
    if (L.g.nh <= kSmallRing)
        k_plane_fwd<T, kSmallRing, CROSS><<<pl.blocks, pl.threads, 0, h->stream>>>(
            L.g, L.G, L.gk, b, x, parity, tw, twN, S, rb);
    else
        k_plane_fwd<T, kPlaneLds, CROSS><<<pl.blocks, pl.threads, 0, h->stream>>>(
            L.g, L.G, L.gk, b, x, parity, tw, twN, S, rb);
    LAUNCH_CHECK();
    const long long lanes = 2LL * pl.rows * (L.g.nh + 1);
    const unsigned tblocks = (unsigned)cdiv(lanes, kTriBlock);
    const T* piv = PB::piv(m) + plane_pivot_offset(L.g, parity);
    auto tri = [&](auto TB) {
        k_plane_tri<T, CROSS, decltype(TB)::value><<<tblocks, kTriBlock, 0, h->stream>>>(
            L.g, L.G, L.gk, parity, piv, PB::S(h));
    };
    switch (tri_batch_of(m.plane_tb)) {
    case 4: tri(IM<4>{}); break;
    case 16: tri(IM<16>{}); break;
    default: tri(IM<kTriBatch>{}); break;
    }
    LAUNCH_CHECK();
    if (L.g.nh <= kSmallRing)
        k_plane_inv<T, kSmallRing><<<pl.blocks, pl.threads, 0, h->stream>>>(L.g, parity, tw, twN,
                                                                            S, x, rb);
    else
        k_plane_inv<T, kPlaneLds><<<pl.blocks, pl.threads, 0, h->stream>>>(L.g, parity, tw, twN, S,
                                                                           x, rb);
    LAUNCH_CHECK();
}

template <typename T>
void plane_half_sweep(cps_handle* h, int l, int parity, const T* b, T* x)
{
    if (h->mode == MODE_RT) plane_half_sweep_t<T, true>(h, l, parity, b, x);
    else plane_half_sweep_t<T, false>(h, l, parity, b, x);
}

// Gauss-Seidel sweeps over all colours (reverse order for post-smoothing).
// from_zero: x is zero on entry; with two colours it is then not even read
// (nor initialised) before the first pass writes it, otherwise it is filled.
// With the plane smoother a sweep is the two zebra half-sweeps (parity 0
// then 1, reversed for post-smoothing).
// dot (two colours on marching levels): the last two passes, which leave
// every cell final, write partial sums of b . x at dot[0 ..) and after
// them; returns the number of partial sums written (0 without dot).
// first_done (from zero, two colours): the caller has already made the
// zero-iterate first pass (x = b / D on colour 0).
template <typename T>
long long smooth(cps_handle* h, int l, const T* b, T* x, int sweeps, bool reverse,
                 bool from_zero = false, double* dot = nullptr, bool first_done = false)
{
    if (h->opts.smoother == 1) {
        if (from_zero) fill<T>(h, x, h->lv[l].n, T(0));
        for (int s = 0; s < sweeps; ++s)
            for (int k = 0; k < 2; ++k) plane_half_sweep<T>(h, l, reverse ? 1 - k : k, b, x);
        return 0;
    }
    const bool skip = from_zero && h->ncol == 2;
    if (from_zero && !skip) fill<T>(h, x, h->lv[l].n, T(0));
    long long parts = 0;
    const int last = sweeps * h->ncol;
    auto pass_at = [&](int pass) {
        const int k = pass % h->ncol;
        const bool with_dot = dot && h->ncol == 2 && pass >= last - 2;
        parts += gs_pass<T>(h, l, reverse ? h->ncol - 1 - k : k, b, x, skip && pass == 0,
                            with_dot ? dot + parts : nullptr, !(skip && pass == 0));
    };
    const int first = skip ? 1 : 0;
    if (skip && !first_done) pass_at(0);
    // the full passes run back to back: one event pair around all of them
    ProfScope ps(h, CPS_KERNEL_GS, l, last - first);
    for (int pass = first; pass < last; ++pass) pass_at(pass);
    return parts;
}

// r = b - A x; partial sums of r^2 into h->partial when want_norm.
// red: x has just been smoothed red-black with the black pass last, and on a
// row-pair level only r's red cells are formed (the black ones are zero, and
// are left stale: only restrict_to(red) reads this r).  Returns the number
// of partial sums written.
template <typename T>
long long residual(cps_handle* h, int l, const T* b, const T* x, T* r, bool want_norm,
                   bool red = false)
{
    const Level<T> L = view<T>(h, l);
    const int bpa = (int)nblk(L.g.rowlen);
    double* part = want_norm ? h->partial.p : nullptr;
    ProfScope ps(h, CPS_KERNEL_RESIDUAL, l);
    if (marching(h)) {
        const MarchShape ms = stencil_shape(L.g);
        if (row_pairs(L.g)) {
            if (l == 0)
                k_residual_march2<T, 0><<<ms.grid, kBlock, 0, h->stream>>>(
                    L.g, L.G, L.gk, ms.bpa, ms.ch, b, x, r, part, red ? 1 : 0);
            else
                k_residual_march2<T, 1><<<ms.grid, kBlock, 0, h->stream>>>(
                    L.g, L.G, L.gk, ms.bpa, ms.ch, b, x, r, part, red ? 1 : 0);
            LAUNCH_CHECK();
            return ms.grid;
        }
        auto launch = [&](auto U, auto T_) {
            k_residual_march<T, decltype(U)::value, decltype(T_)::value>
                <<<ms.grid, kBlock, 0, h->stream>>>(L.g, L.G, L.gk, ms.bpa, ms.ch, b, x, r, part);
        };
        const bool u = L.g.nh % 64 == 0;
        if (l == 0) u ? launch(BA<true>{}, IM<0>{}) : launch(BA<false>{}, IM<0>{});
        else u ? launch(BA<true>{}, IM<1>{}) : launch(BA<false>{}, IM<1>{});
        LAUNCH_CHECK();
        return ms.grid;
    }
    dispatch4(h->mode, h->axi, L.g.nh % 64 == 0, l == 0 ? 0 : 1, [&](auto M, auto A, auto U, auto T_) {
        k_residual<T, decltype(M)::value, decltype(A)::value, decltype(U)::value, decltype(T_)::value>
            <<<grid_of(L.g.nr, bpa), kBlock, 0, h->stream>>>(L.g, L.G, L.gk, bpa, b, x, r, part);
    });
    LAUNCH_CHECK();
    return grid_of(L.g.nr, bpa);
}

// y = A x (level l); with dotv, partial sums of y . dotv.  Returns the
// number of partial sums written.
template <typename T>
long long apply(cps_handle* h, int l, const T* x, T* y, const T* dotv)
{
    const Level<T> L = view<T>(h, l);
    const int bpa = (int)nblk(L.g.rowlen);
    double* part = dotv ? h->partial.p : nullptr;
    ProfScope ps(h, CPS_KERNEL_APPLY, l);
    if (marching(h)) {
        const MarchShape ms = stencil_shape(L.g);
        if (row_pairs(L.g)) {
            if (l == 0)
                k_apply_march2<T, 0><<<ms.grid, kBlock, 0, h->stream>>>(L.g, L.G, L.gk, ms.bpa,
                                                                       ms.ch, x, y, part, dotv);
            else
                k_apply_march2<T, 1><<<ms.grid, kBlock, 0, h->stream>>>(L.g, L.G, L.gk, ms.bpa,
                                                                       ms.ch, x, y, part, dotv);
            LAUNCH_CHECK();
            return ms.grid;
        }
        auto launch = [&](auto U, auto T_) {
            k_apply_march<T, decltype(U)::value, decltype(T_)::value>
                <<<ms.grid, kBlock, 0, h->stream>>>(L.g, L.G, L.gk, ms.bpa, ms.ch, x, y, part, dotv);
        };
        const bool u = L.g.nh % 64 == 0;
        if (l == 0) u ? launch(BA<true>{}, IM<0>{}) : launch(BA<false>{}, IM<0>{});
        else u ? launch(BA<true>{}, IM<1>{}) : launch(BA<false>{}, IM<1>{});
        LAUNCH_CHECK();
        return ms.grid;
    }
    dispatch4(h->mode, h->axi, L.g.nh % 64 == 0, l == 0 ? 0 : 1, [&](auto M, auto A, auto U, auto T_) {
        k_apply<T, decltype(M)::value, decltype(A)::value, decltype(U)::value, decltype(T_)::value>
            <<<grid_of(L.g.nr, bpa), kBlock, 0, h->stream>>>(L.g, L.G, L.gk, bpa, x, y, part, dotv);
    });
    LAUNCH_CHECK();
    return grid_of(L.g.nr, bpa);
}

// ops: the conjugate-gradient scalar updates done in the same launch
// (RED_* of k_reduce_cg)
void reduce(cps_handle* h, long long nparts, int slot, long long first = 0, int ops = 0)
{
    if (ops)
        k_reduce_cg<<<1, kBlock, 0, h->stream>>>(h->partial.p + first, nparts, h->sc.p, slot, ops);
    else
        k_reduce<<<1, kBlock, 0, h->stream>>>(h->partial.p + first, nparts, h->sc.p + slot,
                                              nullptr);
    LAUNCH_CHECK();
}

// The same for the norm an outer iteration ends with: the sum also goes to
// the host mirror (coherent pinned memory), which body_norm reads after the
// stream is synchronised, so no copy follows the launch.
void reduce_norm(cps_handle* h, long long nparts, int slot)
{
    k_reduce<<<1, kBlock, 0, h->stream>>>(h->partial.p, nparts, h->sc.p + slot, h->hsc + slot);
    LAUNCH_CHECK();
}

template <typename T, typename U>
void dot(cps_handle* h, long long n, const T* u, const U* v, int slot, int ops = 0)
{
    k_dot<T, U><<<vgrid(n), kBlock, 0, h->stream>>>(n, u, v, h->partial.p);
    LAUNCH_CHECK();
    reduce(h, vgrid(n), slot, 0, ops);
}

// red: r is residual(red)'s output, of which only the red cells are read.
template <typename T>
void restrict_to(cps_handle* h, int l, const T* r, T* bc, bool red = false)
{
    const Geo& f = h->lv[l].geo;
    const Geo& c = h->lv[l + 1].geo;
    const MarchShape ms = restrict_shape(c);
    ProfScope ps(h, CPS_KERNEL_RESTRICT, l);
    if (!restrict_rows(c))
        k_restrict<T><<<ms.grid, kBlock, 0, h->stream>>>(f, c, ms.bpa, ms.ch, r, bc, red ? 1 : 0);
    else if (red)
        k_restrict_rows<T, 1><<<ms.grid, kBlock, 0, h->stream>>>(f, c, ms.bpa, ms.ch, r, bc);
    else
        k_restrict_rows<T, 0><<<ms.grid, kBlock, 0, h->stream>>>(f, c, ms.bpa, ms.ch, r, bc);
    LAUNCH_CHECK();
}

// bc = P^T r with r = b - A x on level l's red cells (0 on the black ones)
// in one pass: the V-cycle's transfer where resrestrict_segs allows it
// (timed in the restriction's class).
template <typename T>
void resrestrict(cps_handle* h, int l, const T* b, const T* x, T* bc)
{
    const Level<T> F = view<T>(h, l);
    const Geo& c = h->lv[l + 1].geo;
    const int segs = resrestrict_segs(F.g, c);
    if (segs == 0) fail(CPS_E_INVALID, "internal: no fused transfer from level %d", l);
    const MarchShape ms = resrestrict_shape<T>(c, segs);
    ProfScope ps(h, CPS_KERNEL_RESTRICT, l);
    if (segs == 2)
        k_resrestrict<T, 2><<<ms.grid, 64 * rr_waves(2), 0, h->stream>>>(
            F.g, F.G, F.gk, c, ms.bpa, ms.ch, b, x, bc);
    else
        k_resrestrict<T, 1><<<ms.grid, 64 * rr_waves(1), 0, h->stream>>>(
            F.g, F.G, F.gk, c, ms.bpa, ms.ch, b, x, bc);
    LAUNCH_CHECK();
}

// the V-cycle forms only the red residual on level l (point red-black
// smoothing ends on the black pass; row-pair levels)
bool red_residual(const cps_handle* h, int l)
{
    return h->opts.smoother == 0 && marching(h) && h->ncol == 2 && row_pairs(h->lv[l].geo);
}

// red: only level l's red cells are corrected (a red-black post-smoothing
// follows, whose first pass overwrites every black cell unread)
template <typename T>
void prolong_add(cps_handle* h, int l, const T* e, T* x, bool red = false)
{
    const Geo& f = h->lv[l].geo;
    const Geo& c = h->lv[l + 1].geo;
    const MarchShape ms = march_shape(c);
    ProfScope ps(h, CPS_KERNEL_PROLONG, l);
    if (red) k_prolong<T, 1><<<ms.grid, kBlock, 0, h->stream>>>(f, c, ms.bpa, ms.ch, e, x);
    else k_prolong<T, 0><<<ms.grid, kBlock, 0, h->stream>>>(f, c, ms.bpa, ms.ch, e, x);
    LAUNCH_CHECK();
}

template <typename T>
void coarse_solve(cps_handle* h, const T* b, T* e)
{
    const int n = h->nc;
    k_coarse_gemv<T><<<(n + 3) / 4, kBlock, 0, h->stream>>>(n, h->Ainv.p, b, e);
    LAUNCH_CHECK();
}

// The tile path of a small level (tile.hpp): pre-smoothing from zero,
// residual and restriction into bc; prolongation of e and post-smoothing
// from xi into xo.
template <typename T>
void vpre_tile(cps_handle* h, int l, const T* b, T* x, T* bc)
{
    const Level<T> L = view<T>(h, l);
    k_vpre_tile<T><<<tile_count(L.g), kTileThreads, 0, h->stream>>>(L.g, L.G, L.gk, b, x,
                                                                     h->lv[l + 1].geo, bc);
    LAUNCH_CHECK();
}

template <typename T>
void vpost_tile(cps_handle* h, int l, const T* b, const T* xi, T* xo, const T* e)
{
    const Level<T> L = view<T>(h, l);
    k_vpost_tile<T><<<tile_count(L.g), kTileThreads, 0, h->stream>>>(L.g, L.G, L.gk, b, xi, xo,
                                                                      h->lv[l + 1].geo, e);
    LAUNCH_CHECK();
}

// One V(2,2) cycle with level-0 right-hand side b0 and iterate x0 (in place).
// dot: the last level-0 passes leave partial sums of b0 . x0 in h->partial;
// returns their number (0 when the cycle cannot provide them).
// zero_done (from zero, the per-kernel finest level): x0 already holds the
// zero-iterate first pass (the conjugate-gradient step made it).
template <typename T>
long long vcycle(cps_handle* h, const T* b0, T* x0, bool x0_zero = false, bool dot = false,
                 bool zero_done = false)
{
    const int L = h->L;
    if (L == 1) {
        coarse_solve<T>(h, b0, x0);
        return 0;
    }
    // the finest level takes the tile path only from a zero iterate (its
    // pre-smoothing starts from zero): pre writes the scratch iterate xt and
    // post reads it and writes x0, so no block reads what another overwrote
    const bool tile0 = h->lv[0].tile && x0_zero;
    for (int l = 0; l < L - 1; ++l) {
        const T* b = l == 0 ? b0 : bl<T>(h, l);
        T* x = l == 0 ? x0 : xl<T>(h, l);
        if (l == 0 ? tile0 : h->lv[l].tile) { // smoothing, residual, restriction
            vpre_tile<T>(h, l, b, l == 0 ? xtl<T>(h, 0) : x, bl<T>(h, l + 1));
            continue;
        }
        // coarse corrections start from zero
        smooth<T>(h, l, b, x, 2, false, l > 0 || x0_zero, nullptr, l == 0 && zero_done);
        // point red-black smoothing ends on the black pass: on row-pair
        // levels only the red residual is formed and restricted (in one pass
        // where the level's shape allows it)
        const bool red = red_residual(h, l);
        if (red && resrestrict_segs(h->lv[l].geo, h->lv[l + 1].geo) > 0) {
            resrestrict<T>(h, l, b, x, bl<T>(h, l + 1));
            continue;
        }
        residual<T>(h, l, b, x, rl<T>(h, l), false, red);
        restrict_to<T>(h, l, rl<T>(h, l), bl<T>(h, l + 1), red);
    }
    coarse_solve<T>(h, bl<T>(h, L - 1), xl<T>(h, L - 1));
    long long parts = 0;
    for (int l = L - 2; l >= 0; --l) {
        const T* b = l == 0 ? b0 : bl<T>(h, l);
        T* x = l == 0 ? x0 : xl<T>(h, l);
        const T* e = l + 1 == L - 1 ? xl<T>(h, l + 1) : xfin<T>(h, l + 1);
        if (l == 0 && tile0) { // prolongation and smoothing, xt -> x0 (no dot sums)
            vpost_tile<T>(h, 0, b, xtl<T>(h, 0), x, e);
            continue;
        }
        if (l > 0 && h->lv[l].tile) { // prolongation and smoothing, into xt
            vpost_tile<T>(h, l, b, x, xtl<T>(h, l), e);
            continue;
        }
        // point red-black post-smoothing starts with the black pass: only
        // the red cells need the correction
        prolong_add<T>(h, l, e, x, h->opts.smoother == 0 && h->ncol == 2);
        const bool d = dot && l == 0 && marching(h);
        parts = smooth<T>(h, l, b, x, 2, true, false, d ? h->partial.p : nullptr);
    }
    return parts;
}

// out = M^-1 in : one V-cycle from zero, FP64 or FP32 inside (scaled by
// sc[S_SCALE] so that FP32 sees O(1) values).  rz_slot >= 0: also
// sc[rz_slot] = in . out; zq: also sc[S_ZQ] = out . zq.  Both are taken
// from passes that already touch the vectors where possible (the last
// level-0 smoothing passes in FP64, the cast back in the mixed form).
// Mixed form only: rhs_cast -- the FP32 right-hand side (in / scale) is
// already in place (the conjugate-gradient step wrote it); out == nullptr --
// the correction stays in FP32 (the next kernel forms it where it reads it)
// and only the dot products are taken.  rz_ops / zq_ops: scalar updates done
// by the launch that stores r.z / z.q (RED_* of k_reduce_cg).  zero_done
// (FP64): out already holds the cycle's zero-iterate first pass of in.
void precondition(cps_handle* h, const double* in, double* out, int rz_slot = -1,
                  const double* zq = nullptr, bool rhs_cast = false, int rz_ops = 0,
                  int zq_ops = 0, bool zero_done = false)
{
    const long long n = h->lv[0].n;
    if (h->opts.precision == 0) {
        long long parts;
        {
            ProfScope ps(h, CPS_KERNEL_VCYCLE, 0);
            parts = vcycle<double>(h, in, out, true, rz_slot >= 0, zero_done);
        }
        if (rz_slot >= 0) {
            if (parts) reduce(h, parts, rz_slot, 0, rz_ops);
            else dot<double, double>(h, n, in, out, rz_slot, rz_ops);
        }
        if (zq) dot<double, double>(h, n, out, zq, S_ZQ, zq_ops);
    } else {
        float* b = h->lv[0].b32.p;
        float* x = h->lv[0].x32.p;
        if (!rhs_cast) {
            k_cast<double, float><<<nblk(n), kBlock, 0, h->stream>>>(n, in, b, h->sc.p, S_SCALE,
                                                                     1);
            LAUNCH_CHECK();
        }
        {
            ProfScope ps(h, CPS_KERNEL_VCYCLE, 0);
            vcycle<float>(h, b, x, true);
        }
        if (rz_slot < 0 && !zq) {
            k_cast<float, double><<<nblk(n), kBlock, 0, h->stream>>>(n, x, out, h->sc.p, S_SCALE, 0);
            LAUNCH_CHECK();
            return;
        }
        const int vg = vgrid(n);
        k_cast_dots<<<vg, kBlock, 0, h->stream>>>(n, x, out, h->sc.p, S_SCALE, in, zq,
                                                  h->partial.p, h->partial.p + vg);
        LAUNCH_CHECK();
        if (rz_slot >= 0) reduce(h, vg, rz_slot, 0, rz_ops);
        if (zq) reduce(h, vg, S_ZQ, vg, zq_ops);
    }
}

// Outer-iteration bodies: captured once per handle into a hipGraph and
// replayed (one launch per iteration), or launched kernel by kernel when
// the handle runs eagerly, is being profiled (per-launch events) or runs on
// the null stream (which cannot be captured).  A body ends by copying the
// residual norm to the pinned host mirror; the caller synchronises.
enum { G_CG0 = 0, G_CG1 = 1, G_BICG = 2, G_RICH = 3 };

template <typename F>
void run_body(cps_handle* h, int key, F&& body)
{
    if (h->opts.eager || h->prof || !h->stream) {
        body();
        return;
    }
    hipGraphExec_t& ex = h->gexec[key];
    if (!ex) {
        std::shared_lock<std::shared_mutex> cap(g_capture_mu); // no free or sync meanwhile
        hipGraph_t g = nullptr;
        HIPC(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
        try {
            body();
        } catch (...) {
            hipGraph_t g2 = nullptr;
            (void)hipStreamEndCapture(h->stream, &g2);
            if (g2) (void)hipGraphDestroy(g2);
            throw;
        }
        HIPC(hipStreamEndCapture(h->stream, &g));
        const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) ex = nullptr;
        HIPC(e);
    }
    HIPC(hipGraphLaunch(ex, h->stream));
}

// the residual norm the last body left in the host mirror
double body_norm(cps_handle* h, int slot)
{
    HIPC(hipStreamSynchronize(h->stream));
    return h->hsc[slot];
}

double read_scalar(cps_handle* h, int slot)
{
    HIPC(hipMemcpyAsync(h->hsc + slot, h->sc.p + slot, sizeof(double), hipMemcpyDeviceToHost,
                        h->stream));
    HIPC(hipStreamSynchronize(h->stream));
    return h->hsc[slot];
}

#define SCALAR_KERNEL(h, k)                                 \
    do {                                                    \
        k<<<1, 1, 0, (h)->stream>>>((h)->sc.p);             \
        LAUNCH_CHECK();                                     \
    } while (0)

} // namespace

#include "autotune.hpp"

namespace {

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------

int level_plan(const cps_grid* g, int dims[kMaxLevels][3])
{
    int L = 1;
    dims[0][0] = g->n_r;
    dims[0][1] = g->n_theta;
    dims[0][2] = g->n_phi;
    for (;;) {
        const int* p = dims[L - 1];
        // halving keeps n_phi even on the coarser level (colourings and the
        // parity-split layout wrap around phi only for even n_phi)
        const bool can = p[0] % 2 == 0 && p[1] % 2 == 0 && p[2] % 4 == 0 && p[0] >= 4 &&
                         p[1] >= 4 && p[2] >= 4;
        const long long cells = (long long)p[0] * p[1] * p[2];
        const bool want = g->n_levels > 0 ? L < g->n_levels : cells > 1024;
        if (!want) break;
        if (!can || L == kMaxLevels) {
            if (g->n_levels > 0) fail(CPS_E_INVALID, "cannot build %d levels", g->n_levels);
            break;
        }
        dims[L][0] = p[0] / 2;
        dims[L][1] = p[1] / 2;
        dims[L][2] = p[2] / 2;
        ++L;
    }
    return L;
}

void validate_opts(const cps_opts* o)
{
    if (o && (o->precision < 0 || o->precision > 1)) fail(CPS_E_INVALID, "bad precision");
    if (o && (o->accel < 0 || o->accel > 2)) fail(CPS_E_INVALID, "bad accel");
    if (o && (o->tune < 0 || o->tune > 2)) fail(CPS_E_INVALID, "bad tune");
    if (o && (o->eager < 0 || o->eager > 1)) fail(CPS_E_INVALID, "bad eager");
    if (o && (o->smoother < 0 || o->smoother > 2)) fail(CPS_E_INVALID, "bad smoother");
}

void validate(const cps_grid* g, const cps_metrics* m, const cps_opts* o)
{
    if (!g) fail(CPS_E_INVALID, "grid is NULL");
    if (g->n_r < 1 || g->n_theta < 1 || g->n_phi < 1)
        fail(CPS_E_INVALID, "dims must be positive (%d %d %d)", g->n_r, g->n_theta, g->n_phi);
    if ((long long)g->n_r * g->n_theta * g->n_phi > (1LL << 31))
        fail(CPS_E_INVALID, "grid too large");
    if (g->map < CPS_MAP_IDENTITY || g->map > CPS_MAP_TRIAXIAL) fail(CPS_E_INVALID, "bad map");
    if (!(g->r_outer > g->r_inner)) fail(CPS_E_INVALID, "r_outer must exceed r_inner");
    if (g->map != CPS_MAP_IDENTITY && !(g->r_inner > 0)) fail(CPS_E_INVALID, "r_inner must be > 0");
    if (!(g->theta1 > g->theta0)) fail(CPS_E_INVALID, "theta1 must exceed theta0");
    // theta0 = 0 / theta1 = pi: a full sphere, whose polar faces have zero
    // area and carry no flux (no coupling across the pole is needed)
    if (g->map != CPS_MAP_IDENTITY && !(g->theta0 >= 0 && g->theta1 <= M_PI))
        fail(CPS_E_INVALID, "theta0 and theta1 must lie in [0, pi]");
    if (g->radial_stretch < 0) fail(CPS_E_INVALID, "radial_stretch must be >= 0");
    if (g->n_levels < 0 || g->n_levels > kMaxLevels) fail(CPS_E_INVALID, "bad n_levels");
    if (m && m->method != CPS_METRICS_MAP_CENTRAL && m->method != CPS_METRICS_PAPER_VERTEX &&
        m->method != CPS_METRICS_USER_FACE)
        fail(CPS_E_INVALID, "bad metrics method");
    if (m && m->method == CPS_METRICS_USER_FACE && !m->face_G)
        fail(CPS_E_INVALID, "caller-supplied metrics need face_G");
    validate_opts(o);
}

// Face metrics of every level from the map (FP64, plus FP32 copies for the
// mixed form), the stencil class, and the dense inverse of the coarsest
// operator.  Buffers are allocated on first use and reused when the
// operator is recomputed for a new map of the same dims (remap); returns
// the stencil class (MODE_*) found.
// Inverse pivots of the plane smoother's r-line eliminations on every
// smoothed level, in the precision the cycles run in.  They depend on the
// metrics only: computed at set-up and again when the metrics change.
void plane_factors(cps_handle* h)
{
    const bool mixed = h->opts.precision == 1;
    for (int l = 0; l + 1 < h->L; ++l) {
        const LevelMem& m = h->lv[l];
        for (int k = 0; k < 2; ++k) {
            const long long sys = (long long)((m.nt - k + 1) / 2) * (m.np / 2 + 1);
            const long long off = plane_pivot_offset(m.geo, k);
            const bool cross = h->mode == MODE_RT;
            if (mixed && cross)
                k_plane_factor<float, true><<<nblk(sys), kBlock, 0, h->stream>>>(
                    m.geo, m.G32.p, m.gk, k, m.lam32.p, m.pv32.p + off);
            else if (mixed)
                k_plane_factor<float, false><<<nblk(sys), kBlock, 0, h->stream>>>(
                    m.geo, m.G32.p, m.gk, k, m.lam32.p, m.pv32.p + off);
            else if (cross)
                k_plane_factor<double, true><<<nblk(sys), kBlock, 0, h->stream>>>(
                    m.geo, m.G64.p, m.gk, k, m.lam64.p, m.pv64.p + off);
            else
                k_plane_factor<double, false><<<nblk(sys), kBlock, 0, h->stream>>>(
                    m.geo, m.G64.p, m.gk, k, m.lam64.p, m.pv64.p + off);
            LAUNCH_CHECK();
        }
    }
}

// OR of the per-block flags a metrics kernel left in `dflags`.
int gather_flags(cps_handle* h, const Buf<int>& dflags, long long blocks)
{
    std::vector<int> hflags(blocks);
    HIPC(hipMemcpyAsync(hflags.data(), dflags.p, hflags.size() * sizeof(int),
                        hipMemcpyDeviceToHost, h->stream));
    HIPC(hipStreamSynchronize(h->stream));
    int all = 0;
    for (int f : hflags) all |= f;
    return all;
}

// Caller-supplied metrics (CPS_METRICS_USER_FACE): the finest level's array
// goes to the device in natural layout, where its wall faces are zeroed and
// it is checked and classified (k_user_metrics flags).  The natural array
// stays in `unat` for compute_operator.  Sets h->axi; returns the flags.
int upload_user_metrics(cps_handle* h, Buf<double>& unat)
{
    const long long n = (long long)h->grid.n_r * h->grid.n_theta * h->grid.n_phi;
    unat.alloc(9 * n);
    upload(unat.p, h->met.face_G, 9 * n * sizeof(double));
    Buf<int> dflags;
    dflags.alloc(nblk(n) + 1);
    k_user_metrics<<<nblk(n), kBlock, 0, h->stream>>>(h->grid.n_r, h->grid.n_theta,
                                                      h->grid.n_phi, unat.p, dflags.p);
    LAUNCH_CHECK();
    const int flags = gather_flags(h, dflags, nblk(n));
    if (flags & 1)
        fail(CPS_E_INVALID, "face_G holds a non-finite entry or a negative diagonal entry");
    h->axi = !(flags & 8);
    return flags;
}

// Every level's storage from the natural finest-level array: level 0 as
// given, each coarser one by k_coarsen_metrics from the level below.
void store_user_metrics(cps_handle* h, Buf<double>& unat)
{
    Buf<double> fine, coarse;
    for (int l = 0; l < h->L; ++l) {
        LevelMem& m = h->lv[l];
        if (!m.G64.p) m.G64.alloc(9 * m.gk);
        const double* U = unat.p;
        if (l > 0) {
            const LevelMem& f = h->lv[l - 1];
            coarse.alloc(9 * m.n);
            k_coarsen_metrics<<<nblk(m.n), kBlock, 0, h->stream>>>(f.nr, f.nt, f.np,
                                                                   l == 1 ? unat.p : fine.p,
                                                                   coarse.p);
            LAUNCH_CHECK();
            HIPC(hipStreamSynchronize(h->stream)); // before `fine` is freed below
            std::swap(fine.p, coarse.p);
            std::swap(fine.n, coarse.n);
            coarse.release();
            U = fine.p;
        }
        k_store_metrics<<<nblk(m.gk), kBlock, 0, h->stream>>>(m.nr, m.nt, m.np, m.nc, U,
                                                              m.G64.p);
        LAUNCH_CHECK();
    }
    HIPC(hipStreamSynchronize(h->stream));
}

int compute_operator(cps_handle* h, Buf<double>* unat = nullptr, int user_flags = 0)
{
    const cps_grid& g = h->grid;
    MapParams mp{g.map, g.r_inner, g.r_outer, g.theta0, g.theta1, g.radial_stretch, g.flattening,
                 g.skew};
    int flags_all = 0;
    if (unat) {
        store_user_metrics(h, *unat);
        flags_all = user_flags & 6;
    } else {
        Buf<int> dflags;
        long long maxn = 0;
        for (int l = 0; l < h->L; ++l) maxn = std::max(maxn, h->lv[l].gk);
        dflags.alloc(nblk(maxn) + 1);
        for (int l = 0; l < h->L; ++l) {
            LevelMem& m = h->lv[l];
            if (!m.G64.p) m.G64.alloc(9 * m.gk);
            k_metrics<<<nblk(m.gk), kBlock, 0, h->stream>>>(mp, m.nr, m.nt, m.np, m.nc,
                                                             h->met.method, m.G64.p, dflags.p);
            LAUNCH_CHECK();
            flags_all |= gather_flags(h, dflags, nblk(m.gk));
        }
    }
    if (flags_all & 1) fail(CPS_E_INVALID, "a face of the map has det <= 0");
    const int mode = (flags_all & 4) ? MODE_FULL : ((flags_all & 2) ? MODE_RT : MODE_ORTHO);
    if (h->Ainv.p && mode != h->mode)
        fail(CPS_E_INVALID, "the new map changes the stencil class of the hierarchy");
    h->mode = mode;
    h->ncol = h->mode == MODE_ORTHO ? 2 : 4;
    if (h->opts.precision == 1)
        for (int l = 0; l < h->L; ++l) {
            LevelMem& m = h->lv[l];
            if (!m.G32.p) m.G32.alloc(9 * m.gk);
            k_to_f32<<<nblk(9 * m.gk), kBlock, 0, h->stream>>>(9 * m.gk, m.G64.p, m.G32.p);
            LAUNCH_CHECK();
        }
    // coarsest dense inverse of A_c + alpha 1 1^T
    const int n = h->nc;
    {
        // scratch of the inversion: kept by hierarchies whose map is
        // recomputed in place (a pooled service entry), so that a remap
        // allocates and frees nothing (a free synchronises the device)
        Buf<double>& A = h->gjA;
        Buf<double>& M0 = h->gjM;
        Buf<double>& E = h->gjE;
        Buf<double>& Xp = h->gjXp;
        Buf<int>& used = h->gjUsed;
        Buf<int>& piv = h->gjPiv;
        Buf<int>& bad = h->gjBad;
        auto need = [](auto& b, size_t count) {
            if (b.n != count || !b.p) b.alloc(count);
        };
        need(A, (size_t)n * n);
        need(M0, (size_t)n * 2 * n);
        need(E, (size_t)n * kGJ);
        need(Xp, (size_t)kGJ * 2 * n);
        need(used, n);
        need(piv, n);
        need(bad, 1);
        if (!h->Ainv.p) h->Ainv.alloc((size_t)n * n);
        HIPC(hipMemsetAsync(A.p, 0, (size_t)n * n * sizeof(double), h->stream));
        const Level<double> Lc = view<double>(h, h->L - 1);
        dispatch(h->mode, h->axi, [&](auto M, auto AX) {
            k_dense_rows<decltype(M)::value, decltype(AX)::value>
                <<<nblk(27LL * n), kBlock, 0, h->stream>>>(Lc, A.p);
        });
        LAUNCH_CHECK();
        const unsigned gblocks = std::min<long long>(nblk(2LL * n * n), 1024);
        k_augment<<<gblocks, kBlock, 0, h->stream>>>(n, A.p, M0.p);
        LAUNCH_CHECK();
        k_fill<int><<<nblk(n), kBlock, 0, h->stream>>>(n, used.p, INT_MAX);
        k_fill<int><<<nblk(n), kBlock, 0, h->stream>>>(n, piv.p, 0);
        k_fill<int><<<1, kBlock, 0, h->stream>>>(1, bad.p, 0);
        LAUNCH_CHECK();
        // blocked Gauss-Jordan: a panel of kGJ pivot steps, then the rank-kGJ
        // update of the columns past the panel
        const int R = cdiv(n, kGJThreads); // rows per thread: 1, 2 or 4 (n <= 4096)
        const int KB = R == 1 ? 16 : (R == 2 ? 8 : 4);
        for (int c0 = 0; c0 < n; c0 += KB) {
            if (R == 1)
                k_gj_panel<1, 16><<<1, kGJThreads, 0, h->stream>>>(n, c0, M0.p, E.p, used.p,
                                                                   piv.p, bad.p);
            else if (R == 2)
                k_gj_panel<2, 8><<<1, kGJThreads, 0, h->stream>>>(n, c0, M0.p, E.p, used.p,
                                                                  piv.p, bad.p);
            else
                k_gj_panel<4, 4><<<1, kGJThreads, 0, h->stream>>>(n, c0, M0.p, E.p, used.p,
                                                                  piv.p, bad.p);
            const int kb = std::min(KB, n - c0);
            k_gj_pivrows<<<nblk((long long)kb * 2 * n), kBlock, 0, h->stream>>>(n, c0, kb, M0.p,
                                                                               piv.p, Xp.p);
            const long long rest = 2LL * n - c0 - kb;
            const long long blocks = cdiv(rest, 64) * (long long)cdiv(n, kBlock / 64);
            k_gj_update<<<(unsigned)blocks, kBlock, 0, h->stream>>>(n, c0, kb, M0.p, E.p, Xp.p,
                                                                   used.p);
        }
        LAUNCH_CHECK();
        k_gj_extract<<<nblk((long long)n * n), kBlock, 0, h->stream>>>(n, M0.p, piv.p, h->Ainv.p);
        LAUNCH_CHECK();
        int hbad = 0;
        HIPC(hipMemcpyAsync(&hbad, bad.p, sizeof(int), hipMemcpyDeviceToHost, h->stream));
        HIPC(hipStreamSynchronize(h->stream));
        if (!h->keep_gj) {
            A.release(); M0.release(); E.release(); Xp.release();
            used.release(); piv.release(); bad.release();
        }
        if (hbad) fail(CPS_E_INVALID, "coarsest operator is singular");
    }
    if (h->lv[0].pv64.p || h->lv[0].pv32.p) plane_factors(h); // new metrics of a set-up hierarchy
    h->cm_valid = false; // the projection step's face tables follow the map
    h->lf_valid[0] = h->lf_valid[1] = false;
    return mode;
}

// Level plan of a grid with the checks the kernels rely on; returns L.
int checked_plan(const cps_grid& g, int dims[kMaxLevels][3])
{
    const int L = level_plan(&g, dims);
    for (int l = 0; l < L; ++l) {
        if (dims[l][2] % 2)
            fail(CPS_E_INVALID, "n_phi must be even on every level (level %d has %d)", l,
                 dims[l][2]);
        if (l + 1 < L && (dims[l][0] % 2 || dims[l][1] % 2))
            fail(CPS_E_INVALID, "level %d dims must be even", l);
    }
    const long long nc = (long long)dims[L - 1][0] * dims[L - 1][1] * dims[L - 1][2];
    if (nc > kMaxCoarse)
        fail(CPS_E_INVALID, "coarsest level has %lld cells (max %lld): choose even dims", nc,
             kMaxCoarse);
    return L;
}

// The plane smoother applies: phi-invariant metrics with no cross terms or
// the r-theta ones only, and n_phi / 2 a power of two in [2, kPlaneLds] on
// every smoothed level.
bool plane_eligible(const cps_handle* h)
{
    if (!plane_class_ok(h)) return false;
    for (int l = 0; l + 1 < h->L; ++l) {
        const int nh = h->lv[l].np / 2;
        if (nh < 2 || nh > kPlaneLds || (nh & (nh - 1))) return false;
    }
    return true;
}

// Tables and scratch of the plane smoother (phi-invariant hierarchies with
// no cross terms or r-theta ones only, whose smoothed levels have
// power-of-two rings of <= 2048).
void setup_plane(cps_handle* h)
{
    if (!plane_class_ok(h))
        fail(CPS_E_INVALID, "the plane smoother needs phi-invariant metrics without "
                            "phi cross terms (a 7- or 11-point axisymmetric operator)");
    const bool mixed = h->opts.precision == 1;
    size_t spec = 0;
    for (int l = 0; l + 1 < h->L; ++l) {
        LevelMem& m = h->lv[l];
        const int nh = m.np / 2;
        if (nh < 2 || nh > kPlaneLds || (nh & (nh - 1)))
            fail(CPS_E_INVALID, "the plane smoother needs n_phi a power of two in [4, %d] on "
                 "every smoothed level (level %d has %d)", 2 * kPlaneLds, l, m.np);
        std::vector<double> tw(nh), twN(2 * (nh + 1)), lam(nh + 1);
        for (int q = 0; q < nh / 2; ++q) {
            tw[2 * q] = std::cos(-2.0 * M_PI * q / nh);
            tw[2 * q + 1] = std::sin(-2.0 * M_PI * q / nh);
        }
        for (int k = 0; k <= nh; ++k) {
            twN[2 * k] = std::cos(-2.0 * M_PI * k / m.np);
            twN[2 * k + 1] = std::sin(-2.0 * M_PI * k / m.np);
            lam[k] = 2.0 * std::cos(2.0 * M_PI * k / m.np) - 2.0;
        }
        auto up64 = [&](Buf<double>& d, const std::vector<double>& v) {
            d.alloc(v.size());
            upload(d.p, v.data(), v.size() * sizeof(double));
        };
        auto up32 = [&](Buf<float>& d, const std::vector<double>& v) {
            std::vector<float> f(v.begin(), v.end());
            d.alloc(f.size());
            upload(d.p, f.data(), f.size() * sizeof(float));
        };
        up64(m.tw64, tw); up64(m.twN64, twN); up64(m.lam64, lam);
        if (mixed) { up32(m.tw32, tw); up32(m.twN32, twN); up32(m.lam32, lam); }
        spec = std::max(spec, (size_t)m.nr * ((m.nt + 1) / 2) * (nh + 1));
        // pivots of both parities, in the precision of the cycles (FP64 for
        // the FP64 hierarchy and its per-step entry points)
        const size_t npiv = (size_t)m.nr * m.nt * (nh + 1);
        if (mixed) m.pv32.alloc(npiv);
        else m.pv64.alloc(npiv);
    }
    if (!mixed) h->ps64.alloc(2 * spec);
    else h->ps32.alloc(2 * spec);
    plane_factors(h);
}

void build(cps_handle* h)
{
    int dims[kMaxLevels][3];
    h->L = checked_plan(h->grid, dims);
    Buf<double> unat; // caller-supplied metrics, natural layout (set-up only)
    int uflags = 0;
    if (h->met.method == CPS_METRICS_USER_FACE) {
        uflags = upload_user_metrics(h, unat);
        h->met.face_G = nullptr; // the caller's array is not retained
    } else {
        h->axi = h->grid.map != CPS_MAP_TRIAXIAL;
    }
    for (int l = 0; l < h->L; ++l) {
        LevelMem& m = h->lv[l];
        m.nr = dims[l][0];
        m.nt = dims[l][1];
        m.np = dims[l][2];
        m.nc = h->axi ? 1 : m.np;
        m.n = (long long)m.nr * m.nt * m.np;
        m.gk = (long long)m.nr * m.nt * m.nc;
        m.geo = make_geo(m.nr, m.nt, m.np);
    }
    h->nc = (int)h->lv[h->L - 1].n;
    compute_operator(h, unat.p ? &unat : nullptr, uflags);
    unat.release();
    // per-level vectors
    const bool mixed = h->opts.precision == 1;
    for (int l = 0; l < h->L; ++l) {
        LevelMem& m = h->lv[l];
        if (l > 0) {
            if (!mixed) {
                m.x64.alloc(m.n);
                m.b64.alloc(m.n);
            }
        }
        if (!mixed && l < h->L - 1) m.r64.alloc(m.n);
        if (mixed) {
            m.x32.alloc(m.n);
            m.b32.alloc(m.n);
            if (l < h->L - 1) m.r32.alloc(m.n);
        }
    }
    const long long n0 = h->lv[0].n;
    // two passes' (or two reductions') partial sums side by side
    h->partial.alloc(2 * std::max<long long>(nblk(n0), kMaxGrid) + 64);
    h->sc.alloc(S_COUNT);
    {
        MemLock lk(g_capture_mu);
        // coherent: reduce_norm's kernel stores the norms here directly
        HIPC(hipHostMalloc(&h->hsc, S_COUNT * sizeof(double), hipHostMallocCoherent));
    }
    h->x0.alloc(n0);
    h->b0.alloc(n0);
    h->r.alloc(n0);
    if (h->opts.accel >= 1) {
        h->z.alloc(n0);
        h->pd.alloc(n0);
        h->q.alloc(n0);
        h->ph.alloc(n0); // BiCGStab's M^-1 p, or the second CG direction buffer
    }
    if (h->opts.accel == 2) {
        h->r0.alloc(n0); h->v.alloc(n0); h->s.alloc(n0); h->t.alloc(n0);
        h->sh.alloc(n0);
    }
    if (h->opts.smoother == 2) h->opts.smoother = plane_eligible(h) ? 1 : 0; // automatic
    if (h->opts.smoother == 1) setup_plane(h);
    // small levels of the point smoother run the tile path (not the
    // coarsest: it is solved directly; the finest only when the cycle starts
    // from zero, and then its dot products come from a separate reduction)
    for (int l = 0; l + 1 < h->L; ++l) {
        LevelMem& m = h->lv[l];
        m.tile = marching(h) && h->ncol == 2 && h->opts.smoother == 0 && tile_fits(m.geo, mixed);
        if (!m.tile) continue;
        if (mixed) m.xt32.alloc(m.n);
        else m.xt64.alloc(m.n);
    }
    autotune(h, h->opts.tune);
    HIPC(hipStreamSynchronize(h->stream));
}

void destroy(cps_handle* h)
{
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (int l = 0; l < kMaxLevels; ++l) {
        LevelMem& m = h->lv[l];
        m.G64.release(); m.G32.release();
        m.x64.release(); m.b64.release(); m.r64.release();
        m.xt64.release(); m.xt32.release();
        m.x32.release(); m.b32.release(); m.r32.release();
    }
    h->Ainv.release(); h->partial.release(); h->sc.release();
    h->x0.release(); h->b0.release(); h->r.release(); h->z.release(); h->pd.release(); h->q.release();
    h->r0.release(); h->v.release(); h->s.release(); h->t.release(); h->ph.release();
    h->sh.release();
    h->pC.release(); h->pJf.release(); h->pJc.release(); h->prhs.release(); h->prot.release();
    h->plf[0].release(); h->plf[1].release(); h->pls.release(); h->plam.release();
    h->ptw.release(); h->ptwN.release();
    {
        MemLock lk(g_capture_mu); // graph teardown and the pinned free
        for (hipGraphExec_t& g : h->gexec)
            if (g) (void)hipGraphExecDestroy(g);
        if (h->hsc) (void)hipHostFree(h->hsc);
    }
    for (auto& v : h->ev)
        for (hipEvent_t e : v) (void)hipEventDestroy(e);
    delete h;
}

// ---------------------------------------------------------------------------
// solve
// ---------------------------------------------------------------------------

cps_status check_norm(double rr, double bb, double tol, double* rel)
{
    *rel = std::sqrt(rr / bb);
    if (!std::isfinite(*rel)) return CPS_E_DIVERGED;
    return *rel <= tol ? CPS_OK : CPS_E_NOT_CONVERGED;
}

// The Krylov recurrences update r without forming b - A x, and rounding
// lets the two drift apart; a solve that the recurrence calls converged is
// checked on the residual of the iterate itself: y = A x into q, r = b0 - y
// (r then holds it), *rel = ||r|| / ||b0||.  The batched form takes the same
// steps with the same kernel bodies, so both see the same bits.
cps_status true_residual(cps_handle* h, double bb, double tol, double* rel)
{
    const long long n = h->lv[0].n;
    apply<double>(h, 0, h->x0.p, h->q.p, nullptr);
    k_sub<<<nblk(n), kBlock, 0, h->stream>>>(n, h->b0.p, h->q.p, h->r.p);
    LAUNCH_CHECK();
    dot<double, double>(h, n, h->r.p, h->r.p, S_RR);
    return check_norm(read_scalar(h, S_RR), bb, tol, rel);
}

cps_status solve(cps_handle* h, const double* rhs, double* p_out, double tol, cps_info* info)
{
    const auto t0 = std::chrono::steady_clock::now();
    const long long n = h->lv[0].n;
    const int maxit = h->opts.max_iters > 0 ? h->opts.max_iters : 200;
    const bool mixed = h->opts.precision == 1;
    double* x = h->x0.p; // iterate, parity-split order
    // b0 = rhs - mean(rhs) in split order; bb = ||b0||^2
    dot<double, double>(h, n, rhs, nullptr, S_SUM);
    k_to_split<double, double><<<nblk(n), kBlock, 0, h->stream>>>(h->lv[0].geo, rhs, h->b0.p,
                                                                   h->sc.p + S_SUM);
    LAUNCH_CHECK();
    dot<double, double>(h, n, h->b0.p, h->b0.p, S_BB);
    k_sqrt_scalar<<<1, 1, 0, h->stream>>>(h->sc.p, S_SCALE, S_BB);
    LAUNCH_CHECK();
    fill<double>(h, x, n, 0.0);
    fill<double>(h, p_out, n, 0.0);
    HIPC(hipMemcpyAsync(h->hsc, h->sc.p, S_COUNT * sizeof(double), hipMemcpyDeviceToHost,
                        h->stream));
    HIPC(hipStreamSynchronize(h->stream));
    const double bb = h->hsc[S_BB];
    const double mean = h->hsc[S_SUM] / (double)n;
    int it = 0;
    double rel = 0.0;
    cps_status st = CPS_OK;
    if (!std::isfinite(bb)) {
        st = CPS_E_DIVERGED;
        rel = NAN;
    } else if (bb > 0.0) {
        st = CPS_E_NOT_CONVERGED;
        if (h->opts.accel == 0) {
            // stationary: x <- x + V(b - A x)
            if (!mixed) {
                for (it = 1; it <= maxit; ++it) {
                    run_body(h, G_RICH, [&] {
                        vcycle<double>(h, h->b0.p, x);
                        reduce_norm(h, residual<double>(h, 0, h->b0.p, x, h->r.p, true), S_RR);
                    });
                    st = check_norm(body_norm(h, S_RR), bb, tol, &rel);
                    if (st != CPS_E_NOT_CONVERGED) break;
                }
            } else {
                k_copy<double><<<nblk(n), kBlock, 0, h->stream>>>(n, h->b0.p, h->r.p);
                LAUNCH_CHECK();
                k_copy_scalar<<<1, 1, 0, h->stream>>>(h->sc.p, S_RR, S_BB);
                LAUNCH_CHECK();
                float* b32 = h->lv[0].b32.p;
                float* x32 = h->lv[0].x32.p;
                for (it = 1; it <= maxit; ++it) {
                    // s = ||r||; FP32 cycle on r/s; x += s e; FP64 residual
                    run_body(h, G_RICH, [&] {
                        k_sqrt_scalar<<<1, 1, 0, h->stream>>>(h->sc.p, S_SCALE, S_RR);
                        k_cast<double, float><<<nblk(n), kBlock, 0, h->stream>>>(n, h->r.p, b32, h->sc.p, S_SCALE, 1);
                        LAUNCH_CHECK();
                        vcycle<float>(h, b32, x32, true);
                        k_ir_update<float><<<nblk(n), kBlock, 0, h->stream>>>(n, x, x32, h->sc.p + S_SCALE);
                        LAUNCH_CHECK();
                        reduce_norm(h, residual<double>(h, 0, h->b0.p, x, h->r.p, true), S_RR);
                    });
                    st = check_norm(body_norm(h, S_RR), bb, tol, &rel);
                    if (st != CPS_E_NOT_CONVERGED) break;
                }
            }
        } else if (h->opts.accel == 1) {
            // preconditioned CG; flexible (Polak-Ribiere) when the
            // preconditioner runs in FP32 or the operator has cross terms
            // (mildly non-symmetric: the flexible form converges there in
            // fewer V-cycles than BiCGStab's two per iteration).  The search
            // direction alternates between two buffers: p = z + beta p_old
            // is formed inside the product q = A p where the level allows it.
            const int flexible = (mixed || h->mode != MODE_ORTHO) ? 1 : 0;
            double* r = h->r.p;
            double* z = h->z.p;
            double* p = h->pd.p;
            double* pn = h->ph.p;
            double* q = h->q.p;
            const Geo& g0 = h->lv[0].geo;
            const bool fused = marching(h) && row_pairs(g0);
            k_copy<double><<<nblk(n), kBlock, 0, h->stream>>>(n, h->b0.p, r);
            LAUNCH_CHECK();
            precondition(h, r, z, S_RZ);
            k_copy<double><<<nblk(n), kBlock, 0, h->stream>>>(n, z, p);
            LAUNCH_CHECK();
            reduce(h, apply<double>(h, 0, p, q, p), S_PQ, 0, RED_ALPHA | RED_SHIFT_ALPHA);
            // the mixed form on the fused path: the step also casts the new
            // residual into the FP32 right-hand side, and the direction is
            // formed from the FP32 correction (no FP64 cast pass, z not stored)
            const bool cast_fused = fused && mixed;
            float* r32 = cast_fused ? h->lv[0].b32.p : nullptr;
            // FP64 point smoothing with the per-kernel finest level: the step
            // also makes the next cycle's zero-iterate first pass, z = r / D
            // on the red cells, and forms q = A p again from p, so the
            // direction kernel does not store q (k_cg_step_z)
            const bool zfused = fused && !mixed && h->opts.smoother == 0 && h->ncol == 2 &&
                                !h->lv[0].tile;
            // x += alpha p, r -= alpha q and ||r||^2 (the first iteration's
            // step, and the tail of every later body; alpha comes from the
            // launch that stored p.q).  On the fused path the next direction
            // kernel applies x += alpha p instead (it streams p anyway), and
            // the last update runs after the loop.
            double* plast = p; // direction of the last step
            auto step = [&](double* pk) {
                if (zfused) { // q = A p formed again from p (the direction kernel keeps no q)
                    const MarchShape ms = stencil_shape(g0);
                    k_cg_step_z<<<ms.grid, kBlock, 0, h->stream>>>(g0, h->lv[0].G64.p,
                                                                   h->lv[0].gk, ms.bpa, ms.ch,
                                                                   h->sc.p, pk, r, z,
                                                                   h->partial.p);
                    LAUNCH_CHECK();
                    reduce_norm(h, ms.grid, S_RR);
                } else {
                    k_cg_step<<<vgrid(n), kBlock, 0, h->stream>>>(n, h->sc.p, fused ? nullptr : x,
                                                                  r, pk, q, h->partial.p, r32);
                    LAUNCH_CHECK();
                    reduce_norm(h, vgrid(n), S_RR);
                }
            };
            step(p);
            it = 1;
            st = check_norm(body_norm(h, S_RR), bb, tol, &rel);
            // later iterations: new direction from the preconditioned
            // residual, then the step; with the fused product the direction
            // alternates between two buffers, so two bodies by parity.  The
            // iterate's pending updates are applied every other iteration:
            // the even body leaves alpha p_old pending, the odd one applies
            // both (the older direction is still in the buffer it overwrites)
            double* pprev = nullptr; // the direction an even body left pending
            for (;;) {
                while (st == CPS_E_NOT_CONVERGED && it < maxit) {
                    ++it;
                    const int parity = fused ? (it & 1) : 0;
                    double* pc = parity ? pn : p; // direction of the previous iteration
                    double* pnx = parity ? p : pn;
                    run_body(h, G_CG0 + parity, [&] {
                        // the launch that stores the new r.z keeps the old one
                        // and forms beta (flexible: the one that stores z.q)
                        precondition(h, r, cast_fused ? nullptr : z, S_RZ, flexible ? q : nullptr,
                                     cast_fused, flexible ? RED_SHIFT_RZ : RED_SHIFT_RZ | RED_BETA,
                                     flexible ? RED_FBETA : 0, zfused);
                        if (fused) {
                            const MarchShape ms = stencil_shape(g0);
                            {
                                ProfScope ps(h, CPS_KERNEL_APPLY, 0); // the product only
                                // the odd body applies both pending updates of
                                // the iterate, the even body none
                                auto kd = parity ? k_apply_dir_march2<double, 0, 2>
                                                 : k_apply_dir_march2<double, 0, 0>;
                                auto kc = parity ? k_apply_dircast_march2<2>
                                                 : k_apply_dircast_march2<0>;
                                if (cast_fused)
                                    kc<<<ms.grid, kBlock, 0, h->stream>>>(
                                        g0, h->lv[0].G64.p, h->lv[0].gk, ms.bpa, ms.ch,
                                        h->lv[0].x32.p, h->sc.p, S_SCALE, S_BETA, pc, pnx, q,
                                        h->partial.p, x);
                                else
                                    kd<<<ms.grid, kBlock, 0, h->stream>>>(
                                        g0, h->lv[0].G64.p, h->lv[0].gk, ms.bpa, ms.ch, z, pc,
                                        h->sc.p + S_BETA, pnx, zfused ? nullptr : q,
                                        h->partial.p, x, h->sc.p);
                                LAUNCH_CHECK();
                            }
                            reduce(h, ms.grid, S_PQ, 0, RED_ALPHA | RED_SHIFT_ALPHA);
                            step(pnx);
                        } else {
                            k_cg_dir<<<nblk(n), kBlock, 0, h->stream>>>(n, h->sc.p, z, p);
                            LAUNCH_CHECK();
                            reduce(h, apply<double>(h, 0, p, q, p), S_PQ, 0, RED_ALPHA);
                            step(p);
                        }
                    });
                    if (fused) {
                        plast = pnx;
                        pprev = parity ? nullptr : pc;
                    }
                    st = check_norm(body_norm(h, S_RR), bb, tol, &rel);
                }
                if (fused) { // the updates the last steps left pending, in order
                    if (pprev) {
                        k_cg_x<<<nblk(n), kBlock, 0, h->stream>>>(n, h->sc.p, pprev, x,
                                                                   S_ALPHA_OLD);
                        LAUNCH_CHECK();
                    }
                    k_cg_x<<<nblk(n), kBlock, 0, h->stream>>>(n, h->sc.p, plast, x, S_ALPHA);
                    LAUNCH_CHECK();
                    pprev = nullptr;
                }
                if (st != CPS_OK) break;
                st = true_residual(h, bb, tol, &rel);
                if (st != CPS_E_NOT_CONVERGED || it >= maxit) break;
                // restart from the residual of the iterate: the next direction
                // is the preconditioned residual alone (its previous direction
                // is zero, and so are the pending updates that the fused
                // product applies with it and the direction before it)
                fill<double>(h, p, n, 0.0);
                fill<double>(h, pn, n, 0.0);
                // the next body expects the zero-iterate pass of the new r
                if (zfused) gs_pass<double>(h, 0, 0, r, z, true);
                if (cast_fused) {
                    k_cast<double, float><<<nblk(n), kBlock, 0, h->stream>>>(n, r, r32, h->sc.p,
                                                                             S_SCALE, 1);
                    LAUNCH_CHECK();
                }
            }
        } else {
            // BiCGStab (accel = 2), right-preconditioned by the V-cycle
            double* r = h->r.p;
            double* p = h->pd.p;
            k_copy<double><<<nblk(n), kBlock, 0, h->stream>>>(n, h->b0.p, r);
            LAUNCH_CHECK();
            auto start = [&] { // (re)start from the residual in r
                k_copy<double><<<nblk(n), kBlock, 0, h->stream>>>(n, r, h->r0.p);
                LAUNCH_CHECK();
                fill<double>(h, p, n, 0.0);
                fill<double>(h, h->v.p, n, 0.0);
                k_set_scalar<<<1, 1, 0, h->stream>>>(h->sc.p, S_RHO, 1.0); // becomes rho_old
                k_set_scalar<<<1, 1, 0, h->stream>>>(h->sc.p, S_ALPHA, 1.0);
                k_set_scalar<<<1, 1, 0, h->stream>>>(h->sc.p, S_OMEGA, 1.0);
                LAUNCH_CHECK();
            };
            start();
            for (it = 1; it <= maxit; ++it) {
                run_body(h, G_BICG, [&] {
                    k_copy_scalar<<<1, 1, 0, h->stream>>>(h->sc.p, S_RHO_OLD, S_RHO);
                    LAUNCH_CHECK();
                    dot<double, double>(h, n, h->r0.p, r, S_RHO);
                    SCALAR_KERNEL(h, k_bicg_beta);
                    k_bicg_dir<<<nblk(n), kBlock, 0, h->stream>>>(n, h->sc.p, r, h->v.p, p);
                    LAUNCH_CHECK();
                    precondition(h, p, h->ph.p);
                    reduce(h, apply<double>(h, 0, h->ph.p, h->v.p, h->r0.p), S_R0V);
                    SCALAR_KERNEL(h, k_bicg_alpha);
                    k_bicg_s<<<nblk(n), kBlock, 0, h->stream>>>(n, h->sc.p, r, h->v.p, h->s.p);
                    LAUNCH_CHECK();
                    precondition(h, h->s.p, h->sh.p);
                    reduce(h, apply<double>(h, 0, h->sh.p, h->t.p, h->s.p), S_TS);
                    dot<double, double>(h, n, h->t.p, h->t.p, S_TT);
                    SCALAR_KERNEL(h, k_bicg_omega);
                    k_bicg_step<<<vgrid(n), kBlock, 0, h->stream>>>(n, h->sc.p, x, r, h->ph.p,
                                                                   h->sh.p, h->s.p, h->t.p,
                                                                   h->partial.p);
                    LAUNCH_CHECK();
                    reduce_norm(h, vgrid(n), S_RR);
                });
                st = check_norm(body_norm(h, S_RR), bb, tol, &rel);
                if (st == CPS_OK) { // the recurrence says so: check b - A x
                    st = true_residual(h, bb, tol, &rel);
                    if (st == CPS_E_NOT_CONVERGED && it < maxit) start();
                }
                if (st != CPS_E_NOT_CONVERGED) break;
            }
        }
        if (it > maxit) it = maxit;
        // zero-mean result in natural order
        dot<double, double>(h, n, x, nullptr, S_SUM);
        k_from_split<double, double><<<nblk(n), kBlock, 0, h->stream>>>(h->lv[0].geo, x, p_out,
                                                                         h->sc.p + S_SUM);
        LAUNCH_CHECK();
    }
    HIPC(hipStreamSynchronize(h->stream));
    if (info) {
        info->iterations = it;
        info->rel_residual = rel;
        info->rhs_mean_removed = mean;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (st == CPS_E_NOT_CONVERGED)
        g_err = "iteration cap reached at relative residual " + std::to_string(rel);
    else if (st == CPS_E_DIVERGED)
        g_err = "residual norm is not finite";
    return st;
}

template <typename F>
cps_status guarded(F&& f)
{
    try {
        f();
        return CPS_OK;
    } catch (const Fail& e) {
        return e.st;
    } catch (const std::bad_alloc&) {
        g_err = "host allocation failed";
        return CPS_E_OOM;
    }
}

// Device copy of a natural-order level vector in parity-split order (the
// buffer is owned by `tmp`), and the copy back.  Used by the per-step entry
// points, whose arguments are in natural order.
double* split_copy(cps_handle* h, int l, const double* nat, Buf<double>& tmp)
{
    const long long n = h->lv[l].n;
    tmp.alloc(n);
    k_to_split<double, double><<<nblk(n), kBlock, 0, h->stream>>>(h->lv[l].geo, nat, tmp.p, nullptr);
    LAUNCH_CHECK();
    return tmp.p;
}

void natural_copy(cps_handle* h, int l, const double* split, double* nat)
{
    const long long n = h->lv[l].n;
    k_from_split<double, double><<<nblk(n), kBlock, 0, h->stream>>>(h->lv[l].geo, split, nat, nullptr);
    LAUNCH_CHECK();
    HIPC(hipStreamSynchronize(h->stream));
}

void need_level(const cps_handle* h, int l, bool fine)
{
    if (!h) fail(CPS_E_INVALID, "handle is NULL");
    if (l < 0 || l >= h->L || (fine && l >= h->L - 1))
        fail(CPS_E_INVALID, "level %d out of range", l);
    if (h->opts.precision != 0) fail(CPS_E_INVALID, "debug entry points need an FP64 handle");
}

} // namespace

// batched form (same translation unit: shares the hierarchy code above)
#include "batch.hpp"
// solve service (same translation unit)
#include "service.hpp"

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// projection step (eq. (PC_6) right-hand side, eq. (PC_7))
// ---------------------------------------------------------------------------

namespace {

// Face tables of the finest grid for the projection step, on first use and
// after every recomputation of the metrics.
int csym(const cps_handle* h)
{
    if (!h->axi) return kPerCell;
    return h->grid.map == CPS_MAP_IDENTITY ? kInvariant : kRotational;
}

// The projection step and the line solves form C rows from the map's chords.
void need_map(const cps_handle* h)
{
    if (h->met.method == CPS_METRICS_USER_FACE)
        fail(CPS_E_INVALID, "the projection step and the line solves need the map's chords; this "
                            "handle was set up with caller-supplied face metrics");
}

void ensure_cmetrics(cps_handle* h)
{
    need_map(h);
    if (h->cm_valid) return;
    const LevelMem& m = h->lv[0];
    const int nc = csym(h) == kPerCell ? m.np : 1;
    const long long F = (long long)(m.nr + 1) * (m.nt + 1) * nc;
    const long long nj = (long long)m.nr * m.nt * nc;
    if (h->pC.n != (size_t)(9 * F)) h->pC.alloc(9 * F);
    if (h->pJf.n != (size_t)(3 * F)) h->pJf.alloc(3 * F);
    if (h->pJc.n != (size_t)nj) h->pJc.alloc(nj);
    const cps_grid& g = h->grid;
    MapParams mp{g.map, g.r_inner, g.r_outer, g.theta0, g.theta1, g.radial_stretch, g.flattening,
                 g.skew};
    k_crows<<<nblk(F), kBlock, 0, h->stream>>>(mp, m.nr, m.nt, m.np, nc, h->met.method, h->pC.p,
                                               h->pJf.p);
    LAUNCH_CHECK();
    k_cell_jdet<<<nblk(nj), kBlock, 0, h->stream>>>(m.nr, m.nt, nc, h->pJf.p, h->pJc.p);
    LAUNCH_CHECK();
    // cos, sin of the azimuth 2 pi c / n_phi for c = 0 .. n_phi (the turn of
    // cell c's faces against cell 0's about the polar axis)
    std::vector<double> rot(2 * (m.np + 1));
    for (int c = 0; c <= m.np; ++c) {
        rot[2 * c] = std::cos(2.0 * M_PI * c / m.np);
        rot[2 * c + 1] = std::sin(2.0 * M_PI * c / m.np);
    }
    h->prot.alloc(rot.size());
    HIPC(hipMemcpyAsync(h->prot.p, rot.data(), rot.size() * sizeof(double),
                        hipMemcpyHostToDevice, h->stream));
    HIPC(hipStreamSynchronize(h->stream));
    h->cm_valid = true;
}

CRows crows(const cps_handle* h)
{
    const LevelMem& m = h->lv[0];
    const int nc = csym(h) == kPerCell ? m.np : 1;
    return CRows{h->pC.p, (long long)(m.nr + 1) * (m.nt + 1) * nc, m.nt + 1, nc, h->prot.p};
}

// launch f.template operator()<SYM>() for the handle's symmetry
template <typename F>
void with_csym(const cps_handle* h, F&& f)
{
    switch (csym(h)) {
    case kPerCell: f(std::integral_constant<int, kPerCell>{}); break;
    case kInvariant: f(std::integral_constant<int, kInvariant>{}); break;
    default: f(std::integral_constant<int, kRotational>{}); break;
    }
}

void divergence(cps_handle* h, const double* u, double* rhs)
{
    ensure_cmetrics(h);
    const LevelMem& m = h->lv[0];
    ProfScope ps(h, CPS_KERNEL_DIVERGENCE, 0);
    with_csym(h, [&](auto S) {
        if (m.nt % 2 == 0)
            k_divergence2<decltype(S)::value>
                <<<(unsigned)proj2_grid(m.nr, m.nt, m.np), kBlock, 0, h->stream>>>(
                    m.nr, m.nt, m.np, crows(h), u, rhs);
        else
            k_divergence<decltype(S)::value>
                <<<(unsigned)proj_grid(m.nr, m.nt, m.np), kBlock, 0, h->stream>>>(
                    m.nr, m.nt, m.np, crows(h), u, rhs);
    });
    LAUNCH_CHECK();
}

void correct(cps_handle* h, const double* phi, double* u)
{
    ensure_cmetrics(h);
    const LevelMem& m = h->lv[0];
    ProfScope ps(h, CPS_KERNEL_CORRECT, 0);
    with_csym(h, [&](auto S) {
        k_correct<decltype(S)::value><<<(unsigned)proj_grid(m.nr, m.nt, m.np), kBlock, 0,
                                        h->stream>>>(m.nr, m.nt, m.np, crows(h), h->pJc.p, phi,
                                                     u);
    });
    LAUNCH_CHECK();
}

} // namespace

// ---------------------------------------------------------------------------
// ADI line solves (eq. (solve_2)-(solve_4))
// ---------------------------------------------------------------------------

namespace {

bool same_bc(const LineBC& x, const LineBC& y)
{
    return x.type_lo == y.type_lo && x.type_hi == y.type_hi && x.v_lo == y.v_lo &&
           x.v_hi == y.v_hi;
}

// ring transform applies: n_phi / 2 a power of two in [2, kPlaneLds], both
// fields 16-byte aligned (they are read and written as pairs)
bool fft_lines(const cps_handle* h, const double* rhs, const double* psi)
{
    const int nh = h->lv[0].np / 2;
    return nh >= 2 && nh <= kPlaneLds && (nh & (nh - 1)) == 0 &&
           ((uintptr_t)rhs % 16) == 0 && ((uintptr_t)psi % 16) == 0;
}

void ring_tables(cps_handle* h, double* tw, double* twN, double* lam)
{
    const int np = h->lv[0].np;
    k_ring_tables<<<nblk(np / 2 + 1), kBlock, 0, h->stream>>>(np, tw, twN, lam);
    LAUNCH_CHECK();
}

void ensure_ring_tables(cps_handle* h)
{
    if (h->plam.p) return;
    const int nh = h->lv[0].np / 2;
    h->ptw.alloc(nh);
    h->ptwN.alloc(2 * (nh + 1));
    h->plam.alloc(nh + 1);
    ring_tables(h, h->ptw.p, h->ptwN.p, h->plam.p);
}

// The fixed device array of the allocation-free line solve.  In host code
// `line_scratch` names a host-side stand-in, not device memory: kernels get
// the address hipGetSymbolAddress returns for the current device.
constexpr size_t kLineScratchWords = CPS_LINE_SCRATCH_BYTES / sizeof(double);
__device__ __align__(256) double line_scratch[kLineScratchWords];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// Device address of line_scratch on the current device, resolved once per
// device (at set-up, so that a later call under graph capture finds it).
double* line_scratch_ptr()
{
    int dev = 0;
    HIPC(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) fail(CPS_E_INVALID, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        HIPC(hipGetSymbolAddress(&p, HIP_SYMBOL(line_scratch)));
        g_scratch_dev[dev] = static_cast<double*>(p);
    }
    return g_scratch_dev[dev];
}

// cps_line_solve with its tables formed in line_scratch on every call:
// the same kernels in the same order, launches only.
void line_solve_noalloc(cps_handle* h, int dir, double coef, const LineBC& bc,
                        const double* rhs, double* psi)
{
    const LevelMem& m = h->lv[0];
    need_map(h);
    if (csym(h) == kPerCell)
        fail(CPS_E_INVALID, "line solves need phi-invariant metrics (box, sphere, oblate)");
    auto even = [](long long w) { return (w + 1) & ~1LL; }; // 16-byte aligned parts
    const long long F = (long long)(m.nr + 1) * (m.nt + 1), nj = (long long)m.nr * m.nt;
    const int lines = dir == 0 ? m.nt : m.nr, n = dir == 0 ? m.nr : m.nt, nh = m.np / 2;
    const long long tables = dir < 2 ? even(3LL * lines * n + 2LL * lines)
                                     : even(nh) + even(2LL * (nh + 1)) + even(nh + 1);
    const long long words = even(9 * F) + even(3 * F) + even(nj) + tables;
    if (words > (long long)kLineScratchWords)
        fail(CPS_E_INVALID, "the line solve's tables need %lld bytes, more than the %zu of the "
             "allocation-free array", 8 * words, (size_t)CPS_LINE_SCRATCH_BYTES);
    if (dir == 2 && !fft_lines(h, rhs, psi))
        fail(CPS_E_INVALID, "the allocation-free phi-line solve needs n_phi / 2 a power of two "
             "in [2, %d] and 16-byte aligned fields", kPlaneLds);
    double* C = line_scratch_ptr();
    double* Jf = C + even(9 * F);
    double* Jc = Jf + even(3 * F);
    double* T = Jc + even(nj);
    const cps_grid& g = h->grid;
    const MapParams mp{g.map, g.r_inner, g.r_outer, g.theta0, g.theta1, g.radial_stretch,
                       g.flattening, g.skew};
    k_crows<<<nblk(F), kBlock, 0, h->stream>>>(mp, m.nr, m.nt, m.np, 1, h->met.method, C, Jf);
    LAUNCH_CHECK();
    k_cell_jdet<<<nblk(nj), kBlock, 0, h->stream>>>(m.nr, m.nt, 1, Jf, Jc);
    LAUNCH_CHECK();
    const CRows R{C, F, m.nt + 1, 1, nullptr};
    if (dir < 2) {
        double* Fm = T;
        double* Fi = Fm + (size_t)lines * n;
        double* Fh = Fi + (size_t)lines * n;
        double* Fx = Fh + (size_t)lines * n;
        k_line_factor<<<nblk(lines), kBlock, 0, h->stream>>>(m.nr, m.nt, dir, coef, bc, R, Jf, Jc,
                                                             Fm, Fi, Fh, Fx);
        LAUNCH_CHECK();
        const long long threads = (long long)lines * m.np;
        if (dir == 0)
            k_line_open<0><<<nblk(threads), kBlock, 0, h->stream>>>(m.nr, m.nt, m.np, Fm, Fi, Fh,
                                                                    Fx, rhs, psi);
        else
            k_line_open<1><<<nblk(threads), kBlock, 0, h->stream>>>(m.nr, m.nt, m.np, Fm, Fi, Fh,
                                                                    Fx, rhs, psi);
        LAUNCH_CHECK();
        return;
    }
    double* tw = T;
    double* twN = tw + even(nh);
    double* lam = twN + even(2LL * (nh + 1));
    ring_tables(h, tw, twN, lam);
    const FftLineLaunch pl = fft_line_launch(m.nr, m.nt, m.np);
    const auto* tw2 = reinterpret_cast<const Vec2<double>*>(tw);
    const auto* twN2 = reinterpret_cast<const Vec2<double>*>(twN);
    if (nh <= kSmallRing)
        k_line_fft<kSmallRing><<<pl.blocks, pl.threads, 0, h->stream>>>(
            m.nr, m.nt, m.np, coef, R, Jf, Jc, tw2, twN2, lam, rhs, psi);
    else
        k_line_fft<kPlaneLds><<<pl.blocks, pl.threads, 0, h->stream>>>(
            m.nr, m.nt, m.np, coef, R, Jf, Jc, tw2, twN2, lam, rhs, psi);
    LAUNCH_CHECK();
}

void line_solve(cps_handle* h, int dir, double coef, const LineBC& bc, const double* rhs,
                double* psi)
{
    ensure_cmetrics(h);
    const LevelMem& m = h->lv[0];
    const CRows R = crows(h);
    if (dir < 2) {
        const int lines = dir == 0 ? m.nt : m.nr, n = dir == 0 ? m.nr : m.nt;
        Buf<double>& F = h->plf[dir];
        const size_t need = 3 * (size_t)lines * n + 2 * (size_t)lines;
        double* Fm;
        double *Fi, *Fh, *Fx;
        auto views = [&] {
            Fm = F.p;
            Fi = Fm + (size_t)lines * n;
            Fh = Fi + (size_t)lines * n;
            Fx = Fh + (size_t)lines * n;
        };
        // the elimination depends on (coef, walls) and the metrics only: an
        // ADI step repeats it every time step, so it is kept
        if (!h->lf_valid[dir] || h->lf_coef[dir] != coef || !same_bc(h->lf_bc[dir], bc)) {
            if (F.n < need) F.alloc(need);
            views();
            k_line_factor<<<nblk(lines), kBlock, 0, h->stream>>>(m.nr, m.nt, dir, coef, bc, R,
                                                                 h->pJf.p, h->pJc.p, Fm, Fi, Fh,
                                                                 Fx);
            LAUNCH_CHECK();
            h->lf_valid[dir] = true;
            h->lf_coef[dir] = coef;
            h->lf_bc[dir] = bc;
        }
        views();
        const long long threads = (long long)lines * m.np;
        if (dir == 0)
            k_line_open<0><<<nblk(threads), kBlock, 0, h->stream>>>(m.nr, m.nt, m.np, Fm, Fi, Fh,
                                                                    Fx, rhs, psi);
        else
            k_line_open<1><<<nblk(threads), kBlock, 0, h->stream>>>(m.nr, m.nt, m.np, Fm, Fi, Fh,
                                                                    Fx, rhs, psi);
        LAUNCH_CHECK();
        return;
    }
    if (fft_lines(h, rhs, psi)) {
        ensure_ring_tables(h);
        const FftLineLaunch pl = fft_line_launch(m.nr, m.nt, m.np);
        const auto* tw = reinterpret_cast<const Vec2<double>*>(h->ptw.p);
        const auto* twN = reinterpret_cast<const Vec2<double>*>(h->ptwN.p);
        if (m.np / 2 <= kSmallRing)
            k_line_fft<kSmallRing><<<pl.blocks, pl.threads, 0, h->stream>>>(
                m.nr, m.nt, m.np, coef, R, h->pJf.p, h->pJc.p, tw, twN, h->plam.p, rhs, psi);
        else
            k_line_fft<kPlaneLds><<<pl.blocks, pl.threads, 0, h->stream>>>(
                m.nr, m.nt, m.np, coef, R, h->pJf.p, h->pJc.p, tw, twN, h->plam.p, rhs, psi);
        LAUNCH_CHECK();
        return;
    }
    if (h->pls.n < (size_t)(2 * m.n)) h->pls.alloc(2 * m.n);
    k_line_periodic<<<nblk((long long)m.nr * m.nt), kBlock, 0, h->stream>>>(
        m.nr, m.nt, m.np, coef, R, h->pJf.p, h->pJc.p, rhs, psi, h->pls.p, h->pls.p + m.n);
    LAUNCH_CHECK();
}

} // namespace

extern "C" {

void cps_grid_default(cps_grid* g)
{
    if (!g) return;
    std::memset(g, 0, sizeof *g);
    g->n_r = g->n_theta = g->n_phi = 32;
    g->map = CPS_MAP_SPHERE;
    g->r_inner = 1.5;
    g->r_outer = 2.5;
    g->theta0 = 0.05;
    g->theta1 = M_PI - 0.05;
}

const char* cps_last_error(void) { return g_err.c_str(); }

cps_status cps_setup(const cps_grid* grid, const cps_metrics* metrics, const cps_opts* opts,
                     cps_handle** out)
{
    if (!out) {
        g_err = "out is NULL";
        return CPS_E_INVALID;
    }
    *out = nullptr;
    cps_handle* h = nullptr;
    cps_status st = guarded([&] {
        validate(grid, metrics, opts);
        h = new cps_handle();
        h->grid = *grid;
        if (metrics) h->met = *metrics;
        if (opts) h->opts = *opts;
        h->stream = (hipStream_t)h->opts.stream;
        build(h);
        line_scratch_ptr(); // the allocation-free line solve's array on this device
    });
    if (st != CPS_OK) {
        destroy(h);
        return st;
    }
    *out = h;
    return CPS_OK;
}

cps_status cps_solve(cps_handle* h, const double* rhs, double* p, double tol, cps_info* info)
{
    cps_status st = CPS_OK;
    cps_status g = guarded([&] {
        if (!h || !rhs || !p) fail(CPS_E_INVALID, "NULL argument");
        if (rhs == p) fail(CPS_E_INVALID, "rhs and p must not alias");
        if (!(tol > 0)) fail(CPS_E_INVALID, "tol must be positive");
        st = solve(h, rhs, p, tol, info);
    });
    return g != CPS_OK ? g : st;
}

void cps_destroy(cps_handle* h) { destroy(h); }

cps_status cps_levels(const cps_handle* h, int32_t* n_levels, int32_t* dims_out,
                      int32_t* ncolours, int32_t* phi_invariant)
{
    return guarded([&] {
        if (!h) fail(CPS_E_INVALID, "handle is NULL");
        if (n_levels) *n_levels = h->L;
        if (dims_out)
            for (int l = 0; l < h->L; ++l) {
                dims_out[3 * l] = h->lv[l].nr;
                dims_out[3 * l + 1] = h->lv[l].nt;
                dims_out[3 * l + 2] = h->lv[l].np;
            }
        if (ncolours) *ncolours = h->ncol;
        if (phi_invariant) *phi_invariant = h->axi ? 1 : 0;
    });
}

cps_status cps_debug_metrics(cps_handle* h, int32_t level, double* G_out)
{
    return guarded([&] {
        need_level(h, level, false);
        const LevelMem& m = h->lv[level];
        k_expand_metrics<<<nblk(m.n), kBlock, 0, h->stream>>>(m.geo, h->axi ? 1 : 0, m.G64.p, G_out);
        LAUNCH_CHECK();
        HIPC(hipStreamSynchronize(h->stream));
    });
}

cps_status cps_debug_apply(cps_handle* h, int32_t level, const double* x, double* y)
{
    return guarded([&] {
        need_level(h, level, false);
        Buf<double> xs, ys;
        const double* xp = split_copy(h, level, x, xs);
        ys.alloc(h->lv[level].n);
        apply<double>(h, level, xp, ys.p, nullptr);
        natural_copy(h, level, ys.p, y);
    });
}

cps_status cps_debug_residual(cps_handle* h, int32_t level, const double* b, const double* x,
                              double* r, double* norm2)
{
    return guarded([&] {
        need_level(h, level, false);
        Buf<double> bs, xs, rs;
        const double* bp = split_copy(h, level, b, bs);
        const double* xp = split_copy(h, level, x, xs);
        rs.alloc(h->lv[level].n);
        reduce(h, residual<double>(h, level, bp, xp, rs.p, true), S_RR);
        natural_copy(h, level, rs.p, r);
        const double v = read_scalar(h, S_RR);
        if (norm2) *norm2 = v;
    });
}

cps_status cps_debug_gs_pass(cps_handle* h, int32_t level, int32_t colour, const double* b,
                             double* x)
{
    return guarded([&] {
        need_level(h, level, true);
        if (colour < 0 || colour >= h->ncol) fail(CPS_E_INVALID, "bad colour");
        Buf<double> bs, xs;
        const double* bp = split_copy(h, level, b, bs);
        double* xp = split_copy(h, level, x, xs);
        gs_pass<double>(h, level, colour, bp, xp);
        natural_copy(h, level, xp, x);
    });
}

cps_status cps_debug_plane_sweep(cps_handle* h, int32_t level, int32_t parity, const double* b,
                                 double* x)
{
    return guarded([&] {
        need_level(h, level, true);
        if (parity < 0 || parity > 1) fail(CPS_E_INVALID, "bad parity");
        if (h->opts.smoother != 1) fail(CPS_E_INVALID, "handle not set up with smoother = 1");
        Buf<double> bs, xs;
        const double* bp = split_copy(h, level, b, bs);
        double* xp = split_copy(h, level, x, xs);
        plane_half_sweep<double>(h, level, parity, bp, xp);
        natural_copy(h, level, xp, x);
    });
}

cps_status cps_debug_restrict(cps_handle* h, int32_t level, const double* r, double* bc)
{
    return guarded([&] {
        need_level(h, level, true);
        Buf<double> rs, cs;
        const double* rp = split_copy(h, level, r, rs);
        cs.alloc(h->lv[level + 1].n);
        restrict_to<double>(h, level, rp, cs.p);
        natural_copy(h, level + 1, cs.p, bc);
    });
}

cps_status cps_debug_residual_restrict(cps_handle* h, int32_t level, const double* b,
                                       const double* x, double* bc)
{
    return guarded([&] {
        need_level(h, level, true);
        if (!red_residual(h, level))
            fail(CPS_E_INVALID, "level %d forms the whole residual (no red-black row-pair level)",
                 level);
        Buf<double> bs, xs, cs;
        const double* bp = split_copy(h, level, b, bs);
        const double* xp = split_copy(h, level, x, xs);
        cs.alloc(h->lv[level + 1].n);
        if (resrestrict_segs(h->lv[level].geo, h->lv[level + 1].geo) > 0) {
            resrestrict<double>(h, level, bp, xp, cs.p);
        } else {
            residual<double>(h, level, bp, xp, rl<double>(h, level), false, true);
            restrict_to<double>(h, level, rl<double>(h, level), cs.p, true);
        }
        natural_copy(h, level + 1, cs.p, bc);
    });
}

cps_status cps_debug_prolong(cps_handle* h, int32_t level, const double* e, double* x)
{
    return guarded([&] {
        need_level(h, level, true);
        Buf<double> es, xs;
        const double* ep = split_copy(h, level + 1, e, es);
        double* xp = split_copy(h, level, x, xs);
        prolong_add<double>(h, level, ep, xp);
        natural_copy(h, level, xp, x);
    });
}

cps_status cps_debug_coarse_solve(cps_handle* h, const double* b, double* e)
{
    return guarded([&] {
        need_level(h, 0, false);
        const int lc = h->L - 1;
        Buf<double> bs, es;
        const double* bp = split_copy(h, lc, b, bs);
        es.alloc(h->lv[lc].n);
        coarse_solve<double>(h, bp, es.p);
        natural_copy(h, lc, es.p, e);
    });
}

cps_status cps_debug_vcycle(cps_handle* h, const double* b, double* x)
{
    return guarded([&] {
        need_level(h, 0, false);
        Buf<double> bs, xs;
        const double* bp = split_copy(h, 0, b, bs);
        double* xp = split_copy(h, 0, x, xs);
        vcycle<double>(h, bp, xp);
        natural_copy(h, 0, xp, x);
    });
}

cps_status cps_profile_enable(cps_handle* h, int32_t enable)
{
    return guarded([&] {
        if (!h) fail(CPS_E_INVALID, "handle is NULL");
        h->prof = enable != 0;
        for (auto& u : h->ev_used) u = 0;
        for (auto& c : h->ev_launches) c = 0;
    });
}

cps_status cps_profile_select(cps_handle* h, uint32_t class_mask)
{
    return guarded([&] {
        if (!h) fail(CPS_E_INVALID, "handle is NULL");
        h->prof_mask = class_mask;
    });
}

cps_status cps_profile_read(cps_handle* h, int32_t kernel_class, double* total_ms,
                            int64_t* launches)
{
    return guarded([&] {
        if (!h) fail(CPS_E_INVALID, "handle is NULL");
        if (kernel_class < 0 || kernel_class >= CPS_KERNEL_CLASSES)
            fail(CPS_E_INVALID, "bad kernel class");
        HIPC(hipStreamSynchronize(h->stream));
        double tot = 0.0;
        const size_t u = h->ev_used[kernel_class];
        for (size_t i = 0; i + 1 < u; i += 2) {
            float ms = 0.f;
            HIPC(hipEventElapsedTime(&ms, h->ev[kernel_class][i], h->ev[kernel_class][i + 1]));
            tot += ms;
        }
        if (total_ms) *total_ms = tot;
        if (launches) *launches = h->ev_launches[kernel_class];
        h->ev_used[kernel_class] = 0;
        h->ev_launches[kernel_class] = 0;
    });
}

cps_status cps_time_vcycle(cps_handle* h, int32_t cycles, int32_t reps, double* us_per_cycle,
                           int64_t* launches_per_cycle)
{
    return guarded([&] {
        if (!h || !us_per_cycle) fail(CPS_E_INVALID, "NULL argument");
        if (cycles < 1 || reps < 1) fail(CPS_E_INVALID, "cycles and reps must be >= 1");
        if (!h->stream) fail(CPS_E_INVALID, "the null stream cannot be captured: set a stream");
        if (h->prof) fail(CPS_E_INVALID, "profiling is on (its events cannot be captured)");
        const long long n = h->lv[0].n;
        const bool mixed = h->opts.precision == 1;
        if (mixed) fill<float>(h, h->lv[0].b32.p, n, 1.0f);
        else fill<double>(h, h->r.p, n, 1.0);
        hipGraph_t g = nullptr;
        hipGraphExec_t ex = nullptr;
        {
            std::shared_lock<std::shared_mutex> cap(g_capture_mu); // no free or sync meanwhile
            HIPC(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
            try {
                for (int c = 0; c < cycles; ++c) {
                    if (mixed) vcycle<float>(h, h->lv[0].b32.p, h->lv[0].x32.p, true);
                    else vcycle<double>(h, h->r.p, h->x0.p, true);
                }
            } catch (...) {
                hipGraph_t g2 = nullptr;
                (void)hipStreamEndCapture(h->stream, &g2);
                if (g2) (void)hipGraphDestroy(g2);
                throw;
            }
            HIPC(hipStreamEndCapture(h->stream, &g));
        }
        int64_t kernels = 0;
        size_t nodes = 0;
        hipError_t e = hipGraphGetNodes(g, nullptr, &nodes);
        if (e == hipSuccess && nodes > 0) {
            std::vector<hipGraphNode_t> list(nodes);
            e = hipGraphGetNodes(g, list.data(), &nodes);
            for (size_t i = 0; i < nodes && e == hipSuccess; ++i) {
                hipGraphNodeType t;
                e = hipGraphNodeGetType(list[i], &t);
                if (e == hipSuccess && t == hipGraphNodeTypeKernel) ++kernels;
            }
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIPC(e);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        float ms = 0.f;
        hipError_t err = hipEventCreate(&e0);
        if (err == hipSuccess) err = hipEventCreate(&e1);
        if (err == hipSuccess) err = hipGraphLaunch(ex, h->stream);
        if (err == hipSuccess) err = hipEventRecord(e0, h->stream);
        for (int i = 0; i < reps && err == hipSuccess; ++i) err = hipGraphLaunch(ex, h->stream);
        if (err == hipSuccess) err = hipEventRecord(e1, h->stream);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        (void)hipStreamSynchronize(h->stream);
        {
            MemLock lk(g_capture_mu); // graph teardown
            (void)hipGraphExecDestroy(ex);
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        HIPC(err);
        *us_per_cycle = (double)ms * 1e3 / ((double)reps * cycles);
        if (launches_per_cycle) *launches_per_cycle = kernels / cycles;
    });
}

cps_status cps_divergence(cps_handle* h, const double* u, double* rhs)
{
    return guarded([&] {
        if (!h || !u || !rhs) fail(CPS_E_INVALID, "NULL argument");
        const long long n = h->lv[0].n;
        if (rhs + n > u && rhs < u + 3 * n) fail(CPS_E_INVALID, "rhs and u must not overlap");
        divergence(h, u, rhs);
    });
}

cps_status cps_correct(cps_handle* h, const double* phi, double* u)
{
    return guarded([&] {
        if (!h || !phi || !u) fail(CPS_E_INVALID, "NULL argument");
        const long long n = h->lv[0].n;
        if (phi + n > u && phi < u + 3 * n) fail(CPS_E_INVALID, "phi and u must not overlap");
        correct(h, phi, u);
    });
}

cps_status cps_project(cps_handle* h, double* u, double* phi, double tol, cps_info* info)
{
    cps_status st = CPS_OK;
    cps_status g = guarded([&] {
        if (!h || !u || !phi) fail(CPS_E_INVALID, "NULL argument");
        if (!(tol > 0)) fail(CPS_E_INVALID, "tol must be positive");
        const long long n = h->lv[0].n;
        if (phi + n > u && phi < u + 3 * n) fail(CPS_E_INVALID, "phi and u must not overlap");
        if (h->prhs.n != (size_t)h->lv[0].n) h->prhs.alloc(h->lv[0].n);
        divergence(h, u, h->prhs.p);
        st = solve(h, h->prhs.p, phi, tol, info);
        if (st == CPS_OK) correct(h, phi, u);
    });
    return g != CPS_OK ? g : st;
}

} // extern "C"

namespace {

// Argument checks shared by both line-solve entry points.
LineBC line_args(const cps_handle* h, int32_t dir, double coef, const cps_line_bc* bc,
                 const double* rhs, const double* psi)
{
    if (!h || !rhs || !psi) fail(CPS_E_INVALID, "NULL argument");
    if (dir < 0 || dir > 2) fail(CPS_E_INVALID, "dir must be 0 (r), 1 (theta) or 2 (phi)");
    if (!(coef >= 0.0) || !std::isfinite(coef)) fail(CPS_E_INVALID, "coef must be >= 0");
    if (!h->axi)
        fail(CPS_E_INVALID, "line solves need phi-invariant metrics (box, sphere, oblate)");
    if (dir == 2 && h->lv[0].np < 3) fail(CPS_E_INVALID, "periodic lines need n_phi >= 3");
    const long long n = h->lv[0].n;
    if (rhs != psi && rhs + n > psi && rhs < psi + n)
        fail(CPS_E_INVALID, "rhs and psi must be the same array or not overlap");
    LineBC b{0, 0, 0.0, 0.0};
    if (bc) {
        if (bc->type_lo < 0 || bc->type_lo > 1 || bc->type_hi < 0 || bc->type_hi > 1)
            fail(CPS_E_INVALID, "bc types must be 0 (no flux) or 1 (value)");
        b = LineBC{bc->type_lo, bc->type_hi, bc->value_lo, bc->value_hi};
    }
    return b;
}

} // namespace

extern "C" {

cps_status cps_line_solve(cps_handle* h, int32_t dir, double coef, const cps_line_bc* bc,
                          const double* rhs, double* psi)
{
    return guarded([&] {
        const LineBC b = line_args(h, dir, coef, bc, rhs, psi);
        line_solve(h, dir, coef, b, rhs, psi);
    });
}

cps_status cps_line_solve_noalloc(cps_handle* h, int32_t dir, double coef, const cps_line_bc* bc,
                                  const double* rhs, double* psi)
{
    return guarded([&] {
        const LineBC b = line_args(h, dir, coef, bc, rhs, psi);
        line_solve_noalloc(h, dir, coef, b, rhs, psi);
    });
}

cps_status cps_debug_copy(const double* src, double* dst, int64_t n, void* stream)
{
    return guarded([&] {
        if (n < 0 || (n && (!src || !dst))) fail(CPS_E_INVALID, "bad copy arguments");
        if (n == 0) return;
        k_copy<double><<<nblk(n), kBlock, 0, (hipStream_t)stream>>>(n, src, dst);
        LAUNCH_CHECK();
        HIPC(hipStreamSynchronize((hipStream_t)stream));
    });
}

} // extern "C"
