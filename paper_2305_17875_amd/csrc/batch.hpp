// batch.hpp -- batched form: many independent shell problems of uneven size
// advanced together.  Included by cps.hip (one translation unit).
//
// Each problem owns a hierarchy built exactly as for cps_solve with FP32
// V-cycles inside FP64 refinement and Krylov acceleration.  Every phase of
// the iteration is ONE launch for all problems that take part in it: a
// device work table gives each block its problem and its logical index
// among the blocks that problem's own launch would have, and per-problem
// descriptors hold the problem's geometry and buffers.  Each problem thus
// sees exactly the arithmetic and reduction order of its own solve: the
// result of a problem is the same alone and in the batch, bit for bit.
// Problems are grouped by stencil and smoother: with the point smoother,
// 7-point with phi-invariant metrics (marching kernels) and the rest
// (generic kernels); with the plane smoother, the 7-point and the 11-point
// (r-theta cross terms) axisymmetric classes.  All run flexible CG.  The
// iteration bodies of the groups are captured once in hipGraphs and replayed; the
// only host round trip per iteration gathers the residual norms, retires
// converged problems and uploads the active flags.

namespace cps {

// Plane-smoother half-sweep kernels of the batched form: the bodies of
// k_plane_fwd / k_plane_tri / k_plane_inv with each block's problem and
// logical index from the work table (rings of <= kSmallRing complex values,
// whose launches take kBlock threads).
template <bool CROSS>
__global__ void __launch_bounds__(kBlock) kb_plane_fwd(const BItem* __restrict__ items,
                                                       const int* __restrict__ active,
                                                       const PDesc<float>* __restrict__ pd,
                                                       int level, int parity)
{
    CPS_BATCH_BLOCK
    __shared__ Vec2<float> buf[kPlaneLds], twS[kPlaneLds / 2];
    const LDesc<float>& d = pd[it.prob].lv[level];
    d_plane_fwd<float, kSmallRing, CROSS>(bk.L, buf, twS, d.g, d.G, d.gk, d.b, d.x, parity,
                                          d.ptw, d.ptwN, d.pS, d.prb);
}

template <bool CROSS>
__global__ void __launch_bounds__(kBlock) kb_plane_tri(const BItem* __restrict__ items,
                                                       const int* __restrict__ active,
                                                       const PDesc<float>* __restrict__ pd,
                                                       int level, int parity)
{
    CPS_BATCH_BLOCK
    const LDesc<float>& d = pd[it.prob].lv[level];
    // the default r-steps in flight: one depth per launch keeps the
    // kernel's registers those of that depth (the depth schedules the same
    // arithmetic, so the bits equal the single solve's with its tuned one)
    d_plane_tri<float, CROSS>((long long)bk.L * blockDim.x + threadIdx.x, d.g, d.G, d.gk,
                              parity, d.ppiv + plane_pivot_offset(d.g, parity),
                              reinterpret_cast<float*>(d.pS));
}

__global__ void __launch_bounds__(kBlock) kb_plane_inv(const BItem* __restrict__ items,
                                                       const int* __restrict__ active,
                                                       const PDesc<float>* __restrict__ pd,
                                                       int level, int parity)
{
    CPS_BATCH_BLOCK
    __shared__ Vec2<float> buf[kPlaneLds], twS[kPlaneLds / 2];
    const LDesc<float>& d = pd[it.prob].lv[level];
    d_plane_inv<float, kSmallRing>(bk.L, buf, twS, d.g, parity, d.ptw, d.ptwN, d.pS, d.x,
                                   d.prb);
}

} // namespace cps

namespace {

struct ItemTable {
    Buf<BItem> d;
    int count = 0;
};

struct BatchGroup {
    int mode = MODE_ORTHO;
    bool axi = true, march = true, flexible_cg = true, plane = false;
    int ncol = 2;
    std::vector<int> probs;
    int Lmax = 0;
    ItemTable gs[kMaxLevels], res[kMaxLevels], xfer[kMaxLevels], fill[kMaxLevels];
    // restriction of the problems that form their residual apart (xfer:
    // every problem's prolongation); rr: the fused red residual and
    // restriction, by ring segments (1, 2)
    ItemTable rst[kMaxLevels], rr[kMaxLevels][2];
    ItemTable tile[kMaxLevels]; // problems whose level takes the tile path: its tiles
    ItemTable pfwd[kMaxLevels][2], ptri[kMaxLevels][2]; // plane half-sweeps by parity
    ItemTable coarse, apply, vred, elem;
    hipGraphExec_t gA = nullptr, gB = nullptr;
    hipGraph_t graphA = nullptr, graphB = nullptr;
};

void build_items(ItemTable& t, const std::vector<std::pair<int, int>>& pg)
{
    std::vector<BItem> v;
    for (auto& q : pg)
        for (int L = 0; L < q.second; ++L) v.push_back(BItem{q.first, (unsigned)L, (unsigned)q.second});
    t.count = (int)v.size();
    t.d.alloc(v.size());
    if (!v.empty()) upload(t.d.p, v.data(), v.size() * sizeof(BItem));
}

} // namespace

struct cps_batch {
    int n = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<cps_handle*> h;
    BatchGroup grp[4]; // point smoother: 7-point, the other stencil class; plane: 7-, 11-point
    std::vector<PDesc<float>> hpd;
    Buf<PDesc<float>> pd;
    Buf<int> active;
    int* hactive = nullptr;
    Buf<double> gath;
    double* hgath = nullptr;
    ItemTable all_vred, all_elem; // every problem, for the set-up and final steps
};

namespace {

template <typename K, typename... A>
void blaunch(cps_batch* B, const ItemTable& t, K kernel, A... args)
{
    if (!t.count) return;
    kernel<<<t.count, kBlock, 0, B->stream>>>(t.d.p, B->active.p, B->pd.p, args...);
    LAUNCH_CHECK();
}

// the same for kernels of other block sizes (tiles, the fused transfer)
template <typename K, typename... A>
void blaunch_n(cps_batch* B, const ItemTable& t, int threads, K kernel, A... args)
{
    if (!t.count) return;
    kernel<<<t.count, threads, 0, B->stream>>>(t.d.p, B->active.p, B->pd.p, args...);
    LAUNCH_CHECK();
}
template <typename K, typename... A>
void blaunch_tile(cps_batch* B, const ItemTable& t, K kernel, A... args)
{
    blaunch_n(B, t, kTileThreads, kernel, args...);
}

void bscalar(cps_batch* B, int op, int dst = 0, int src = 0, double value = 0.0)
{
    kb_scalar<float><<<cdiv(B->n, kBlock), kBlock, 0, B->stream>>>(B->active.p, B->pd.p, B->n, op,
                                                                   dst, src, value);
    LAUNCH_CHECK();
}

void breduce(cps_batch* B, int apply, int slot)
{
    kb_reduce<float><<<B->n, kBlock, 0, B->stream>>>(B->active.p, B->pd.p, apply, slot);
    LAUNCH_CHECK();
}

void bdot(cps_batch* B, const ItemTable& vred, int u, int v, int slot)
{
    blaunch(B, vred, kb_dot<float>, u, v);
    breduce(B, 0, slot);
}

void b_smooth(cps_batch* B, BatchGroup& G, int l, bool reverse, bool from_zero)
{
    if (G.plane) { // as smooth() with the plane smoother: two sweeps of two half-sweeps
        if (from_zero) blaunch(B, G.fill[l], kb_fill_level<float>, l);
        const bool cross = G.mode == MODE_RT;
        for (int s = 0; s < 2; ++s)
            for (int k = 0; k < 2; ++k) {
                const int parity = reverse ? 1 - k : k;
                blaunch(B, G.pfwd[l][parity], cross ? kb_plane_fwd<true> : kb_plane_fwd<false>, l,
                        parity);
                blaunch(B, G.ptri[l][parity], cross ? kb_plane_tri<true> : kb_plane_tri<false>, l,
                        parity);
                blaunch(B, G.pfwd[l][parity], kb_plane_inv, l, parity);
            }
        return;
    }
    const bool skip = from_zero && G.ncol == 2;
    if (from_zero && !skip) blaunch(B, G.fill[l], kb_fill_level<float>, l);
    for (int s = 0; s < 2; ++s)
        for (int k = 0; k < G.ncol; ++k) {
            const int col = reverse ? G.ncol - 1 - k : k;
            const int zero = (skip && s == 0 && k == 0) ? 1 : 0;
            if (G.march) {
                blaunch(B, G.gs[l], kb_gs_march<float>, l, col, zero);
            } else {
                dispatch(G.mode, G.axi, [&](auto M, auto A) {
                    blaunch(B, G.gs[l], kb_gs<float, decltype(M)::value, decltype(A)::value>, l, col,
                            zero);
                });
            }
        }
}

// one V(2,2) cycle from zero for every problem of the group (level-0 b/x
// of the FP32 hierarchy); a problem takes part in level l while l is above
// its own coarsest level
void b_vcycle(cps_batch* B, BatchGroup& G)
{
    for (int l = 0; l + 1 < G.Lmax; ++l) {
        // problems whose level l takes the tile path (as vcycle() does)
        blaunch_tile(B, G.tile[l], kb_vpre_tile<float>, l);
        if (!G.gs[l].count) continue;
        b_smooth(B, G, l, false, true);
        // as vcycle(): after point red-black smoothing, the red residual on
        // row-pair levels (the kernels check the level's shape)
        const int red = !G.plane && G.mode == MODE_ORTHO && G.axi ? 1 : 0;
        dispatch(G.mode, G.axi, [&](auto M, auto A) {
            blaunch(B, G.res[l], kb_residual<float, decltype(M)::value, decltype(A)::value>, l, red);
        });
        blaunch(B, G.rst[l], kb_restrict<float>, l, red);
        // where the shape allows it, the red residual inside the restriction
        blaunch_n(B, G.rr[l][0], 64 * rr_waves(1), kb_resrestrict<float, 1>, l);
        blaunch_n(B, G.rr[l][1], 64 * rr_waves(2), kb_resrestrict<float, 2>, l);
    }
    blaunch(B, G.coarse, kb_coarse<float>);
    for (int l = G.Lmax - 2; l >= 0; --l) {
        blaunch_tile(B, G.tile[l], kb_vpost_tile<float>, l);
        if (!G.gs[l].count) continue;
        // point red-black post-smoothing starts with the black pass: only
        // the red cells need the correction (as vcycle())
        if (!G.plane && G.ncol == 2) blaunch(B, G.xfer[l], kb_prolong<float, 1>, l);
        else blaunch(B, G.xfer[l], kb_prolong<float, 0>, l);
        b_smooth(B, G, l, true, false);
    }
}

void b_precondition(cps_batch* B, BatchGroup& G, int in, int out)
{
    blaunch(B, G.elem, kb_cast_in<float>, in);
    b_vcycle(B, G);
    blaunch(B, G.elem, kb_cast_out<float>, out);
}

void b_apply(cps_batch* B, BatchGroup& G, int in, int out, int dot, int slot)
{
    dispatch(G.mode, G.axi, [&](auto M, auto A) {
        blaunch(B, G.apply, kb_apply64<float, decltype(M)::value, decltype(A)::value>, in, out, dot);
    });
    breduce(B, 1, slot);
}

// iteration bodies (the same steps, in the same order, as solve())
void fcg_part_a(cps_batch* B, BatchGroup& G)
{
    b_apply(B, G, V_P, V_Q, V_P, S_PQ);
    bscalar(B, SOP_CG_ALPHA);
    blaunch(B, G.vred, kb_cg_step<float>);
    breduce(B, 0, S_RR);
}

void fcg_part_b(cps_batch* B, BatchGroup& G)
{
    bscalar(B, SOP_COPY, S_RZ_OLD, S_RZ);
    b_precondition(B, G, V_R, V_Z);
    bdot(B, G.vred, V_R, V_Z, S_RZ);
    bdot(B, G.vred, V_Z, V_Q, S_ZQ);
    bscalar(B, SOP_FCG_BETA);
    blaunch(B, G.elem, kb_elem<float>, (int)EOP_CG_DIR, (int)V_Z, (int)V_P, 0);
}

void bicg_body(cps_batch* B, BatchGroup& G)
{
    bdot(B, G.vred, V_R0, V_R, S_RHO);
    bscalar(B, SOP_BICG_BETA);
    blaunch(B, G.elem, kb_elem<float>, (int)EOP_BICG_DIR, (int)V_R, (int)V_V, (int)V_P);
    b_precondition(B, G, V_P, V_PH);
    b_apply(B, G, V_PH, V_V, V_R0, S_R0V);
    bscalar(B, SOP_BICG_ALPHA);
    blaunch(B, G.elem, kb_elem<float>, (int)EOP_BICG_S, (int)V_R, (int)V_V, (int)V_S);
    b_precondition(B, G, V_S, V_SH);
    b_apply(B, G, V_SH, V_T, V_S, S_TS);
    bdot(B, G.vred, V_T, V_T, S_TT);
    bscalar(B, SOP_BICG_OMEGA);
    blaunch(B, G.vred, kb_bicg_step<float>);
    breduce(B, 0, S_RR);
}

template <typename F>
void capture(cps_batch* B, hipGraph_t& graph, hipGraphExec_t& exec, F&& f)
{
    std::shared_lock<std::shared_mutex> cap(g_capture_mu); // no free or sync meanwhile
    HIPC(hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal));
    try {
        f();
    } catch (...) {
        hipGraph_t g2 = nullptr;
        (void)hipStreamEndCapture(B->stream, &g2);
        if (g2) (void)hipGraphDestroy(g2);
        throw;
    }
    HIPC(hipStreamEndCapture(B->stream, &graph));
    HIPC(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
}

void gather(cps_batch* B, int slot)
{
    kb_gather<float><<<cdiv(B->n, kBlock), kBlock, 0, B->stream>>>(B->pd.p, B->n, slot, B->gath.p);
    LAUNCH_CHECK();
    HIPC(hipMemcpyAsync(B->hgath, B->gath.p, B->n * sizeof(double), hipMemcpyDeviceToHost, B->stream));
    HIPC(hipStreamSynchronize(B->stream));
}

void upload_active(cps_batch* B)
{
    HIPC(hipMemcpyAsync(B->active.p, B->hactive, B->n * sizeof(int), hipMemcpyHostToDevice,
                        B->stream));
}

void upload_desc(cps_batch* B)
{
    HIPC(hipMemcpyAsync(B->pd.p, B->hpd.data(), B->n * sizeof(PDesc<float>), hipMemcpyHostToDevice,
                        B->stream));
}

PDesc<float> make_desc(cps_handle* h)
{
    PDesc<float> d;
    std::memset(&d, 0, sizeof d);
    d.L = h->L;
    d.nc = h->nc;
    d.ncol = h->ncol;
    d.Ainv = h->Ainv.p;
    d.G64 = h->lv[0].G64.p;
    d.gk64 = h->lv[0].gk;
    const Geo& g0 = h->lv[0].geo;
    d.parts_apply = marching(h) ? stencil_shape(g0).grid : grid_of(g0.nr, cdiv(g0.rowlen, kBlock));
    d.parts_vec = vgrid(h->lv[0].n);
    double* v[V_COUNT] = {h->x0.p, h->b0.p, h->r.p, h->z.p, h->pd.p, h->q.p, h->r0.p,
                          h->v.p,  h->s.p,  h->t.p, h->ph.p, h->sh.p, nullptr, nullptr};
    for (int k = 0; k < V_COUNT; ++k) d.vec[k] = v[k];
    d.sc = h->sc.p;
    d.partial = h->partial.p;
    for (int l = 0; l < h->L; ++l) {
        const LevelMem& m = h->lv[l];
        d.lv[l] = LDesc<float>{m.geo, m.G32.p, m.gk, m.x32.p, m.b32.p, m.r32.p, m.gs_ch};
        d.lv[l].tile = m.tile ? 1 : 0;
        d.lv[l].xt = m.xt32.p;
        if (h->opts.smoother == 1 && l + 1 < h->L) {
            d.lv[l].ptw = reinterpret_cast<const Vec2<float>*>(m.tw32.p);
            d.lv[l].ptwN = reinterpret_cast<const Vec2<float>*>(m.twN32.p);
            d.lv[l].plam = m.lam32.p;
            d.lv[l].ppiv = m.pv32.p;
            d.lv[l].pS = reinterpret_cast<Vec2<float>*>(h->ps32.p);
            d.lv[l].prb = m.plane_rb;
        }
    }
    return d;
}

void build_group_tables(cps_batch* B, BatchGroup& G)
{
    using PG = std::vector<std::pair<int, int>>;
    G.Lmax = 0;
    for (int p : G.probs) G.Lmax = std::max(G.Lmax, B->h[p]->L);
    const bool red = !G.plane && G.mode == MODE_ORTHO && G.axi;
    for (int l = 0; l + 1 < G.Lmax; ++l) {
        PG gs, res, xf, fl, tl, rs, rr1, rr2;
        for (int p : G.probs) {
            cps_handle* h = B->h[p];
            if (l + 1 >= h->L) continue;
            const Geo& g = h->lv[l].geo;
            if (h->lv[l].tile) {
                tl.push_back({p, tile_count(g)});
                continue;
            }
            const Geo& c = h->lv[l + 1].geo;
            const int segs = red && G.march ? resrestrict_segs(g, c) : 0;
            if (G.march) gs.push_back({p, gs_shape<float>(g, h->lv[l].gs_ch).grid});
            else gs.push_back({p, (int)grid_of(g.nr, gs_bpa(g, h->ncol))});
            if (segs) {
                (segs == 1 ? rr1 : rr2).push_back({p, resrestrict_shape<float>(c, segs).grid});
            } else {
                if (G.march) res.push_back({p, stencil_shape(g).grid});
                else res.push_back({p, (int)grid_of(g.nr, cdiv(g.rowlen, kBlock))});
                rs.push_back({p, march_shape(c).grid});
            }
            xf.push_back({p, march_shape(c).grid});
            fl.push_back({p, (int)nblk(h->lv[l].n)});
        }
        build_items(G.gs[l], gs);
        build_items(G.res[l], res);
        build_items(G.rst[l], rs);
        build_items(G.rr[l][0], rr1);
        build_items(G.rr[l][1], rr2);
        build_items(G.xfer[l], xf);
        build_items(G.fill[l], fl);
        build_items(G.tile[l], tl);
        if (G.plane)
            for (int k = 0; k < 2; ++k) {
                PG pf, pt;
                for (int p : G.probs) {
                    cps_handle* h = B->h[p];
                    if (l + 1 >= h->L) continue;
                    const Geo& g = h->lv[l].geo;
                    const PlaneLaunch pl = plane_launch(g, k, h->lv[l].plane_rb);
                    pf.push_back({p, pl.blocks});
                    pt.push_back({p, cdiv(2LL * pl.rows * (g.nh + 1), kBlock)});
                }
                build_items(G.pfwd[l][k], pf);
                build_items(G.ptri[l][k], pt);
            }
    }
    PG co, ap, vr, el;
    for (int p : G.probs) {
        cps_handle* h = B->h[p];
        co.push_back({p, (h->nc + 3) / 4});
        ap.push_back({p, (int)B->hpd[p].parts_apply});
        vr.push_back({p, (int)vgrid(h->lv[0].n)});
        el.push_back({p, (int)nblk(h->lv[0].n)});
    }
    build_items(G.coarse, co);
    build_items(G.apply, ap);
    build_items(G.vred, vr);
    build_items(G.elem, el);
}

void batch_destroy(cps_batch* B)
{
    if (!B) return;
    if (B->stream) (void)hipStreamSynchronize(B->stream);
    for (auto& G : B->grp) {
        MemLock lk(g_capture_mu); // graph teardown
        if (G.gA) (void)hipGraphExecDestroy(G.gA);
        if (G.gB) (void)hipGraphExecDestroy(G.gB);
        if (G.graphA) (void)hipGraphDestroy(G.graphA);
        if (G.graphB) (void)hipGraphDestroy(G.graphB);
    }
    for (cps_handle* h : B->h) destroy(h);
    {
        MemLock lk(g_capture_mu);
        if (B->hactive) (void)hipHostFree(B->hactive);
        if (B->hgath) (void)hipHostFree(B->hgath);
    }
    hipStream_t s = B->own_stream ? B->stream : nullptr;
    delete B;
    if (s) (void)hipStreamDestroy(s);
}

void batch_build(cps_batch* B, int n, const cps_grid* grids, const cps_metrics* metrics,
                 const cps_opts* opts)
{
    B->n = n;
    if (opts && opts->stream) {
        B->stream = (hipStream_t)opts->stream;
    } else {
        // default priority; non-blocking (see the service workers' streams)
        HIPC(hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking));
        B->own_stream = true;
    }
    cps_opts o = opts ? *opts : cps_opts{};
    o.precision = 1;
    o.accel = 1;
    o.stream = B->stream;
    B->h.assign(n, nullptr);
    for (int p = 0; p < n; ++p) {
        validate(&grids[p], metrics, &o);
        cps_handle* h = new cps_handle();
        B->h[p] = h;
        h->grid = grids[p];
        if (metrics) h->met = *metrics;
        h->opts = o;
        h->stream = B->stream;
        build(h);
    }
    B->hpd.resize(n);
    for (int p = 0; p < n; ++p) B->hpd[p] = make_desc(B->h[p]);
    B->pd.alloc(n);
    B->active.alloc(n);
    B->gath.alloc(n);
    {
        MemLock lk(g_capture_mu);
        HIPC(hipHostMalloc(&B->hactive, n * sizeof(int), hipHostMallocDefault));
        HIPC(hipHostMalloc(&B->hgath, n * sizeof(double), hipHostMallocDefault));
    }
    // groups
    BatchGroup& g0 = B->grp[0];
    BatchGroup& g1 = B->grp[1];
    BatchGroup& g2 = B->grp[2];
    BatchGroup& g3 = B->grp[3];
    g0.mode = MODE_ORTHO; g0.axi = true; g0.march = true; g0.ncol = 2; g0.flexible_cg = true;
    g2.mode = MODE_ORTHO; g2.axi = true; g2.march = true; g2.ncol = 2; g2.flexible_cg = true;
    g2.plane = true;
    // r-theta cross terms with the plane smoother: generic residual and
    // transfer kernels of that class
    g3.mode = MODE_RT; g3.axi = true; g3.march = false; g3.ncol = 4; g3.flexible_cg = true;
    g3.plane = true;
    int mode1 = -1;
    bool axi1 = true;
    for (int p = 0; p < n; ++p) {
        cps_handle* h = B->h[p];
        if (h->opts.smoother == 1) {
            for (int l = 0; l + 1 < h->L; ++l)
                if (h->lv[l].np / 2 > kSmallRing)
                    fail(CPS_E_INVALID, "the batched plane smoother takes n_phi <= %d "
                         "(problem %d)", 2 * kSmallRing, p);
            (h->mode == MODE_RT ? g3 : g2).probs.push_back(p);
        } else if (marching(h)) {
            g0.probs.push_back(p);
        } else {
            if (mode1 >= 0 && (h->mode != mode1 || h->axi != axi1))
                fail(CPS_E_INVALID, "a batch may hold one stencil class besides the 7-point one");
            mode1 = h->mode;
            axi1 = h->axi;
            g1.probs.push_back(p);
        }
    }
    g1.mode = mode1 < 0 ? MODE_RT : mode1;
    g1.axi = axi1;
    g1.march = false;
    g1.ncol = mode1 == MODE_ORTHO ? 2 : 4;
    g1.flexible_cg = true; // as cps_solve with accel = 1 for every stencil class
    for (auto& G : B->grp)
        if (!G.probs.empty()) build_group_tables(B, G);
    std::vector<std::pair<int, int>> vr, el;
    for (int p = 0; p < n; ++p) {
        vr.push_back({p, (int)vgrid(B->h[p]->lv[0].n)});
        el.push_back({p, (int)nblk(B->h[p]->lv[0].n)});
    }
    build_items(B->all_vred, vr);
    build_items(B->all_elem, el);
    upload_desc(B);
    // capture the iteration bodies
    for (auto& G : B->grp) {
        if (G.probs.empty()) continue;
        if (G.flexible_cg) {
            capture(B, G.graphA, G.gA, [&] { fcg_part_a(B, G); });
            capture(B, G.graphB, G.gB, [&] { fcg_part_b(B, G); });
        } else {
            capture(B, G.graphA, G.gA, [&] { bicg_body(B, G); });
        }
    }
    HIPC(hipStreamSynchronize(B->stream));
}

void set_active(cps_batch* B, const std::vector<int>& on)
{
    for (int p = 0; p < B->n; ++p) B->hactive[p] = on[p];
    upload_active(B);
}

// The problems marked in `check` met the tolerance by the conjugate-gradient
// recurrence: as solve() does, form r = b0 - A x (y = A x into q) and decide
// on its norm.  A problem that misses the tolerance restarts from that
// residual: its direction is zeroed, so the next part B takes p = z.  Leaves
// the active flags at `check` (the caller sets its own next).
void true_residuals(cps_batch* B, BatchGroup& G, const std::vector<int>& check,
                    const std::vector<double>& bb, double tol, std::vector<double>& rel,
                    std::vector<cps_status>& st)
{
    set_active(B, check);
    dispatch(G.mode, G.axi, [&](auto M, auto A) {
        blaunch(B, G.apply, kb_apply64<float, decltype(M)::value, decltype(A)::value>, (int)V_X,
                (int)V_Q, -1);
    });
    blaunch(B, G.elem, kb_elem<float>, (int)EOP_SUB, (int)V_B0, (int)V_Q, (int)V_R);
    bdot(B, G.vred, V_R, V_R, S_RR);
    gather(B, S_RR); // synchronises: the flags below may be rewritten
    std::vector<int> again(B->n, 0);
    bool any = false;
    for (int p = 0; p < B->n; ++p) {
        if (!check[p]) continue;
        st[p] = check_norm(B->hgath[p], bb[p], tol, &rel[p]);
        if (st[p] == CPS_E_NOT_CONVERGED) again[p] = 1, any = true;
    }
    if (!any) return;
    set_active(B, again);
    blaunch(B, G.elem, kb_elem<float>, (int)EOP_FILL, (int)V_P, 0, 0);
    HIPC(hipStreamSynchronize(B->stream)); // before the flags are rewritten
}

cps_status batch_solve(cps_batch* B, const double* const* rhs, double* const* out, double tol,
                       cps_info* infos)
{
    const auto t0 = std::chrono::steady_clock::now();
    const int n = B->n;
    for (int p = 0; p < n; ++p) {
        if (!rhs[p] || !out[p]) fail(CPS_E_INVALID, "NULL rhs or p for problem %d", p);
        B->hpd[p].vec[V_RHS] = const_cast<double*>(rhs[p]);
        B->hpd[p].vec[V_OUT] = out[p];
    }
    upload_desc(B);
    std::vector<int> on(n, 1), iters(n, 0);
    std::vector<double> bb(n), mean(n), rel(n, 0.0);
    std::vector<cps_status> st(n, CPS_OK);
    set_active(B, on);
    // b0 = rhs - mean, ||b0||^2, scale, x = 0, p = 0   (as in solve())
    blaunch(B, B->all_vred, kb_dot<float>, (int)V_RHS, -1);
    breduce(B, 0, S_SUM);
    blaunch(B, B->all_elem, kb_elem<float>, (int)EOP_TO_SPLIT, (int)V_RHS, (int)V_B0, (int)S_SUM);
    bdot(B, B->all_vred, V_B0, V_B0, S_BB);
    bscalar(B, SOP_SQRT, S_SCALE, S_BB);
    blaunch(B, B->all_elem, kb_elem<float>, (int)EOP_FILL, (int)V_X, 0, 0);
    blaunch(B, B->all_elem, kb_elem<float>, (int)EOP_FILL, (int)V_OUT, 0, 0);
    gather(B, S_SUM);
    for (int p = 0; p < n; ++p) mean[p] = B->hgath[p] / (double)B->h[p]->lv[0].n;
    gather(B, S_BB);
    std::vector<int> live(n, 0); // problems that iterate
    for (int p = 0; p < n; ++p) {
        bb[p] = B->hgath[p];
        if (!std::isfinite(bb[p])) {
            st[p] = CPS_E_DIVERGED;
            rel[p] = NAN;
        } else if (bb[p] > 0.0) {
            live[p] = 1;
            st[p] = CPS_E_NOT_CONVERGED;
        }
    }
    for (int gi = 0; gi < 4; ++gi) {
        BatchGroup& G = B->grp[gi];
        if (G.probs.empty()) continue;
        std::vector<int> act(n, 0);
        bool any = false;
        for (int p : G.probs) {
            act[p] = live[p];
            any = any || live[p];
        }
        if (!any) continue;
        set_active(B, act);
        int maxit = 0;
        for (int p : G.probs) {
            const int m = B->h[p]->opts.max_iters > 0 ? B->h[p]->opts.max_iters : 200;
            maxit = std::max(maxit, m);
        }
        if (G.flexible_cg) {
            blaunch(B, G.elem, kb_elem<float>, (int)EOP_COPY, (int)V_B0, (int)V_R, 0);
            b_precondition(B, G, V_R, V_Z);
            bdot(B, G.vred, V_R, V_Z, S_RZ);
            blaunch(B, G.elem, kb_elem<float>, (int)EOP_COPY, (int)V_Z, (int)V_P, 0);
        } else {
            blaunch(B, G.elem, kb_elem<float>, (int)EOP_COPY, (int)V_B0, (int)V_R, 0);
            blaunch(B, G.elem, kb_elem<float>, (int)EOP_COPY, (int)V_B0, (int)V_R0, 0);
            blaunch(B, G.elem, kb_elem<float>, (int)EOP_FILL, (int)V_P, 0, 0);
            blaunch(B, G.elem, kb_elem<float>, (int)EOP_FILL, (int)V_V, 0, 0);
            bscalar(B, SOP_SET, S_RHO_OLD, 0, 1.0);
            bscalar(B, SOP_SET, S_ALPHA, 0, 1.0);
            bscalar(B, SOP_SET, S_OMEGA, 0, 1.0);
        }
        for (int it = 1; it <= maxit; ++it) {
            HIPC(hipGraphLaunch(G.gA, B->stream));
            gather(B, S_RR);
            bool left = false;
            std::vector<int> check(n, 0); // the recurrence met the tolerance
            bool any_check = false;
            for (int p : G.probs) {
                if (!act[p]) continue;
                iters[p] = it;
                const cps_status s = check_norm(B->hgath[p], bb[p], tol, &rel[p]);
                st[p] = s;
                if (s == CPS_OK) check[p] = 1, any_check = true;
            }
            if (any_check) // as solve(): the residual of the iterate decides
                true_residuals(B, G, check, bb, tol, rel, st);
            for (int p : G.probs) {
                if (!act[p]) continue;
                const int m = B->h[p]->opts.max_iters > 0 ? B->h[p]->opts.max_iters : 200;
                if (st[p] != CPS_E_NOT_CONVERGED || it >= m) act[p] = 0;
                left = left || act[p];
            }
            if (!left) break;
            set_active(B, act);
            if (G.flexible_cg) {
                HIPC(hipGraphLaunch(G.gB, B->stream));
            } else {
                bscalar(B, SOP_COPY, S_RHO_OLD, S_RHO);
            }
        }
    }
    // zero-mean results in natural order for every problem that iterated
    set_active(B, live);
    bdot(B, B->all_vred, V_X, -1, S_SUM);
    blaunch(B, B->all_elem, kb_elem<float>, (int)EOP_FROM_SPLIT, (int)V_X, (int)V_OUT, (int)S_SUM);
    HIPC(hipStreamSynchronize(B->stream));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    cps_status worst = CPS_OK;
    for (int p = 0; p < n; ++p) {
        if (infos) {
            infos[p].iterations = iters[p];
            infos[p].rel_residual = rel[p];
            infos[p].rhs_mean_removed = mean[p];
            infos[p].seconds = secs;
        }
        if (st[p] == CPS_E_DIVERGED) worst = CPS_E_DIVERGED;
        else if (st[p] == CPS_E_NOT_CONVERGED && worst == CPS_OK) worst = CPS_E_NOT_CONVERGED;
    }
    if (worst != CPS_OK) g_err = "some problems of the batch did not converge (see infos)";
    return worst;
}

} // namespace

extern "C" {

cps_status cps_batch_setup(int32_t n, const cps_grid* grids, const cps_metrics* metrics,
                           const cps_opts* opts, cps_batch** out)
{
    if (!out) {
        g_err = "out is NULL";
        return CPS_E_INVALID;
    }
    *out = nullptr;
    cps_batch* B = nullptr;
    cps_status st = guarded([&] {
        if (n < 1 || !grids) fail(CPS_E_INVALID, "need n >= 1 grids");
        if (opts && opts->precision != 1)
            fail(CPS_E_INVALID, "the batched form runs FP32 V-cycles inside FP64 refinement "
                                "(precision = 1)");
        if (opts && (opts->smoother < 0 || opts->smoother > 2))
            fail(CPS_E_INVALID, "bad smoother");
        if (metrics && metrics->method == CPS_METRICS_USER_FACE)
            fail(CPS_E_INVALID, "the batched form forms its metrics from each problem's map");
        B = new cps_batch();
        batch_build(B, n, grids, metrics, opts);
    });
    if (st != CPS_OK) {
        batch_destroy(B);
        return st;
    }
    *out = B;
    return CPS_OK;
}

cps_status cps_batch_solve(cps_batch* b, const double* const* rhs, double* const* p, double tol,
                           cps_info* infos)
{
    cps_status st = CPS_OK;
    cps_status g = guarded([&] {
        if (!b || !rhs || !p) fail(CPS_E_INVALID, "NULL argument");
        if (!(tol > 0)) fail(CPS_E_INVALID, "tol must be positive");
        st = batch_solve(b, rhs, p, tol, infos);
    });
    return g != CPS_OK ? g : st;
}

void cps_batch_destroy(cps_batch* b) { batch_destroy(b); }

} // extern "C"
