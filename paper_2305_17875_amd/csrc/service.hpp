// service.hpp -- solve service: requests of different grid sizes and maps
// are admitted by HBM budget and free slots, their hierarchies stay
// resident for reuse, and admitted requests run concurrently on their
// slots' streams, so their work overlaps on the device.
// Included by cps.hip (one translation unit).
//
// Admission is first-come first-served.  A request takes an idle resident
// hierarchy of the same dims and stencil class if one exists (recomputing
// the metrics and coarse inverse in place when the map differs); otherwise
// a new hierarchy is built if the budget allows, after evicting idle
// hierarchies of other shapes (least recently used first).  A request that
// does not fit waits until running requests finish.  Every request is
// solved by the same code as cps_solve, so its result equals the result of
// the same problem solved alone.

namespace {

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct SvcReq {
    uint64_t id = 0;
    cps_grid grid{};
    cps_metrics met{};
    double tol = 1e-10;
    long long n = 0;
    const double* rhs = nullptr; // the caller's host arrays, held until the wait
    double* p = nullptr;
    cps_info info{};
    cps_status st = CPS_OK;
    bool done = false;
    std::string err;
    double t_submit = 0, t_start = 0, t_done = 0;
};

struct PoolEnt {
    cps_handle* h = nullptr;
    Buf<double> rhs, p; // device staging of one request of this shape
    size_t bytes = 0;
    bool busy = false;
    double last = 0;
};

int stencil_class(const cps_grid& g)
{
    return g.map == CPS_MAP_TRIAXIAL ? 2 : (g.map == CPS_MAP_OBLATE ? 1 : 0);
}

bool same_dims(const cps_grid& a, const cps_grid& b)
{
    return a.n_r == b.n_r && a.n_theta == b.n_theta && a.n_phi == b.n_phi &&
           a.n_levels == b.n_levels && stencil_class(a) == stencil_class(b);
}

bool same_map(const cps_grid& a, const cps_grid& b)
{
    return same_dims(a, b) && a.map == b.map && a.r_inner == b.r_inner && a.r_outer == b.r_outer &&
           a.theta0 == b.theta0 && a.theta1 == b.theta1 && a.radial_stretch == b.radial_stretch &&
           a.flattening == b.flattening && a.skew == b.skew;
}

size_t handle_bytes(const cps_handle* h)
{
    size_t s = 0;
    auto add = [&](const auto& b) { s += b.n * sizeof(*b.p); };
    for (int l = 0; l < h->L; ++l) {
        const LevelMem& m = h->lv[l];
        add(m.G64); add(m.G32); add(m.x64); add(m.b64); add(m.r64);
        add(m.x32); add(m.b32); add(m.r32); add(m.xt64); add(m.xt32);
    }
    add(h->Ainv); add(h->partial); add(h->sc);
    add(h->x0); add(h->b0); add(h->r); add(h->z); add(h->pd); add(h->q);
    add(h->r0); add(h->v); add(h->s); add(h->t); add(h->ph); add(h->sh);
    add(h->ps64); add(h->ps32);
    add(h->gjA); add(h->gjM); add(h->gjE); add(h->gjXp);
    add(h->gjUsed); add(h->gjPiv); add(h->gjBad);
    for (int l = 0; l < h->L; ++l) {
        const LevelMem& m = h->lv[l];
        add(m.tw64); add(m.twN64); add(m.lam64); add(m.tw32); add(m.twN32); add(m.lam32);
        add(m.pv64); add(m.pv32);
    }
    return s;
}

// device bytes a hierarchy of this grid will take, including the
// Gauss-Jordan buffers of the coarsest inverse (which a service hierarchy
// keeps for its remaps)
size_t estimate_bytes(const cps_grid& g, const cps_opts& o)
{
    int dims[kMaxLevels][3];
    const int L = checked_plan(g, dims); // validated at submission
    const bool axi = g.map != CPS_MAP_TRIAXIAL, mixed = o.precision == 1;
    size_t s = 0;
    for (int l = 0; l < L; ++l) {
        const size_t n = (size_t)dims[l][0] * dims[l][1] * dims[l][2];
        const size_t gk = (size_t)dims[l][0] * dims[l][1] * (axi ? 1 : dims[l][2]);
        s += 9 * gk * 8;
        if (mixed) s += 9 * gk * 4 + n * 4 * (l + 1 < L ? 3 : 2);
        else s += n * 8 * ((l > 0 ? 2 : 0) + (l + 1 < L ? 1 : 0));
        // the tile path's second iterate (small levels, point smoother)
        if (l + 1 < L && n <= (size_t)tile_max_cells(mixed)) s += n * (mixed ? 4 : 8);
    }
    const size_t n0 = (size_t)g.n_r * g.n_theta * g.n_phi;
    const size_t nc = (size_t)dims[L - 1][0] * dims[L - 1][1] * dims[L - 1][2];
    s += n0 * 8 * (3 + 2 + (o.accel >= 1 ? 4 : 0) + (o.accel == 2 ? 5 : 0));
    bool plane_dims = L > 1;
    for (int l = 0; l + 1 < L; ++l) {
        const int nh = dims[l][2] / 2;
        plane_dims = plane_dims && nh >= 2 && nh <= kPlaneLds && (nh & (nh - 1)) == 0;
    }
    if (o.smoother == 1 || (o.smoother == 2 && plane_dims)) {
        // spectra of one parity, pivots of every smoothed level, tables
        const size_t w = mixed ? 4 : 8;
        s += (size_t)dims[0][0] * ((dims[0][1] + 1) / 2) * (dims[0][2] / 2 + 1) * 2 * w +
             (size_t)L * (2 * dims[0][2] + 8) * 8 * 2;
        for (int l = 0; l + 1 < L; ++l)
            s += (size_t)dims[l][0] * dims[l][1] * (dims[l][2] / 2 + 1) * w;
    }
    s += (2 * std::max<size_t>(n0 / kBlock + 1, kMaxGrid) + 64 + S_COUNT) * 8 +
         nc * nc * 8 * 4 + nc * kGJ * 8 * 3 + (2 * nc + 1) * 4;
    return s;
}

} // namespace

struct cps_service {
    size_t budget = 0;
    int slots = 1;
    cps_opts opts{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<SvcReq*> queue;
    std::map<uint64_t, SvcReq*> reqs;
    std::vector<std::unique_ptr<PoolEnt>> pool;
    size_t pool_bytes = 0, reserved = 0;
    std::vector<std::thread> workers;
    bool stop = false;
    uint64_t next_id = 1;
    // statistics
    std::vector<double> lat_ms;
    double unknowns = 0, t_first = -1, t_last = 0;
    uint64_t submitted = 0, completed = 0, failed = 0, built = 0, reused = 0, remapped = 0,
             evicted = 0;
    int active = 0, peak_active = 0;
};

namespace {

void svc_finish(cps_service* S, SvcReq* R)
{
    R->t_done = now_s();
    R->done = true;
    const double ms = (R->t_done - R->t_submit) * 1e3;
    if (R->st == CPS_OK) {
        S->completed++;
        S->lat_ms.push_back(ms);
        S->unknowns += (double)R->n;
        S->t_last = std::max(S->t_last, R->t_done);
    } else {
        S->failed++;
    }
    S->cv.notify_all();
}

// A new hierarchy for the request on `stream` (destroyed again on failure).
cps_handle* new_hierarchy(const cps_service* S, const SvcReq* R, hipStream_t stream)
{
    cps_handle* h = new cps_handle();
    h->grid = R->grid;
    h->met = R->met;
    h->opts = S->opts;
    h->stream = stream;
    h->keep_gj = true; // remaps recompute the coarsest inverse in place
    try {
        build(h);
    } catch (...) {
        destroy(h);
        throw;
    }
    return h;
}

// Take the next request the budget admits (FIFO).  Returns false when the
// service stops.  On return, *pe is the reused pool entry or null (then
// *est bytes were reserved for a new one); `dead` holds evicted hierarchies
// the caller frees outside the lock.
bool svc_admit(cps_service* S, std::unique_lock<std::mutex>& lk, SvcReq** out, PoolEnt** pe,
               size_t* est, std::vector<std::unique_ptr<PoolEnt>>& dead)
{
    for (;;) {
        if (S->stop) return false;
        if (!S->queue.empty()) {
            SvcReq* head = S->queue.front();
            PoolEnt* best = nullptr;
            for (auto& e : S->pool) {
                if (e->busy || !same_dims(e->h->grid, head->grid)) continue;
                if (same_map(e->h->grid, head->grid) && e->h->met.method == head->met.method) {
                    best = e.get();
                    break;
                }
                if (!best) best = e.get();
            }
            if (best) {
                best->busy = true;
                *pe = best;
                *out = head;
                S->queue.pop_front();
                S->reused++;
                return true;
            }
            const size_t need = estimate_bytes(head->grid, S->opts);
            while (S->pool_bytes + S->reserved + need > S->budget) {
                size_t idx = S->pool.size();
                for (size_t i = 0; i < S->pool.size(); ++i)
                    if (!S->pool[i]->busy &&
                        (idx == S->pool.size() || S->pool[i]->last < S->pool[idx]->last))
                        idx = i;
                if (idx == S->pool.size()) break; // every resident hierarchy is busy
                S->pool_bytes -= S->pool[idx]->bytes;
                dead.push_back(std::move(S->pool[idx]));
                S->pool.erase(S->pool.begin() + idx);
                S->evicted++;
            }
            if (S->pool_bytes + S->reserved + need <= S->budget) {
                *pe = nullptr;
                *est = need;
                *out = head;
                S->queue.pop_front();
                S->reserved += need;
                return true;
            }
            if (S->pool.empty() && S->reserved == 0) { // can never fit
                S->queue.pop_front();
                head->st = CPS_E_OOM;
                head->err = "request needs about " + std::to_string(need) +
                            " bytes of device memory, above the service's budget";
                svc_finish(S, head);
                continue;
            }
        }
        if (!dead.empty()) return true; // free them first, then look again
        S->cv.wait(lk);
    }
}

void svc_worker(cps_service* S)
{
    (void)hipSetDevice(S->device);
    hipStream_t stream = nullptr;
    // default priority; non-blocking: null-stream work elsewhere in the
    // process must not synchronise with (and so invalidate) this stream's
    // graph captures
    if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) return;
    for (;;) {
        SvcReq* R = nullptr;
        PoolEnt* pe = nullptr;
        size_t est = 0;
        std::vector<std::unique_ptr<PoolEnt>> dead;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            const bool go = svc_admit(S, lk, &R, &pe, &est, dead);
            if (go && R) {
                S->active++;
                S->peak_active = std::max(S->peak_active, S->active);
            }
            if (!go) {
                lk.unlock();
                for (auto& d : dead) destroy(d->h);
                break;
            }
        }
        for (auto& d : dead) destroy(d->h);
        dead.clear(); // frees the staging buffers, outside the lock
        if (!R) continue;
        R->t_start = now_s();
        cps_handle* h = pe ? pe->h : nullptr;
        std::unique_ptr<PoolEnt> fresh;
        bool remapped = false;
        try {
            if (h) {
                h->stream = stream;
                if (!same_map(h->grid, R->grid) || h->met.method != R->met.method) {
                    h->grid = R->grid;
                    h->met = R->met;
                    bool ok = true;
                    try {
                        compute_operator(h);
                    } catch (const Fail&) {
                        ok = false;
                    }
                    if (ok) {
                        remapped = true;
                    } else {
                        // the map is of another stencil class (a shape parameter
                        // of 0, say) or invalid: rebuild the entry from scratch
                        destroy(h);
                        h = pe->h = nullptr;
                        h = pe->h = new_hierarchy(S, R, stream);
                    }
                }
            } else {
                fresh = std::make_unique<PoolEnt>();
                h = fresh->h = new_hierarchy(S, R, stream);
                fresh->rhs.alloc(R->n);
                fresh->p.alloc(R->n);
            }
            PoolEnt* e = pe ? pe : fresh.get();
            if ((long long)e->rhs.n < R->n) { // an entry rebuilt in place keeps its dims
                e->rhs.alloc(R->n);
                e->p.alloc(R->n);
            }
            HIPC(hipMemcpyAsync(e->rhs.p, R->rhs, R->n * sizeof(double), hipMemcpyHostToDevice,
                                stream));
            R->st = solve(h, e->rhs.p, e->p.p, R->tol, &R->info);
            HIPC(hipMemcpyAsync(R->p, e->p.p, R->n * sizeof(double), hipMemcpyDeviceToHost,
                                stream));
            HIPC(hipStreamSynchronize(stream));
            if (R->st != CPS_OK) R->err = g_err;
        } catch (const Fail& f) {
            R->st = f.st;
            R->err = g_err;
        } catch (const std::bad_alloc&) {
            R->st = CPS_E_OOM;
            R->err = "host allocation failed";
        }
        if (h) h->stream = nullptr; // another worker may take the entry next
        std::lock_guard<std::mutex> lk(S->mu);
        if (remapped) S->remapped++;
        if (pe) {
            if (!pe->h) { // rebuild failed: drop the entry
                for (size_t i = 0; i < S->pool.size(); ++i)
                    if (S->pool[i].get() == pe) {
                        S->pool_bytes -= pe->bytes;
                        S->pool.erase(S->pool.begin() + i);
                        break;
                    }
            } else {
                const size_t b = handle_bytes(pe->h) + 2 * pe->rhs.n * sizeof(double);
                S->pool_bytes = S->pool_bytes - pe->bytes + b;
                pe->bytes = b;
                pe->busy = false;
                pe->last = now_s();
            }
        } else {
            S->reserved -= est;
            if (fresh && fresh->h) {
                fresh->bytes = handle_bytes(fresh->h) + 2 * fresh->rhs.n * sizeof(double);
                fresh->last = now_s();
                S->pool_bytes += fresh->bytes;
                S->pool.push_back(std::move(fresh));
                S->built++;
            }
        }
        S->active--;
        svc_finish(S, R);
    }
    (void)hipStreamDestroy(stream);
}

void service_destroy(cps_service* S)
{
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv.notify_all();
    }
    for (auto& t : S->workers)
        if (t.joinable()) t.join();
    for (auto& e : S->pool) destroy(e->h);
    for (auto& kv : S->reqs) delete kv.second;
    delete S;
}

double percentile(std::vector<double> v, double q)
{
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (v.size() - 1);
    const size_t i = (size_t)pos;
    const double f = pos - i;
    return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

} // namespace

extern "C" {

cps_status cps_service_create(size_t hbm_budget_bytes, int32_t max_slots, const cps_opts* opts,
                              cps_service** out)
{
    if (!out) {
        g_err = "out is NULL";
        return CPS_E_INVALID;
    }
    *out = nullptr;
    cps_service* S = nullptr;
    cps_status st = guarded([&] {
        if (max_slots < 1 || max_slots > 64) fail(CPS_E_INVALID, "max_slots must be 1..64");
        if (hbm_budget_bytes == 0) fail(CPS_E_INVALID, "HBM budget must be positive");
        if (opts && opts->stream) fail(CPS_E_INVALID, "the service uses its own streams");
        S = new cps_service();
        S->budget = hbm_budget_bytes;
        S->slots = max_slots;
        if (opts) S->opts = *opts;
        validate_opts(&S->opts);
        HIPC(hipGetDevice(&S->device));
        for (int i = 0; i < max_slots; ++i) S->workers.emplace_back(svc_worker, S);
    });
    if (st != CPS_OK) {
        service_destroy(S);
        return st;
    }
    *out = S;
    return CPS_OK;
}

cps_status cps_service_submit(cps_service* S, const cps_grid* grid, const cps_metrics* metrics,
                              const double* rhs_host, double* p_host, double tol,
                              uint64_t* ticket)
{
    return guarded([&] {
        if (!S || !grid || !rhs_host || !p_host || !ticket) fail(CPS_E_INVALID, "NULL argument");
        if (!(tol > 0)) fail(CPS_E_INVALID, "tol must be positive");
        validate(grid, metrics, &S->opts);
        if (metrics && metrics->method == CPS_METRICS_USER_FACE)
            fail(CPS_E_INVALID, "the service forms each request's metrics from its map (pooled "
                                "hierarchies are matched by the map)");
        int dims[kMaxLevels][3];
        (void)checked_plan(*grid, dims);
        auto R = std::make_unique<SvcReq>();
        R->grid = *grid;
        if (metrics) R->met = *metrics;
        R->tol = tol;
        R->n = (long long)grid->n_r * grid->n_theta * grid->n_phi;
        R->rhs = rhs_host;
        R->p = p_host;
        R->t_submit = now_s();
        std::lock_guard<std::mutex> lk(S->mu);
        R->id = S->next_id++;
        *ticket = R->id;
        S->submitted++;
        if (S->t_first < 0) S->t_first = R->t_submit;
        S->queue.push_back(R.get());
        S->reqs[R->id] = R.get();
        R.release();
        S->cv.notify_all();
    });
}

cps_status cps_service_wait(cps_service* S, uint64_t ticket, cps_info* info)
{
    SvcReq* R = nullptr;
    cps_status g = guarded([&] {
        if (!S) fail(CPS_E_INVALID, "NULL service");
        std::unique_lock<std::mutex> lk(S->mu);
        auto it = S->reqs.find(ticket);
        if (it == S->reqs.end()) fail(CPS_E_INVALID, "unknown ticket");
        R = it->second;
        S->cv.wait(lk, [&] { return R->done; });
        S->reqs.erase(it);
    });
    if (g != CPS_OK) return g;
    if (info) *info = R->info;
    const cps_status st = R->st;
    if (st != CPS_OK) g_err = R->err;
    delete R;
    return st;
}

cps_status cps_service_footprint(const cps_grid* grid, const cps_opts* opts, uint64_t* bytes)
{
    return guarded([&] {
        if (!bytes) fail(CPS_E_INVALID, "bytes is NULL");
        validate(grid, nullptr, opts);
        int dims[kMaxLevels][3];
        (void)checked_plan(*grid, dims);
        cps_opts o{};
        if (opts) o = *opts;
        *bytes = estimate_bytes(*grid, o);
    });
}

cps_status cps_service_stats(cps_service* S, cps_service_report* out)
{
    return guarded([&] {
        if (!S || !out) fail(CPS_E_INVALID, "NULL argument");
        std::lock_guard<std::mutex> lk(S->mu);
        std::memset(out, 0, sizeof *out);
        out->submitted = S->submitted;
        out->completed = S->completed;
        out->failed = S->failed;
        out->queued = S->queue.size();
        out->active = S->active;
        out->peak_active = S->peak_active;
        out->p50_ms = percentile(S->lat_ms, 0.50);
        out->p99_ms = percentile(S->lat_ms, 0.99);
        out->max_ms = S->lat_ms.empty() ? 0.0 : *std::max_element(S->lat_ms.begin(), S->lat_ms.end());
        double sum = 0;
        for (double v : S->lat_ms) sum += v;
        out->mean_ms = S->lat_ms.empty() ? 0.0 : sum / S->lat_ms.size();
        const double span = S->t_last - S->t_first;
        out->unknowns_per_s = span > 0 ? S->unknowns / span : 0.0;
        out->hbm_in_use = S->pool_bytes + S->reserved;
        out->hbm_budget = S->budget;
        out->hierarchies_built = S->built;
        out->hierarchies_reused = S->reused;
        out->map_rebuilds = S->remapped;
        out->evictions = S->evicted;
    });
}

void cps_service_destroy(cps_service* S) { service_destroy(S); }

} // extern "C"
