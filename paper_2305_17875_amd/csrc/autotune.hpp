// autotune.hpp -- chooses the marching chunk (planes per block) of the
// Gauss-Seidel colour pass, and the plane smoother's launch shapes (rings per
// block, r-steps in flight), for every level shape and precision by timing
// the candidates on the device, and keeps the choices in a JSON cache.
// Included by cps.hip (one translation unit).
//
// The chunk only changes how blocks walk the planes: every cell's update is
// the same arithmetic, and the colour pass has no reduction, so a tuned
// solve gives the same bits as an untuned one.
//
// Cache: the file named by the environment variable CPS_TUNE_CACHE (none =
// in-process only), a flat JSON object {"gs_march/f64/192x256x512": 24, ...}.

namespace {

std::mutex g_tune_mu;
std::map<std::string, int> g_tune;
bool g_tune_loaded = false;

std::string tune_key(const char* prec, const Geo& g)
{
    char buf[96];
    snprintf(buf, sizeof buf, "gs_march/%s/%dx%dx%d", prec, g.nr, g.nt, g.np);
    return buf;
}

void tune_load_locked()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = getenv("CPS_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    std::string s;
    char buf[4096];
    size_t k;
    while ((k = fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, k);
    fclose(f);
    // "key": integer pairs
    size_t i = 0;
    while ((i = s.find('"', i)) != std::string::npos) {
        const size_t j = s.find('"', i + 1);
        if (j == std::string::npos) break;
        const std::string key = s.substr(i + 1, j - i - 1);
        size_t c = s.find(':', j);
        if (c == std::string::npos) break;
        const int v = atoi(s.c_str() + c + 1);
        if (v > 0) g_tune[key] = v;
        i = s.find_first_of(",}", c);
        if (i == std::string::npos) break;
    }
}

void tune_save_locked()
{
    const char* path = getenv("CPS_TUNE_CACHE");
    if (!path || !*path) return;
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return;
    fprintf(f, "{\n");
    size_t k = 0;
    for (auto& e : g_tune)
        fprintf(f, "  \"%s\": %d%s\n", e.first.c_str(), e.second, ++k < g_tune.size() ? "," : "");
    fprintf(f, "}\n");
    fclose(f);
    rename(tmp.c_str(), path);
}

// median time (ms) of `reps` colour passes with chunk ch on level l
template <typename T>
double time_gs(cps_handle* h, int l, T* b, T* x, int ch, int reps)
{
    const int saved = h->lv[l].gs_ch;
    h->lv[l].gs_ch = ch;
    hipEvent_t e0, e1;
    HIPC(hipEventCreate(&e0));
    HIPC(hipEventCreate(&e1));
    std::vector<float> ms;
    for (int r = 0; r < reps + 1; ++r) {
        HIPC(hipEventRecord(e0, h->stream));
        gs_pass<T>(h, l, r & 1, b, x);
        HIPC(hipEventRecord(e1, h->stream));
        HIPC(hipEventSynchronize(e1));
        float t = 0.f;
        HIPC(hipEventElapsedTime(&t, e0, e1));
        if (r) ms.push_back(t); // the first run warms caches and code
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->lv[l].gs_ch = saved;
    std::sort(ms.begin(), ms.end());
    return ms[ms.size() / 2];
}

// Tunes (or looks up) the chunk of every smoothed level of a marching
// hierarchy.  mode 1: time shapes missing from the cache; 2: retime all.
template <typename T>
void autotune_levels(cps_handle* h, int mode)
{
    const char* prec = std::is_same<T, double>::value ? "f64" : "f32";
    for (int l = 0; l + 1 < h->L; ++l) {
        const Geo& g = h->lv[l].geo;
        const std::string key = tune_key(prec, g);
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            tune_load_locked();
            auto it = g_tune.find(key);
            if (it != g_tune.end() && mode < 2) {
                h->lv[l].gs_ch = std::min(it->second, g.nr);
                continue;
            }
        }
        if (mode == 0) continue;
        // scratch: the level's own x and b, zeroed
        T* x = l == 0 ? nullptr : xl<T>(h, l);
        T* b = l == 0 ? nullptr : bl<T>(h, l);
        Buf<T> sx, sb;
        if (l == 0) {
            sx.alloc(h->lv[0].n);
            sb.alloc(h->lv[0].n);
            x = sx.p;
            b = sb.p;
        }
        fill<T>(h, x, h->lv[l].n, T(0));
        fill<T>(h, b, h->lv[l].n, T(0));
        std::vector<int> cand = {0, 1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64};
        int best = 0;
        double tbest = 1e30;
        std::vector<int> seen;
        for (int c : cand) {
            const MarchShape ms = stencil_shape(g, c);
            if (c > g.nr || std::find(seen.begin(), seen.end(), ms.ch) != seen.end()) continue;
            seen.push_back(ms.ch);
            const double t = time_gs<T>(h, l, b, x, ms.ch, 5);
            if (t < tbest) {
                tbest = t;
                best = ms.ch;
            }
        }
        h->lv[l].gs_ch = best;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = best;
        tune_save_locked();
    }
}

// median time (ms) of `reps` zebra sweeps (both half-sweeps) on level l with
// the plane smoother's launch shapes rb, tb
template <typename T>
double time_plane(cps_handle* h, int l, T* b, T* x, int rb, int tb, int reps)
{
    LevelMem& m = h->lv[l];
    const int srb = m.plane_rb, stb = m.plane_tb;
    m.plane_rb = rb;
    m.plane_tb = tb;
    hipEvent_t e0, e1;
    HIPC(hipEventCreate(&e0));
    HIPC(hipEventCreate(&e1));
    std::vector<float> ms;
    for (int r = 0; r < reps + 1; ++r) {
        HIPC(hipEventRecord(e0, h->stream));
        plane_half_sweep<T>(h, l, 0, b, x);
        plane_half_sweep<T>(h, l, 1, b, x);
        HIPC(hipEventRecord(e1, h->stream));
        HIPC(hipEventSynchronize(e1));
        float t = 0.f;
        HIPC(hipEventElapsedTime(&t, e0, e1));
        if (r) ms.push_back(t);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    m.plane_rb = srb;
    m.plane_tb = stb;
    std::sort(ms.begin(), ms.end());
    return ms[ms.size() / 2];
}

// The plane smoother's launch shapes of every smoothed level: rings per
// block of the transforms (the largest that fits, half and a quarter of it)
// and r-steps in flight per lane of the elimination (4, 8, 16).  Neither
// changes any arithmetic: a tuned solve gives the same bits.  Cached under
// "plane/<precision>/<stencil>/<dims>" as 100 rb + tb.
template <typename T>
void autotune_plane(cps_handle* h, int mode)
{
    const char* prec = std::is_same<T, double>::value ? "f64" : "f32";
    const char* cls = h->mode == MODE_RT ? "rt" : "ortho";
    for (int l = 0; l + 1 < h->L; ++l) {
        LevelMem& m = h->lv[l];
        const Geo& g = m.geo;
        char key[96];
        snprintf(key, sizeof key, "plane/%s/%s/%dx%dx%d", prec, cls, g.nr, g.nt, g.np);
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            tune_load_locked();
            auto it = g_tune.find(key);
            if (it != g_tune.end() && mode < 2) {
                m.plane_rb = it->second / 100;
                m.plane_tb = it->second % 100;
                continue;
            }
        }
        if (mode == 0) continue;
        T* x = l == 0 ? nullptr : xl<T>(h, l);
        T* b = l == 0 ? nullptr : bl<T>(h, l);
        Buf<T> sx, sb;
        if (l == 0) {
            sx.alloc(m.n);
            sb.alloc(m.n);
            x = sx.p;
            b = sb.p;
        }
        fill<T>(h, x, m.n, T(0));
        fill<T>(h, b, m.n, T(1));
        const int rb0 = plane_launch(g, 0).rb;
        int best_rb = rb0, best_tb = kTriBatch;
        double tbest = 1e30;
        for (int rb : {rb0, rb0 / 2, rb0 / 4}) {
            if (rb < 1 || (rb != rb0 && rb == best_rb)) continue;
            const double t = time_plane<T>(h, l, b, x, rb, kTriBatch, 5);
            if (t < tbest) tbest = t, best_rb = rb;
        }
        for (int tb : {4, 16}) {
            const double t = time_plane<T>(h, l, b, x, best_rb, tb, 5);
            if (t < tbest) tbest = t, best_tb = tb;
        }
        m.plane_rb = best_rb;
        m.plane_tb = best_tb;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = 100 * best_rb + best_tb;
        tune_save_locked();
    }
}

void autotune(cps_handle* h, int mode)
{
    if (h->opts.smoother == 1) {
        if (h->opts.precision == 0) autotune_plane<double>(h, mode);
        else autotune_plane<float>(h, mode);
        return;
    }
    if (!marching(h)) return; // the generic colour pass has no chunk to tune
    if (h->opts.precision == 0) autotune_levels<double>(h, mode);
    else autotune_levels<float>(h, mode);
}

} // namespace
