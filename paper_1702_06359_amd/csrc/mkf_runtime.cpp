// Host runtime and C ABI of the track builder (everything except serving).
#include "mkf_runtime.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>

namespace mkf {

static thread_local char g_err[512] = "";

mkf_status fail(mkf_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

// ---------------------------------------------------------------- memory

static std::atomic<unsigned long long> g_broken{0};   // one bit per device

void note_device_error(hipError_t e)
{
    switch (e) {
    case hipErrorIllegalAddress:
    case hipErrorLaunchFailure:
    case hipErrorAssert: {
        int dev = 0;
        (void)hipGetDevice(&dev);
        g_broken.fetch_or(1ull << (dev & 63));
        break;
    }
    default:
        break;
    }
}

bool device_broken(int device) { return (g_broken.load() >> (device & 63)) & 1ull; }

void *CtxHeap::alloc(size_t bytes)
{
    if (bytes == 0) bytes = 256;
    if (ctx->has_alloc) return ctx->alloc.alloc(bytes, (void *)ctx->stream, ctx->alloc.user);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
}

void CtxHeap::release(void *p)
{
    if (!p) return;
    if (ctx->has_alloc) ctx->alloc.free(p, (void *)ctx->stream, ctx->alloc.user);
    else (void)hipFree(p);
}

SlabHeap::SlabHeap(char *base, size_t bytes) : base_(base), cap_(bytes) { free_[0] = bytes; }

void *SlabHeap::alloc(size_t bytes)
{
    bytes = (bytes + 255) & ~size_t(255);
    std::lock_guard<std::mutex> lk(mu_);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second < bytes) continue;
        const size_t off = it->first, sz = it->second;
        free_.erase(it);
        if (sz > bytes) free_[off + bytes] = sz - bytes;
        taken_[off] = bytes;
        used_ += bytes;
        return base_ + off;
    }
    return nullptr;
}

void SlabHeap::release(void *p)
{
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu_);
    const size_t off = static_cast<char *>(p) - base_;
    auto t = taken_.find(off);
    if (t == taken_.end()) return;
    size_t sz = t->second;
    taken_.erase(t);
    used_ -= sz;
    size_t start = off;
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && nx->first == off + sz) {
        sz += nx->second;
        free_.erase(nx);
    }
    auto pv = free_.lower_bound(off);
    if (pv != free_.begin()) {
        --pv;
        if (pv->first + pv->second == off) {
            start = pv->first;
            sz += pv->second;
            free_.erase(pv);
        }
    }
    free_[start] = sz;
}

// ---------------------------------------------------------------- layout

namespace {

struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *b) : base(static_cast<char *>(b)) {}
    template <class T>
    T *take(size_t count)
    {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

// The event's inputs come first (hits, seeds, tracks, as the host packs
// them: one copy moves them all), then the index, outputs and descriptor.
size_t carve_data(const EventShape &s, void *base, DevEvent *v, DevEvent **dev_view, size_t *input_end = nullptr)
{
    Carver c(base);
    const size_t n = (size_t)s.n_hits(), ns = (size_t)s.n_seeds, nt = (size_t)s.n_tracks, nl = (size_t)s.n_layers;
    v->hits = c.take<float4>(n);
    v->seed_par = c.take<float>(6 * ns);
    v->seed_cov = c.take<float>(21 * ns);
    v->seed_hits = c.take<int>((size_t)s.n_seed_layers * ns);
    v->seed_order = c.take<int>(ns);
    v->track_par = c.take<float>(6 * nt);
    v->track_cov = c.take<float>(21 * nt);
    v->track_hits = c.take<int>(nl * nt);
    if (input_end) *input_end = c.off;
    v->binned = c.take<float4>(n);
    v->bin_of = c.take<int>(n);
    v->bin_rank = c.take<int>(n);
    v->out_par = c.take<double>(6 * ns);
    v->out_cov = c.take<double>(21 * ns);
    v->out_hits = c.take<int>(nl * ns);
    v->out_nhits = c.take<int>(ns);
    v->out_nholes = c.take<int>(ns);
    v->out_chi2 = c.take<double>(ns);
    v->out_status = c.take<int>(ns);
    v->fit_par = c.take<double>(6 * nt);
    v->fit_cov = c.take<double>(21 * nt);
    v->fit_chi2 = c.take<double>(nt);
    v->fit_nupd = c.take<int>(nt);
    v->fit_status = c.take<int>(nt);
    v->rf_par = c.take<double>(6 * ns);
    v->rf_cov = c.take<double>(21 * ns);
    v->rf_chi2 = c.take<double>(ns);
    v->rf_nupd = c.take<int>(ns);
    v->rf_status = c.take<int>(ns);
    v->stats = c.take<unsigned long long>(5);
    DevEvent *dv = c.take<DevEvent>(1);
    if (dev_view) *dev_view = dv;
    return c.off;
}

size_t carve_index(const EventShape &s, int nb, void *base, DevEvent *v)
{
    Carver c(base);
    v->bin_count = c.take<int>((size_t)s.n_layers * nb);
    v->bin_off = c.take<int>((size_t)s.n_layers * bin_off_stride(nb));
    return c.off;
}

int plain_slots(int n_seeds, int G)
{
    const int spw = kWave / G;
    return ((n_seeds + spw - 1) / spw) * kWave;
}

size_t carve_plain(const EventShape &s, int slots, void *base, DevEvent *v)
{
    Carver c(base);
    const size_t S = (size_t)slots;
    v->st_par = c.take<float>(6 * S);
    v->st_cov = c.take<float>(21 * S);
    v->st_trig = c.take<float>(4 * S);
    v->st_chi2 = c.take<float>(S);
    v->st_meta = c.take<int>(S);
    v->st_hist = c.take<int>((size_t)s.n_layers * S);
    v->st_slots = slots;
    return c.off;
}

bool finite_all(const double *p, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

// FP64 -> FP32 with the check that the value is, and stays, finite.
bool narrow(const double *src, float *dst, size_t n)
{
    bool ok = true;
    for (size_t i = 0; i < n; ++i) {
        const float f = (float)src[i];
        dst[i] = f;
        ok &= std::isfinite(f);
    }
    return ok;
}

// Host threads that pack inputs, started on first use and kept for the life
// of the process.  A caller posts a job (n tasks, at most `threads` workers
// including itself), takes tasks itself and waits until every task is done;
// jobs of concurrent callers share the workers.
class HostPool {
  public:
    static HostPool &get()
    {
        static HostPool *pool = new HostPool();   // never destroyed: workers may outlive static destructors
        return *pool;
    }

    void run(int n_tasks, int threads, const std::function<void(int)> &f)
    {
        Job job;
        job.f = &f;
        job.n = n_tasks;
        job.helpers = std::min(threads, n_tasks) - 1;
        if (job.helpers > 0 && !workers_.empty()) {
            std::lock_guard<std::mutex> lk(mu_);
            jobs_.push_back(&job);
            cv_.notify_all();
        }
        work(job);
        std::unique_lock<std::mutex> lk(mu_);
        auto it = std::find(jobs_.begin(), jobs_.end(), &job);
        if (it != jobs_.end()) jobs_.erase(it);
        done_cv_.wait(lk, [&] { return job.done.load() == job.n && job.active == 0; });
    }

  private:
    struct Job {
        const std::function<void(int)> *f = nullptr;
        int n = 0;
        int helpers = 0;                 // workers still allowed to join (under mu_)
        int active = 0;                  // workers inside the job (under mu_)
        std::atomic<int> next{0};
        std::atomic<int> done{0};
    };

    HostPool()
    {
        const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
        const int n = (int)std::min(15u, hw > 1 ? hw - 1 : 0u);
        for (int i = 0; i < n; ++i) workers_.emplace_back([this] { loop(); });
        for (auto &t : workers_) t.detach();
    }

    void work(Job &job)
    {
        for (int t = job.next.fetch_add(1); t < job.n; t = job.next.fetch_add(1)) {
            (*job.f)(t);
            if (job.done.fetch_add(1) + 1 == job.n) {
                std::lock_guard<std::mutex> lk(mu_);
                done_cv_.notify_all();
            }
        }
    }

    void loop()
    {
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            Job *job = nullptr;
            for (Job *j : jobs_)
                if (j->helpers > 0 && j->next.load() < j->n) {
                    job = j;
                    break;
                }
            if (!job) {
                cv_.wait(lk);
                continue;
            }
            --job->helpers;
            ++job->active;
            lk.unlock();
            work(*job);
            lk.lock();
            --job->active;
            done_cv_.notify_all();
        }
    }

    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    std::deque<Job *> jobs_;
    std::vector<std::thread> workers_;
};

// Runs f(task) for task = 0 .. n_tasks-1 on up to `threads` host threads.
template <class F>
void run_tasks(int n_tasks, int threads, F f)
{
    threads = std::max(1, std::min(threads, n_tasks));
    if (threads == 1) {
        for (int t = 0; t < n_tasks; ++t) f(t);
        return;
    }
    const std::function<void(int)> fn = f;
    HostPool::get().run(n_tasks, threads, fn);
}


void derive_params(mkf_ctx *ctx)
{
    Params &P = ctx->params;
    const mkf_config &c = ctx->cfg;
    const mkf_tuning &t = ctx->tuning;
    std::memset(&P, 0, sizeof(P));
    for (int L = 0; L < c.n_layers; ++L) {
        LayerParam &lp = P.layer[L];
        lp.r = (float)c.layer_r[L];
        lp.x0 = (float)c.layer_x0[L];
        lp.inv_dphi = (float)(t.bins_phi / (2.0 * M_PI));
        lp.inv_r = (float)(1.0 / c.layer_r[L]);
        lp.kind = c.layer_kind[L];
        lp.half_thick = (float)(0.5 * c.layer_thickness[L]);
        if (lp.kind == 0) {
            lp.half_z = (float)c.layer_half_z[L];
            lp.inv_dz = (float)(t.bins_z / (2.0 * c.layer_half_z[L]));
            lp.grid_lo = -lp.half_z;
        } else {
            lp.zplane = (float)c.layer_z[L];
            lp.inv_dz = (float)(t.bins_z / (c.layer_r[L] - c.layer_rmin[L]));
            lp.grid_lo = (float)c.layer_rmin[L];
        }
    }
    P.n_layers = c.n_layers;
    P.n_seed_layers = c.n_seed_layers;
    P.max_cands = c.max_cands;
    P.max_holes = c.max_holes;
    P.hole_always = (c.flags & MKF_HOLE_ALWAYS) ? 1 : 0;
    P.update3d = (c.flags & MKF_UPDATE_3D) ? 1 : 0;
    P.geo = (c.layer_kind[0] == 1 ? 1 : 0) | (c.layer_thickness[0] > 0.0 || P.update3d ? 2 : 0);
    P.bins_phi = t.bins_phi;
    P.bins_z = t.bins_z;
    P.w_per_qpt = (float)(-0.00299792458 * c.bz);
    P.var_u = (float)(c.sigma_rphi * c.sigma_rphi);
    P.var_z = (float)(c.sigma_z * c.sigma_z);
    P.var_r = (float)(c.sigma_r * c.sigma_r);
    P.chi2_cut = (float)c.chi2_cut;
    P.mass2 = (float)(c.mass * c.mass);
    P.win_scale = 1.05f;
}

mkf_status check_config(const mkf_config *c)
{
    if (!c) return fail(MKF_E_INVALID, "config is NULL");
    if (c->n_seed_layers < 1 || c->n_layers <= c->n_seed_layers || c->n_layers > kMaxLayers)
        return fail(MKF_E_INVALID, "need 1 <= n_seed_layers < n_layers <= %d", kMaxLayers);
    if (c->max_cands < 1 || c->max_cands > kMaxCands) return fail(MKF_E_INVALID, "max_cands must be 1..%d", kMaxCands);
    if (c->max_holes < 0 || c->max_holes > 7) return fail(MKF_E_INVALID, "max_holes must be 0..7");
    if (c->flags & ~(MKF_HOLE_ALWAYS | MKF_UPDATE_3D)) return fail(MKF_E_INVALID, "unknown config flags");
    bool any_disk = false;
    for (int L = 0; L < c->n_layers; ++L) {
        const int kind = c->layer_kind[L];
        if (kind != 0 && kind != 1) return fail(MKF_E_INVALID, "layer_kind must be 0 (cylinder) or 1 (disk)");
        if (!(c->layer_r[L] > 0) || !std::isfinite(c->layer_r[L])) return fail(MKF_E_INVALID, "layer_r must be positive");
        if (kind == 0) {
            if (L > 0 && c->layer_kind[L - 1] == 0 && !(c->layer_r[L] > c->layer_r[L - 1]))
                return fail(MKF_E_INVALID, "consecutive cylinder radii must increase");
            if (!(c->layer_half_z[L] > 0) || !std::isfinite(c->layer_half_z[L]))
                return fail(MKF_E_INVALID, "layer_half_z must be positive");
        } else {
            any_disk = true;
            if (!std::isfinite(c->layer_z[L]) || c->layer_z[L] == 0.0)
                return fail(MKF_E_INVALID, "a disk needs a finite nonzero layer_z");
            if (!(c->layer_rmin[L] >= 0) || !(c->layer_rmin[L] < c->layer_r[L]))
                return fail(MKF_E_INVALID, "a disk needs 0 <= layer_rmin < layer_r");
        }
        if (!(c->layer_x0[L] >= 0) || !std::isfinite(c->layer_x0[L])) return fail(MKF_E_INVALID, "layer_x0 must be >= 0");
    }
    if ((any_disk || (c->flags & MKF_UPDATE_3D)) && (!(c->sigma_r > 0) || !std::isfinite(c->sigma_r)))
        return fail(MKF_E_INVALID, "sigma_r must be positive with a disk or the 3x3 measurement");
    for (int L = 1; L < c->n_layers; ++L)
        if (c->layer_kind[L] != c->layer_kind[0])
            return fail(MKF_E_INVALID, "layers must be all cylinders or all disks (mixed lists are not supported)");
    for (int L = 0; L < c->n_layers; ++L) {
        const double t = c->layer_thickness[L];
        if (!(t >= 0.0) || !std::isfinite(t)) return fail(MKF_E_INVALID, "layer_thickness must be >= 0");
        if ((t > 0.0) != (c->layer_thickness[0] > 0.0))
            return fail(MKF_E_INVALID, "layers must be all thin or all thick (mixed lists are not supported)");
        const double ref = c->layer_kind[L] == 0 ? c->layer_r[L] : std::fabs(c->layer_z[L]);
        if (!(0.5 * t < ref)) return fail(MKF_E_INVALID, "layer_thickness must be below twice the layer's r or |z|");
    }
    if (!std::isfinite(c->bz)) return fail(MKF_E_INVALID, "bz must be finite");
    if (!(c->sigma_rphi > 0) || !(c->sigma_z > 0) || !std::isfinite(c->sigma_rphi) || !std::isfinite(c->sigma_z))
        return fail(MKF_E_INVALID, "hit resolutions must be positive");
    if (!(c->chi2_cut > 0) || !std::isfinite(c->chi2_cut)) return fail(MKF_E_INVALID, "chi2_cut must be positive");
    if (!(c->mass >= 0) || !std::isfinite(c->mass)) return fail(MKF_E_INVALID, "mass must be >= 0");
    return MKF_OK;
}

mkf_status check_tuning(const mkf_config &c, mkf_tuning *t)
{
    static const int kLanes[] = {1, 2, 4, 6, 8};
    if (t->lanes_per_seed == 0) {
        for (int g : kLanes)
            if (g >= c.max_cands) {
                t->lanes_per_seed = g;
                break;
            }
    }
    const int G = t->lanes_per_seed;
    if (G != 1 && G != 2 && G != 4 && G != 6 && G != 8)
        return fail(MKF_E_INVALID, "lanes_per_seed must be 1, 2, 4, 6 or 8");
    if (G < c.max_cands) return fail(MKF_E_INVALID, "lanes_per_seed must be >= max_cands");
    if (t->waves_per_block == 0) t->waves_per_block = 1;
    if (t->waves_per_block < 1 || t->waves_per_block > 4) return fail(MKF_E_INVALID, "waves_per_block must be 1..4");
    if (t->bins_phi == 0) t->bins_phi = 2048;
    if (t->bins_z == 0) t->bins_z = 32;
    if (t->bins_phi < 1 || t->bins_phi > 4096 || t->bins_z < 1 || t->bins_z > 1024 ||
        (long long)t->bins_phi * t->bins_z > (1 << 20))
        return fail(MKF_E_INVALID, "bins out of range (phi 1..4096, z 1..1024, product <= 2^20)");
    if (t->persistent != 0 && t->persistent != 1) return fail(MKF_E_INVALID, "persistent must be 0 or 1");
    if (t->blocks_per_cu == 0) t->blocks_per_cu = 4;
    if (t->blocks_per_cu < 1 || t->blocks_per_cu > 32) return fail(MKF_E_INVALID, "blocks_per_cu must be 1..32");
    return MKF_OK;
}

void timers_collect(mkf_ctx *ctx, bool wait);

void timer_begin(mkf_ctx *ctx, int which, hipStream_t s)
{
    Timer &t = ctx->timers[which];
    if (s != ctx->stream) return;
    if (t.count == Timer::kRing) timers_collect(ctx, true);
    (void)hipEventRecord(t.start[(t.head + t.count) % Timer::kRing], s);
    t.open = true;
}

void timer_end(mkf_ctx *ctx, int which, hipStream_t s, long long launches)
{
    Timer &t = ctx->timers[which];
    if (s != ctx->stream || !t.open) return;
    const int slot = (t.head + t.count) % Timer::kRing;
    (void)hipEventRecord(t.stop[slot], s);
    t.ring_launches[slot] = launches;
    ++t.count;
    t.open = false;
}

// Adds the recorded intervals to the totals: all of them (waiting for the
// device) or only those already complete.
void timers_collect(mkf_ctx *ctx, bool wait)
{
    for (auto &t : ctx->timers) {
        while (t.count > 0) {
            const int slot = t.head;
            if (wait) (void)hipEventSynchronize(t.stop[slot]);
            else if (hipEventQuery(t.stop[slot]) != hipSuccess) break;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, t.start[slot], t.stop[slot]) == hipSuccess) {
                t.total_ms += ms;
                t.launches += t.ring_launches[slot];
            }
            t.head = (t.head + 1) % Timer::kRing;
            --t.count;
        }
    }
}

EventRec *find_event(mkf_ctx *ctx, int32_t h)
{
    auto it = ctx->events.find(h);
    return it == ctx->events.end() ? nullptr : it->second.get();
}

void drop_graphs_with(mkf_ctx *ctx, int32_t handle)
{
    auto &g = ctx->graphs;
    for (size_t i = 0; i < g.size();) {
        const bool hit = handle < 0 || std::find(g[i]->handles.begin(), g[i]->handles.end(), handle) != g[i]->handles.end();
        if (hit) {
            (void)hipStreamSynchronize(ctx->stream);   // a queued replay may still use its scratch
            (void)hipGraphExecDestroy(g[i]->exec);
            ctx->heap.release(g[i]->scratch);
            g.erase(g.begin() + i);
        } else {
            ++i;
        }
    }
}

void drop_plain_graph(EventRec *rec)
{
    if (rec->plain_graph) (void)hipGraphExecDestroy(rec->plain_graph);
    rec->plain_graph = nullptr;
}

mkf_status upload_view(EventRec *rec, hipStream_t s)
{
    MKF_HIP(hipMemcpyAsync(rec->dev_view, &rec->view, sizeof(DevEvent), hipMemcpyHostToDevice, s));
    MKF_HIP(hipStreamSynchronize(s));
    return MKF_OK;
}

mkf_status ensure_batch_scratch(mkf_ctx *ctx, int n)
{
    const size_t need = batch_scratch_bytes(n);
    if (ctx->batch_dev_bytes < need || ctx->batch_host_bytes < need) {
        MKF_HIP(hipStreamSynchronize(ctx->stream));   // queued work may still read the buffers
        ctx->stage_pending = false;
        ctx->staged_image.clear();
    }
    if (ctx->batch_dev_bytes < need) {
        ctx->heap.release(ctx->batch_dev);
        ctx->batch_dev = ctx->heap.alloc(need);
        ctx->batch_dev_bytes = ctx->batch_dev ? need : 0;
        if (!ctx->batch_dev) return fail(MKF_E_NOMEM, "batch scratch of %zu bytes", need);
    }
    if (ctx->batch_host_bytes < need) {
        if (ctx->batch_host) (void)hipHostFree(ctx->batch_host);
        ctx->batch_host = nullptr;
        ctx->batch_host_bytes = 0;
        MKF_HIP(hipHostMalloc(&ctx->batch_host, need, hipHostMallocDefault));
        ctx->batch_host_bytes = need;
    }
    return MKF_OK;
}

mkf_status gather_events(mkf_ctx *ctx, const int32_t *handles, int32_t n, std::vector<EventRec *> *recs)
{
    if (n < 0 || (n > 0 && !handles)) return fail(MKF_E_INVALID, "bad handle list");
    if ((long long)n * ctx->cfg.n_layers > 65535)
        return fail(MKF_E_INVALID, "at most %d events per batch", 65535 / ctx->cfg.n_layers);
    std::vector<int32_t> seen(handles, handles + n);
    std::sort(seen.begin(), seen.end());
    if (std::adjacent_find(seen.begin(), seen.end()) != seen.end())
        return fail(MKF_E_INVALID, "an event appears twice in the batch");
    recs->clear();
    for (int i = 0; i < n; ++i) {
        EventRec *r = find_event(ctx, handles[i]);
        if (!r) return fail(MKF_E_NOTFOUND, "unknown event handle %d", handles[i]);
        recs->push_back(r);
    }
    return MKF_OK;
}

}  // namespace

size_t event_data_bytes(const EventShape &s)
{
    DevEvent v{};
    return carve_data(s, nullptr, &v, nullptr);
}

int pack_threads(size_t n_values)
{
    // a thread per ~100k values of FP64 input, up to 16
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    return (int)std::min<size_t>({(size_t)16, (size_t)hw, 1 + n_values / 100000});
}

size_t event_input_bytes(const EventShape &s)
{
    DevEvent v{};
    size_t end = 0;
    carve_data(s, nullptr, &v, nullptr, &end);
    return end;
}

size_t event_index_bytes(const EventShape &s, int nb)
{
    DevEvent v{};
    return carve_index(s, nb, nullptr, &v);
}

size_t batch_scratch_bytes(int n)
{
    size_t b = ((size_t)n * sizeof(DevEvent) + 255) & ~size_t(255);
    b += 4 * (((size_t)(n + 1) * sizeof(int) + 255) & ~size_t(255));
    return b + 256;
}

int resolve_lanes(const mkf_ctx *ctx) { return ctx->tuning.lanes_per_seed; }
int seeds_per_item(int G) { return kWave / G; }

// ---------------------------------------------------------------- events

// Counts and pointers of an event: its shape.  The values are checked while
// they are packed (pack_event).
mkf_status validate_event(const mkf_ctx *ctx, const mkf_event *ev, EventShape *shape)
{
    const mkf_config &c = ctx->cfg;
    if (!ev) return fail(MKF_E_INVALID, "event is NULL");
    if (ev->n_layers != c.n_layers) return fail(MKF_E_INVALID, "event has %d layers, config %d", ev->n_layers, c.n_layers);
    if (ev->n_seeds < 0 || ev->n_tracks < 0) return fail(MKF_E_INVALID, "negative seed or track count");
    if (!ev->n_hits || !ev->hit_xyz) return fail(MKF_E_INVALID, "n_hits / hit_xyz is NULL");
    EventShape s;
    s.n_layers = c.n_layers;
    s.n_seed_layers = c.n_seed_layers;
    s.n_seeds = ev->n_seeds;
    s.n_tracks = ev->n_tracks;
    long long tot = 0;
    for (int L = 0; L < c.n_layers; ++L) {
        const int n = ev->n_hits[L];
        if (n < 0 || n > kMaxHitsPerLayer) return fail(MKF_E_INVALID, "layer %d: %d hits out of range", L, n);
        if (n > 0 && !ev->hit_xyz[L]) return fail(MKF_E_INVALID, "layer %d: hit_xyz is NULL", L);
        s.layer_off[L] = (int)tot;
        tot += n;
        if (tot > (1LL << 30)) return fail(MKF_E_INVALID, "too many hits in one event");
    }
    s.layer_off[c.n_layers] = (int)tot;
    if (ev->n_seeds > 0 && (!ev->seed_par || !ev->seed_cov || !ev->seed_hits))
        return fail(MKF_E_INVALID, "seed arrays are NULL");
    if (ev->n_tracks > 0 && (!ev->track_par || !ev->track_cov || !ev->track_hits))
        return fail(MKF_E_INVALID, "track arrays are NULL");
    *shape = s;
    return MKF_OK;
}

// Checks a state (finite, theta in (0, pi), off the axis) and the hit
// indices of one seed or track; writes its FP32 state and covariance.
static bool pack_state(const double *par, const double *cov, float *fpar, float *fcov, const int32_t *hits,
                       int32_t *ohits, int n_hit_layers, const int32_t *n_hits, int *bad_hit)
{
    if (!narrow(par, fpar, 6) || !narrow(cov, fcov, 21)) return false;
    if (!(par[5] > 0 && par[5] < M_PI) || !(par[0] * par[0] + par[1] * par[1] > 0)) return false;
    for (int L = 0; L < n_hit_layers; ++L) {
        const int32_t h = hits[L];
        if (h < -1 || h >= n_hits[L]) {
            *bad_hit = 1;
            return false;
        }
        ohits[L] = h;
    }
    return true;
}

// Packs an event's inputs into `image` in the device layout of its data
// block (carve_data) and checks every value on the way: each hit becomes
// the FP32 form the kernels read (geo: bit 0 disks, bit 1 layers of finite
// thickness or the 3x3 measurement), computed in FP64; seeds and tracks
// FP32 states and covariances, finite, theta in (0, pi), hit indices in
// range.  The layers and the seeds are packed in parallel for large events.
// The seeds in order of the azimuth of their direction: a counting sort over
// 1024 sectors that keeps the caller's order within a sector.  The batched
// builder takes the seeds of one wavefront, and of the wavefronts that run
// together, from neighbouring sectors, so the hits and bins their windows read
// are shared in cache instead of each wavefront reading a different part of
// every layer.  The outputs stay in the caller's order.
constexpr int kSeedSectors = 1024;

static inline uint16_t seed_sector(double phi)
{
    const double x = (phi + M_PI) * (kSeedSectors / (2 * M_PI));
    return (uint16_t)(x >= 0.0 ? (x < kSeedSectors ? (int)x : kSeedSectors - 1) : 0);   // NaN: sector 0
}

static void order_seeds(const std::vector<uint16_t> &sector, int *order)
{
    int start[kSeedSectors + 1] = {0};
    for (uint16_t k : sector) ++start[k + 1];
    for (int k = 0; k < kSeedSectors; ++k) start[k + 1] += start[k];
    for (int i = 0; i < (int)sector.size(); ++i) order[start[sector[i]]++] = i;
}

mkf_status pack_event(const mkf_event *ev, const EventShape &sh, int geo, void *image, int threads, std::string *why)
{
    DevEvent v{};
    carve_data(sh, image, &v, nullptr);
    const int nl = sh.n_layers, nsl = sh.n_seed_layers;
    const int chunk = 4096;
    const int seed_tasks = (sh.n_seeds + chunk - 1) / chunk, track_tasks = (sh.n_tracks + chunk - 1) / chunk;
    const int n_tasks = nl + seed_tasks + track_tasks;
    // first failure of each task: (index, kind), index -1 for none
    std::vector<int> bad(n_tasks, -1), kind(n_tasks, 0);
    std::vector<uint16_t> sector(sh.n_seeds);   // azimuth sector of each seed, taken while it is packed
    run_tasks(n_tasks, threads, [&](int t) {
        if (t < nl) {
            // a hit as the kernels read it: its direction and second grid
            // coordinate computed here in FP64 and rounded once
            const int n = ev->n_hits[t];
            const double *h = ev->hit_xyz[t];
            float4 *o = const_cast<float4 *>(v.hits) + sh.layer_off[t];
            const bool xyz = (geo & 2) != 0, disk = (geo & 1) != 0;
            for (int i = 0; i < n; ++i) {
                const double x = h[3 * i], y = h[3 * i + 1], z = h[3 * i + 2];
                const double r = std::sqrt(x * x + y * y);
                float4 f;
                if (xyz) f = make_float4((float)x, (float)y, (float)z, 0.f);
                else if (disk) f = make_float4((float)(x / r), (float)(y / r), (float)r, (float)z);
                else f = make_float4((float)(x / r), (float)(y / r), (float)z, (float)r);
                o[i] = f;
                if (!(r > 0) || !std::isfinite(f.x) || !std::isfinite(f.y) || !std::isfinite(f.z) ||
                    !std::isfinite(f.w) || (xyz && !((double)f.x * f.x + (double)f.y * f.y > 0))) {
                    bad[t] = i;
                    return;
                }
            }
            return;
        }
        const bool seeds = t < nl + seed_tasks;
        const int i0 = (seeds ? t - nl : t - nl - seed_tasks) * chunk;
        const int i1 = std::min(i0 + chunk, seeds ? sh.n_seeds : sh.n_tracks);
        for (int i = i0; i < i1; ++i) {
            int bad_hit = 0;
            const bool ok = seeds ? pack_state(ev->seed_par + 6 * (size_t)i, ev->seed_cov + 21 * (size_t)i,
                                               const_cast<float *>(v.seed_par) + 6 * (size_t)i,
                                               const_cast<float *>(v.seed_cov) + 21 * (size_t)i,
                                               ev->seed_hits + (size_t)i * nsl,
                                               const_cast<int *>(v.seed_hits) + (size_t)i * nsl, nsl, ev->n_hits,
                                               &bad_hit)
                                  : pack_state(ev->track_par + 6 * (size_t)i, ev->track_cov + 21 * (size_t)i,
                                               const_cast<float *>(v.track_par) + 6 * (size_t)i,
                                               const_cast<float *>(v.track_cov) + 21 * (size_t)i,
                                               ev->track_hits + (size_t)i * nl,
                                               const_cast<int *>(v.track_hits) + (size_t)i * nl, nl, ev->n_hits,
                                               &bad_hit);
            if (!ok) {
                bad[t] = i;
                kind[t] = bad_hit;
                return;
            }
            if (seeds) sector[i] = seed_sector(ev->seed_par[6 * (size_t)i + 4]);
        }
    });
    for (int t = 0; t < n_tasks; ++t) {
        if (bad[t] < 0) continue;
        char msg[200];
        if (t < nl) {
            std::snprintf(msg, sizeof(msg), "layer %d hit %d: not finite (in FP32) or on the axis", t, bad[t]);
        } else {
            const char *what = t < nl + seed_tasks ? "seed" : "track";
            if (kind[t]) std::snprintf(msg, sizeof(msg), "%s %d: hit index out of range", what, bad[t]);
            else std::snprintf(msg, sizeof(msg), "%s %d: state or covariance not finite (in FP32), theta outside "
                                                 "(0, pi) or position on the axis", what, bad[t]);
        }
        *why = msg;
        return MKF_E_INVALID;
    }
    order_seeds(sector, const_cast<int *>(v.seed_order));
    return MKF_OK;
}

mkf_status create_event(mkf_ctx *ctx, const EventShape &shape, DeviceHeap *heap, std::unique_ptr<EventRec> *out)
{
    auto rec = std::make_unique<EventRec>();
    rec->shape = shape;
    rec->heap = heap;
    const size_t bytes = event_data_bytes(shape);
    rec->data = heap->alloc(bytes);
    if (!rec->data) return fail(MKF_E_NOMEM, "event data: %zu bytes", bytes);
    DevEvent &v = rec->view;
    std::memset(&v, 0, sizeof(v));
    carve_data(shape, rec->data, &v, &rec->dev_view);
    v.n_layers = shape.n_layers;
    v.n_seeds = shape.n_seeds;
    v.n_tracks = shape.n_tracks;
    v.n_hits = shape.n_hits();
    for (int L = 0; L <= shape.n_layers; ++L) v.layer_off[L] = shape.layer_off[L];
    (void)ctx;
    *out = std::move(rec);
    return MKF_OK;
}

// Copies an event's packed inputs (pack_event) into its device data block.
mkf_status upload_packed(EventRec *rec, const void *image, hipStream_t s)
{
    const size_t bytes = event_input_bytes(rec->shape);
    if (bytes) MKF_HIP(hipMemcpyAsync(rec->data, image, bytes, hipMemcpyHostToDevice, s));
    return MKF_OK;
}

void destroy_event(mkf_ctx *ctx, EventRec *rec)
{
    (void)ctx;
    drop_plain_graph(rec);
    rec->heap->release(rec->plain);
    rec->heap->release(rec->index);
    rec->heap->release(rec->data);
    rec->heap->release(rec->beam);
    rec->plain = rec->index = rec->data = rec->beam = nullptr;
}

// Storage for every rank of the final beam of an event (max_cands per seed).
mkf_status ensure_beam(mkf_ctx *ctx, EventRec *rec)
{
    if (rec->beam) return MKF_OK;
    const size_t n = (size_t)rec->shape.n_seeds * ctx->cfg.max_cands, nl = (size_t)rec->shape.n_layers;
    auto carve = [&](void *base) {
        Carver c(base);
        DevEvent &v = rec->beam_view;
        v.beam_par = c.take<double>(6 * n);
        v.beam_cov = c.take<double>(21 * n);
        v.beam_chi2 = c.take<double>(n);
        v.beam_hits = c.take<int>(nl * n);
        v.beam_nhits = c.take<int>(n);
        v.beam_nholes = c.take<int>(n);
        v.beam_status = c.take<int>(n);
        return c.off;
    };
    const size_t bytes = carve(nullptr);
    rec->beam = rec->heap->alloc(bytes);
    if (!rec->beam) return fail(MKF_E_NOMEM, "final beam: %zu bytes", bytes);
    carve(rec->beam);
    return MKF_OK;
}

// Make sure the event's index tables match the current bin grid.  *rebuilt is
// set when the tables were (re)allocated and the index must be built.
mkf_status ensure_index(mkf_ctx *ctx, EventRec *rec, bool *rebuilt, hipStream_t s)
{
    return ensure_index_grid(ctx, rec, ctx->tuning.bins_phi, ctx->tuning.bins_z, rebuilt, s);
}

int max_layer_hits(const EventShape &s)
{
    int m = 0;
    for (int L = 0; L < s.n_layers; ++L) m = std::max(m, s.layer_off[L + 1] - s.layer_off[L]);
    return m;
}

int event_bins(const EventShape &s, int bins_phi, int bins_z)
{
    const int k = event_grid_shift(max_layer_hits(s), bins_phi, bins_z);
    return (bins_phi >> k) * (bins_z >> k);
}

mkf_status ensure_index_grid(mkf_ctx *ctx, EventRec *rec, int bp, int bz, bool *rebuilt, hipStream_t s)
{
    *rebuilt = false;
    if (rec->index && rec->index_bins_phi == bp && rec->index_bins_z == bz) return MKF_OK;
    if (rec->index) MKF_HIP(hipStreamSynchronize(ctx->stream));   // queued builds may still read it
    rec->heap->release(rec->index);
    // the event's own grid: the context's, coarsened for a small event
    const int k = event_grid_shift(max_layer_hits(rec->shape), bp, bz);
    const int nb = (bp >> k) * (bz >> k);
    const size_t bytes = event_index_bytes(rec->shape, nb);
    rec->index = rec->heap->alloc(bytes);
    if (!rec->index) {
        rec->index_bins_phi = rec->index_bins_z = 0;
        return fail(MKF_E_NOMEM, "hit index: %zu bytes", bytes);
    }
    carve_index(rec->shape, nb, rec->index, &rec->view);
    rec->view.grid_k = k;
    // the index build expects zero bin counts (and leaves them at zero)
    MKF_HIP(launch_fill_i32(rec->view.bin_count, 0, rec->shape.n_layers * nb, s));
    rec->index_bins_phi = bp;
    rec->index_bins_z = bz;
    drop_plain_graph(rec);
    *rebuilt = true;
    return MKF_OK;
}

// Lays out the batch descriptors of recs[0..n) - the event views, the work,
// hit, track and seed prefixes and the work-queue counter - into `image`
// (batch_scratch_bytes(n) bytes, all written) and points `args` at the same
// layout starting at device address `dev`.  Allocates nothing.
mkf_status compose_batch(EventRec *const *recs, int n, int spi, bool beam, char *image, char *dev, BatchArgs *args)
{
    size_t off = 0;
    auto place = [&](size_t bytes) {
        const size_t o = off;
        off = (off + bytes + 255) & ~size_t(255);
        return o;
    };
    const size_t o_ev = place((size_t)n * sizeof(DevEvent));
    const size_t o_item = place((size_t)(n + 1) * sizeof(int));
    const size_t o_hit = place((size_t)(n + 1) * sizeof(int));
    const size_t o_trk = place((size_t)(n + 1) * sizeof(int));
    const size_t o_seed = place((size_t)(n + 1) * sizeof(int));
    const size_t o_q = place(sizeof(unsigned));
    std::memset(image, 0, off);
    char *h = image;
    DevEvent *ev = reinterpret_cast<DevEvent *>(h + o_ev);
    int *ip = reinterpret_cast<int *>(h + o_item);
    int *hp = reinterpret_cast<int *>(h + o_hit);
    int *tp = reinterpret_cast<int *>(h + o_trk);
    int *sp = reinterpret_cast<int *>(h + o_seed);
    long long items = 0, hits = 0, trks = 0, seeds = 0;
    int max_layer = 0, max_bins = 0;
    for (int i = 0; i < n; ++i) {
        const EventShape &sh = recs[i]->shape;
        for (int L = 0; L < sh.n_layers; ++L) max_layer = std::max(max_layer, sh.layer_off[L + 1] - sh.layer_off[L]);
        const int k = recs[i]->view.grid_k;
        max_bins = std::max(max_bins, (recs[i]->index_bins_phi >> k) * (recs[i]->index_bins_z >> k));
        ev[i] = recs[i]->view;
        if (beam) {   // this launch also writes every rank of the final beam
            const DevEvent &b = recs[i]->beam_view;
            ev[i].beam_par = b.beam_par;
            ev[i].beam_cov = b.beam_cov;
            ev[i].beam_hits = b.beam_hits;
            ev[i].beam_nhits = b.beam_nhits;
            ev[i].beam_nholes = b.beam_nholes;
            ev[i].beam_chi2 = b.beam_chi2;
            ev[i].beam_status = b.beam_status;
        }
        ip[i] = (int)items;
        hp[i] = (int)hits;
        tp[i] = (int)trks;
        sp[i] = (int)seeds;
        seeds += recs[i]->shape.n_seeds;
        items += (recs[i]->shape.n_seeds + spi - 1) / spi;
        hits += recs[i]->shape.n_hits();
        trks += recs[i]->shape.n_tracks;
    }
    if (items > INT32_MAX || hits > INT32_MAX || trks > INT32_MAX || seeds > INT32_MAX)
        return fail(MKF_E_INVALID, "batch too large");
    ip[n] = (int)items;
    hp[n] = (int)hits;
    tp[n] = (int)trks;
    sp[n] = (int)seeds;
    args->events = reinterpret_cast<const DevEvent *>(dev + o_ev);
    args->item_prefix = reinterpret_cast<const int *>(dev + o_item);
    args->hit_prefix = reinterpret_cast<const int *>(dev + o_hit);
    args->track_prefix = reinterpret_cast<const int *>(dev + o_trk);
    args->seed_prefix = reinterpret_cast<const int *>(dev + o_seed);
    args->queue = reinterpret_cast<unsigned *>(dev + o_q);
    args->n_events = n;
    args->total_items = (int)items;
    args->total_hits = (int)hits;
    args->total_tracks = (int)trks;
    args->total_seeds = (int)seeds;
    args->seeds_per_item = spi;
    args->max_layer_hits = max_layer;
    args->max_bins = max_bins;
    return MKF_OK;
}

mkf_status stage_batch(mkf_ctx *ctx, const std::vector<EventRec *> &recs, void *dev, void *host, int spi,
                       BatchArgs *args, hipStream_t s, bool beam)
{
    const int n = (int)recs.size();
    std::vector<char> image(batch_scratch_bytes(n));
    mkf_status st = compose_batch(recs.data(), n, spi, beam, image.data(), static_cast<char *>(dev), args);
    if (st != MKF_OK) return st;
    // The context's own buffer keeps the last image: an identical batch (same
    // events, views and tuning) is not copied again.  Its pinned staging
    // buffer is rewritten only once the previous copy out of it has run.
    const bool own = dev == ctx->batch_dev;
    if (!own || image != ctx->staged_image) {
        if (host == ctx->batch_host && ctx->stage_pending) {
            MKF_HIP(hipEventSynchronize(ctx->stage_done));
            ctx->stage_pending = false;
        }
        std::memcpy(host, image.data(), image.size());
        MKF_HIP(hipMemcpyAsync(dev, host, image.size(), hipMemcpyHostToDevice, s));
        if (host == ctx->batch_host) {
            MKF_HIP(hipEventRecord(ctx->stage_done, s));
            ctx->stage_pending = true;
        }
        if (own) ctx->staged_image.swap(image);
    }
    return MKF_OK;
}

// The batched pipeline on stream s: optional counter reset and re-index,
// then the build kernel.
mkf_status run_pipeline(mkf_ctx *ctx, const BatchArgs &args, const std::vector<EventRec *> &recs, uint32_t flags,
                        bool timed, hipStream_t s)
{
    (void)recs;
    return run_pipeline_with(ctx, ctx->params, ctx->tuning, args, flags, timed, s);
}

mkf_status run_pipeline_with(mkf_ctx *ctx, const Params &P, const mkf_tuning &t, const BatchArgs &args,
                             uint32_t flags, bool timed, hipStream_t s)
{
    const bool stats = flags & MKF_BATCH_STATS, reindex = flags & MKF_BATCH_REINDEX;
    // bin counts are left at zero by every index build; fresh tables are
    // cleared when they are allocated
    if (stats) MKF_HIP(launch_batch_zero(args, s));
    if (reindex) {
        if (timed) timer_begin(ctx, 1, s);
        MKF_HIP(launch_index(P, args, s));
        if (timed) timer_end(ctx, 1, s, 1);   // one index build of the batch
    }
    if (t.persistent) MKF_HIP(launch_fill_i32(reinterpret_cast<int *>(args.queue), 0, 1, s));
    if (timed) timer_begin(ctx, 0, s);
    MKF_HIP(launch_build_batch(P, args, t.lanes_per_seed, t.waves_per_block, t.persistent,
                               ctx->n_cu * t.blocks_per_cu, stats, s));
    if (timed) timer_end(ctx, 0, s, 1);
    if (flags & MKF_BATCH_FIT) {
        if (timed) timer_begin(ctx, 2, s);
        MKF_HIP(launch_refit(P, args, s));
        if (timed) timer_end(ctx, 2, s, 1);
    }
    return MKF_OK;
}

static mkf_status copy_d2h(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    if (!dst || bytes == 0) return MKF_OK;
    MKF_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
    return MKF_OK;
}

mkf_status copy_tracks_out(mkf_ctx *ctx, const EventRec *rec, const mkf_tracks *out, hipStream_t s)
{
    (void)ctx;
    const DevEvent &v = rec->view;
    const size_t n = (size_t)rec->shape.n_seeds, nl = (size_t)rec->shape.n_layers;
    mkf_status st;
    if ((st = copy_d2h(out->par, v.out_par, 48 * n, s)) != MKF_OK) return st;
    if ((st = copy_d2h(out->cov, v.out_cov, 168 * n, s)) != MKF_OK) return st;
    if ((st = copy_d2h(out->hits, v.out_hits, 4 * nl * n, s)) != MKF_OK) return st;
    if ((st = copy_d2h(out->n_hits, v.out_nhits, 4 * n, s)) != MKF_OK) return st;
    if ((st = copy_d2h(out->n_holes, v.out_nholes, 4 * n, s)) != MKF_OK) return st;
    if ((st = copy_d2h(out->chi2, v.out_chi2, 8 * n, s)) != MKF_OK) return st;
    if ((st = copy_d2h(out->status, v.out_status, 4 * n, s)) != MKF_OK) return st;
    if (out->ndof) {
        // 2 measured coordinates per hit, minus the 5 track parameters
        if ((st = copy_d2h(out->ndof, v.out_nhits, 4 * n, s)) != MKF_OK) return st;
    }
    return MKF_OK;
}

static void finish_ndof(const mkf_tracks *out)
{
    if (!out || !out->ndof) return;
    for (int i = 0; i < out->n; ++i) out->ndof[i] = 2 * out->ndof[i] - 5;
}

static mkf_status check_tracks(const mkf_tracks *out, int n, const char *what)
{
    if (!out) return MKF_OK;
    if (out->n != n) return fail(MKF_E_INVALID, "%s: output has %d rows, need %d", what, out->n, n);
    return MKF_OK;
}

}  // namespace mkf

using namespace mkf;

// ====================================================================== ABI

extern "C" {

const char *mkf_version(void) { return "mkf 0.1 (gfx950, FP32 Kalman filter)"; }

const char *mkf_last_error(const mkf_ctx *ctx)
{
    (void)ctx;   // the message is per thread
    return g_err;
}

int32_t mkf_ctx_broken(const mkf_ctx *ctx) { return ctx && device_broken(ctx->device) ? 1 : 0; }

mkf_status mkf_create(const mkf_config *cfg, const mkf_allocator *alloc, void *hip_stream, mkf_ctx **out)
{
    if (!out) return fail(MKF_E_INVALID, "out is NULL");
    mkf_status st = check_config(cfg);
    if (st != MKF_OK) return st;
    if (alloc && (!alloc->alloc || !alloc->free)) return fail(MKF_E_INVALID, "allocator needs alloc and free");
    int dev = 0;
    MKF_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    MKF_HIP(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(MKF_E_DEVICE, "device %d is %s, this library is built for gfx950", dev, prop.gcnArchName);
    auto ctx = std::make_unique<mkf_ctx>();
    ctx->cfg = *cfg;
    ctx->device = dev;
    ctx->n_cu = prop.multiProcessorCount;
    ctx->heap.ctx = ctx.get();
    if (alloc) {
        ctx->alloc = *alloc;
        ctx->has_alloc = true;
    }
    if (hip_stream) {
        ctx->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        MKF_HIP(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
        ctx->own_stream = true;
    }
    std::memset(&ctx->tuning, 0, sizeof(ctx->tuning));
    if ((st = check_tuning(ctx->cfg, &ctx->tuning)) != MKF_OK) return st;
    derive_params(ctx.get());
    for (auto &t : ctx->timers)
        for (int i = 0; i < Timer::kRing; ++i) {
            MKF_HIP(hipEventCreate(&t.start[i]));
            MKF_HIP(hipEventCreate(&t.stop[i]));
        }
    MKF_HIP(hipEventCreateWithFlags(&ctx->stage_done, hipEventDisableTiming));
    // device address of this GPU's fixed batch-descriptor array (the
    // no-allocation builder); looked up once per device
    MKF_HIP(noalloc_scratch_init(dev));
    *out = ctx.release();
    return MKF_OK;
}

void mkf_destroy(mkf_ctx *ctx)
{
    if (!ctx) return;
    shutdown_server(ctx);
    (void)hipStreamSynchronize(ctx->stream);
    drop_graphs_with(ctx, -1);
    for (auto &kv : ctx->events) destroy_event(ctx, kv.second.get());
    ctx->events.clear();
    ctx->heap.release(ctx->batch_dev);
    if (ctx->batch_host) (void)hipHostFree(ctx->batch_host);
    if (ctx->load_pin) (void)hipHostFree(ctx->load_pin);
    for (auto &t : ctx->timers)
        for (int i = 0; i < Timer::kRing; ++i) {
            if (t.start[i]) (void)hipEventDestroy(t.start[i]);
            if (t.stop[i]) (void)hipEventDestroy(t.stop[i]);
        }
    if (ctx->stage_done) (void)hipEventDestroy(ctx->stage_done);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

mkf_status mkf_set_tuning(mkf_ctx *ctx, const mkf_tuning *t)
{
    if (!ctx || !t) return fail(MKF_E_INVALID, "NULL argument");
    mkf_tuning nt = *t;
    mkf_status st = check_tuning(ctx->cfg, &nt);
    if (st != MKF_OK) return st;
    if (build_lds_bytes(ctx->params.geo, ctx->cfg.n_layers, nt.waves_per_block) > 65536)
        return fail(MKF_E_INVALID, "waves_per_block too large for %d layers", ctx->cfg.n_layers);
    ctx->tuning = nt;
    derive_params(ctx);
    drop_graphs_with(ctx, -1);
    for (auto &kv : ctx->events) drop_plain_graph(kv.second.get());
    return MKF_OK;
}

mkf_status mkf_get_tuning(const mkf_ctx *ctx, mkf_tuning *t)
{
    if (!ctx || !t) return fail(MKF_E_INVALID, "NULL argument");
    *t = ctx->tuning;
    return MKF_OK;
}

mkf_status mkf_load_events(mkf_ctx *ctx, const mkf_event *evs, int32_t n, int32_t *handles)
{
    if (!ctx || !handles || n < 0 || (n > 0 && !evs)) return fail(MKF_E_INVALID, "NULL argument");
    if ((long long)n * ctx->cfg.n_layers > 65535)
        return fail(MKF_E_INVALID, "at most %d events per call", 65535 / ctx->cfg.n_layers);
    if (n == 0) return MKF_OK;
    std::vector<EventShape> shapes(n);
    std::vector<size_t> off(n + 1, 0);
    size_t values = 0;
    for (int i = 0; i < n; ++i) {
        mkf_status st = validate_event(ctx, &evs[i], &shapes[i]);
        if (st != MKF_OK) return n == 1 ? st : fail(st, "event %d: %s", i, mkf_last_error(ctx));
        off[i + 1] = off[i] + ((event_input_bytes(shapes[i]) + 255) & ~size_t(255));
        values += (size_t)shapes[i].n_hits() * 3 + (size_t)(shapes[i].n_seeds + shapes[i].n_tracks) * 27;
    }
    // every load ends waiting for the stream, so the staging is free
    if (ctx->load_pin_bytes < off[n]) {
        if (ctx->load_pin) (void)hipHostFree(ctx->load_pin);
        ctx->load_pin = nullptr;
        ctx->load_pin_bytes = 0;
        MKF_HIP(hipHostMalloc(&ctx->load_pin, off[n], hipHostMallocDefault));
        ctx->load_pin_bytes = off[n];
    }
    char *pin = static_cast<char *>(ctx->load_pin);
    std::vector<std::unique_ptr<EventRec>> recs(n);
    auto undo = [&](mkf_status st) {
        (void)hipStreamSynchronize(ctx->stream);
        for (auto &r : recs)
            if (r) destroy_event(ctx, r.get());
        return st;
    };
    hipStream_t s = ctx->stream;
    mkf_status st;
    // device memory first (the allocator may call back into the caller, so
    // on this thread); then every event is packed and its copy queued as soon
    // as its packing ends, so that the copies overlap the packing of the
    // others
    for (int i = 0; i < n; ++i)
        if ((st = create_event(ctx, shapes[i], &ctx->heap, &recs[i])) != MKF_OK) return undo(st);
    std::vector<mkf_status> sts(n, MKF_OK);
    std::vector<std::string> why(n);
    std::vector<hipError_t> copied(n, hipSuccess);
    auto pack_send = [&](int i, int th) {
        sts[i] = pack_event(&evs[i], shapes[i], ctx->params.geo, pin + off[i], th, &why[i]);
        const size_t bytes = event_input_bytes(shapes[i]);
        if (sts[i] == MKF_OK && bytes)
            copied[i] = hipMemcpyAsync(recs[i]->data, pin + off[i], bytes, hipMemcpyHostToDevice, s);
    };
    const int threads = pack_threads(values);
    if (n == 1) pack_send(0, threads);
    else run_tasks(n, threads, [&](int i) { pack_send(i, 1); });
    for (int i = 0; i < n; ++i)
        if (sts[i] != MKF_OK) return undo(n == 1 ? fail(sts[i], "%s", why[i].c_str())
                                                 : fail(sts[i], "event %d: %s", i, why[i].c_str()));
    for (int i = 0; i < n; ++i)
        if (copied[i] != hipSuccess) {
            note_device_error(copied[i]);
            return undo(fail(MKF_E_DEVICE, "load: %s", hipGetErrorString(copied[i])));
        }
    for (int i = 0; i < n; ++i) {
        bool rebuilt = false;
        if ((st = ensure_index(ctx, recs[i].get(), &rebuilt, s)) != MKF_OK) return undo(st);
        const hipError_t e = hipMemcpyAsync(recs[i]->dev_view, &recs[i]->view, sizeof(DevEvent),
                                            hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return undo(fail(MKF_E_DEVICE, "load: %s", hipGetErrorString(e)));
    }
    if ((st = ensure_batch_scratch(ctx, n)) != MKF_OK) return undo(st);
    std::vector<EventRec *> raw(n);
    for (int i = 0; i < n; ++i) raw[i] = recs[i].get();
    BatchArgs args{};
    if ((st = stage_batch(ctx, raw, ctx->batch_dev, ctx->batch_host, seeds_per_item(ctx->tuning.lanes_per_seed),
                          &args, s)) != MKF_OK)
        return undo(st);
    hipError_t e = launch_batch_zero(args, s);
    if (e == hipSuccess) e = launch_index(ctx->params, args, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        note_device_error(e);
        return undo(fail(MKF_E_DEVICE, "load: %s", hipGetErrorString(e)));
    }
    for (int i = 0; i < n; ++i) {
        const int32_t h = ctx->next_handle++;
        ctx->events[h] = std::move(recs[i]);
        handles[i] = h;
    }
    return MKF_OK;
}

mkf_status mkf_load_event(mkf_ctx *ctx, const mkf_event *ev, int32_t *handle)
{
    if (!ctx || !handle || !ev) return fail(MKF_E_INVALID, "NULL argument");
    return mkf_load_events(ctx, ev, 1, handle);
}

mkf_status mkf_unload_event(mkf_ctx *ctx, int32_t handle)
{
    if (!ctx) return fail(MKF_E_INVALID, "NULL context");
    auto it = ctx->events.find(handle);
    if (it == ctx->events.end()) return fail(MKF_E_NOTFOUND, "unknown event handle %d", handle);
    MKF_HIP(hipStreamSynchronize(ctx->stream));
    drop_graphs_with(ctx, handle);
    destroy_event(ctx, it->second.get());
    ctx->events.erase(it);
    return MKF_OK;
}

static mkf_status reindex_if_needed(mkf_ctx *ctx, const std::vector<EventRec *> &recs, bool *any)
{
    *any = false;
    for (EventRec *r : recs) {
        bool rebuilt = false;
        mkf_status st = ensure_index(ctx, r, &rebuilt, ctx->stream);
        if (st != MKF_OK) return st;
        if (rebuilt) {
            if ((st = upload_view(r, ctx->stream)) != MKF_OK) return st;
            drop_graphs_with(ctx, -1);
            *any = true;
        }
    }
    return MKF_OK;
}

mkf_status mkf_build(mkf_ctx *ctx, int32_t handle, mkf_tracks *out)
{
    if (!ctx) return fail(MKF_E_INVALID, "NULL context");
    EventRec *rec = find_event(ctx, handle);
    if (!rec) return fail(MKF_E_NOTFOUND, "unknown event handle %d", handle);
    mkf_status st = check_tracks(out, rec->shape.n_seeds, "build");
    if (st != MKF_OK) return st;
    std::vector<EventRec *> one{rec};
    bool need_index = false;
    if ((st = reindex_if_needed(ctx, one, &need_index)) != MKF_OK) return st;
    const int G = ctx->tuning.lanes_per_seed, wpb = ctx->tuning.waves_per_block;
    if (need_index) {
        if ((st = ensure_batch_scratch(ctx, 1)) != MKF_OK) return st;
        BatchArgs args{};
        if ((st = stage_batch(ctx, one, ctx->batch_dev, ctx->batch_host, seeds_per_item(G), &args, ctx->stream)) !=
            MKF_OK)
            return st;
        MKF_HIP(launch_index(ctx->params, args, ctx->stream));
    }
    if (rec->plain_G != G || !rec->plain) {
        if (rec->plain) MKF_HIP(hipStreamSynchronize(ctx->stream));
        drop_plain_graph(rec);
        rec->heap->release(rec->plain);
        const int slots = plain_slots(rec->shape.n_seeds, G);
        const size_t bytes = carve_plain(rec->shape, slots, nullptr, &rec->view);
        rec->plain = rec->heap->alloc(bytes);
        if (!rec->plain) {
            rec->plain_G = 0;
            return fail(MKF_E_NOMEM, "builder state: %zu bytes", bytes);
        }
        carve_plain(rec->shape, slots, rec->plain, &rec->view);
        rec->plain_G = G;
        if ((st = upload_view(rec, ctx->stream)) != MKF_OK) return st;
    }
    const int n_launch = rec->shape.n_layers - rec->shape.n_seed_layers;
    if (rec->shape.n_seeds > 0) {
        if (!rec->plain_graph || rec->plain_graph_G != G || rec->plain_graph_wpb != wpb) {
            drop_plain_graph(rec);
            hipGraph_t graph = nullptr;
            MKF_HIP(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
            hipError_t cap = hipSuccess;
            for (int L = rec->shape.n_seed_layers; L < rec->shape.n_layers && cap == hipSuccess; ++L)
                cap = launch_build_layer(ctx->params, rec->dev_view, rec->view, L, G, wpb, false, ctx->stream);
            hipError_t end = hipStreamEndCapture(ctx->stream, &graph);
            if (cap != hipSuccess || end != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return fail(MKF_E_DEVICE, "capturing the layer loop: %s",
                            hipGetErrorString(cap != hipSuccess ? cap : end));
            }
            hipError_t ins = hipGraphInstantiate(&rec->plain_graph, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ins != hipSuccess) return fail(MKF_E_DEVICE, "instantiating the layer loop: %s", hipGetErrorString(ins));
            rec->plain_graph_G = G;
            rec->plain_graph_wpb = wpb;
        }
        timer_begin(ctx, 0, ctx->stream);
        MKF_HIP(hipGraphLaunch(rec->plain_graph, ctx->stream));
        timer_end(ctx, 0, ctx->stream, n_launch);
    }
    if (out && (st = copy_tracks_out(ctx, rec, out, ctx->stream)) != MKF_OK) return st;
    MKF_HIP(hipStreamSynchronize(ctx->stream));
    timers_collect(ctx, true);
    finish_ndof(out);
    return MKF_OK;
}

mkf_status mkf_build_batch(mkf_ctx *ctx, const int32_t *handles, int32_t n, uint32_t flags, mkf_tracks *outs)
{
    if (!ctx) return fail(MKF_E_INVALID, "NULL context");
    if (flags & ~(MKF_BATCH_REINDEX | MKF_BATCH_STATS | MKF_BATCH_GRAPH | MKF_BATCH_ASYNC | MKF_BATCH_FIT |
                  MKF_BATCH_BEAM))
        return fail(MKF_E_INVALID, "unknown flags");
    const bool beam = flags & MKF_BATCH_BEAM;
    const bool async = flags & MKF_BATCH_ASYNC;
    flags &= ~MKF_BATCH_ASYNC;
    if (async && outs) return fail(MKF_E_INVALID, "an asynchronous batch returns no host outputs (outs must be NULL)");
    std::vector<EventRec *> recs;
    mkf_status st = gather_events(ctx, handles, n, &recs);
    if (st != MKF_OK) return st;
    if (outs)
        for (int i = 0; i < n; ++i)
            if ((st = check_tracks(&outs[i], recs[i]->shape.n_seeds, "build_batch")) != MKF_OK) return st;
    if (n == 0) return MKF_OK;
    if (beam)
        for (EventRec *r : recs)
            if ((st = ensure_beam(ctx, r)) != MKF_OK) return st;
    bool need_index = false;
    if ((st = reindex_if_needed(ctx, recs, &need_index)) != MKF_OK) return st;
    if (need_index) flags |= MKF_BATCH_REINDEX;
    const int spi = seeds_per_item(ctx->tuning.lanes_per_seed);
    if (flags & MKF_BATCH_GRAPH) {
        BatchGraph *bg = nullptr;
        std::vector<int32_t> key(handles, handles + n);
        for (auto &g : ctx->graphs)
            if (g->handles == key && g->flags == flags && std::memcmp(&g->tuning, &ctx->tuning, sizeof(mkf_tuning)) == 0)
                bg = g.get();
        if (!bg) {
            auto g = std::make_unique<BatchGraph>();
            g->handles = key;
            g->flags = flags;
            g->tuning = ctx->tuning;
            g->scratch = ctx->heap.alloc(batch_scratch_bytes(n));
            if (!g->scratch) return fail(MKF_E_NOMEM, "graph scratch");
            if ((st = ensure_batch_scratch(ctx, n)) != MKF_OK) {
                ctx->heap.release(g->scratch);
                return st;
            }
            BatchArgs args{};
            if ((st = stage_batch(ctx, recs, g->scratch, ctx->batch_host, spi, &args, ctx->stream, beam)) != MKF_OK) {
                ctx->heap.release(g->scratch);
                return st;
            }
            hipError_t e = hipStreamSynchronize(ctx->stream);
            if (e != hipSuccess) {
                ctx->heap.release(g->scratch);
                return fail(MKF_E_DEVICE, "staging: %s", hipGetErrorString(e));
            }
            hipGraph_t graph = nullptr;
            MKF_HIP(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
            mkf_status cst = run_pipeline(ctx, args, recs, flags, false, ctx->stream);
            hipError_t end = hipStreamEndCapture(ctx->stream, &graph);
            if (cst != MKF_OK || end != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                ctx->heap.release(g->scratch);
                return cst != MKF_OK ? cst : fail(MKF_E_DEVICE, "capture: %s", hipGetErrorString(end));
            }
            hipError_t ins = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ins != hipSuccess) {
                ctx->heap.release(g->scratch);
                return fail(MKF_E_DEVICE, "instantiate: %s", hipGetErrorString(ins));
            }
            bg = g.get();
            ctx->graphs.push_back(std::move(g));
        }
        timer_begin(ctx, 0, ctx->stream);
        MKF_HIP(hipGraphLaunch(bg->exec, ctx->stream));
        timer_end(ctx, 0, ctx->stream, 1);
    } else {
        if ((st = ensure_batch_scratch(ctx, n)) != MKF_OK) return st;
        BatchArgs args{};
        if ((st = stage_batch(ctx, recs, ctx->batch_dev, ctx->batch_host, spi, &args, ctx->stream, beam)) != MKF_OK)
            return st;
        if ((st = run_pipeline(ctx, args, recs, flags, true, ctx->stream)) != MKF_OK) return st;
    }
    if (async) {
        timers_collect(ctx, false);
        return MKF_OK;
    }
    if (outs)
        for (int i = 0; i < n; ++i)
            if ((st = copy_tracks_out(ctx, recs[i], &outs[i], ctx->stream)) != MKF_OK) return st;
    MKF_HIP(hipStreamSynchronize(ctx->stream));
    timers_collect(ctx, true);
    if (outs)
        for (int i = 0; i < n; ++i) finish_ndof(&outs[i]);
    return MKF_OK;
}

mkf_status mkf_build_batch_noalloc(mkf_ctx *ctx, const int32_t *handles, int32_t n, uint32_t flags,
                                   mkf_tracks *outs)
{
    if (!ctx) return fail(MKF_E_INVALID, "NULL context");
    if (flags & ~(MKF_BATCH_REINDEX | MKF_BATCH_STATS | MKF_BATCH_ASYNC | MKF_BATCH_FIT))
        return fail(MKF_E_INVALID, "only MKF_BATCH_REINDEX, _STATS, _ASYNC and _FIT build without allocating");
    const bool async = flags & MKF_BATCH_ASYNC;
    flags &= ~MKF_BATCH_ASYNC;
    if (async && outs) return fail(MKF_E_INVALID, "an asynchronous batch returns no host outputs (outs must be NULL)");
    if (n < 0 || (n > 0 && !handles)) return fail(MKF_E_INVALID, "bad handle list");
    if (n > kNoAllocMaxEvents)
        return fail(MKF_E_INVALID, "%d events: the no-allocation builder takes at most %d", n, kNoAllocMaxEvents);
    if ((long long)n * ctx->cfg.n_layers > 65535)
        return fail(MKF_E_INVALID, "at most %d events per batch", 65535 / ctx->cfg.n_layers);
    char *dev = static_cast<char *>(noalloc_scratch(ctx->device));
    if (!dev) return fail(MKF_E_DEVICE, "no descriptor array on device %d", ctx->device);
    EventRec *recs[kNoAllocMaxEvents];
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < i; ++j)
            if (handles[j] == handles[i]) return fail(MKF_E_INVALID, "an event appears twice in the batch");
        recs[i] = find_event(ctx, handles[i]);
        if (!recs[i]) return fail(MKF_E_NOTFOUND, "unknown event handle %d", handles[i]);
        if (!recs[i]->index || recs[i]->index_bins_phi != ctx->tuning.bins_phi ||
            recs[i]->index_bins_z != ctx->tuning.bins_z)
            return fail(MKF_E_STATE, "event %d has no index for the current bin grid (mkf_build_batch makes one)",
                        handles[i]);
        if (outs && outs[i].n != recs[i]->shape.n_seeds)
            return fail(MKF_E_INVALID, "build_batch_noalloc: output has %d rows, need %d", outs[i].n,
                        recs[i]->shape.n_seeds);
    }
    if (n == 0) return MKF_OK;
    // the descriptors go through one host image and the device array of this
    // GPU; earlier work of this context may still read the array
    static std::mutex image_mu;
    static char image[kNoAllocScratchBytes];
    MKF_HIP(hipStreamSynchronize(ctx->stream));
    BatchArgs args{};
    {
        std::lock_guard<std::mutex> lk(image_mu);
        mkf_status st = compose_batch(recs, n, seeds_per_item(ctx->tuning.lanes_per_seed), false, image, dev, &args);
        if (st != MKF_OK) return st;
        MKF_HIP(hipMemcpyAsync(dev, image, batch_scratch_bytes(n), hipMemcpyHostToDevice, ctx->stream));
        MKF_HIP(hipStreamSynchronize(ctx->stream));
    }
    mkf_status st = run_pipeline_with(ctx, ctx->params, ctx->tuning, args, flags, true, ctx->stream);
    if (st != MKF_OK) return st;
    if (async) {
        timers_collect(ctx, false);
        return MKF_OK;
    }
    if (outs)
        for (int i = 0; i < n; ++i)
            if ((st = copy_tracks_out(ctx, recs[i], &outs[i], ctx->stream)) != MKF_OK) return st;
    MKF_HIP(hipStreamSynchronize(ctx->stream));
    timers_collect(ctx, true);
    if (outs)
        for (int i = 0; i < n; ++i) finish_ndof(&outs[i]);
    return MKF_OK;
}

mkf_status mkf_fetch_tracks(mkf_ctx *ctx, int32_t handle, mkf_tracks *out)
{
    if (!ctx || !out) return fail(MKF_E_INVALID, "NULL argument");
    EventRec *rec = find_event(ctx, handle);
    if (!rec) return fail(MKF_E_NOTFOUND, "unknown event handle %d", handle);
    mkf_status st = check_tracks(out, rec->shape.n_seeds, "fetch");
    if (st != MKF_OK) return st;
    if ((st = copy_tracks_out(ctx, rec, out, ctx->stream)) != MKF_OK) return st;
    MKF_HIP(hipStreamSynchronize(ctx->stream));
    finish_ndof(out);
    return MKF_OK;
}

mkf_status mkf_fetch_fit(mkf_ctx *ctx, int32_t handle, mkf_tracks *out)
{
    if (!ctx || !out) return fail(MKF_E_INVALID, "NULL argument");
    EventRec *rec = find_event(ctx, handle);
    if (!rec) return fail(MKF_E_NOTFOUND, "unknown event handle %d", handle);
    mkf_status st = check_tracks(out, rec->shape.n_seeds, "fetch_fit");
    if (st != MKF_OK) return st;
    const DevEvent &v = rec->view;
    const size_t n = (size_t)rec->shape.n_seeds, nl = (size_t)rec->shape.n_layers;
    hipStream_t s = ctx->stream;
    if ((st = copy_d2h(out->par, v.rf_par, 48 * n, s)) != MKF_OK || (st = copy_d2h(out->cov, v.rf_cov, 168 * n, s)) != MKF_OK ||
        (st = copy_d2h(out->hits, v.out_hits, 4 * nl * n, s)) != MKF_OK ||
        (st = copy_d2h(out->n_hits, v.rf_nupd, 4 * n, s)) != MKF_OK ||
        (st = copy_d2h(out->n_holes, v.out_nholes, 4 * n, s)) != MKF_OK ||
        (st = copy_d2h(out->chi2, v.rf_chi2, 8 * n, s)) != MKF_OK ||
        (st = copy_d2h(out->status, v.rf_status, 4 * n, s)) != MKF_OK ||
        (st = copy_d2h(out->ndof, v.rf_nupd, 4 * n, s)) != MKF_OK)
        return st;
    MKF_HIP(hipStreamSynchronize(ctx->stream));
    finish_ndof(out);
    return MKF_OK;
}

mkf_status mkf_fetch_beam(mkf_ctx *ctx, int32_t handle, mkf_tracks *out)
{
    if (!ctx || !out) return fail(MKF_E_INVALID, "NULL argument");
    EventRec *rec = find_event(ctx, handle);
    if (!rec) return fail(MKF_E_NOTFOUND, "unknown event handle %d", handle);
    if (!rec->beam) return fail(MKF_E_STATE, "no build of this event kept its beam (MKF_BATCH_BEAM)");
    const size_t n = (size_t)rec->shape.n_seeds * ctx->cfg.max_cands, nl = (size_t)rec->shape.n_layers;
    mkf_status st = check_tracks(out, (int)n, "fetch_beam");
    if (st != MKF_OK) return st;
    const DevEvent &v = rec->beam_view;
    hipStream_t s = ctx->stream;
    if ((st = copy_d2h(out->par, v.beam_par, 48 * n, s)) != MKF_OK ||
        (st = copy_d2h(out->cov, v.beam_cov, 168 * n, s)) != MKF_OK ||
        (st = copy_d2h(out->hits, v.beam_hits, 4 * nl * n, s)) != MKF_OK ||
        (st = copy_d2h(out->n_hits, v.beam_nhits, 4 * n, s)) != MKF_OK ||
        (st = copy_d2h(out->n_holes, v.beam_nholes, 4 * n, s)) != MKF_OK ||
        (st = copy_d2h(out->chi2, v.beam_chi2, 8 * n, s)) != MKF_OK ||
        (st = copy_d2h(out->status, v.beam_status, 4 * n, s)) != MKF_OK ||
        (st = copy_d2h(out->ndof, v.beam_nhits, 4 * n, s)) != MKF_OK)
        return st;
    MKF_HIP(hipStreamSynchronize(ctx->stream));
    if (out->ndof)
        for (size_t i = 0; i < n; ++i) out->ndof[i] = out->status && out->status[i] < 0 ? 0 : 2 * out->ndof[i] - 5;
    return MKF_OK;
}

mkf_status mkf_index_grid(mkf_ctx *ctx, int32_t handle, int32_t *bins_phi, int32_t *bins_z)
{
    if (!ctx || !bins_phi || !bins_z) return fail(MKF_E_INVALID, "NULL argument");
    EventRec *rec = find_event(ctx, handle);
    if (!rec) return fail(MKF_E_NOTFOUND, "unknown event handle %d", handle);
    if (!rec->index || rec->index_bins_phi != ctx->tuning.bins_phi || rec->index_bins_z != ctx->tuning.bins_z)
        return fail(MKF_E_STATE, "the index was built for another bin grid");
    *bins_phi = rec->index_bins_phi >> rec->view.grid_k;
    *bins_z = rec->index_bins_z >> rec->view.grid_k;
    return MKF_OK;
}

mkf_status mkf_fetch_index(mkf_ctx *ctx, int32_t handle, int32_t layer, int32_t *bin_off, int32_t *bin_of,
                           int32_t *order)
{
    if (!ctx) return fail(MKF_E_INVALID, "NULL context");
    EventRec *rec = find_event(ctx, handle);
    if (!rec) return fail(MKF_E_NOTFOUND, "unknown event handle %d", handle);
    if (layer < 0 || layer >= rec->shape.n_layers) return fail(MKF_E_INVALID, "layer %d out of range", layer);
    if (!rec->index || rec->index_bins_phi != ctx->tuning.bins_phi || rec->index_bins_z != ctx->tuning.bins_z)
        return fail(MKF_E_STATE, "the index was built for another bin grid");
    const int k = rec->view.grid_k;
    const int nb = (ctx->tuning.bins_phi >> k) * (ctx->tuning.bins_z >> k);
    const int h0 = rec->shape.layer_off[layer], n = rec->shape.layer_off[layer + 1] - h0;
    const DevEvent &v = rec->view;
    std::vector<int32_t> off(bin_off ? nb + 1 : 0);
    std::vector<float4> binned(order ? n : 0);
    hipStream_t s = ctx->stream;
    if (bin_off)
        MKF_HIP(hipMemcpyAsync(off.data(), v.bin_off + (size_t)layer * bin_off_stride(nb), 4 * (size_t)(nb + 1),
                               hipMemcpyDeviceToHost, s));
    if (bin_of && n) MKF_HIP(hipMemcpyAsync(bin_of, v.bin_of + h0, 4 * (size_t)n, hipMemcpyDeviceToHost, s));
    if (order && n) MKF_HIP(hipMemcpyAsync(binned.data(), v.binned + h0, sizeof(float4) * (size_t)n,
                                           hipMemcpyDeviceToHost, s));
    MKF_HIP(hipStreamSynchronize(s));
    if (bin_off)
        for (int i = 0; i <= nb; ++i) bin_off[i] = off[i] - h0;
    if (order)
        for (int i = 0; i < n; ++i) {
            int32_t id;
            std::memcpy(&id, &binned[i].w, 4);
            order[i] = id;
        }
    return MKF_OK;
}

mkf_status mkf_get_stats(mkf_ctx *ctx, int32_t handle, mkf_build_stats *out)
{
    if (!ctx || !out) return fail(MKF_E_INVALID, "NULL argument");
    EventRec *rec = find_event(ctx, handle);
    if (!rec) return fail(MKF_E_NOTFOUND, "unknown event handle %d", handle);
    unsigned long long v[5];
    MKF_HIP(hipMemcpyAsync(v, rec->view.stats, sizeof(v), hipMemcpyDeviceToHost, ctx->stream));
    MKF_HIP(hipStreamSynchronize(ctx->stream));
    out->cand_layers = (int64_t)v[0];
    out->chi2_evals = (int64_t)v[1];
    out->accepted = (int64_t)v[2];
    out->updates = (int64_t)v[3];
    out->hits_scanned = (int64_t)v[4];
    return MKF_OK;
}

static mkf_status copy_fit_out(const EventRec *rec, const DevEvent &v, const mkf_tracks *out, hipStream_t s)
{
    const size_t n = (size_t)rec->shape.n_tracks, nl = (size_t)rec->shape.n_layers;
    mkf_status st;
    if ((st = copy_d2h(out->par, v.fit_par, 48 * n, s)) != MKF_OK) return st;
    if ((st = copy_d2h(out->cov, v.fit_cov, 168 * n, s)) != MKF_OK) return st;
    if ((st = copy_d2h(out->hits, v.track_hits, 4 * nl * n, s)) != MKF_OK) return st;
    if ((st = copy_d2h(out->n_hits, v.fit_nupd, 4 * n, s)) != MKF_OK) return st;
    if ((st = copy_d2h(out->n_holes, v.fit_nupd, 4 * n, s)) != MKF_OK) return st;
    if ((st = copy_d2h(out->chi2, v.fit_chi2, 8 * n, s)) != MKF_OK) return st;
    if ((st = copy_d2h(out->status, v.fit_status, 4 * n, s)) != MKF_OK) return st;
    if ((st = copy_d2h(out->ndof, v.fit_nupd, 4 * n, s)) != MKF_OK) return st;
    return MKF_OK;
}

static void finish_fit_out(const mkf_tracks *out, int n_layers)
{
    if (!out) return;
    for (int i = 0; i < out->n; ++i) {
        if (out->n_holes) out->n_holes[i] = n_layers - out->n_holes[i];
        if (out->ndof) out->ndof[i] = 2 * out->ndof[i] - 5;
    }
}

mkf_status mkf_fit_batch(mkf_ctx *ctx, const int32_t *handles, int32_t n, mkf_tracks *outs)
{
    if (!ctx) return fail(MKF_E_INVALID, "NULL context");
    std::vector<EventRec *> recs;
    mkf_status st = gather_events(ctx, handles, n, &recs);
    if (st != MKF_OK) return st;
    if (outs)
        for (int i = 0; i < n; ++i)
            if ((st = check_tracks(&outs[i], recs[i]->shape.n_tracks, "fit_batch")) != MKF_OK) return st;
    if (n == 0) return MKF_OK;
    if ((st = ensure_batch_scratch(ctx, n)) != MKF_OK) return st;
    BatchArgs args{};
    if ((st = stage_batch(ctx, recs, ctx->batch_dev, ctx->batch_host, seeds_per_item(ctx->tuning.lanes_per_seed),
                          &args, ctx->stream)) != MKF_OK)
        return st;
    timer_begin(ctx, 2, ctx->stream);
    MKF_HIP(launch_fit(ctx->params, args, ctx->stream));
    timer_end(ctx, 2, ctx->stream, 1);
    if (outs)
        for (int i = 0; i < n; ++i)
            if ((st = copy_fit_out(recs[i], recs[i]->view, &outs[i], ctx->stream)) != MKF_OK) return st;
    MKF_HIP(hipStreamSynchronize(ctx->stream));
    timers_collect(ctx, true);
    if (outs)
        for (int i = 0; i < n; ++i) finish_fit_out(&outs[i], recs[i]->shape.n_layers);
    return MKF_OK;
}

mkf_status mkf_fit(mkf_ctx *ctx, int32_t handle, int32_t n_tracks, const double *init_par, const double *init_cov,
                   const int32_t *track_hits, mkf_tracks *out)
{
    if (!ctx) return fail(MKF_E_INVALID, "NULL context");
    EventRec *rec = find_event(ctx, handle);
    if (!rec) return fail(MKF_E_NOTFOUND, "unknown event handle %d", handle);
    mkf_status st = check_tracks(out, n_tracks, "fit");
    if (st != MKF_OK) return st;
    if (n_tracks < 0) return fail(MKF_E_INVALID, "negative track count");
    if (n_tracks > 0 && (!init_par || !init_cov || !track_hits)) return fail(MKF_E_INVALID, "track arrays are NULL");
    if (n_tracks == 0) return MKF_OK;
    // a temporary event view: the loaded event's hits with these tracks, whose
    // inputs are checked and narrowed to FP32 in the load staging and copied
    // in one piece
    EventShape ts = rec->shape;
    ts.n_seeds = 0;
    ts.n_tracks = n_tracks;
    const size_t nt = (size_t)n_tracks, nl = (size_t)ts.n_layers;
    auto layout = [&](char *base, DevEvent *v) {
        size_t o = 0;
        auto take = [&](size_t b) {
            char *p = base + o;
            o = (o + b + 255) & ~size_t(255);
            return p;
        };
        v->track_par = reinterpret_cast<float *>(take(24 * nt));
        v->track_cov = reinterpret_cast<float *>(take(84 * nt));
        v->track_hits = reinterpret_cast<int *>(take(4 * nl * nt));
        const size_t inputs = o;
        v->fit_par = reinterpret_cast<double *>(take(48 * nt));
        v->fit_cov = reinterpret_cast<double *>(take(168 * nt));
        v->fit_chi2 = reinterpret_cast<double *>(take(8 * nt));
        v->fit_nupd = reinterpret_cast<int *>(take(4 * nt));
        v->fit_status = reinterpret_cast<int *>(take(4 * nt));
        return std::make_pair(inputs, o);
    };
    DevEvent hv{};
    const auto sizes = layout(nullptr, &hv);
    if (ctx->load_pin_bytes < sizes.first) {
        if (ctx->load_pin) (void)hipHostFree(ctx->load_pin);
        ctx->load_pin = nullptr;
        ctx->load_pin_bytes = 0;
        MKF_HIP(hipHostMalloc(&ctx->load_pin, sizes.first, hipHostMallocDefault));
        ctx->load_pin_bytes = sizes.first;
    }
    layout(static_cast<char *>(ctx->load_pin), &hv);
    std::vector<int32_t> nh(nl);
    for (size_t L = 0; L < nl; ++L) nh[L] = rec->shape.layer_off[L + 1] - rec->shape.layer_off[L];
    for (int i = 0; i < n_tracks; ++i) {
        int bad_hit = 0;
        if (!pack_state(init_par + 6 * (size_t)i, init_cov + 21 * (size_t)i, const_cast<float *>(hv.track_par) + 6 * (size_t)i,
                        const_cast<float *>(hv.track_cov) + 21 * (size_t)i, track_hits + (size_t)i * nl,
                        const_cast<int *>(hv.track_hits) + (size_t)i * nl, (int)nl, nh.data(), &bad_hit))
            return fail(MKF_E_INVALID, bad_hit ? "track %d: hit index out of range"
                                               : "track %d: state or covariance not finite (in FP32), theta "
                                                 "outside (0, pi) or position on the axis", i);
    }
    char *buf = static_cast<char *>(ctx->heap.alloc(sizes.second + sizeof(DevEvent) + 256));
    if (!buf) return fail(MKF_E_NOMEM, "fit buffers: %zu bytes", sizes.second);
    DevEvent v = rec->view;
    v.n_seeds = 0;
    v.n_tracks = n_tracks;
    layout(buf, &v);
    auto cleanup = [&](mkf_status s) {
        (void)hipStreamSynchronize(ctx->stream);
        ctx->heap.release(buf);
        return s;
    };
    hipStream_t s = ctx->stream;
    if (hipMemcpyAsync(buf, ctx->load_pin, sizes.first, hipMemcpyHostToDevice, s) != hipSuccess)
        return cleanup(fail(MKF_E_DEVICE, "fit upload failed"));
    if ((st = ensure_batch_scratch(ctx, 1)) != MKF_OK) return cleanup(st);
    EventRec tmp;
    tmp.shape = ts;
    tmp.view = v;
    std::vector<EventRec *> one{&tmp};
    BatchArgs args{};
    if ((st = stage_batch(ctx, one, ctx->batch_dev, ctx->batch_host, 64, &args, s)) != MKF_OK) return cleanup(st);
    timer_begin(ctx, 2, s);
    hipError_t e = launch_fit(ctx->params, args, s);
    timer_end(ctx, 2, s, 1);
    if (e != hipSuccess) return cleanup(fail(MKF_E_DEVICE, "fit launch: %s", hipGetErrorString(e)));
    if (out && (st = copy_fit_out(&tmp, v, out, s)) != MKF_OK) return cleanup(st);
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return cleanup(fail(MKF_E_DEVICE, "fit: %s", hipGetErrorString(e)));
    timers_collect(ctx, true);
    finish_fit_out(out, ts.n_layers);
    return cleanup(MKF_OK);
}

mkf_status mkf_timer_read(mkf_ctx *ctx, int32_t which, double *total_ms, int64_t *launches)
{
    if (!ctx || which < 0 || which > 2) return fail(MKF_E_INVALID, "bad timer");
    MKF_HIP(hipStreamSynchronize(ctx->stream));
    timers_collect(ctx, true);
    if (total_ms) *total_ms = ctx->timers[which].total_ms;
    if (launches) *launches = ctx->timers[which].launches;
    return MKF_OK;
}

mkf_status mkf_timer_reset(mkf_ctx *ctx)
{
    if (!ctx) return fail(MKF_E_INVALID, "NULL context");
    MKF_HIP(hipStreamSynchronize(ctx->stream));
    timers_collect(ctx, true);
    for (auto &t : ctx->timers) {
        t.total_ms = 0;
        t.launches = 0;
    }
    return MKF_OK;
}

mkf_status mkf_sync(mkf_ctx *ctx)
{
    if (!ctx) return fail(MKF_E_INVALID, "NULL context");
    MKF_HIP(hipStreamSynchronize(ctx->stream));
    timers_collect(ctx, true);
    return MKF_OK;
}

mkf_status mkf_autotune(mkf_ctx *ctx, const int32_t *handles, int32_t n, mkf_tuning *best)
{
    if (!ctx) return fail(MKF_E_INVALID, "NULL context");
    std::vector<EventRec *> recs;
    mkf_status st = gather_events(ctx, handles, n, &recs);
    if (st != MKF_OK) return st;
    if (n == 0) return fail(MKF_E_INVALID, "no events to tune on");
    const mkf_tuning start = ctx->tuning;
    auto measure = [&](const mkf_tuning &t, double *ms) -> mkf_status {
        mkf_status s2 = mkf_set_tuning(ctx, &t);
        if (s2 != MKF_OK) return s2;
        s2 = mkf_build_batch(ctx, handles, n, MKF_BATCH_REINDEX, nullptr);
        if (s2 != MKF_OK) return s2;
        double best_ms = 1e30;
        for (int rep = 0; rep < 3; ++rep) {
            MKF_HIP(hipStreamSynchronize(ctx->stream));
            const auto t0 = std::chrono::steady_clock::now();
            s2 = mkf_build_batch(ctx, handles, n, MKF_BATCH_REINDEX, nullptr);
            if (s2 != MKF_OK) return s2;
            const auto t1 = std::chrono::steady_clock::now();
            best_ms = std::min(best_ms, std::chrono::duration<double, std::milli>(t1 - t0).count());
        }
        *ms = best_ms;
        return MKF_OK;
    };
    mkf_tuning cur = start;
    double cur_ms = 0;
    if ((st = measure(cur, &cur_ms)) != MKF_OK) return st;
    std::vector<int> lanes;
    for (int G : {1, 2, 4, 6, 8})
        if (G >= ctx->cfg.max_cands) lanes.push_back(G);
    const std::vector<int> waves = {1, 2, 4};
    const std::vector<int> bphi = {128, 256, 512, 1024, 2048};
    const std::vector<int> bz = {4, 8, 16, 32, 64};
    const std::vector<int> pers = {0, 1};
    const std::vector<int> bpc = {2, 4, 8, 16};
    for (int pass = 0; pass < 2; ++pass) {
        for (int dim = 0; dim < 6; ++dim) {
            const std::vector<int> &vals = dim == 0 ? lanes : dim == 1 ? waves : dim == 2 ? bphi : dim == 3 ? bz
                                                                                        : dim == 4 ? pers : bpc;
            for (int v : vals) {
                mkf_tuning t = cur;
                int *field = dim == 0 ? &t.lanes_per_seed : dim == 1 ? &t.waves_per_block : dim == 2 ? &t.bins_phi
                             : dim == 3 ? &t.bins_z : dim == 4 ? &t.persistent : &t.blocks_per_cu;
                if (*field == v) continue;
                *field = v;
                double ms = 0;
                if (measure(t, &ms) != MKF_OK) continue;
                if (ms < cur_ms * 0.98) {
                    cur = t;
                    cur_ms = ms;
                }
            }
        }
    }
    if ((st = mkf_set_tuning(ctx, &cur)) != MKF_OK) return st;
    if (best) *best = ctx->tuning;
    return MKF_OK;
}

mkf_status mkf_calib_copy(mkf_ctx *ctx, const void *src_dev, void *dst_dev, size_t bytes)
{
    if (!ctx || !src_dev || !dst_dev || bytes % 16) return fail(MKF_E_INVALID, "bad copy arguments");
    MKF_HIP(launch_copy(src_dev, dst_dev, bytes, ctx->stream));
    MKF_HIP(hipStreamSynchronize(ctx->stream));
    return MKF_OK;
}

mkf_status mkf_calib_fma(mkf_ctx *ctx, float *dst_dev, int32_t n_blocks, int32_t iters, double *ms, double *flop)
{
    if (!ctx || !dst_dev || n_blocks < 1 || iters < 4 || iters % 4 || !ms || !flop)
        return fail(MKF_E_INVALID, "bad FMA calibration arguments");
    hipEvent_t ev[2] = {nullptr, nullptr};
    MKF_HIP(hipEventCreate(&ev[0]));
    hipError_t e = hipEventCreate(&ev[1]);
    if (e == hipSuccess) e = hipEventRecord(ev[0], ctx->stream);
    if (e == hipSuccess) e = launch_calib_fma(dst_dev, n_blocks, iters, ctx->stream);
    if (e == hipSuccess) e = hipEventRecord(ev[1], ctx->stream);
    if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, ev[0], ev[1]);
    hipEventDestroy(ev[0]);
    if (ev[1]) hipEventDestroy(ev[1]);
    MKF_HIP(e);
    *ms = t;
    *flop = 2.0 * calib_fma_chains() * (double)iters * 256.0 * (double)n_blocks;
    return MKF_OK;
}

}  // extern "C"
