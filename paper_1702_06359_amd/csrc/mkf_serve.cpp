// Serving: continuous batching of events as they arrive.
//
// Submit copies an event into pinned host staging and queues a ticket.  A
// scheduler thread admits queued tickets in arrival order while the device
// budget (a slab reserved once, sub-allocated first-fit) and the in-flight
// limit allow, uploads them, builds their hit indices and runs one batched
// build for everything admitted together, on one of several streams, so that
// batches admitted later overlap the ones still on the device.  Results come
// back through pinned staging; the scheduler marks a ticket done when it
// observes its batch's completion event.
#include "mkf_runtime.hpp"

#include <chrono>
#include <cstring>

namespace mkf {

namespace {

using Clock = std::chrono::steady_clock;
constexpr int kStreams = 4;

// Reuses pinned host buffers by power-of-two size class.
class PinnedPool {
  public:
    void *get(size_t bytes, size_t *cls)
    {
        size_t c = 4096;
        while (c < bytes) c <<= 1;
        *cls = c;
        {
            std::lock_guard<std::mutex> lk(mu_);
            auto it = free_.find(c);
            if (it != free_.end() && !it->second.empty()) {
                void *p = it->second.back();
                it->second.pop_back();
                return p;
            }
        }
        void *p = nullptr;
        if (hipHostMalloc(&p, c, hipHostMallocDefault) != hipSuccess) return nullptr;
        return p;
    }
    void put(void *p, size_t cls)
    {
        if (!p) return;
        std::lock_guard<std::mutex> lk(mu_);
        free_[cls].push_back(p);
    }
    ~PinnedPool()
    {
        for (auto &kv : free_)
            for (void *p : kv.second) (void)hipHostFree(p);
    }

  private:
    std::mutex mu_;
    std::map<size_t, std::vector<void *>> free_;
};

struct Ticket {
    uint64_t id = 0;
    EventShape shape;
    mkf_tracks out{};
    void *in_pin = nullptr;
    size_t in_cls = 0;
    void *out_pin = nullptr;
    size_t out_cls = 0;
    size_t dev_bytes = 0;
    Clock::time_point t_submit, t_done;
    int state = 0;    // 0 queued, 1 running, 2 done
    mkf_status status = MKF_OK;
    std::unique_ptr<EventRec> rec;
};

// byte offsets of one event inside its pinned input staging
struct InLayout {
    size_t hits, seed_par, seed_cov, seed_hits, total;
};

InLayout in_layout(const EventShape &s)
{
    InLayout l{};
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off = (off + b + 255) & ~size_t(255);
        return o;
    };
    l.hits = take(24 * (size_t)s.n_hits());
    l.seed_par = take(48 * (size_t)s.n_seeds);
    l.seed_cov = take(168 * (size_t)s.n_seeds);
    l.seed_hits = take(4 * (size_t)s.n_seed_layers * s.n_seeds);
    l.total = off;
    return l;
}

struct OutLayout {
    size_t par, cov, hits, nhits, nholes, chi2, status, total;
};

OutLayout out_layout(const EventShape &s)
{
    OutLayout l{};
    size_t off = 0;
    const size_t n = (size_t)s.n_seeds;
    auto take = [&](size_t b) {
        const size_t o = off;
        off = (off + b + 255) & ~size_t(255);
        return o;
    };
    l.par = take(48 * n);
    l.cov = take(168 * n);
    l.hits = take(4 * (size_t)s.n_layers * n);
    l.nhits = take(4 * n);
    l.nholes = take(4 * n);
    l.chi2 = take(8 * n);
    l.status = take(4 * n);
    l.total = off;
    return l;
}

struct Running {
    std::vector<Ticket *> tickets;
    int stream = 0;
    hipEvent_t done = nullptr;
    void *scratch_dev = nullptr;
    void *scratch_host = nullptr;
    size_t scratch_cls = 0;
};

}  // namespace

struct Server {
    mkf_ctx *ctx = nullptr;
    void *slab_base = nullptr;
    std::unique_ptr<SlabHeap> slab;
    int max_in_flight = 0;
    int max_batch = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Ticket *> pending;
    std::unordered_map<uint64_t, std::unique_ptr<Ticket>> tickets;
    std::vector<Running> running;
    int in_flight = 0;
    bool stop = false;
    uint64_t next_id = 1;
    hipStream_t streams[kStreams] = {};
    bool stream_busy[kStreams] = {};
    PinnedPool pinned;
    std::thread thr;

    size_t footprint(const EventShape &s) const
    {
        return event_data_bytes(s) + event_index_bytes(s, ctx->tuning.bins_phi * ctx->tuning.bins_z) + 4096;
    }

    void finish_batch(Running &b)
    {
        for (Ticket *t : b.tickets) {
            const OutLayout ol = out_layout(t->shape);
            const char *o = static_cast<const char *>(t->out_pin);
            const size_t n = (size_t)t->shape.n_seeds;
            if (t->out.par) std::memcpy(t->out.par, o + ol.par, 48 * n);
            if (t->out.cov) std::memcpy(t->out.cov, o + ol.cov, 168 * n);
            if (t->out.hits) std::memcpy(t->out.hits, o + ol.hits, 4 * (size_t)t->shape.n_layers * n);
            if (t->out.n_hits) std::memcpy(t->out.n_hits, o + ol.nhits, 4 * n);
            if (t->out.n_holes) std::memcpy(t->out.n_holes, o + ol.nholes, 4 * n);
            if (t->out.chi2) std::memcpy(t->out.chi2, o + ol.chi2, 8 * n);
            if (t->out.status) std::memcpy(t->out.status, o + ol.status, 4 * n);
            if (t->out.ndof) {
                const int *nh = reinterpret_cast<const int *>(o + ol.nhits);
                for (size_t i = 0; i < n; ++i) t->out.ndof[i] = 2 * nh[i] - 5;
            }
            destroy_event(ctx, t->rec.get());
            t->rec.reset();
            pinned.put(t->in_pin, t->in_cls);
            pinned.put(t->out_pin, t->out_cls);
            t->in_pin = t->out_pin = nullptr;
        }
        slab->release(b.scratch_dev);
        pinned.put(b.scratch_host, b.scratch_cls);
        (void)hipEventDestroy(b.done);
        stream_busy[b.stream] = false;
        const auto now = Clock::now();
        std::lock_guard<std::mutex> lk(mu);
        for (Ticket *t : b.tickets) {
            t->t_done = now;
            t->state = 2;
        }
        in_flight -= (int)b.tickets.size();
        cv.notify_all();
    }

    void fail_batch(std::vector<Ticket *> &batch, mkf_status st)
    {
        const auto now = Clock::now();
        for (Ticket *t : batch) {
            if (t->rec) destroy_event(ctx, t->rec.get());
            t->rec.reset();
            pinned.put(t->in_pin, t->in_cls);
            pinned.put(t->out_pin, t->out_cls);
            t->in_pin = t->out_pin = nullptr;
        }
        std::lock_guard<std::mutex> lk(mu);
        for (Ticket *t : batch) {
            t->status = st;
            t->t_done = now;
            t->state = 2;
        }
        in_flight -= (int)batch.size();
        cv.notify_all();
    }

    // Upload, index and build one admitted batch on stream si.
    mkf_status launch(std::vector<Ticket *> &batch, int si, Running *run)
    {
        hipStream_t s = streams[si];
        std::vector<EventRec *> recs;
        for (Ticket *t : batch) {
            const InLayout il = in_layout(t->shape);
            const char *in = static_cast<const char *>(t->in_pin);
            DevEvent &v = t->rec->view;
            if (t->shape.n_hits())
                MKF_HIP(hipMemcpyAsync(const_cast<double *>(v.raw_xyz), in + il.hits, 24 * (size_t)t->shape.n_hits(),
                                       hipMemcpyHostToDevice, s));
            const size_t ns = (size_t)t->shape.n_seeds;
            if (ns) {
                MKF_HIP(hipMemcpyAsync(const_cast<double *>(v.seed_par), in + il.seed_par, 48 * ns,
                                       hipMemcpyHostToDevice, s));
                MKF_HIP(hipMemcpyAsync(const_cast<double *>(v.seed_cov), in + il.seed_cov, 168 * ns,
                                       hipMemcpyHostToDevice, s));
                MKF_HIP(hipMemcpyAsync(const_cast<int *>(v.seed_hits), in + il.seed_hits,
                                       4 * (size_t)t->shape.n_seed_layers * ns, hipMemcpyHostToDevice, s));
            }
            recs.push_back(t->rec.get());
        }
        const size_t sb = batch_scratch_bytes((int)batch.size());
        run->scratch_dev = slab->alloc(sb);
        if (!run->scratch_dev) return fail(MKF_E_NOMEM, "batch scratch");
        run->scratch_host = pinned.get(sb, &run->scratch_cls);
        if (!run->scratch_host) return fail(MKF_E_NOMEM, "pinned batch scratch");
        BatchArgs args{};
        mkf_status st = stage_batch(ctx, recs, run->scratch_dev, run->scratch_host,
                                    seeds_per_item(ctx->tuning.lanes_per_seed), &args, s);
        if (st != MKF_OK) return st;
        if ((st = run_pipeline(ctx, args, recs, MKF_BATCH_REINDEX, false, s)) != MKF_OK) return st;
        for (Ticket *t : batch) {
            const OutLayout ol = out_layout(t->shape);
            char *o = static_cast<char *>(t->out_pin);
            const DevEvent &v = t->rec->view;
            const size_t n = (size_t)t->shape.n_seeds;
            if (!n) continue;
            MKF_HIP(hipMemcpyAsync(o + ol.par, v.out_par, 48 * n, hipMemcpyDeviceToHost, s));
            MKF_HIP(hipMemcpyAsync(o + ol.cov, v.out_cov, 168 * n, hipMemcpyDeviceToHost, s));
            MKF_HIP(hipMemcpyAsync(o + ol.hits, v.out_hits, 4 * (size_t)t->shape.n_layers * n, hipMemcpyDeviceToHost, s));
            MKF_HIP(hipMemcpyAsync(o + ol.nhits, v.out_nhits, 4 * n, hipMemcpyDeviceToHost, s));
            MKF_HIP(hipMemcpyAsync(o + ol.nholes, v.out_nholes, 4 * n, hipMemcpyDeviceToHost, s));
            MKF_HIP(hipMemcpyAsync(o + ol.chi2, v.out_chi2, 8 * n, hipMemcpyDeviceToHost, s));
            MKF_HIP(hipMemcpyAsync(o + ol.status, v.out_status, 4 * n, hipMemcpyDeviceToHost, s));
        }
        MKF_HIP(hipEventCreateWithFlags(&run->done, hipEventDisableTiming));
        MKF_HIP(hipEventRecord(run->done, s));
        run->stream = si;
        run->tickets = batch;
        return MKF_OK;
    }

    void loop()
    {
        (void)hipSetDevice(ctx->device);
        for (;;) {
            bool progress = false;
            // completions
            for (size_t i = 0; i < running.size();) {
                if (hipEventQuery(running[i].done) == hipSuccess) {
                    finish_batch(running[i]);
                    running.erase(running.begin() + i);
                    progress = true;
                } else {
                    ++i;
                }
            }
            // admission, in arrival order, while memory, slots and a stream are free
            int si = -1;
            for (int k = 0; k < kStreams; ++k)
                if (!stream_busy[k]) {
                    si = k;
                    break;
                }
            std::vector<Ticket *> batch;
            {
                std::unique_lock<std::mutex> lk(mu);
                if (stop && pending.empty() && running.empty()) return;
                while (si >= 0 && !pending.empty() && in_flight < max_in_flight &&
                       (max_batch == 0 || (int)batch.size() < max_batch)) {
                    Ticket *t = pending.front();
                    std::unique_ptr<EventRec> rec;
                    if (create_event(ctx, t->shape, slab.get(), &rec) != MKF_OK) break;
                    bool rebuilt = false;
                    if (ensure_index(ctx, rec.get(), &rebuilt, streams[si]) != MKF_OK) {
                        destroy_event(ctx, rec.get());
                        break;
                    }
                    t->rec = std::move(rec);
                    t->state = 1;
                    pending.pop_front();
                    batch.push_back(t);
                    ++in_flight;
                }
                if (batch.empty() && !progress) {
                    cv.wait_for(lk, std::chrono::microseconds(50));
                    continue;
                }
            }
            if (!batch.empty()) {
                Running run;
                mkf_status st = launch(batch, si, &run);
                if (st != MKF_OK) {
                    (void)hipStreamSynchronize(streams[si]);
                    slab->release(run.scratch_dev);
                    pinned.put(run.scratch_host, run.scratch_cls);
                    if (run.done) (void)hipEventDestroy(run.done);
                    fail_batch(batch, st);
                } else {
                    stream_busy[si] = true;
                    running.push_back(run);
                }
            }
        }
    }
};

void ServerDeleter::operator()(Server *s) const { delete s; }

void shutdown_server(mkf_ctx *ctx)
{
    Server *sv = ctx->server.get();
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        // queued tickets are abandoned
        for (Ticket *t : sv->pending) {
            sv->pinned.put(t->in_pin, t->in_cls);
            sv->pinned.put(t->out_pin, t->out_cls);
            t->in_pin = t->out_pin = nullptr;
        }
        sv->pending.clear();
        sv->cv.notify_all();
    }
    if (sv->thr.joinable()) sv->thr.join();
    for (auto &s : sv->streams)
        if (s) {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
    sv->tickets.clear();
    sv->slab.reset();
    ctx->heap.release(sv->slab_base);
    ctx->server.reset();
}

}  // namespace mkf

using namespace mkf;

extern "C" {

mkf_status mkf_serve_config(mkf_ctx *ctx, uint64_t hbm_budget_bytes, int32_t max_in_flight, int32_t max_batch_events)
{
    if (!ctx) return fail(MKF_E_INVALID, "NULL context");
    if (hbm_budget_bytes < (1u << 20) || max_in_flight < 1 || max_batch_events < 0)
        return fail(MKF_E_INVALID, "budget >= 1 MiB, max_in_flight >= 1, max_batch_events >= 0");
    if (ctx->server) {
        std::lock_guard<std::mutex> lk(ctx->server->mu);
        if (!ctx->server->pending.empty() || ctx->server->in_flight > 0)
            return fail(MKF_E_STATE, "serving has tickets in flight");
    }
    shutdown_server(ctx);
    std::unique_ptr<Server, ServerDeleter> sv(new Server());
    sv->ctx = ctx;
    sv->slab_base = ctx->heap.alloc(hbm_budget_bytes);
    if (!sv->slab_base) return fail(MKF_E_NOMEM, "cannot reserve %llu bytes", (unsigned long long)hbm_budget_bytes);
    sv->slab = std::make_unique<SlabHeap>(static_cast<char *>(sv->slab_base), hbm_budget_bytes);
    sv->max_in_flight = max_in_flight;
    sv->max_batch = max_batch_events;
    for (auto &s : sv->streams) {
        hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e != hipSuccess) {
            ctx->heap.release(sv->slab_base);
            return fail(MKF_E_DEVICE, "stream: %s", hipGetErrorString(e));
        }
    }
    ctx->server = std::move(sv);
    Server *raw = ctx->server.get();
    raw->thr = std::thread([raw] { raw->loop(); });
    return MKF_OK;
}

mkf_status mkf_serve_submit(mkf_ctx *ctx, const mkf_event *ev, mkf_tracks *out, uint64_t *ticket)
{
    if (!ctx || !out || !ticket) return fail(MKF_E_INVALID, "NULL argument");
    Server *sv = ctx->server.get();
    if (!sv) return fail(MKF_E_STATE, "serving is not configured");
    EventShape shape;
    mkf_status st = validate_event(ctx, ev, &shape);
    if (st != MKF_OK) return st;
    if (out->n != shape.n_seeds) return fail(MKF_E_INVALID, "output has %d rows, need %d", out->n, shape.n_seeds);
    shape.n_tracks = 0;   // serving builds; tracks for fitting are not staged
    const size_t need = sv->footprint(shape) + batch_scratch_bytes(1);
    if (need > sv->slab->capacity()) return fail(MKF_E_NOMEM, "event needs %zu bytes, budget %zu", need, sv->slab->capacity());
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->pending.size() >= 65536) return fail(MKF_E_AGAIN, "submission queue full");
    }
    auto t = std::make_unique<Ticket>();
    t->shape = shape;
    t->out = *out;
    const InLayout il = in_layout(shape);
    const OutLayout ol = out_layout(shape);
    t->in_pin = sv->pinned.get(il.total, &t->in_cls);
    t->out_pin = sv->pinned.get(ol.total, &t->out_cls);
    if (!t->in_pin || !t->out_pin) {
        sv->pinned.put(t->in_pin, t->in_cls);
        sv->pinned.put(t->out_pin, t->out_cls);
        return fail(MKF_E_NOMEM, "pinned staging");
    }
    char *in = static_cast<char *>(t->in_pin);
    for (int L = 0; L < shape.n_layers; ++L)
        std::memcpy(in + il.hits + 24 * (size_t)shape.layer_off[L], ev->hit_xyz[L], 24 * (size_t)ev->n_hits[L]);
    const size_t ns = (size_t)shape.n_seeds;
    if (ns) {
        std::memcpy(in + il.seed_par, ev->seed_par, 48 * ns);
        std::memcpy(in + il.seed_cov, ev->seed_cov, 168 * ns);
        std::memcpy(in + il.seed_hits, ev->seed_hits, 4 * (size_t)shape.n_seed_layers * ns);
    }
    t->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(sv->mu);
    t->id = sv->next_id++;
    *ticket = t->id;
    sv->pending.push_back(t.get());
    sv->tickets[t->id] = std::move(t);
    sv->cv.notify_all();
    return MKF_OK;
}

mkf_status mkf_serve_poll(mkf_ctx *ctx, uint64_t ticket, int32_t *done, int32_t *ticket_status, double *latency_s)
{
    if (!ctx || !done) return fail(MKF_E_INVALID, "NULL argument");
    Server *sv = ctx->server.get();
    if (!sv) return fail(MKF_E_STATE, "serving is not configured");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->tickets.find(ticket);
    if (it == sv->tickets.end()) return fail(MKF_E_NOTFOUND, "unknown ticket");
    Ticket *t = it->second.get();
    *done = t->state == 2 ? 1 : 0;
    if (t->state == 2) {
        if (ticket_status) *ticket_status = t->status;
        if (latency_s) *latency_s = std::chrono::duration<double>(t->t_done - t->t_submit).count();
        sv->tickets.erase(it);
    }
    return MKF_OK;
}

mkf_status mkf_serve_cancel(mkf_ctx *ctx, uint64_t ticket)
{
    if (!ctx) return fail(MKF_E_INVALID, "NULL context");
    Server *sv = ctx->server.get();
    if (!sv) return fail(MKF_E_STATE, "serving is not configured");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->tickets.find(ticket);
    if (it == sv->tickets.end()) return fail(MKF_E_NOTFOUND, "unknown ticket");
    Ticket *t = it->second.get();
    if (t->state != 0) return fail(MKF_E_STATE, "ticket already admitted");
    sv->pending.erase(std::find(sv->pending.begin(), sv->pending.end(), t));
    sv->pinned.put(t->in_pin, t->in_cls);
    sv->pinned.put(t->out_pin, t->out_cls);
    sv->tickets.erase(it);
    return MKF_OK;
}

mkf_status mkf_serve_drain(mkf_ctx *ctx)
{
    if (!ctx) return fail(MKF_E_INVALID, "NULL context");
    Server *sv = ctx->server.get();
    if (!sv) return fail(MKF_E_STATE, "serving is not configured");
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv.wait(lk, [sv] { return sv->pending.empty() && sv->in_flight == 0; });
    return MKF_OK;
}

}  // extern "C"
