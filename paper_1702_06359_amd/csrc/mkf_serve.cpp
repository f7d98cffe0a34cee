// Serving: continuous batching of events as they arrive.
//
// An event is admitted when it is submitted: it takes one of the in-flight
// slots and reserves its device footprint against the budget (a slab
// reserved once, sub-allocated first-fit), or the submit returns
// MKF_E_AGAIN.  Its arrays are copied into pinned host staging.  A scheduler
// thread gives each free stream whatever has been admitted and not yet
// started: it uploads those events, builds their hit indices and runs one
// batched build for all of them, so events submitted later start while
// earlier ones are still on the device.  Results come back through pinned
// staging; the scheduler marks a ticket done when it observes its batch's
// completion event.  The launch shapes and parameters are the context's at
// mkf_serve_config, kept by the server, so later tuning changes of the
// context do not reach events in flight.
#include "mkf_runtime.hpp"

#include <algorithm>
#include <chrono>
#include <cstring>

namespace mkf {

namespace {

using Clock = std::chrono::steady_clock;
constexpr int kStreams = 4;

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

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
    size_t reserved = 0;          // budget bytes held from submit to completion
    Clock::time_point t_submit, t_done;
    int state = 0;                // 0 admitted, 1 running, 2 done
    mkf_status status = MKF_OK;
    std::unique_ptr<EventRec> rec;
};

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
        off = round256(off + b);
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
};

}  // namespace

struct Server {
    mkf_ctx *ctx = nullptr;
    Params params{};              // the context's parameters and launch shapes at configuration
    mkf_tuning tuning{};
    void *slab_base = nullptr;
    std::unique_ptr<SlabHeap> slab;
    int max_in_flight = 0;
    int max_batch = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Ticket *> admitted;   // submitted, not yet started
    std::unordered_map<uint64_t, std::unique_ptr<Ticket>> tickets;
    std::vector<Running> running;
    int in_flight = 0;               // submitted and not finished
    size_t reserved = 0;             // budget promised to those tickets
    bool stop = false;
    uint64_t next_id = 1;
    hipStream_t streams[kStreams] = {};
    bool stream_busy[kStreams] = {};
    // per-stream batch descriptors (device and pinned host), sized for the
    // largest batch at configuration, outside the event budget
    void *scratch_dev[kStreams] = {};
    void *scratch_host[kStreams] = {};
    PinnedPool pinned;
    std::thread thr;

    // device bytes of one event: its data and its hit index, as the slab
    // rounds them
    size_t footprint(const EventShape &s) const
    {
        return round256(event_data_bytes(s)) + round256(event_index_bytes(s, event_bins(s, tuning.bins_phi, tuning.bins_z)));
    }

    void release_ticket_resources(Ticket *t)
    {
        if (t->rec) destroy_event(ctx, t->rec.get());
        t->rec.reset();
        pinned.put(t->in_pin, t->in_cls);
        pinned.put(t->out_pin, t->out_cls);
        t->in_pin = t->out_pin = nullptr;
    }

    // marks tickets done (under the lock) and frees their slots and budget
    void complete(const std::vector<Ticket *> &ts, mkf_status st)
    {
        const auto now = Clock::now();
        std::lock_guard<std::mutex> lk(mu);
        for (Ticket *t : ts) {
            t->status = st;
            t->t_done = now;
            t->state = 2;
            reserved -= t->reserved;
            t->reserved = 0;
        }
        in_flight -= (int)ts.size();
        cv.notify_all();
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
            release_ticket_resources(t);
        }
        (void)hipEventDestroy(b.done);
        stream_busy[b.stream] = false;
        complete(b.tickets, MKF_OK);
    }

    void fail_batch(const std::vector<Ticket *> &batch, int si, mkf_status st)
    {
        (void)hipStreamSynchronize(streams[si]);   // nothing queued may still use the buffers
        for (Ticket *t : batch) release_ticket_resources(t);
        stream_busy[si] = false;
        complete(batch, st);
    }

    // Upload, index and build one batch on stream si.
    mkf_status launch(std::vector<Ticket *> &batch, int si, Running *run)
    {
        hipStream_t s = streams[si];
        std::vector<EventRec *> recs;
        for (Ticket *t : batch) {
            mkf_status st = upload_packed(t->rec.get(), t->in_pin, s);   // hits and seeds, FP32, one copy
            if (st != MKF_OK) return st;
            recs.push_back(t->rec.get());
        }
        BatchArgs args{};
        mkf_status st = stage_batch(ctx, recs, scratch_dev[si], scratch_host[si],
                                    seeds_per_item(tuning.lanes_per_seed), &args, s);
        if (st != MKF_OK) return st;
        if ((st = run_pipeline_with(ctx, params, tuning, args, MKF_BATCH_REINDEX, false, s)) != MKF_OK) return st;
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
            // completions; an error other than "not ready" fails the batch
            for (size_t i = 0; i < running.size();) {
                const hipError_t q = hipEventQuery(running[i].done);
                if (q == hipErrorNotReady) {
                    ++i;
                    continue;
                }
                if (q == hipSuccess) {
                    finish_batch(running[i]);
                } else {
                    note_device_error(q);
                    (void)hipEventDestroy(running[i].done);
                    fail_batch(running[i].tickets, running[i].stream, MKF_E_DEVICE);
                }
                running.erase(running.begin() + i);
                progress = true;
            }
            // start whatever is admitted on a free stream, in submission order,
            // while the slab can place the events
            int si = -1;
            for (int k = 0; k < kStreams; ++k)
                if (!stream_busy[k]) {
                    si = k;
                    break;
                }
            std::vector<Ticket *> batch;
            {
                std::unique_lock<std::mutex> lk(mu);
                if (stop && admitted.empty() && running.empty()) return;
                while (si >= 0 && !admitted.empty() && (max_batch == 0 || (int)batch.size() < max_batch)) {
                    Ticket *t = admitted.front();
                    std::unique_ptr<EventRec> rec;
                    if (create_event(ctx, t->shape, slab.get(), &rec) != MKF_OK) break;   // wait for memory
                    bool rebuilt = false;
                    if (ensure_index_grid(ctx, rec.get(), tuning.bins_phi, tuning.bins_z, &rebuilt, streams[si]) !=
                        MKF_OK) {
                        destroy_event(ctx, rec.get());
                        break;
                    }
                    t->rec = std::move(rec);
                    t->state = 1;
                    admitted.pop_front();
                    batch.push_back(t);
                }
                if (batch.empty() && !progress) {
                    cv.wait_for(lk, std::chrono::microseconds(50));
                    continue;
                }
            }
            if (!batch.empty()) {
                stream_busy[si] = true;
                Running run;
                const mkf_status st = launch(batch, si, &run);
                if (st != MKF_OK) {
                    if (run.done) (void)hipEventDestroy(run.done);
                    fail_batch(batch, si, st);
                } else {
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
        // tickets not started are abandoned
        for (Ticket *t : sv->admitted) {
            sv->pinned.put(t->in_pin, t->in_cls);
            sv->pinned.put(t->out_pin, t->out_cls);
            t->in_pin = t->out_pin = nullptr;
        }
        sv->admitted.clear();
        sv->cv.notify_all();
    }
    if (sv->thr.joinable()) sv->thr.join();
    for (auto &s : sv->streams)
        if (s) {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
    for (int k = 0; k < kStreams; ++k) {
        ctx->heap.release(sv->scratch_dev[k]);
        if (sv->scratch_host[k]) (void)hipHostFree(sv->scratch_host[k]);
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
        if (!ctx->server->admitted.empty() || ctx->server->in_flight > 0)
            return fail(MKF_E_STATE, "serving has tickets in flight");
    }
    shutdown_server(ctx);
    std::unique_ptr<Server, ServerDeleter> sv(new Server());
    sv->ctx = ctx;
    sv->params = ctx->params;
    sv->tuning = ctx->tuning;
    sv->max_in_flight = max_in_flight;
    sv->max_batch = max_batch_events;
    auto undo = [&](mkf_status st) {
        for (int k = 0; k < kStreams; ++k) {
            if (sv->streams[k]) (void)hipStreamDestroy(sv->streams[k]);
            ctx->heap.release(sv->scratch_dev[k]);
            if (sv->scratch_host[k]) (void)hipHostFree(sv->scratch_host[k]);
        }
        ctx->heap.release(sv->slab_base);
        return st;
    };
    sv->slab_base = ctx->heap.alloc(hbm_budget_bytes);
    if (!sv->slab_base) return fail(MKF_E_NOMEM, "cannot reserve %llu bytes", (unsigned long long)hbm_budget_bytes);
    sv->slab = std::make_unique<SlabHeap>(static_cast<char *>(sv->slab_base), hbm_budget_bytes);
    const int largest = max_batch_events > 0 ? std::min(max_batch_events, max_in_flight) : max_in_flight;
    const size_t sb = batch_scratch_bytes(largest);
    for (int k = 0; k < kStreams; ++k) {
        hipError_t e = hipStreamCreateWithFlags(&sv->streams[k], hipStreamNonBlocking);
        if (e != hipSuccess) return undo(fail(MKF_E_DEVICE, "stream: %s", hipGetErrorString(e)));
        sv->scratch_dev[k] = ctx->heap.alloc(sb);
        if (!sv->scratch_dev[k]) return undo(fail(MKF_E_NOMEM, "batch descriptors: %zu bytes", sb));
        e = hipHostMalloc(&sv->scratch_host[k], sb, hipHostMallocDefault);
        if (e != hipSuccess) {
            sv->scratch_host[k] = nullptr;
            return undo(fail(MKF_E_NOMEM, "pinned batch descriptors: %s", hipGetErrorString(e)));
        }
    }
    ctx->server = std::move(sv);
    Server *raw = ctx->server.get();
    raw->thr = std::thread([raw] { raw->loop(); });
    return MKF_OK;
}

mkf_status mkf_serve_submit(mkf_ctx *ctx, const mkf_event *ev, mkf_tracks *out, uint64_t *ticket)
{
    const auto t_entry = Clock::now();
    if (!ctx || !out || !ticket) return fail(MKF_E_INVALID, "NULL argument");
    Server *sv = ctx->server.get();
    if (!sv) return fail(MKF_E_STATE, "serving is not configured");
    // the shape first (cheap), so that a submit refused for want of a slot
    // or budget costs little; the values once admitted
    EventShape shape;
    mkf_status st = validate_event(ctx, ev, &shape);
    if (st != MKF_OK) return st;
    if (out->n != shape.n_seeds) return fail(MKF_E_INVALID, "output has %d rows, need %d", out->n, shape.n_seeds);
    shape.n_tracks = 0;   // serving builds; tracks for fitting are not staged
    const size_t need = sv->footprint(shape);
    if (need > sv->slab->capacity()) return fail(MKF_E_NOMEM, "event needs %zu bytes, budget %zu", need, sv->slab->capacity());
    auto t = std::make_unique<Ticket>();
    t->t_submit = t_entry;
    t->shape = shape;
    t->out = *out;
    t->reserved = need;
    {   // admission: a free in-flight slot and room in the budget
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->stop) return fail(MKF_E_STATE, "serving is shutting down");
        if (sv->in_flight >= sv->max_in_flight) return fail(MKF_E_AGAIN, "all %d in-flight slots are taken", sv->max_in_flight);
        if (sv->reserved + need > sv->slab->capacity())
            return fail(MKF_E_AGAIN, "budget: %zu of %zu bytes held, event needs %zu", sv->reserved,
                        sv->slab->capacity(), need);
        ++sv->in_flight;
        sv->reserved += need;
    }
    auto unreserve = [&]() {
        std::lock_guard<std::mutex> lk(sv->mu);
        --sv->in_flight;
        sv->reserved -= need;
        sv->cv.notify_all();
    };
    const OutLayout ol = out_layout(shape);
    t->in_pin = sv->pinned.get(event_input_bytes(shape), &t->in_cls);
    t->out_pin = sv->pinned.get(ol.total, &t->out_cls);
    if (!t->in_pin || !t->out_pin) {
        sv->pinned.put(t->in_pin, t->in_cls);
        sv->pinned.put(t->out_pin, t->out_cls);
        unreserve();
        return fail(MKF_E_NOMEM, "pinned staging");
    }
    // the values are checked while they are narrowed to FP32 into the staging
    mkf_event seeds_only = *ev;
    seeds_only.n_tracks = 0;   // serving builds; tracks for fitting are not staged
    std::string why;
    const size_t values = (size_t)shape.n_hits() * 3 + (size_t)shape.n_seeds * 27;
    if ((st = pack_event(&seeds_only, shape, sv->params.geo, t->in_pin, pack_threads(values), &why)) != MKF_OK) {
        sv->pinned.put(t->in_pin, t->in_cls);
        sv->pinned.put(t->out_pin, t->out_cls);
        unreserve();
        return fail(st, "%s", why.c_str());
    }
    std::lock_guard<std::mutex> lk(sv->mu);
    t->id = sv->next_id++;
    *ticket = t->id;
    sv->admitted.push_back(t.get());
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
    if (t->state != 0) return fail(MKF_E_STATE, "ticket already started");
    sv->admitted.erase(std::find(sv->admitted.begin(), sv->admitted.end(), t));
    sv->pinned.put(t->in_pin, t->in_cls);
    sv->pinned.put(t->out_pin, t->out_cls);
    --sv->in_flight;
    sv->reserved -= t->reserved;
    sv->tickets.erase(it);
    sv->cv.notify_all();
    return MKF_OK;
}

mkf_status mkf_serve_drain(mkf_ctx *ctx)
{
    if (!ctx) return fail(MKF_E_INVALID, "NULL context");
    Server *sv = ctx->server.get();
    if (!sv) return fail(MKF_E_STATE, "serving is not configured");
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv.wait(lk, [sv] { return sv->admitted.empty() && sv->in_flight == 0; });
    return MKF_OK;
}

}  // extern "C"
