// Host runtime of the track builder: context, device memory, loaded events.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdarg>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mkf_internal.hpp"

namespace mkf {

// thread-local message of the last failure
mkf_status fail(mkf_status st, const char *fmt, ...);

// Records errors after which the device's HIP context is unusable (a faulting
// kernel); mkf_ctx_broken reports them.
void note_device_error(hipError_t e);
bool device_broken(int device);

#define MKF_HIP(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) {                                                                \
            ::mkf::note_device_error(e_);                                                      \
            return ::mkf::fail(MKF_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_));          \
        }                                                                                      \
    } while (0)

// Source of device memory for events: the caller's hooks / hipMalloc, or
// the serving slab.
struct DeviceHeap {
    virtual ~DeviceHeap() = default;
    virtual void *alloc(size_t bytes) = 0;
    virtual void release(void *p) = 0;
};

// First-fit sub-allocator over one reserved device slab (serving budget).
class SlabHeap : public DeviceHeap {
  public:
    SlabHeap(char *base, size_t bytes);
    void *alloc(size_t bytes) override;
    void release(void *p) override;
    size_t used() const { return used_; }
    size_t capacity() const { return cap_; }

  private:
    char *base_;
    size_t cap_;
    size_t used_ = 0;
    std::map<size_t, size_t> free_;     // offset -> size
    std::map<size_t, size_t> taken_;    // offset -> size
    std::mutex mu_;
};

// Sizes of one event, from which its device layout follows.
struct EventShape {
    int n_layers = 0;
    int n_seed_layers = 0;
    int n_seeds = 0;
    int n_tracks = 0;
    int layer_off[kMaxLayers + 1] = {0};
    int n_hits() const { return layer_off[n_layers]; }
};

size_t event_data_bytes(const EventShape &s);
size_t event_input_bytes(const EventShape &s);   // the packed inputs at the start of the data block
size_t event_index_bytes(const EventShape &s, int n_bins);
int max_layer_hits(const EventShape &s);
int event_bins(const EventShape &s, int bins_phi, int bins_z);   // bins per layer of the event's grid

// One loaded event.
struct EventRec {
    EventShape shape;
    DeviceHeap *heap = nullptr;
    void *data = nullptr;          // hits, seeds, tracks, outputs, stats, descriptor
    void *index = nullptr;         // bin counts and offsets
    void *plain = nullptr;         // per-layer builder state
    void *beam = nullptr;          // every rank of the final beam (allocated on first request)
    DevEvent beam_view{};          // its arrays (only the beam_* members are set)
    int index_bins_phi = 0, index_bins_z = 0;   // grid the index was built for (0 = none)
    int plain_G = 0;
    DevEvent view{};               // host copy of the device descriptor
    DevEvent *dev_view = nullptr;  // device copy (inside `data`)
    hipGraphExec_t plain_graph = nullptr;
    int plain_graph_G = 0;
    int plain_graph_wpb = 0;
};

struct BatchGraph {
    std::vector<int32_t> handles;
    uint32_t flags = 0;
    mkf_tuning tuning{};
    void *scratch = nullptr;       // descriptors + prefixes + queue, owned
    hipGraphExec_t exec = nullptr;
};

// Device time of the timed phases: a ring of event pairs, so that calls
// that return before the device finishes (asynchronous batches) each keep
// their own interval until it is collected.
struct Timer {
    static constexpr int kRing = 32;
    hipEvent_t start[kRing] = {}, stop[kRing] = {};
    long long ring_launches[kRing] = {};
    int head = 0, count = 0;   // recorded intervals not yet collected
    bool open = false;         // between timer_begin and timer_end
    double total_ms = 0.0;
    long long launches = 0;
};

struct Server;   // serving state (mkf_serve.cpp)
struct ServerDeleter {
    void operator()(Server *s) const;
};

struct CtxHeap : public DeviceHeap {
    mkf_ctx *ctx = nullptr;
    void *alloc(size_t bytes) override;
    void release(void *p) override;
};

}  // namespace mkf

struct mkf_ctx {
    mkf_config cfg{};
    mkf_tuning tuning{};
    mkf::Params params{};          // derived from cfg + tuning
    int device = 0;
    int n_cu = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool has_alloc = false;
    mkf_allocator alloc{};
    mkf::CtxHeap heap;
    std::unordered_map<int32_t, std::unique_ptr<mkf::EventRec>> events;
    int32_t next_handle = 1;
    // batch scratch (descriptor array + prefixes + queue), device and pinned host
    void *batch_dev = nullptr;
    size_t batch_dev_bytes = 0;
    void *batch_host = nullptr;
    size_t batch_host_bytes = 0;
    hipEvent_t stage_done = nullptr;    // last copy out of batch_host
    bool stage_pending = false;
    std::vector<char> staged_image;     // what batch_dev holds (empty: unknown)
    void *load_pin = nullptr;           // pinned staging of the packed inputs of loads and fits
    size_t load_pin_bytes = 0;
    std::vector<std::unique_ptr<mkf::BatchGraph>> graphs;
    mkf::Timer timers[3];
    std::unique_ptr<mkf::Server, mkf::ServerDeleter> server;
};

namespace mkf {

// context-level helpers used by the ABI and the scheduler
// the counts and pointers of an event (its shape); values are checked by pack_event
mkf_status validate_event(const mkf_ctx *ctx, const mkf_event *ev, EventShape *shape);
// the event's inputs, checked and narrowed to FP32, in its device layout
// (event_input_bytes of them)
mkf_status pack_event(const mkf_event *ev, const EventShape &shape, int geo, void *image, int threads,
                      std::string *why);
int pack_threads(size_t n_values);   // host threads worth using for packing that many values
mkf_status create_event(mkf_ctx *ctx, const EventShape &shape, DeviceHeap *heap, std::unique_ptr<EventRec> *out);
mkf_status upload_packed(EventRec *rec, const void *image, hipStream_t s);
void destroy_event(mkf_ctx *ctx, EventRec *rec);
mkf_status ensure_index(mkf_ctx *ctx, EventRec *rec, bool *rebuilt, hipStream_t s);
mkf_status ensure_index_grid(mkf_ctx *ctx, EventRec *rec, int bins_phi, int bins_z, bool *rebuilt, hipStream_t s);
mkf_status compose_batch(EventRec *const *recs, int n, int spi, bool beam, char *image, char *dev, BatchArgs *args);
mkf_status stage_batch(mkf_ctx *ctx, const std::vector<EventRec *> &recs, void *dev, void *host, int spi,
                       BatchArgs *args, hipStream_t s, bool beam = false);
mkf_status ensure_beam(mkf_ctx *ctx, EventRec *rec);
size_t batch_scratch_bytes(int n_events);
int resolve_lanes(const mkf_ctx *ctx);
int seeds_per_item(int G);
mkf_status run_pipeline(mkf_ctx *ctx, const BatchArgs &args, const std::vector<EventRec *> &recs, uint32_t flags,
                        bool timed, hipStream_t s);
// the same with explicit parameters and launch shapes (serving keeps its own)
mkf_status run_pipeline_with(mkf_ctx *ctx, const Params &P, const mkf_tuning &t, const BatchArgs &args,
                             uint32_t flags, bool timed, hipStream_t s);
mkf_status copy_tracks_out(mkf_ctx *ctx, const EventRec *rec, const mkf_tracks *out, hipStream_t s);
void shutdown_server(mkf_ctx *ctx);

}  // namespace mkf
