/* mkf.h - C ABI of the MI355X (gfx950) Kalman-filter track builder.
 *
 * The method is Kalman-filter track reconstruction in a barrel detector
 * (Cerati et al., "Kalman filter tracking on parallel architectures"):
 * seeding gives a first estimate from a few inner hits; building projects
 * each candidate outward layer by layer, collects compatible hits with the
 * KF and branches to several candidates per seed; fitting re-runs the KF
 * over the final hit set (Section 2).  This library implements building and
 * fitting on the GPU; seeds are an input.
 *
 * Conventions for every call:
 *  - Units cm, GeV, tesla, radians; magnetic field along +z.
 *  - A state is (x, y, z, q/pT, phi, theta): global Cartesian position and
 *    polar momentum, the paper's hybrid coordinates (Section 2.2).  q/pT is
 *    signed; phi in (-pi, pi] is the momentum azimuth; theta in (0, pi).
 *  - A covariance is the symmetric 6x6 matrix packed as its 21-entry upper
 *    triangle, row-major: (0,0) (0,1) .. (0,5) (1,1) .. (5,5).
 *  - A hit is identified by its layer and its index in the caller's array
 *    for that layer.
 *  - All host pointers are plain C arrays in the caller's memory, read or
 *    written only during the call unless stated; nothing is retained.
 *  - Every call returns an mkf_status; on error the outputs are untouched and
 *    mkf_last_error(ctx) describes the failure.  Argument checks run on the host
 *    before any device work.  No C++ exception crosses this interface.
 *  - One context is used by one host thread at a time, except
 *    mkf_serve_submit / mkf_serve_poll / mkf_serve_cancel, which are
 *    thread-safe.
 */
#ifndef MKF_H
#define MKF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MKF_MAX_LAYERS 16
#define MKF_MAX_CANDS 8

typedef enum {
    MKF_OK = 0,
    MKF_E_INVALID = -1,   /* bad argument, NaN, count or index out of range */
    MKF_E_NOMEM = -2,     /* device allocation failed or budget too small */
    MKF_E_DEVICE = -3,    /* HIP runtime error */
    MKF_E_AGAIN = -4,     /* serving: no in-flight slot or budget free now, retry later */
    MKF_E_NOTFOUND = -5,  /* unknown event handle or ticket */
    MKF_E_STATE = -6      /* call not valid in the current state */
} mkf_status;

/* config.flags */
#define MKF_HOLE_ALWAYS 0x1u   /* offer a hole child even when hits were accepted */
#define MKF_UPDATE_3D 0x2u     /* 3x3 global-Cartesian measurement: the hit's (x, y, z) with the error
                                  ellipsoid sigma_rphi along the layer, sigma_r radially and sigma_z along z
                                  (the layer normal carries sigma_r on a cylinder, sigma_z on a disk), in
                                  place of the two coordinates on the tangent plane; needs sigma_r > 0 */

/* Detector, field and building parameters (Section 2.2: ideal barrel of
 * cylinders in a uniform longitudinal field, Gaussian hit resolution; the
 * simplified geometry's endcap disks as planes at fixed z).
 * Layer L is a cylinder of radius layer_r[L] (layer_kind 0) or a disk
 * (layer_kind 1) in the plane z = layer_z[L] between radii layer_rmin[L] and
 * layer_r[L].  A cylinder's hits are measured along r*phi (sigma_rphi) and z
 * (sigma_z), a disk's along r*phi and r (sigma_r).  layer_half_z (cylinders)
 * and the disk radii bound the hit index grid only: hits beyond them go to
 * the edge bins, a track may cross a layer anywhere.  layer_x0 is the
 * material of each layer in radiation lengths at normal incidence (0 = none);
 * the path through it grows as 1 / cos of the angle to the layer normal
 * (radial for a cylinder, z for a disk).  Layers are crossed in index order;
 * consecutive cylinders need increasing radii.
 * A layer of thickness t > 0 (Section 2.2's simplified geometry: modules at
 * different radii) holds hits anywhere within t/2 of its average radius (z
 * for a disk).  Building then propagates in two steps: to the average
 * surface, then, for each hit in the window, to the hit's own radius (z),
 * ahead or behind, where its chi2 and the update are taken; the fit goes
 * straight to the hit's surface.  The GPU takes all-thin or all-thick lists. */
typedef struct {
    int32_t n_layers;        /* 4 .. MKF_MAX_LAYERS */
    int32_t n_seed_layers;   /* seeds carry one hit on each of layers 0 .. n_seed_layers-1 */
    int32_t max_cands;       /* candidates kept per seed, 1 .. MKF_MAX_CANDS (1 = best hit) */
    int32_t max_holes;       /* layers a candidate may cross without a hit, 0 .. 7 */
    uint32_t flags;          /* MKF_HOLE_ALWAYS */
    int32_t reserved;
    double layer_r[MKF_MAX_LAYERS];       /* increasing radii */
    double layer_half_z[MKF_MAX_LAYERS];
    double layer_x0[MKF_MAX_LAYERS];
    double bz;               /* tesla */
    double sigma_rphi;       /* hit resolution along the layer, cm */
    double sigma_z;          /* hit resolution along z, cm */
    double chi2_cut;         /* a hit is compatible when its chi2 < chi2_cut */
    double mass;             /* mass hypothesis for the scattering angle, GeV */
    int32_t layer_kind[MKF_MAX_LAYERS];   /* 0 cylinder (all zero: a barrel), 1 disk */
    double layer_z[MKF_MAX_LAYERS];       /* disk plane, cm (nonzero) */
    double layer_rmin[MKF_MAX_LAYERS];    /* disk inner radius, 0 <= rmin < layer_r */
    double sigma_r;          /* disk hit resolution along r, cm (> 0 when a disk exists) */
    double layer_thickness[MKF_MAX_LAYERS];   /* depth of a layer, cm (0: hits on the surface) */
} mkf_config;

/* Device memory hooks.  alloc returns device memory usable on `stream`
 * (the context's HIP stream), or NULL; free releases it.  With no allocator
 * the library uses hipMalloc/hipFree. */
typedef struct {
    void *(*alloc)(size_t bytes, void *stream, void *user);
    void (*free)(void *ptr, void *stream, void *user);
    void *user;
} mkf_allocator;

/* One event (input).  hit_xyz[L] points at n_hits[L] rows of (x, y, z).
 * Seeds (for building) and tracks (for fitting) are both optional.
 *  seed_par  [n_seeds][6]  state on layer n_seed_layers-1 (through its hit)
 *  seed_cov  [n_seeds][21]
 *  seed_hits [n_seeds][n_seed_layers]   hit index per seed layer (-1 = none)
 *  track_par [n_tracks][6]  prior state on layer 0
 *  track_cov [n_tracks][21]
 *  track_hits[n_tracks][n_layers]  hit index per layer, -1 = no hit */
typedef struct {
    int32_t n_layers;
    int32_t n_seeds;
    int32_t n_tracks;
    int32_t reserved;
    const int32_t *n_hits;
    const double *const *hit_xyz;
    const double *seed_par;
    const double *seed_cov;
    const int32_t *seed_hits;
    const double *track_par;
    const double *track_cov;
    const int32_t *track_hits;
} mkf_event;

/* Track output, caller-allocated, one row per seed (building) or per track
 * (fitting).  Any pointer may be NULL to skip that field.
 *  par  [n][6], cov [n][21]: state and covariance on the last surface the
 *        candidate reached (building) or after the last update (fitting);
 *        scattering of that last surface is not included.
 *  hits [n][n_layers]: hit index per layer, -1 = hole or not reached; the
 *        seed layers carry the seed's hits.
 *  n_hits: hits on the track (seed hits included) / updates in the fit.
 *  n_holes: holes taken (building) / layers without a hit (fitting).
 *  chi2: sum of the accepted hits' chi2 on the building layers / over all
 *        updates of the fit.
 *  ndof: 2 * n_hits - 5 (two measured coordinates per hit, five track
 *        parameters).
 *  status: 0 reached the last layer, 1 stopped when no hit and no hole was
 *        left, 2 the helix does not reach the next layer. */
typedef struct {
    int32_t n;
    int32_t reserved;
    double *par;
    double *cov;
    int32_t *hits;
    int32_t *n_hits;
    int32_t *n_holes;
    double *chi2;
    int32_t *ndof;
    int32_t *status;
} mkf_tracks;

/* Launch shapes.  None of them changes any result. */
typedef struct {
    int32_t lanes_per_seed;   /* 1, 2, 4, 6 or 8, >= max_cands; 0 = smallest valid */
    int32_t waves_per_block;  /* 1 .. 4; 0 = 1 */
    int32_t bins_phi;         /* hit-index bins in phi per layer, 1 .. 4096; 0 = 2048 */
    int32_t bins_z;           /* hit-index bins in z per layer, 1 .. 1024; 0 = 32 */
    int32_t persistent;       /* batched build: 1 = persistent waves on a device work queue,
                                 0 = one wave per work item dispatched by the hardware (default) */
    int32_t blocks_per_cu;    /* persistent grid size per compute unit, 1 .. 32; 0 = 4 */
} mkf_tuning;

/* Counters of the last build of an event (zero unless MKF_BATCH_STATS). */
typedef struct {
    int64_t cand_layers;      /* candidate propagations to a layer */
    int64_t chi2_evals;       /* (candidate, hit) pairs inside the search window */
    int64_t accepted;         /* pairs with chi2 < cut */
    int64_t updates;          /* Kalman updates of surviving hit children */
    int64_t hits_scanned;     /* hits read from the window's bins */
} mkf_build_stats;

typedef struct mkf_ctx mkf_ctx;

/* Library version string, static storage. */
const char *mkf_version(void);

/* Create a context on the current HIP device: the detector, field and
 * building parameters that every later call of the context uses (Section 2:
 * seeds are propagated outward layer by layer and branch to several
 * candidates; Section 2.2: the geometry, the uniform field and the hit
 * resolution).  cfg: building parameters (copied).  alloc: may be NULL.
 * hip_stream: a hipStream_t to run on (NULL = a stream the library
 * creates).  *out receives the context.  Errors: MKF_E_INVALID for an
 * inconsistent config, MKF_E_DEVICE when no gfx950 device is current. */
mkf_status mkf_create(const mkf_config *cfg, const mkf_allocator *alloc, void *hip_stream,
                      mkf_ctx **out);

/* Destroy a context and everything it owns (events, serving state).  Waits
 * for outstanding device work.  NULL is ignored. */
void mkf_destroy(mkf_ctx *ctx);

/* Message of the last failed call on this thread (thread-local storage,
 * valid until the thread's next failing call).  ctx may be NULL: the
 * message is per thread, so it also covers mkf_create failures, which have
 * no context yet. */
const char *mkf_last_error(const mkf_ctx *ctx);

/* 1 when a device error that leaves the GPU's HIP context unusable (a
 * faulting kernel: illegal address, launch failure, ...) was seen on the
 * context's device since the process started; then only mkf_destroy is
 * meaningful.  Any other MKF_E_DEVICE leaves the context usable.  0 for a
 * healthy context or NULL. */
int32_t mkf_ctx_broken(const mkf_ctx *ctx);

/* Change launch shapes (copied).  Loaded events are re-indexed on their next
 * build when the bin grid changes.  MKF_E_INVALID for values out of range. */
mkf_status mkf_set_tuning(mkf_ctx *ctx, const mkf_tuning *t);
mkf_status mkf_get_tuning(const mkf_ctx *ctx, mkf_tuning *t);

/* Load an event: validate on the host while narrowing its coordinates,
 * states and covariances to FP32, copy hits, seeds and tracks to the device
 * and build its (eta, phi)-binned hit index there (Section 3.2.1: the data
 * structures used to select hit candidates).  Synchronous: the host arrays
 * may be freed on return.  *handle identifies the event until
 * mkf_unload_event.  Errors: MKF_E_INVALID (counts, NaN or hit index out of
 * range), MKF_E_NOMEM, MKF_E_DEVICE. */
mkf_status mkf_load_event(mkf_ctx *ctx, const mkf_event *ev, int32_t *handle);

/* Load n events at once: as mkf_load_event for each, with their copies and
 * their hit indices in one pass and one wait (Section 5: on a GPU the setup
 * copies dominate).  The inputs are checked and narrowed to FP32 on up to
 * 16 host threads into pinned staging (12 bytes per hit, 120 per seed),
 * then copied in one piece per event.  handles[n] receives the handles.  On
 * error nothing is loaded and the message names the failing event.  At most
 * 65,535 / n_layers events per call. */
mkf_status mkf_load_events(mkf_ctx *ctx, const mkf_event *evs, int32_t n, int32_t *handles);
mkf_status mkf_unload_event(mkf_ctx *ctx, int32_t handle);

/* Plain builder: one event, one kernel launch per layer with the candidate
 * state in device memory between layers (Section 2: building layer by layer
 * with branching; Section 3.2.1: the beam is re-ranked and pruned after each
 * layer).  Blocks until the tracks are in `out` (out->n must equal the
 * event's n_seeds; out may be NULL to keep the results on the device). */
mkf_status mkf_build(mkf_ctx *ctx, int32_t handle, mkf_tracks *out);

/* mkf_build_batch flags */
#define MKF_BATCH_REINDEX 0x1u   /* rebuild every event's hit index first (same stream) */
#define MKF_BATCH_STATS 0x2u     /* count work (mkf_get_stats); slower */
#define MKF_BATCH_GRAPH 0x4u     /* run the pipeline as a captured hipGraph, cached per handle list */
#define MKF_BATCH_ASYNC 0x8u     /* return once the work is queued on the context stream (outs must be
                                    NULL); results, counters and timers are final after mkf_sync or
                                    any call that waits for the stream (fetch, stats, timers) */
#define MKF_BATCH_FIT 0x10u      /* then fit every built track on the device (mkf_fetch_fit) */
#define MKF_BATCH_BEAM 0x20u     /* also keep every rank of each seed's final beam (mkf_fetch_beam) */

/* Batched builder: all listed events in one launch whose waves each take
 * (event, seed group) work items - one per wave as the hardware dispatches
 * them, or in turn from a device queue with persistent waves - with every
 * layer of a candidate kept in registers (Section 2.3: small units of work
 * with dynamic assignment against uneven events; Section 4: seeds of several
 * events processed together).  Results equal mkf_build's.  outs: n entries
 * or NULL (results stay on the device; see mkf_fetch_tracks). */
mkf_status mkf_build_batch(mkf_ctx *ctx, const int32_t *handles, int32_t n, uint32_t flags,
                           mkf_tracks *outs);

/* mkf_build_batch without any allocation, for callers that cannot allocate
 * device memory during the call (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  The batch descriptors (the
 * events' device views, the work, hit, track and seed prefixes and the
 * work-queue counter) go to a fixed array in device memory that the library
 * holds per GPU for the life of the process, instead of memory allocated by
 * the call; the host image of them is a fixed array too.  Inputs and outputs
 * are as in mkf_build_batch.  Limits: at most 256 events (MKF_E_INVALID
 * beyond), flags MKF_BATCH_REINDEX, _STATS, _ASYNC and _FIT only (the graph
 * and the final beam allocate; MKF_E_INVALID), and every event must hold an
 * index for the current bin grid - it has one from mkf_load_event or any
 * mkf_build_batch since the last grid change - or MKF_E_STATE.  The call
 * waits for the context stream before it rewrites the array, so the calls
 * of one context are ordered; every context on one GPU shares the array,
 * so calls of different contexts that overlap on one GPU race and must not
 * be issued together. */
mkf_status mkf_build_batch_noalloc(mkf_ctx *ctx, const int32_t *handles, int32_t n, uint32_t flags,
                                   mkf_tracks *outs);

/* Copy the last build results of an event to the host. */
mkf_status mkf_fetch_tracks(mkf_ctx *ctx, int32_t handle, mkf_tracks *out);

/* Final fit of the built tracks of an event, from the last mkf_build_batch
 * with MKF_BATCH_FIT (Section 2: once a track is complete, a last KF pass
 * over its hits).  Prior: the helix through the track's hits on layers 0, 1
 * and 2 (circle through the transverse points, z linear in the arc length)
 * at the first hit, covariance diag(1 cm, 10 cm, 1/GeV, 0.1, 0.1)^2 in the
 * frame (u, z, q/pT, phi, theta) of the layer tangent there; then the KF fit
 * over the built hit list as mkf_fit.  out (n = the event's seeds): par/cov
 * after the last update, hits and n_holes of the build, n_hits = updates,
 * chi2, ndof = 2 n_hits - 5, status 0 / 2 (propagation failure) / 3 (no
 * hit on one of layers 0-2, or collinear points: no prior, nothing fitted).
 * Waits for the stream.  Errors: MKF_E_INVALID, MKF_E_NOTFOUND, MKF_E_DEVICE. */
mkf_status mkf_fetch_fit(mkf_ctx *ctx, int32_t handle, mkf_tracks *out);

/* Every rank of each seed's final beam from the last mkf_build_batch with
 * MKF_BATCH_BEAM (Section 3.2.1: up to max_cands candidates survive each
 * layer; the build's output is rank 0).  out->n must equal n_seeds *
 * max_cands; row seed * max_cands + r is rank r, in the beam order (n_hits
 * descending, chi2 ascending), with the same fields as mkf_build's output;
 * ranks beyond the beam have status -1, no hits (-1) and ndof 0.  Waits for
 * the stream.  Errors: MKF_E_INVALID (NULL, wrong n), MKF_E_NOTFOUND,
 * MKF_E_STATE (no build of this event kept its beam), MKF_E_DEVICE. */
mkf_status mkf_fetch_beam(mkf_ctx *ctx, int32_t handle, mkf_tracks *out);

/* The hit index of one layer of a loaded event, as built on the device for
 * the current bin grid (Section 3.2.1: the structures that select the hit
 * candidates of a layer).  bin_off [n_bins + 1]: first position of each bin
 * in the layer's binned order, bin = i_z * bins_phi + i_phi (i_z over z on a
 * cylinder, r on a disk), bin_off[n_bins] = the layer's hit count;
 * bin_of [n_hits of the layer]: the bin of each hit, caller's order;
 * order [n_hits of the layer]: the caller's index of the hit at each binned
 * position.  Any pointer may be NULL.  Waits for the stream.  Errors:
 * MKF_E_INVALID (layer out of range), MKF_E_NOTFOUND, MKF_E_STATE (the
 * index was built for another grid; the next build rebuilds it),
 * MKF_E_DEVICE. */
mkf_status mkf_fetch_index(mkf_ctx *ctx, int32_t handle, int32_t layer, int32_t *bin_off, int32_t *bin_of,
                           int32_t *order);

/* Work counters of the last build of an event. */
/* The bin grid of a loaded event's hit index (Section 3.2.1): the context's
 * grid (mkf_tuning bins_phi x bins_z), coarsened for a small event by
 * halving both axes while its fullest layer keeps at least three bins per hit,
 * both counts stay divisible and at least 64 azimuth bins and 2 rows remain,
 * so that a small event's index and windows suit its hit density.  Writes
 * the event's bins_phi and bins_z.  Errors: MKF_E_INVALID (NULL pointer),
 * MKF_E_NOTFOUND, MKF_E_STATE (no index for the current grid yet). */
mkf_status mkf_index_grid(mkf_ctx *ctx, int32_t handle, int32_t *bins_phi, int32_t *bins_z);

mkf_status mkf_get_stats(mkf_ctx *ctx, int32_t handle, mkf_build_stats *out);

/* KF fit with known hits (Section 2: once the hit set is fixed the filter
 * runs without branching).  For each track: update with its layer-0 hit,
 * then for every further layer add the previous layer's scattering noise,
 * propagate, transport the covariance and update with the assigned hit (or
 * skip).  Inputs are host arrays as in mkf_event (track_*), hits refer to the
 * loaded event `handle`.  Blocks until `out` (n rows) is written. */
mkf_status mkf_fit(mkf_ctx *ctx, int32_t handle, int32_t n_tracks, const double *init_par,
                   const double *init_cov, const int32_t *track_hits, mkf_tracks *out);

/* Fit the tracks loaded with each event (mkf_event.track_*), all events in
 * one launch.  outs: n entries (outs[i].n = that event's n_tracks) or NULL. */
mkf_status mkf_fit_batch(mkf_ctx *ctx, const int32_t *handles, int32_t n, mkf_tracks *outs);

/* Device time of the library's kernels, from HIP events recorded on the
 * context stream around each launch of non-graph calls (waits for the
 * stream first).  which: 0 = build
 * (batched build kernel, or the plain per-layer kernels), 1 = hit index
 * (one count per index build of a batch), 2 = fit.  Returns the summed
 * milliseconds and launch count since the last reset. */
mkf_status mkf_timer_read(mkf_ctx *ctx, int32_t which, double *total_ms, int64_t *launches);
mkf_status mkf_timer_reset(mkf_ctx *ctx);

/* Wait until all work queued on the context stream (asynchronous batches
 * included) has finished.  Errors: MKF_E_INVALID (NULL), MKF_E_DEVICE. */
mkf_status mkf_sync(mkf_ctx *ctx);

/* Autotune: time the batched build of the given events over a grid of
 * launch shapes, keep the fastest (applied to ctx and written to *best).
 * Results do not depend on the choice. */
mkf_status mkf_autotune(mkf_ctx *ctx, const int32_t *handles, int32_t n, mkf_tuning *best);

/* ---- serving (continuous batching) -------------------------------------
 * Section 5: on a GPU the total time is dominated by copying the setup data
 * structures to the device, so events are kept resident there and their
 * copies overlap the builds of other events.  An event is admitted when it
 * is submitted - it takes one of max_in_flight slots and reserves its device
 * footprint (its hits, seeds, outputs and hit index) against the budget -
 * or the submit returns MKF_E_AGAIN.  A scheduler thread starts whatever has
 * been admitted on one of four streams, as one batched build (upload, hit
 * index, build, copy of the tracks back), so events submitted while others
 * are on the device start as soon as a stream is free.  Each event's result
 * does not depend on what it was batched with.  The launch shapes are the
 * context's at mkf_serve_config; a later mkf_set_tuning or mkf_autotune
 * does not change them for serving.  Latency runs from the entry into
 * mkf_serve_submit until the scheduler observes the event's completion. */

/* Configure serving: device-memory budget in bytes (reserved at once, a
 * slab that admitted events are placed in), events in flight (submitted and
 * not finished), events per batched build (0 = all that are waiting).  Also
 * allocates, outside the budget, the batch descriptors of each stream.
 * Errors: MKF_E_INVALID, MKF_E_NOMEM (the budget cannot be reserved),
 * MKF_E_STATE (tickets of a previous configuration still in flight),
 * MKF_E_DEVICE. */
mkf_status mkf_serve_config(mkf_ctx *ctx, uint64_t hbm_budget_bytes, int32_t max_in_flight,
                            int32_t max_batch_events);

/* Submit an event: validated and copied into pinned host staging before
 * return (the event arrays may be freed); `out` must stay valid until the
 * ticket is done.  MKF_E_AGAIN when all in-flight slots are taken or the
 * budget held by the events in flight leaves no room for this one (retry
 * once a ticket has finished), MKF_E_NOMEM when the event can never fit the
 * budget, MKF_E_STATE before mkf_serve_config, MKF_E_INVALID for a bad
 * event. */
mkf_status mkf_serve_submit(mkf_ctx *ctx, const mkf_event *ev, mkf_tracks *out, uint64_t *ticket);

/* Poll a ticket: *done = 1 once finished; *ticket_status is its mkf_status;
 * *latency_s the submit-to-completion time.  A finished ticket is forgotten
 * after the poll that reports it.  MKF_E_NOTFOUND for an unknown ticket. */
mkf_status mkf_serve_poll(mkf_ctx *ctx, uint64_t ticket, int32_t *done, int32_t *ticket_status,
                          double *latency_s);

/* Cancel a ticket that has not started (MKF_E_STATE once started); its slot
 * and budget are released. */
mkf_status mkf_serve_cancel(mkf_ctx *ctx, uint64_t ticket);

/* Block until every submitted ticket has finished. */
mkf_status mkf_serve_drain(mkf_ctx *ctx);

/* ---- measurement helper --------------------------------------------------
 * Plain device-to-device copy of `bytes` (multiple of 16) on the context
 * stream with a simple streaming kernel; used to calibrate hardware memory
 * counters against a known traffic.  Blocks until done. */
mkf_status mkf_calib_copy(mkf_ctx *ctx, const void *src_dev, void *dst_dev, size_t bytes);

/* FP32 multiply-add throughput of the vector ALUs (the ceiling of the
 * ALU-bound kernels, which are built without packed FP32 instructions):
 * n_blocks blocks of 256 threads, each lane running 8 independent chains
 * x <- x * a + b for `iters` rounds (a multiple of 4) with no memory
 * traffic, then storing the sum of its chains to dst_dev[thread] (device
 * memory of n_blocks * 256 floats, owned by the caller).  Launched on the
 * context stream between two HIP events; blocks until done and returns the
 * elapsed device time in *ms and the FLOP executed (2 per multiply-add) in
 * *flop.  Errors: MKF_E_INVALID (null pointers, n_blocks < 1, iters not a
 * positive multiple of 4), MKF_E_DEVICE. */
mkf_status mkf_calib_fma(mkf_ctx *ctx, float *dst_dev, int32_t n_blocks, int32_t iters, double *ms, double *flop);

#ifdef __cplusplus
}
#endif
#endif
