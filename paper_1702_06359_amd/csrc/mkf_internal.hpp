// Internal structures shared by the HIP kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mkf.h"

namespace mkf {

constexpr int kMaxLayers = MKF_MAX_LAYERS;
constexpr int kMaxCands = MKF_MAX_CANDS;
constexpr int kWave = 64;
constexpr uint32_t kHoleId = 0xFFFFFFu;   // hit-id field of a hole or stopped entry
constexpr int kMaxHitsPerLayer = 0xFFFFFE;

// Per-layer geometry and the hit-index grid, in FP32 as the kernels use it.
// The grid's second coordinate is z on a cylinder and r on a disk.
struct LayerParam {
    float r;           // cylinder radius; disk outer radius
    float half_z;
    float x0;
    float inv_dphi;    // bins_phi / (2 pi)
    float inv_dz;      // bins_z / extent of the second coordinate
    float inv_r;
    float grid_lo;     // lower edge of the second coordinate: -half_z, or the disk's r_min
    float zplane;      // disk plane
    int kind;          // 0 cylinder, 1 disk
    float half_thick;  // half the layer's depth (radial or along z); 0: hits on the surface
    int pad[2];
};

// Building and fitting parameters for one launch.
struct Params {
    LayerParam layer[kMaxLayers];
    int n_layers;
    int n_seed_layers;
    int max_cands;
    int max_holes;
    int hole_always;
    int bins_phi;
    int bins_z;
    int geo;             // bit 0: every layer a disk (else a cylinder); bit 1: hits carry (x, y, z) and every
                         // pair is carried to the hit's surface (thick layers, or the 3x3 measurement)
    float w_per_qpt;     // -kappa * B: curvature w = w_per_qpt * q/pT
    float var_u;         // sigma_rphi^2
    float var_z;         // sigma_z^2
    float chi2_cut;
    float mass2;         // scattering mass hypothesis squared
    float win_scale;     // (1 + window margin)
    float var_r;         // sigma_r^2 (disks; the radial axis of the 3x3 measurement)
    int update3d;        // 3x3 global-Cartesian measurement (needs the (x, y, z) hit layout)
};

// Device view of one loaded event.  All pointers are device pointers.
struct DevEvent {
    int n_layers;
    int n_seeds;
    int n_tracks;
    int n_hits;                          // all layers
    int layer_off[kMaxLayers + 1];       // first hit of each layer in the flat hit arrays
    const float4 *hits;                  // [n_hits] caller order, packed by the host from the FP64 input:
                                         // (cos phi_h, sin phi_h, z, r) on a cylinder, (cos, sin, r, z) on a
                                         // disk; (x, y, z, 0) for thick layers and the 3x3 measurement
    float4 *binned;                      // [n_hits] grouped by layer then bin: (c, s, z or r, id bits)
    int *bin_of;                         // [n_hits] bin of each caller-order hit
    int *bin_rank;                       // [n_hits] position of the hit inside its bin
    int *bin_count;                      // [n_layers][n_bins] counts (zero between index builds)
    int *bin_off;                        // [n_layers][bin_off_stride(n_bins)]: n_bins + 1 absolute indices into
                                         // `binned` per layer
    const float *seed_par;               // [n_seeds][6]
    const float *seed_cov;               // [n_seeds][21]
    const int *seed_hits;                // [n_seeds][n_seed_layers]
    const int *seed_order;               // [n_seeds] the seeds by azimuth of their direction: the batched
                                         // builder takes them in this order
    const float *track_par;              // [n_tracks][6]
    const float *track_cov;              // [n_tracks][21]
    const int *track_hits;               // [n_tracks][n_layers]
    // build outputs
    double *out_par;                     // [n_seeds][6]
    double *out_cov;                     // [n_seeds][21]
    int *out_hits;                       // [n_seeds][n_layers]
    int *out_nhits;
    int *out_nholes;
    double *out_chi2;
    int *out_status;
    // fit outputs
    double *fit_par;                     // [n_tracks][6]
    double *fit_cov;                     // [n_tracks][21]
    double *fit_chi2;
    int *fit_nupd;
    int *fit_status;
    double *rf_par;                      // [n_seeds][6] final fit of the built tracks
    double *rf_cov;                      // [n_seeds][21]
    double *rf_chi2;                     // [n_seeds]
    int *rf_nupd;                        // [n_seeds]
    int *rf_status;                      // [n_seeds]
    // the whole final beam (set only for a build that asks for it; null otherwise)
    double *beam_par;                    // [n_seeds * max_cands][6]
    double *beam_cov;                    // [n_seeds * max_cands][21]
    int *beam_hits;                      // [n_seeds * max_cands][n_layers]
    int *beam_nhits;
    int *beam_nholes;
    double *beam_chi2;
    int *beam_status;                    // -1: no candidate at that rank
    unsigned long long *stats;           // [5] mkf_build_stats counters
    // plain per-layer builder state (slots = n_seeds * lanes_per_seed)
    float *st_par;                       // [6][slots]
    float *st_cov;                       // [21][slots]
    float *st_trig;                      // [4][slots] sin, cos of phi and theta
    float *st_chi2;                      // [slots]
    int *st_meta;                        // [slots]
    int *st_hist;                        // [n_layers][slots] parent rank << 24 | hit (0xFFFFFF: hole)
    int st_slots;
    int grid_k;                          // the event's bin grid: (bins_phi >> grid_k) x (bins_z >> grid_k)
};

// A batch: events plus the flattened work decomposition over them.
struct BatchArgs {
    const DevEvent *events;
    const int *item_prefix;      // [n_events + 1] work items (seed groups) before each event
    const int *hit_prefix;       // [n_events + 1] hits before each event
    const int *track_prefix;     // [n_events + 1] tracks before each event
    const int *seed_prefix;      // [n_events + 1] seeds before each event
    unsigned int *queue;         // work-queue counter (persistent kernels)
    int n_events;
    int total_items;
    int total_hits;
    int total_tracks;
    int total_seeds;
    int seeds_per_item;
    int max_layer_hits;          // largest layer of any event (index launch shape)
    int max_bins;                // largest bin grid of any event (index launch shape)
};

// Ints per layer in the bin-offset array: its n_bins + 1 offsets, padded to
// a multiple of four so that every layer's row starts 16-byte aligned.
__host__ __device__ constexpr int bin_off_stride(int n_bins) { return (n_bins + 4) & ~3; }

// The bin grid of one event: the context's grid (bins_phi x bins_z, set for
// the fullest events) coarsened by halving both axes while the event's
// fullest layer keeps at least three bins per hit (the headline's 20,000-
// track events have three), both counts stay divisible, and at least 64
// azimuth bins and 2 rows remain.  Small events so get an index and windows
// sized for their hit density instead of an index as large as the largest.
inline int event_grid_shift(int max_layer_hits, int bins_phi, int bins_z)
{
    int k = 0;
    for (;;) {
        const int k1 = k + 1;
        if ((bins_phi >> k1) << k1 != bins_phi || (bins_z >> k1) << k1 != bins_z) break;
        if ((bins_phi >> k1) < 64 || (bins_z >> k1) < 2) break;
        if ((long long)(bins_phi >> k1) * (bins_z >> k1) < 3LL * max_layer_hits) break;
        k = k1;
    }
    return k;
}

// Batch descriptors of the no-allocation builder: a fixed device array per
// GPU (mkf_kernels.hip), as laid out for up to kNoAllocMaxEvents events.
constexpr int kNoAllocMaxEvents = 256;
constexpr size_t round_up_256(size_t b) { return (b + 255) & ~size_t(255); }
constexpr size_t kNoAllocScratchBytes =
    round_up_256(kNoAllocMaxEvents * sizeof(DevEvent)) + 4 * round_up_256((kNoAllocMaxEvents + 1) * sizeof(int)) + 256;
hipError_t noalloc_scratch_init(int device);   // with `device` current; once per device
void *noalloc_scratch(int device);              // its device address (null before init)

// Launch helpers implemented in mkf_kernels.hip.
size_t build_lds_bytes(int geo, int n_layers, int waves_per_block);   // dynamic LDS of a batched build block
hipError_t launch_fill_i32(int *ptr, int value, int n, hipStream_t s);
hipError_t launch_batch_zero(const BatchArgs &b, hipStream_t s);   // work counters of a batch
hipError_t launch_index(const Params &p, const BatchArgs &b, hipStream_t s);
hipError_t launch_build_batch(const Params &p, const BatchArgs &b, int lanes_per_seed, int waves_per_block,
                              int persistent, int n_blocks, bool stats, hipStream_t s);
hipError_t launch_build_layer(const Params &p, const DevEvent *ev_dev, const DevEvent &ev_host, int layer,
                              int lanes_per_seed, int waves_per_block, bool stats, hipStream_t s);
hipError_t launch_fit(const Params &p, const BatchArgs &b, hipStream_t s);
hipError_t launch_refit(const Params &p, const BatchArgs &b, hipStream_t s);
hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s);
hipError_t launch_calib_fma(float *dst, int n_blocks, int iters, hipStream_t s);   // iters: multiple of 4
int calib_fma_chains();

}  // namespace mkf
