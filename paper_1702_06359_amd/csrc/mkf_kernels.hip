// HIP kernels of the Kalman-filter track builder and fit (gfx950): the hit
// index, the batched and the per-layer builders, the fit and the final fit
// of built tracks, on barrel cylinders or endcap disks, thin or of finite
// thickness, plus two calibration kernels (a streaming copy, an FP32
// multiply-add loop).
//
// Layout: one lane = one track candidate.  A seed owns G consecutive lanes
// (G = lanes_per_seed >= max_cands), so a wavefront carries 64/G seeds and a
// seed's beam never leaves its wavefront: ranking and pruning use lane
// shuffles only.  Candidate state (27 floats) lives in registers; the
// per-layer choice of every kept candidate (parent rank, hit) is recorded in
// LDS (batched builder) or device memory (per-layer builder) and unwound at
// the end to produce the hit list.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>

#include "mkf_device.hpp"

namespace mkf {

// ---------------------------------------------------------------------------
// small helpers

__device__ __forceinline__ int upper_bound_i32(const int *a, int n, int v)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] <= v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ unsigned long long shfl_xor_u64(unsigned long long v, int m)
{
    const unsigned lo = __shfl_xor((unsigned)v, m);
    const unsigned hi = __shfl_xor((unsigned)(v >> 32), m);
    return ((unsigned long long)hi << 32) | lo;
}

__global__ void k_fill_i32(int *__restrict__ p, int v, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Plain streaming copy used to calibrate memory-traffic counters.
__global__ void k_copy16(const float4 *__restrict__ src, float4 *__restrict__ dst, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// FP32 multiply-add throughput of the vector ALUs: every lane runs
// kFmaChains independent chains x <- x a + b for `iters` rounds, with no
// memory traffic, and stores the sum of its chains (so nothing folds away).
constexpr int kFmaChains = 8;

__global__ void __launch_bounds__(256) k_calib_fma(float *__restrict__ out, int iters, float a, float b)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    float x[kFmaChains];
#pragma unroll
    for (int i = 0; i < kFmaChains; ++i) x[i] = (float)(t & 1023) * 1e-3f + (float)i;
    for (int it = 0; it < iters; it += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int i = 0; i < kFmaChains; ++i) x[i] = fmaf(x[i], a, b);
        }
    }
    float sum = 0.f;
#pragma unroll
    for (int i = 0; i < kFmaChains; ++i) sum += x[i];
    store_global(out + t, sum);
}

// Clears the per-event work counters of a batch (a kernel rather than a
// memset so that it can sit in a captured graph).
__global__ void k_batch_zero(const BatchArgs B)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < B.n_events * 5) B.events[g / 5].stats[g % 5] = 0ull;
}

// Geometries the kernels are specialised for: bit 0 disks (else cylinders);
// bit 1 hits that carry their position (x, y, z), to whose own surface every
// (candidate, hit) pair is carried before its chi2 - layers of finite
// thickness (the two-step propagation) and the 3x3 measurement.
constexpr bool geo_disk(int geo) { return (geo & 1) != 0; }
constexpr bool geo_xyz(int geo) { return (geo & 2) != 0; }

// ---------------------------------------------------------------------------
// Hit index: per layer, hits are grouped by an (eta, phi) grid.  On a cylinder
// eta is a function of z, on a disk a function of r, so the grid is (z, phi)
// or (r, phi): bin = iz * bins_phi + iphi.  A counting sort over all events
// of a batch at once.

// An event's bin grid (event_grid_shift): bins_phi x bins_z, and the factor
// 2^-k that turns the context grid's per-layer scales into the event's
// (exact, so the scaled products round as the unscaled ones would).
struct EvGrid {
    int bp, bz;
    float sc;
};

__device__ __forceinline__ EvGrid ev_grid(const Params &P, CEvent &E)
{
    const int k = E.grid_k;
    return EvGrid{P.bins_phi >> k, P.bins_z >> k, __builtin_ldexpf(1.f, -k)};
}

// The bin of a hit as the host packed it: (cos phi_h, sin phi_h, g2, -) with
// g2 = z on a cylinder and r on a disk, or, on layers of finite thickness and
// for the 3x3 measurement, (x, y, z, 0), whose own surface the second
// propagation step needs.  bin = row * bins_phi + (phi bin).
__device__ __forceinline__ int bin_hit(const Params &P, const LayerParam &lp, const EvGrid &g, const float4 v)
{
    // the azimuth to 3.8e-7 rad: far inside the 1e-5 rad the search window
    // adds to its own azimuth range, which uses the same function
    const float phi = fast_atan2(v.y, v.x);
    const float g2 = geo_xyz(P.geo) ? (lp.kind ? sqrtf(fmaf(v.x, v.x, v.y * v.y)) : v.z) : v.z;
    int ip = (int)floorf((phi + kPi) * (lp.inv_dphi * g.sc));
    int iz = (int)floorf((g2 - lp.grid_lo) * (lp.inv_dz * g.sc));
    ip = min(max(ip, 0), g.bp - 1);
    iz = min(max(iz, 0), g.bz - 1);
    return iz * g.bp + ip;
}

// Binning of every hit of a batch, no atomics: grid (chunks, event x
// layer).  Precedes k_index_range.
__global__ void __launch_bounds__(256) k_index_bin(const Params P, const BatchArgs B)
{
    const int e = blockIdx.y / P.n_layers;
    const int L = blockIdx.y - e * P.n_layers;
    CEvent &E = event_desc(B.events, e);
    const int h0 = E.layer_off[L], h1 = E.layer_off[L + 1];
    const LayerParam lp = P.layer[L];
    const EvGrid g = ev_grid(P, E);
    for (int h = h0 + blockIdx.x * blockDim.x + threadIdx.x; h < h1; h += gridDim.x * blockDim.x)
        store_global(E.bin_of + h, bin_hit(P, lp, g, load_global(E.hits + h)));
}

// Bin counters in LDS: one 32-bit counter per bin, or two 16-bit counters per
// word when kShort (layers of at most 65,535 hits, so that neither half
// carries into the other).
template <bool kShort>
__device__ __forceinline__ int lds_count(const unsigned *s_cnt, int i)
{
    return kShort ? (int)((s_cnt[i >> 1] >> ((i & 1) * 16)) & 0xFFFFu) : (int)s_cnt[i];
}

// Adds one to counter `bin` and returns its previous value.
template <bool kShort>
__device__ __forceinline__ int lds_bump(unsigned *s_cnt, int bin)
{
    if (kShort) {
        const int sh = (bin & 1) * 16;
        return (int)((atomicAdd(&s_cnt[bin >> 1], 1u << sh) >> sh) & 0xFFFFu);
    }
    return (int)atomicAdd(&s_cnt[bin], 1u);
}

// In-place exclusive scan of the nr counters in s_cnt, starting from
// `carry`; each offset plus `gbase` is also written to gout[0, nr) as it is
// formed when gout is not null (16-byte aligned).  Each thread owns kPer (a multiple of 8)
// consecutive bins per step: one step for up to 1024 kPer bins in a block of
// 1024.  Every thread of the block calls it; it ends on a barrier.
template <bool kShort, int kPer>
__device__ __forceinline__ void lds_scan_counts(unsigned *s_cnt, int nr, int carry, int *s_wave, int *gout,
                                                int gbase)
{
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6, n_waves = blockDim.x >> 6;
    const int nw = kShort ? (nr + 1) / 2 : nr;
    constexpr int kWords = kShort ? kPer / 2 : kPer;
    for (int base = 0; base < nr; base += blockDim.x * kPer) {
        const int b0 = base + threadIdx.x * kPer;   // a multiple of 8: its words are 16-byte aligned
        const int w0 = kShort ? b0 / 2 : b0;
        unsigned w[kWords];
        if (w0 + kWords <= nw) {
#pragma unroll
            for (int j = 0; j < kWords; j += 4) {
                const uint4 q = *reinterpret_cast<const uint4 *>(s_cnt + w0 + j);
                w[j] = q.x; w[j + 1] = q.y; w[j + 2] = q.z; w[j + 3] = q.w;
            }
        } else {
#pragma unroll
            for (int j = 0; j < kWords; ++j) w[j] = w0 + j < nw ? s_cnt[w0 + j] : 0u;
        }
        int v[kPer];
#pragma unroll
        for (int j = 0; j < kPer; ++j)
            v[j] = b0 + j >= nr ? 0 : kShort ? (int)((w[j >> 1] >> ((j & 1) * 16)) & 0xFFFFu) : (int)w[j];
        int sum = 0;
#pragma unroll
        for (int j = 0; j < kPer; ++j) sum += v[j];
        int x = sum;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int t = __shfl_up(x, o);
            if (lane >= o) x += t;
        }
        if (lane == kWave - 1) s_wave[wave] = x;
        __syncthreads();
        if (wave == 0) {
            int t2 = lane < n_waves ? s_wave[lane] : 0;
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) {
                const int t = __shfl_up(t2, o);
                if (lane >= o) t2 += t;
            }
            if (lane < n_waves) s_wave[lane] = t2;
        }
        __syncthreads();
        int run = carry + (wave > 0 ? s_wave[wave - 1] : 0) + x - sum;
        int o[kPer];
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            o[j] = run;
            if (kShort) {
                if (j & 1) w[j >> 1] |= (unsigned)run << 16;
                else w[j >> 1] = (unsigned)run;
            } else {
                w[j] = (unsigned)run;
            }
            run += v[j];
        }
        if (gout == nullptr) {
        } else if (b0 + kPer <= nr) {
#pragma unroll
            for (int j = 0; j < kPer; j += 4)
                store_global(reinterpret_cast<int4 *>(gout + b0 + j),
                             make_int4(gbase + o[j], gbase + o[j + 1], gbase + o[j + 2], gbase + o[j + 3]));
        } else {
#pragma unroll
            for (int j = 0; j < kPer; ++j)
                if (b0 + j < nr) store_global(gout + b0 + j, gbase + o[j]);
        }
        if (w0 + kWords <= nw) {
#pragma unroll
            for (int j = 0; j < kWords; j += 4)
                *reinterpret_cast<uint4 *>(s_cnt + w0 + j) = make_uint4(w[j], w[j + 1], w[j + 2], w[j + 3]);
        } else {
#pragma unroll
            for (int j = 0; j < kWords; ++j)
                if (w0 + j < nw) s_cnt[w0 + j] = w[j];
        }
        carry += s_wave[n_waves - 1];
        __syncthreads();
    }
}

// Hit index of a layer, its bins split into `nsplit` ranges of `chunk` bins
// (a multiple of 64), after k_index_bin: one 1024-thread block per (event,
// layer, range) reads the bin of every hit of the layer, counts those in its
// range with LDS atomics and those below it, scans its range's counts in LDS
// (the absolute offsets written out as they are formed), then reads the bins
// again and places the hits of its range at their bin's running offset (a
// second LDS atomic).  No device-wide atomic, no count array to clear, no
// rank stored, and no block waits for another; the split fills the machine
// when a batch has few (event, layer) pairs.  The order inside a bin is that
// of the atomics, which does not matter: every hit of a window is tested and
// ties are broken by hit index.  kShort packs two 16-bit counters per word
// (layers of at most 65,535 hits).
template <bool kShort>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) k_index_range(const Params P,
                                                                                              const BatchArgs B,
                                                                                              int nsplit, int chunk)
{
    extern __shared__ unsigned s_cnt[];
    __shared__ int s_wave[16];
    const int part = blockIdx.x % nsplit;
    const int el = blockIdx.x / nsplit;
    const int e = el / P.n_layers;
    const int L = el - e * P.n_layers;
    CEvent &E = event_desc(B.events, e);
    const int h0 = E.layer_off[L], n = E.layer_off[L + 1] - h0;
    const EvGrid g = ev_grid(P, E);
    const int nb = g.bp * g.bz;
    int *off = E.bin_off + L * bin_off_stride(nb);
    const int *bin_of = E.bin_of + h0;
    const float4 *hits = E.hits + h0;
    float4 *binned = E.binned + h0;
    if (part == nsplit - 1 && threadIdx.x == 0) off[nb] = h0 + n;
    const int lo = part * chunk;
    if (lo >= nb) return;                     // an empty range (whole block)
    const int nr = min(chunk, nb - lo);       // bins of this range
    const int nw = kShort ? (nr + 1) / 2 : nr;
    for (int i = threadIdx.x; i < nw; i += blockDim.x) s_cnt[i] = 0u;
    __syncthreads();
    constexpr int kU = 8;
    const int stride = blockDim.x, step = kU * stride;
    const int n_full = n - n % step;
    int below = 0;   // hits of this thread in bins before the range
    for (int i = threadIdx.x; i < n_full; i += step) {
        int b[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) b[u] = load_global(bin_of + i + u * stride) - lo;
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            below += b[u] < 0 ? 1 : 0;
            if ((unsigned)b[u] < (unsigned)nr) lds_bump<kShort>(s_cnt, b[u]);
        }
    }
    for (int i = n_full + threadIdx.x; i < n; i += stride) {
        const int b = load_global(bin_of + i) - lo;
        below += b < 0 ? 1 : 0;
        if ((unsigned)b < (unsigned)nr) lds_bump<kShort>(s_cnt, b);
    }
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6, n_waves = blockDim.x >> 6;
    // block sum of `below`: the offset of the range's first bin in the layer
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) below += __shfl_xor(below, o);
    if (lane == 0) s_wave[wave] = below;
    __syncthreads();
    int carry = 0;
    for (int w = 0; w < n_waves; ++w) carry += s_wave[w];
    __syncthreads();
    // exclusive scan of the counts into offsets relative to the layer, written
    // out absolute; ends on a barrier
    lds_scan_counts<kShort, 16>(s_cnt, nr, carry, s_wave, off + lo, h0);
    // placement: kP hits per thread and step
    constexpr int kP = 4;
    const int pstep = kP * stride;
    const int p_full = n - n % pstep;
    for (int i = threadIdx.x; i < p_full; i += pstep) {
        int b[kP];
#pragma unroll
        for (int u = 0; u < kP; ++u) b[u] = load_global(bin_of + i + u * stride) - lo;
        // the hit loads issued together, outside any branch: lanes whose hit
        // lies in another range all read the layer's first hit (one line)
        float4 v[kP];
#pragma unroll
        for (int u = 0; u < kP; ++u) v[u] = load_global(hits + ((unsigned)b[u] < (unsigned)nr ? i + u * stride : 0));
        // all the atomics, then all the stores: a store between them would
        // make each later branch wait for it
        int pos[kP];
#pragma unroll
        for (int u = 0; u < kP; ++u) pos[u] = (unsigned)b[u] < (unsigned)nr ? lds_bump<kShort>(s_cnt, b[u]) : -1;
#pragma unroll
        for (int u = 0; u < kP; ++u)
            if (pos[u] >= 0)
                store_global(binned + pos[u], make_float4(v[u].x, v[u].y, v[u].z, __int_as_float(i + u * stride)));
    }
    for (int i = p_full + threadIdx.x; i < n; i += stride) {
        const int b = load_global(bin_of + i) - lo;
        if ((unsigned)b < (unsigned)nr) {
            const float4 v = load_global(hits + i);
            const int pos = lds_bump<kShort>(s_cnt, b);
            store_global(binned + pos, make_float4(v.x, v.y, v.z, __int_as_float(i)));
        }
    }
}

// Hit index of one layer in one 1024-thread block per (event, layer), for
// batches with enough (event, layer) pairs to fill the machine: every hit
// binned (bin_of kept) and counted with LDS atomics, the counts scanned in LDS
// (the offsets written out as they are formed), then every hit placed at its
// bin's running offset (a second LDS atomic), so that no rank is stored.  The
// order inside a bin is that of the atomics, which does not matter: every hit
// of a window is tested and ties are broken by hit index.  `kU` hits per
// thread and step, their loads issued together; the ragged end of the layer
// takes steps of one hit so that the full steps carry no bounds tests.  A
// thread reads back only the bins it wrote itself.
template <bool kShort>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(4, 4))) k_index_layer(const Params P,
                                                                                                   const BatchArgs B)
{
    extern __shared__ unsigned s_cnt[];
    __shared__ int s_wave[16];
    const int e = blockIdx.x / P.n_layers;
    const int L = blockIdx.x - e * P.n_layers;
    CEvent &E = event_desc(B.events, e);
    const int h0 = E.layer_off[L], n = E.layer_off[L + 1] - h0;
    const LayerParam lp = P.layer[L];
    const EvGrid g = ev_grid(P, E);
    const int nb = g.bp * g.bz;
    int *off = E.bin_off + L * bin_off_stride(nb);
    const float4 *hits = E.hits + h0;
    int *bin_of = E.bin_of + h0;
    float4 *binned = E.binned + h0;
    const int nw = kShort ? (nb + 1) / 2 : nb;
    for (int i = threadIdx.x; i < nw; i += blockDim.x) s_cnt[i] = 0u;
    __syncthreads();
    constexpr int kU = 8;
    const int stride = blockDim.x, step = kU * stride;
    const int n_full = n - n % step;
    for (int i = threadIdx.x; i < n_full; i += step) {
        float4 v[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) v[u] = load_global(hits + i + u * stride);
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int b = bin_hit(P, lp, g, v[u]);
            store_global(bin_of + i + u * stride, b);
            lds_bump<kShort>(s_cnt, b);
        }
    }
    for (int i = n_full + threadIdx.x; i < n; i += stride) {
        const int b = bin_hit(P, lp, g, load_global(hits + i));
        store_global(bin_of + i, b);
        lds_bump<kShort>(s_cnt, b);
    }
    __syncthreads();
    lds_scan_counts<kShort, 32>(s_cnt, nb, 0, s_wave, nullptr, 0);   // ends on a barrier
    // the offsets written out four consecutive bins per lane, so that each
    // store instruction covers one contiguous kilobyte
    for (int i = 4 * (int)threadIdx.x; i < nb; i += 4 * (int)blockDim.x) {
        if (i + 4 <= nb) {
            store_global(reinterpret_cast<int4 *>(off + i),
                         make_int4(h0 + lds_count<kShort>(s_cnt, i), h0 + lds_count<kShort>(s_cnt, i + 1),
                                   h0 + lds_count<kShort>(s_cnt, i + 2), h0 + lds_count<kShort>(s_cnt, i + 3)));
        } else {
            for (int j = i; j < nb; ++j) store_global(off + j, h0 + lds_count<kShort>(s_cnt, j));
        }
    }
    if (threadIdx.x == 0) off[nb] = h0 + n;
    __syncthreads();   // every offset read before the placement moves them
    for (int i = threadIdx.x; i < n_full; i += step) {
        int b[kU];
        float4 v[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            b[u] = load_global(bin_of + i + u * stride);
            v[u] = load_global(hits + i + u * stride);
        }
        int pos[kU];   // all atomics of the step in flight before the stores
#pragma unroll
        for (int u = 0; u < kU; ++u) pos[u] = lds_bump<kShort>(s_cnt, b[u]);
#pragma unroll
        for (int u = 0; u < kU; ++u)
            store_global(binned + pos[u], make_float4(v[u].x, v[u].y, v[u].z, __int_as_float(i + u * stride)));
    }
    for (int i = n_full + threadIdx.x; i < n; i += stride) {
        const float4 v = load_global(hits + i);
        const int pos = lds_bump<kShort>(s_cnt, load_global(bin_of + i));
        store_global(binned + pos, make_float4(v.x, v.y, v.z, __int_as_float(i)));
    }
}

// Pass 1: bin each caller-order hit and take its position in the bin.  Grid
// (chunks, event x layer).
__global__ void __launch_bounds__(256) k_index_prep(const Params P, const BatchArgs B)
{
    const int e = blockIdx.y / P.n_layers;
    const int L = blockIdx.y - e * P.n_layers;
    CEvent &E = event_desc(B.events, e);
    const int h0 = E.layer_off[L], h1 = E.layer_off[L + 1];
    const LayerParam lp = P.layer[L];
    const EvGrid g = ev_grid(P, E);
    int *cnt = E.bin_count + L * g.bp * g.bz;
    for (int h = h0 + blockIdx.x * blockDim.x + threadIdx.x; h < h1; h += gridDim.x * blockDim.x) {
        const int bin = bin_hit(P, lp, g, load_global(E.hits + h));
        E.bin_of[h] = bin;
        E.bin_rank[h] = atomicAdd(&cnt[bin], 1);
    }
}

// Pass 2: one block per (event, layer): exclusive scan of the bin counts into
// absolute offsets.  Each thread owns 32 consecutive bins, so a layer of up to
// 32768 bins is one step whose loads are all in flight together; the counts are
// cleared on the way so the next index build starts from zero.
__global__ void __launch_bounds__(1024) k_index_scan(const Params P, const BatchArgs B)
{
    constexpr int kPer = 32;   // consecutive bins per thread
    __shared__ int s_wave[16];
    const int e = blockIdx.x / P.n_layers;
    const int L = blockIdx.x - e * P.n_layers;
    CEvent &E = event_desc(B.events, e);
    const EvGrid g = ev_grid(P, E);
    const int nb = g.bp * g.bz;
    int *cnt = E.bin_count + L * nb;
    int *off = E.bin_off + L * bin_off_stride(nb);
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
    const int n_waves = blockDim.x >> 6;
    const bool vec = (nb & 3) == 0;   // then every thread's first bin is 16-byte aligned
    int carry = E.layer_off[L];
    for (int base = 0; base < nb; base += blockDim.x * kPer) {
        const int b0 = base + threadIdx.x * kPer;
        int v[kPer];
        if (vec && b0 + kPer <= nb) {
#pragma unroll
            for (int j = 0; j < kPer; j += 4) {
                const int4 q = *reinterpret_cast<const int4 *>(cnt + b0 + j);
                v[j] = q.x; v[j + 1] = q.y; v[j + 2] = q.z; v[j + 3] = q.w;
            }
        } else {
#pragma unroll
            for (int j = 0; j < kPer; ++j) v[j] = b0 + j < nb ? cnt[b0 + j] : 0;
        }
        int sum = 0;
#pragma unroll
        for (int j = 0; j < kPer; ++j) sum += v[j];
        int x = sum;   // inclusive scan of the per-thread sums inside the wavefront
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int t = __shfl_up(x, o);
            if (lane >= o) x += t;
        }
        if (lane == kWave - 1) s_wave[wave] = x;
        __syncthreads();
        if (wave == 0) {
            int w = lane < n_waves ? s_wave[lane] : 0;
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) {
                const int t = __shfl_up(w, o);
                if (lane >= o) w += t;
            }
            if (lane < n_waves) s_wave[lane] = w;
        }
        __syncthreads();
        int run = carry + (wave > 0 ? s_wave[wave - 1] : 0) + x - sum;
        if (vec && b0 + kPer <= nb) {
#pragma unroll
            for (int j = 0; j < kPer; j += 4) *reinterpret_cast<int4 *>(cnt + b0 + j) = make_int4(0, 0, 0, 0);
#pragma unroll
            for (int j = 0; j < kPer; ++j) {
                off[b0 + j] = run;
                run += v[j];
            }
        } else {
#pragma unroll
            for (int j = 0; j < kPer; ++j) {
                if (b0 + j < nb) {
                    off[b0 + j] = run;
                    cnt[b0 + j] = 0;
                }
                run += v[j];
            }
        }
        carry += s_wave[n_waves - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) off[nb] = E.layer_off[L + 1];
}

// Pass 3: scatter each hit into its bin (order inside a bin is irrelevant:
// every hit of a window is tested and ties are broken by hit index).
__global__ void __launch_bounds__(256) k_index_scatter(const Params P, const BatchArgs B)
{
    const int e = blockIdx.y / P.n_layers;
    const int L = blockIdx.y - e * P.n_layers;
    CEvent &E = event_desc(B.events, e);
    const int h0 = E.layer_off[L], h1 = E.layer_off[L + 1];
    const EvGrid g = ev_grid(P, E);
    const int nb = g.bp * g.bz;
    const int *off = E.bin_off + L * bin_off_stride(nb);
    for (int h = h0 + blockIdx.x * blockDim.x + threadIdx.x; h < h1; h += gridDim.x * blockDim.x) {
        const int pos = load_global(off + load_global(E.bin_of + h)) + load_global(E.bin_rank + h);
        const float4 v = load_global(E.hits + h);
        store_global(E.binned + pos, make_float4(v.x, v.y, v.z, __int_as_float(h - h0)));
    }
}

// The blocks of a launch are dealt to the chip's eight XCDs in turn (block b
// runs on XCD b mod 8), and each XCD has its own L2.  Renumbering them so
// that every XCD takes one contiguous range of the work keeps what that
// range reads (the hits of the few events it covers) in that XCD's L2
// instead of every L2 holding a little of every event.  A bijection of
// [0, n) for any n; blocks of one XCD keep their dispatch order.
constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_contiguous(int b, int n)
{
    const int q = n / kXcds, r = n % kXcds;
    const int x = b % kXcds;
    return x * q + min(x, r) + b / kXcds;
}

// ---------------------------------------------------------------------------
// Track building

struct Lane {
    float p[6];
    float c[21];
    Trig tg;           // sines and cosines of p[4] (phi) and p[5] (theta)
    float chi2;
    int n_hits;
    int n_holes;
    int status;
    int live;
    int stopped;
};

// Per-layer record of every kept candidate: parent rank << 24 | hit index
// (kHoleId for a hole).
struct Hist {
    int *rec;
    int stride;        // elements between layers
    __device__ void put(int L, int lane, int h, int parent) const
    {
        rec[L * stride + lane] = (parent << 24) | (h & (int)kHoleId);
    }
    __device__ int hit(int L, int lane) const
    {
        const int v = rec[L * stride + lane] & (int)kHoleId;
        return v == (int)kHoleId ? -1 : v;
    }
    __device__ int parent(int L, int lane) const { return (int)((unsigned)rec[L * stride + lane] >> 24); }
};

struct Count {
    unsigned long long prop = 0, chi2 = 0, acc = 0, upd = 0, scan = 0;
};

// ---------------------------------------------------------------------------
// Wavefront-cooperative hit search and beam selection.
//
// Each lane owns one candidate whose window is a few (z row, phi segment)
// runs of the binned hit array.  The non-empty runs of all lanes are listed
// in LDS with running offsets; the (candidate, hit) pairs they define are then
// evaluated 64 at a time, one pair per lane whatever candidate it belongs to,
// and the accepted ones are appended to an LDS list.  A wavefront's work so
// follows the total number of hits in its windows instead of its largest
// window, and no lane idles through another lane's chi2.  The next beam of
// every seed is then chosen straight from that list (plus each candidate's
// hole or stop entry) by rounds of LDS atomic minima over the child keys,
// one rank per round; when the list fills up first, it is cut down to the
// entries that can still make a beam.

constexpr int kRuns = 128;         // run records held before their pairs are evaluated
constexpr int kAcc = 2 * kWave;    // accepted entries held (two per lane) before the list is cut down

// kOwn rows of owner data per lane: 3 on thin layers ({x, y, z or r, chi2},
// {Cxx, Cxy, Cyy, Cxz}, {Cyz, Czz, du, dz}); 8 on thick ones, where every
// pair carries its candidate to the hit's own surface and so needs the whole
// predicted state ({x, y, z, chi2}, {q/pT, sin phi, cos phi, sin theta},
// {cos theta, phi, theta, C0}, then C1..C20), from which the kept children
// also take their parent's state.
template <int kOwn>
struct SearchLdsT {
    float4 own[kOwn][kWave];
    int4 run[kRuns];              // {first binned index, first pair index, owner lane, -}
    int2 acc[kAcc];               // {accumulated chi2 bits, hit id << 6 | owner lane}
    unsigned long long best[kWave + 1];   // per seed group: the best child key of the current round; + a sink
    int tally[kWave];             // per owner: child hit count << 16 | accepted entries
    int mark[kWave];              // run starting at each pair slot of the current round
};
template <int kGeo>
using SearchLds = SearchLdsT<geo_xyz(kGeo) ? 8 : 3>;

// LDS written by some lanes of a wavefront and read by others: the wavefront's
// LDS operations are executed in order, so it only takes a compiler barrier
// and the wait for outstanding LDS operations.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Issue priority of a wavefront through the phases of a layer step.  The
// prediction and the Kalman update are long runs of VALU work; the hit search
// and above all the beam selection spend most of their time waiting on LDS
// round trips and hit loads.  Raising the priority of the waiting phases lets
// a wavefront that comes out of a wait issue ahead of the wavefronts in their
// VALU runs (the SIMD picks the highest-priority ready wavefront), so its
// chain of waits ends sooner while the VALU runs fill the gaps.  The levels
// were chosen by timing the headline build; they change no result.
enum : int { kPrioVector = 0, kPrioWindow = 1, kPrioListing = 2, kPrioPairs = 1, kPrioSelect = 3 };
template <int kLevel>
__device__ __forceinline__ void wave_priority()
{
    __builtin_amdgcn_s_setprio(kLevel);
}

__device__ __forceinline__ int lanes_below(unsigned long long m)
{
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// Exclusive prefix sum over the wavefront with DPP moves (no LDS round
// trips): within each row of 16 lanes by shifts of 1, 2, 3, 4 and 8 lanes,
// then across rows by broadcasting lane 15 into rows 1 and 3 and lane 31
// into rows 2 and 3.  Disabled lanes of a step add 0.
__device__ __forceinline__ int wave_exclusive_sum(int x, int lane)
{
    (void)lane;
    int v = x;
    v += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, x, 0x113, 0xf, 0xf, true);   // row_shr:3
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xe, true);   // row_shr:4, banks 1-3
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xc, true);   // row_shr:8, banks 2-3
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, true);   // row_bcast:15 into rows 1, 3
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, true);   // row_bcast:31 into rows 2, 3
    return v - x;
}

// Inclusive prefix maximum over the wavefront of non-negative values, with
// DPP moves: within each row of 16 lanes by shifts of 1, 2, 4 and 8 lanes,
// then across rows by broadcasting lane 15 into rows 1 and 3 and lane 31
// into rows 2 and 3.  Lanes a move does not reach take 0, the identity.
__device__ __forceinline__ int wave_inclusive_max(int v)
{
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true));   // row_shr:1
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true));   // row_shr:2
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true));   // row_shr:4
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true));   // row_shr:8
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, true));   // row_bcast:15 into rows 1, 3
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, true));   // row_bcast:31 into rows 2, 3
    return v;
}

template <int G, bool kStats, int kGeo>
struct WaveSearch {
    static constexpr bool kDisk = geo_disk(kGeo);
    static constexpr bool kXyz = geo_xyz(kGeo);
    static_assert(kAcc == 2 * kWave, "two accepted entries per lane");
    SearchLds<kGeo> &W;
    const float4 *bh;
    const Params &P;
    const int lane;
    Count &cnt;
    int n_runs = 0, n_pairs = 0, n_acc = 0;

    // Child key of accepted entry v and the seed group of its owner (the
    // owner's child hit count is the high half of its tally).
    __device__ __forceinline__ unsigned long long entry_key(const int2 v, int &grp) const
    {
        const int o = v.y & (kWave - 1);
        grp = o / G;
        return child_key(W.tally[o] >> 16, (unsigned)v.x, o - grp * G, (unsigned)v.y >> 6);
    }

    // Up to max_cands rounds over this lane's items (two adjacent slots of
    // the accepted list and one more key): round r takes the minimum key of
    // every seed group with LDS atomics, marks the item that holds it as
    // taken, and hands it to the group's lane of rank r (`mine`).  The items
    // of a group are distinct, so each round takes exactly one per group that
    // has any.  Items out of the round read a sink entry, so that the reads
    // of a round are issued together outside any branch; of two items of one
    // group in a lane only the smaller enters the round (the slots hold runs
    // of one candidate's pairs, so this halves the lanes that meet at one
    // address).  Program order suffices between the reads and writes of one
    // round: a wavefront's LDS instructions execute in order.  Which items are
    // live and which enter a round are kept as wavefront masks in scalar
    // registers, so that a round's bookkeeping is scalar work beside the
    // vector work of the other wavefronts.
    __device__ __forceinline__ void rounds(const unsigned long long (&key)[3], const int (&grp)[3], bool (&live)[3],
                                           bool (&taken)[3], unsigned long long &mine)
    {
        const int my_grp = lane / G, my_rank = lane - my_grp * G;
        mine = ~0ull;
        const unsigned long long L0i = __ballot(live[0]), L1i = __ballot(live[1]), L2i = __ballot(live[2]);
        unsigned long long L0 = L0i, L1 = L1i, L2 = L2i;
        // of slots 0 and 1 in one group, the larger waits while the smaller is live
        const bool same = grp[0] == grp[1];
        const unsigned long long Y0 = __ballot(same & (key[1] < key[0])), Y1 = __ballot(same & (key[0] < key[1]));
        for (int r = 0; r < P.max_cands; ++r) {
            if ((L0 | L1 | L2) == 0) break;
            const unsigned long long I0 = L0 & ~(Y0 & L1), I1 = L1 & ~(Y1 & L0), I2 = L2;
            const bool in0 = __builtin_amdgcn_inverse_ballot_w64(I0);
            const bool in1 = __builtin_amdgcn_inverse_ballot_w64(I1);
            const bool in2 = __builtin_amdgcn_inverse_ballot_w64(I2);
            const int a0 = in0 ? grp[0] : kWave, a1 = in1 ? grp[1] : kWave, a2 = in2 ? grp[2] : kWave;
            if (in0) atomicMin(&W.best[a0], key[0]);
            if (in1) atomicMin(&W.best[a1], key[1]);
            if (in2) atomicMin(&W.best[a2], key[2]);
            wave_lds_sync();
            const unsigned long long b0 = W.best[a0], b1 = W.best[a1], b2 = W.best[a2], bm = W.best[my_grp];
            L0 &= ~(__ballot(b0 == key[0]) & I0);
            L1 &= ~(__ballot(b1 == key[1]) & I1);
            L2 &= ~(__ballot(b2 == key[2]) & I2);
            mine = my_rank == r ? bm : mine;
            wave_lds_sync();
            if (my_rank == r) W.best[my_grp] = ~0ull;
            wave_lds_sync();
        }
        taken[0] |= __builtin_amdgcn_inverse_ballot_w64(L0i & ~L0);
        taken[1] |= __builtin_amdgcn_inverse_ballot_w64(L1i & ~L1);
        taken[2] |= __builtin_amdgcn_inverse_ballot_w64(L2i & ~L2);
        live[0] = __builtin_amdgcn_inverse_ballot_w64(L0);
        live[1] = __builtin_amdgcn_inverse_ballot_w64(L1);
        live[2] = __builtin_amdgcn_inverse_ballot_w64(L2);
    }

    // The accepted list is full: keep only its entries that are among the
    // max_cands best of their seed group so far (any other can no longer
    // make the beam), compacted to the front.
    __device__ __forceinline__ void prune()
    {
        wave_lds_sync();
        int2 v[2];
        unsigned long long key[3] = {~0ull, ~0ull, ~0ull};
        int grp[3] = {0, 0, 0};
        bool live[3] = {false, false, false}, taken[3] = {false, false, false};
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int e = 2 * lane + t;
            live[t] = e < n_acc;
            v[t] = live[t] ? W.acc[e] : make_int2(0, 0);
            if (live[t]) key[t] = entry_key(v[t], grp[t]);
        }
        unsigned long long mine;
        rounds(key, grp, live, taken, mine);
        const unsigned long long m0 = __ballot(taken[0]), m1 = __ballot(taken[1]);
        if (taken[0]) W.acc[lanes_below(m0)] = v[0];
        if (taken[1]) W.acc[__popcll(m0) + lanes_below(m1)] = v[1];
        n_acc = __popcll(m0) + __popcll(m1);
        wave_lds_sync();
    }

    // The next beam: the max_cands best children of every seed group among
    // its accepted entries and its candidates' own entries (`own_key`, ~0
    // for none; a hole or a stopped candidate).  Returns this lane's new
    // entry by its rank in the group (~0: none).
    __device__ __forceinline__ unsigned long long select(unsigned long long own_key)
    {
        wave_lds_sync();
        unsigned long long key[3] = {~0ull, ~0ull, own_key};
        int grp[3] = {0, 0, lane / G};
        bool live[3] = {false, false, own_key != ~0ull}, taken[3] = {false, false, false};
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int e = 2 * lane + t;
            live[t] = e < n_acc;
            if (live[t]) key[t] = entry_key(W.acc[e], grp[t]);
        }
        unsigned long long mine;
        rounds(key, grp, live, taken, mine);
        return mine;
    }

    // Pair slot t0 + lane of a round: its owner and hit (the load is left in
    // flight).  Runs starting in the round mark their slot; the other slots
    // continue the last run started before them.
    __device__ __forceinline__ bool fetch_pair(int t0, int &first, int &o, float4 &hv)
    {
        W.mark[lane] = -1;
        const int r = first + lane;
        const int start = r < n_runs ? W.run[r].y : 0x7FFFFFFF;
        const bool starts = start < t0 + kWave;
        if (starts) W.mark[start - t0] = r;
        const int prev = first - 1;
        first += __popcll(__ballot(starts));
        wave_lds_sync();
        // the last run starting at or before this slot: the marks rise with
        // the slot, so it is their prefix maximum
        const int last = wave_inclusive_max(W.mark[lane] + 1) - 1;
        const int rr = last >= 0 ? last : prev;
        const int pair = t0 + lane;
        const bool valid = pair < n_pairs;
        // every lane loads (a slot past the last pair, the first binned hit),
        // so that the load is issued and waited for outside any branch
        const int4 R = W.run[valid ? rr : 0];
        o = valid ? R.z : 0;
        hv = load_global(bh + (valid ? R.x + (pair - R.y) : 0));
        return valid;
    }

    // test one round's pairs (pair slot of this lane: valid, owner o, hit
    // hv) and append the accepted ones to the list
    __device__ __forceinline__ void test_round(const bool valid, const int o, const float4 hv)
    {
        bool ok = false;
        float tot = 0.f;
        const unsigned hid = (unsigned)__float_as_int(hv.w);   // every lane waits for its load here
        if (valid) {
            if constexpr (!kXyz) {
                const float4 a = W.own[0][o], b = W.own[1][o], c = W.own[2][o];
                const bool fwd = fmaf(a.x, hv.x, a.y * hv.y) > 0.f;
                if (kStats) {
                    cnt.scan++;
                    if (fabsf(hv.z - a.z) <= c.w && fabsf(fmaf(a.x, hv.y, -a.y * hv.x)) <= c.z && fwd)
                        cnt.chi2++;
                }
                const float c2 = kDisk ? hit_chi2_disk(a.x, a.y, b.x, b.y, b.z, hv.x, hv.y, hv.z, P.var_u, P.var_r)
                                       : hit_chi2(a.x, a.y, a.z, b.x, b.y, b.z, b.w, c.x, c.y, hv.x, hv.y, hv.z,
                                                  P.var_u, P.var_z);
                ok = fwd & (c2 < P.chi2_cut);
                tot = a.w + c2;
            } else {
                // two-step: the owner's prediction on the layer's average
                // surface, carried to this hit's own surface
                const float4 r0 = W.own[0][o], r1 = W.own[1][o], r2 = W.own[2][o];
                const bool fwd = fmaf(r0.x, hv.x, r0.y * hv.y) > 0.f;
                float c[21];
                c[0] = r2.w;
#pragma unroll
                for (int i = 0; i < 5; ++i) {
                    const float4 v = W.own[3 + i][o];
                    c[1 + 4 * i] = v.x;
                    c[2 + 4 * i] = v.y;
                    c[3 + 4 * i] = v.z;
                    c[4 + 4 * i] = v.w;
                }
                const float p[6] = {r0.x, r0.y, r0.z, r1.x, 0.f, 0.f};
                const Trig tg{r1.y, r1.z, r1.w, r2.x};
                const float rh = sqrtf(fmaf(hv.x, hv.x, hv.y * hv.y));
                const float irh = fast_rcp(rh);
                float np[6], F[6][6], sn, cn, cp[6];
                const bool reach = kDisk ? step_near_plane(p, tg, hv.z, P.w_per_qpt, np, F, sn, cn)
                                         : step_near_cyl(p, tg, rh, P.w_per_qpt, np, F, sn, cn);
                transport_pos<kDisk>(F, c, cp);
                const float ch = hv.x * irh, sh = hv.y * irh;
                const float c2 =
                    P.update3d ? hit_chi2_3d(np[0], np[1], np[2], cp[0], cp[1], cp[2], cp[3], cp[4], cp[5], hv.x,
                                             hv.y, hv.z, P.var_u, P.var_r, P.var_z)
                    : kDisk    ? hit_chi2_disk(np[0], np[1], cp[0], cp[1], cp[2], ch, sh, rh, P.var_u, P.var_r)
                               : hit_chi2(np[0], np[1], np[2], cp[0], cp[1], cp[2], cp[3], cp[4], cp[5], ch, sh,
                                          hv.z, P.var_u, P.var_z);
                if (kStats) {
                    cnt.scan++;
                    if (fwd && reach) cnt.chi2++;
                }
                ok = fwd & reach & (c2 < P.chi2_cut);
                tot = r0.w + c2;
            }
        }
        const unsigned long long am = __ballot(ok);
        const int n_new = __popcll(am);
        if (n_acc + n_new > kAcc) prune();   // leaves at most kWave entries
        if (ok) {
            W.acc[n_acc + lanes_below(am)] = make_int2(__float_as_int(tot), (int)((hid << 6) | (unsigned)o));
            atomicAdd(&W.tally[o], 1);
        }
        n_acc += n_new;
    }

    // evaluate every pair of the listed runs, one per lane and round; the hits
    // of the next round are loaded while this round's are tested.  Two rounds
    // per iteration, in alternating registers, so that the wait for a round's
    // hits falls after the next round's pair listing.
    __device__ __forceinline__ void evaluate()
    {
        if (n_pairs > 0) {
            wave_lds_sync();
            int first = 0;   // first run not yet started
            int oa, ob;
            float4 ha, hb;
            bool va = fetch_pair(0, first, oa, ha);
            for (int t0 = 0;; t0 += 2 * kWave) {
                const bool vb = fetch_pair(t0 + kWave, first, ob, hb);
                test_round(va, oa, ha);
                if (t0 + kWave >= n_pairs) break;
                va = fetch_pair(t0 + 2 * kWave, first, oa, ha);
                test_round(vb, ob, hb);
                if (t0 + 2 * kWave >= n_pairs) break;
            }
        }
        n_runs = 0;
        n_pairs = 0;
    }

    // list one run per lane (len 0: none)
    __device__ __forceinline__ void add_run(int beg, int len)
    {
        const unsigned long long m = __ballot(len > 0);
        const int n_new = __popcll(m);
        if (n_runs + n_new > kRuns || n_pairs >= (1 << 29)) evaluate();
        const int ex = wave_exclusive_sum(len, lane);
        if (len > 0) W.run[n_runs + lanes_below(m)] = make_int4(beg, n_pairs + ex, lane, 0);
        n_runs += n_new;
        n_pairs += __builtin_amdgcn_readlane(ex + len, kWave - 1);
    }
};

// Windowed search of layer L for the predicted state (pp, pc) of every lane
// with `predicted` set: the best K accepted hits of the lane in (lc, lid),
// sorted by accumulated chi2 then hit id; returns the lane's accepted count.
// All lanes of the wavefront must call it together.
// Half-widths of the window that holds every chi2 < cut hit of a surface,
// for a predicted position (x, y, z) with position covariance (cxx, cxy,
// cyy, czz): du along the layer, dz along the grid's second coordinate g2 (z,
// or r on a disk), and the bound x = du / r on the azimuth (inv_r: 1 / the
// cylinder's radius).
template <bool kDisk>
__device__ __forceinline__ void window_at(const Params &P, float x, float y, float z, float cxx, float cxy, float cyy,
                                          float czz, float inv_r, float scale, float &du, float &dz, float &g2,
                                          float &xr)
{
    {
        const float hd = 0.5f * (cxx - cyy);
        const float lmax = 0.5f * (cxx + cyy) + sqrtf(fmaf(hd, hd, cxy * cxy));
        if (!kDisk) {
            // the chi2 < cut ellipse lies inside |u| <= du, |dz| <= dz, since
            // S_uu(phi_h) <= lambda_max(C_xy) + V_u for every hit direction
            g2 = z;
            du = sqrtf(P.chi2_cut * (lmax + P.var_u)) * scale;
            dz = sqrtf(P.chi2_cut * (czz + P.var_z)) * scale;
            xr = du * inv_r;
        } else {
            // On a disk the position covariance has a radial part too.  Any
            // hit with chi2 < cut lies within d0 = sqrt(cut (lmax + max V))
            // of the predicted point, so its azimuth is within a0 = asin(d0 /
            // rp) of the prediction's.  The hit frame is the prediction's
            // (u_p, r_p) turned by that angle a, so sqrt(u_h^T C u_h) <=
            // sqrt(C_uu) + |a| sqrt(lmax) (likewise for r), which bounds
            // each residual separately: |rp sin a| <= du and
            // |r_h - rp cos a| <= dr.
            g2 = sqrtf(fmaf(x, x, y * y));
            const float irp = fast_rcp(g2);
            const float cp = x * irp, sp = y * irp;
            const float cuu = fmaf(sp * sp, cxx, fmaf(-2.f * sp * cp, cxy, cp * cp * cyy));
            const float crr = fmaf(cp * cp, cxx, fmaf(2.f * sp * cp, cxy, sp * sp * cyy));
            const float d0 = sqrtf(P.chi2_cut * (lmax + fmaxf(P.var_u, P.var_r))) * scale;
            const float x0 = d0 * irp;
            const float a0 = x0 >= 0.7f ? 0.5f * kPi : x0 * __builtin_amdgcn_rsqf(1.f - x0 * x0);
            const float sl = a0 * sqrtf(lmax);
            const float su = sqrtf(fmaxf(cuu, 0.f)) + sl, sr = sqrtf(fmaxf(crr, 0.f)) + sl;
            du = sqrtf(P.chi2_cut * fmaf(su, su, P.var_u)) * scale;
            // rp (1 - cos a) <= du^2 / rp for the low edge of the radius range
            dz = fmaf(du * du, irp, sqrtf(P.chi2_cut * fmaf(sr, sr, P.var_r)) * scale);
            xr = du * irp;
        }
    }
}

// |phi_h - phi| <= asin(x) <= x / sqrt(1 - x^2) for x = du / r
__device__ __forceinline__ float dphi_of(float xr)
{
    return (xr >= 0.7f || !(xr >= 0.f) ? 0.5f * kPi : xr * __builtin_amdgcn_rsqf(1.f - xr * xr)) + 1e-5f;
}

// Windowed search of layer L for the predicted state (pp, pc) of every lane
// with `predicted` set (summed chi2 `chi2`, `n_hits` hits so far): every
// accepted (candidate, hit) pair ends in the search's accepted list; returns
// the lane's accepted count.  All lanes of the wavefront must call it
// together.
template <int G, bool kStats, int kGeo>
__device__ __forceinline__ int search_layer(const float (&pp)[6], const float (&pc)[21], const Trig &tg, float chi2,
                                            int n_hits, bool predicted, int L, const LayerParam &lp, const Params &P,
                                            CEvent &E, int lane, WaveSearch<G, kStats, kGeo> &ws)
{
    SearchLds<kGeo> &W = ws.W;
    constexpr bool kDisk = geo_disk(kGeo), kXyz = geo_xyz(kGeo);
    const EvGrid gr = ev_grid(P, E);
    int n_rows = 0, izlo = 0, n_seg = 1, s0lo = 0, s0hi = -1, s1lo = 0, s1hi = -1;
    float du = 0.f, dz = 0.f, g2 = pp[2];
    if (predicted) {
        const float phipos = fast_atan2(pp[1], pp[0]);
        float lo, hi, g2lo, g2hi;   // azimuth offsets from phipos, second-coordinate range
        bool finite = isfinite(phipos);
        if constexpr (!kXyz) {
            float xr;
            window_at<kDisk>(P, pp[0], pp[1], pp[2], pc[sym(0, 0)], pc[sym(0, 1)], pc[sym(1, 1)], pc[sym(2, 2)],
                             lp.inv_r, P.win_scale, du, dz, g2, xr);
            hi = dphi_of(xr);
            lo = -hi;
            g2lo = g2 - dz;
            g2hi = g2 + dz;
        } else {
            // A thick layer's hits lie between two bounding surfaces: the
            // window is the union of the chi2 < cut windows at both (the
            // predicted point moves along the short arc between them and its
            // covariance changes quadratically with the step), widened by 10 %.
            lo = kInf;
            hi = -kInf;
            g2lo = kInf;
            g2hi = -kInf;
#pragma unroll
            for (int end = -1; end <= 1; end += 2) {
                const float where = (kDisk ? lp.zplane : lp.r) + (float)end * lp.half_thick;
                float np[6], F[6][6], sn, cn, cp[6];
                const bool reach = kDisk ? step_near_plane(pp, tg, where, P.w_per_qpt, np, F, sn, cn)
                                         : step_near_cyl(pp, tg, where, P.w_per_qpt, np, F, sn, cn);
                transport_pos<kDisk>(F, pc, cp);
                float due, dze, g2e, xre;
                window_at<kDisk>(P, np[0], np[1], np[2], cp[0], cp[1], cp[2], cp[5], fast_rcp(where),
                                 P.win_scale * 1.1f, due, dze, g2e, xre);
                const float off = wrap_pi(fast_atan2(np[1], np[0]) - phipos);
                const float dph = dphi_of(xre);
                lo = fminf(lo, off - dph);
                hi = fmaxf(hi, off + dph);
                g2lo = fminf(g2lo, g2e - dze);
                g2hi = fmaxf(g2hi, g2e + dze);
                finite = finite && reach;
            }
            if (!finite) {   // an edge out of reach: the whole layer
                finite = isfinite(phipos);
                lo = -kPi;
                hi = kPi;
                g2lo = -1e30f;
                g2hi = 1e30f;
            }
        }
        const int nphi = gr.bp;
        if (finite && isfinite(lo) && isfinite(hi) && !isnan(g2lo) && !isnan(g2hi)) {
            const float idphi = lp.inv_dphi * gr.sc, idz = lp.inv_dz * gr.sc;
            const int ilo = (int)floorf((phipos + lo + kPi) * idphi);
            const int ihi = (int)floorf((phipos + hi + kPi) * idphi);
            const float zlo = fmaxf((g2lo - 1e-4f - lp.grid_lo) * idz, -1.f);
            const float zhi = fminf((g2hi + 1e-4f - lp.grid_lo) * idz, (float)gr.bz);
            izlo = min(max((int)floorf(zlo), 0), gr.bz - 1);
            const int izhi = min(max((int)floorf(zhi), 0), gr.bz - 1);
            n_rows = izhi - izlo + 1;
            if (ihi - ilo + 1 >= nphi) {
                s0lo = 0;
                s0hi = nphi - 1;
            } else if (ilo < 0) {
                s0lo = ilo + nphi;
                s0hi = nphi - 1;
                s1lo = 0;
                s1hi = ihi;
                n_seg = 2;
            } else if (ihi >= nphi) {
                s0lo = ilo;
                s0hi = nphi - 1;
                s1lo = 0;
                s1hi = ihi - nphi;
                n_seg = 2;
            } else {
                s0lo = ilo;
                s0hi = ihi;
            }
        }
    }
    if constexpr (!kXyz) {
        W.own[0][lane] = make_float4(pp[0], pp[1], g2, chi2);
        W.own[1][lane] = make_float4(pc[sym(0, 0)], pc[sym(0, 1)], pc[sym(1, 1)], pc[sym(0, 2)]);
        W.own[2][lane] = make_float4(pc[sym(1, 2)], pc[sym(2, 2)], du, dz);
    } else {
        W.own[0][lane] = make_float4(pp[0], pp[1], pp[2], chi2);
        W.own[1][lane] = make_float4(pp[3], tg.sph, tg.cph, tg.sth);
        W.own[2][lane] = make_float4(tg.cth, pp[4], pp[5], pc[0]);
#pragma unroll
        for (int i = 0; i < 5; ++i)
            W.own[3 + i][lane] = make_float4(pc[1 + 4 * i], pc[2 + 4 * i], pc[3 + 4 * i], pc[4 + 4 * i]);
    }
    W.tally[lane] = (n_hits + 1) << 16;
    W.best[lane] = ~0ull;

    wave_priority<kPrioListing>();
    const int n_runs = n_rows * n_seg;
    const int *off = E.bin_off + L * bin_off_stride(gr.bp * gr.bz);
    // bin offsets of run q: [off[row + lo], off[row + hi + 1])
    auto run_bounds = [&](int q, int &b, int &e) {
        const int sg = n_seg == 2 ? (q & 1) : 0;
        const int row = (izlo + (n_seg == 2 ? q >> 1 : q)) * gr.bp;
        b = load_global(off + row + (sg ? s1lo : s0lo));
        e = load_global(off + row + (sg ? s1hi : s0hi) + 1);
    };
    int nb = 0, ne = 0;   // next run, loaded one iteration ahead
    if (n_runs > 0) run_bounds(0, nb, ne);
    for (int q = 0; __ballot(q < n_runs) != 0; ++q) {
        const int beg = nb, len = ne - nb;
        nb = ne = 0;
        if (q + 1 < n_runs) run_bounds(q + 1, nb, ne);
        ws.add_run(beg, len);
    }
    wave_priority<kPrioPairs>();
    ws.evaluate();
    wave_lds_sync();
    return W.tally[lane] & 0xFFFF;
}

__device__ __forceinline__ void init_lane(Lane &S, CEvent &E, const Params &P, int seed, bool first_slot)
{
    S.live = first_slot ? 1 : 0;
    S.stopped = 0;
    S.status = 0;
    S.n_holes = 0;
    S.chi2 = 0.f;
    S.n_hits = 0;
    S.tg = Trig{0.f, 1.f, 1.f, 0.f};
#pragma unroll
    for (int i = 0; i < 6; ++i) S.p[i] = 0.f;
#pragma unroll
    for (int i = 0; i < 21; ++i) S.c[i] = 0.f;
    if (!first_slot) return;
#pragma unroll
    for (int i = 0; i < 6; ++i) S.p[i] = load_global(E.seed_par + 6 * (size_t)seed + i);
#pragma unroll
    for (int i = 0; i < 21; ++i) S.c[i] = load_global(E.seed_cov + 21 * (size_t)seed + i);
    for (int L = 0; L < P.n_seed_layers; ++L) S.n_hits += load_global(E.seed_hits + (size_t)seed * P.n_seed_layers + L) >= 0;
    S.tg = trig_of(S.p);
}

// One building layer for every lane of a wavefront (Section 2: propagate the
// candidate to the next layer, collect compatible hits, branch; Section
// 3.2.1: re-rank and prune to max_cands per seed).
template <int G, bool kStats, int kGeo>
__device__ __forceinline__ void layer_step(Lane &S, const int L, const Params &P, CEvent &E,
                                           const int lane, const Hist &H, SearchLds<kGeo> &W, Count &cnt)
{
    constexpr bool kDisk = geo_disk(kGeo), kXyz = geo_xyz(kGeo);
    const int gbase = (lane / G) * G;
    const int slot = lane - gbase;
    const LayerParam lp = P.layer[L];
    const bool active = S.live && !S.stopped;

    // 1. scattering of the layer being left, propagation, transport.  The
    //    prediction replaces the state in place; a lane whose helix misses
    //    the layer keeps its state and stops.
    wave_priority<kPrioVector>();
    bool predicted = false;
    if (active) {
        float np[6], sn, cn;
        const bool ok = predict<kDisk>(S.p, S.tg, kDisk ? lp.zplane : lp.r, P.w_per_qpt, P.layer[L - 1].x0, P.mass2,
                                       np, sn, cn, S.c);
        if (kStats) cnt.prop++;
        if (ok) {
#pragma unroll
            for (int i = 0; i < 6; ++i) S.p[i] = np[i];
            S.tg.sph = sn;
            S.tg.cph = cn;
            predicted = true;
        } else {
            S.stopped = 1;
            S.status = 2;
        }
    }
    const float (&pp)[6] = S.p;
    const float (&pc)[21] = S.c;

    // 2. windowed hit search: every accepted hit child into the search's list
    wave_priority<kPrioWindow>();
    WaveSearch<G, kStats, kGeo> ws{W, E.binned, P, lane, cnt};
    const int nacc = search_layer<G, kStats, kGeo>(pp, pc, S.tg, S.chi2, S.n_hits, predicted, L, lp, P, E, lane, ws);
    if (kStats) cnt.acc += nacc;

    // 3. hole child, or stop on this surface (with the prediction as state)
    //    when neither a hit nor a hole is left
    const bool hole = predicted && (nacc == 0 || P.hole_always) && S.n_holes < P.max_holes;
    if (predicted && nacc == 0 && S.n_holes >= P.max_holes) {
        S.stopped = 1;
        S.status = 1;
    }
    const bool tail = S.live && (S.stopped || hole);

    // 4. keep the max_cands best children of the seed (accepted hits, and
    //    each candidate's hole or stop entry): the lane of rank r takes the
    //    r-th best key of its group
    wave_priority<kPrioSelect>();
    unsigned long long mine = ws.select(tail ? child_key(S.n_hits, __float_as_uint(S.chi2), slot, kHoleId) : ~0ull);
    if (slot >= P.max_cands || lane >= (kWave / G) * G) mine = ~0ull;

    // 5. each kept entry moves to the lane of its rank: fetch the parent's
    //    state and apply the Kalman update with the entry's hit
    wave_priority<kPrioVector>();
    const bool alive = mine != ~0ull;
    const int parent = alive ? key_parent(mine) : slot;
    const int src = alive ? gbase + parent : lane;
    const unsigned hid = key_hit(mine);
    const bool with_hit = alive && hid != kHoleId;
    float4 hv = make_float4(1.f, 0.f, 0.f, 0.f);
    if (with_hit) hv = load_global(E.hits + E.layer_off[L] + (int)hid);   // in flight during the shuffles
    if constexpr (!kXyz) {
#pragma unroll
        for (int i = 0; i < 6; ++i) S.p[i] = __shfl(S.p[i], src);
#pragma unroll
        for (int i = 0; i < 21; ++i) S.c[i] = __shfl(S.c[i], src);
        S.tg.sph = __shfl(S.tg.sph, src);
        S.tg.cph = __shfl(S.tg.cph, src);
        S.tg.sth = __shfl(S.tg.sth, src);
        S.tg.cth = __shfl(S.tg.cth, src);
    } else {
        // the whole prediction of every lane is still in the search LDS, so
        // no lane keeps its state in registers through the search
        const float4 r0 = W.own[0][src], r1 = W.own[1][src], r2 = W.own[2][src];
        S.p[0] = r0.x;
        S.p[1] = r0.y;
        S.p[2] = r0.z;
        S.p[3] = r1.x;
        S.p[4] = r2.y;
        S.p[5] = r2.z;
        S.tg = Trig{r1.y, r1.z, r1.w, r2.x};
        S.c[0] = r2.w;
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            const float4 v = W.own[3 + i][src];
            S.c[1 + 4 * i] = v.x;
            S.c[2 + 4 * i] = v.y;
            S.c[3 + 4 * i] = v.z;
            S.c[4 + 4 * i] = v.w;
        }
    }
    const int p_holes = __shfl(S.n_holes, src);
    const int p_stopped = __shfl(S.stopped, src);
    const int p_status = __shfl(S.status, src);
    S.live = alive;
    if (!alive) return;
    S.n_hits = key_nhits(mine);
    S.chi2 = key_chi2(mine);
    S.n_holes = p_holes;
    S.stopped = p_stopped;
    S.status = p_status;
    if (with_hit) {
        if constexpr (!kXyz) {
            kf_update<kDisk>(S.p, S.c, S.tg, hv.x, hv.y, hv.z, P.var_u, kDisk ? P.var_r : P.var_z);
        } else {
            // second step to the hit's own surface, then the update there
            const float rh = sqrtf(fmaf(hv.x, hv.x, hv.y * hv.y));
            const float irh = fast_rcp(rh);
            float np[6], F[6][6], sn, cn;
            if (kDisk) step_near_plane(S.p, S.tg, hv.z, P.w_per_qpt, np, F, sn, cn);
            else step_near_cyl(S.p, S.tg, rh, P.w_per_qpt, np, F, sn, cn);
            transport<kDisk>(F, S.c);
#pragma unroll
            for (int i = 0; i < 6; ++i) S.p[i] = np[i];
            S.tg.sph = sn;
            S.tg.cph = cn;
            if (P.update3d) kf_update_3d<false>(S.p, S.c, S.tg, hv.x, hv.y, hv.z, P.var_u, P.var_r, P.var_z);
            else kf_update<kDisk>(S.p, S.c, S.tg, hv.x * irh, hv.y * irh, kDisk ? rh : hv.z, P.var_u,
                                  kDisk ? P.var_r : P.var_z);
        }
        if (kStats) cnt.upd++;
        H.put(L, lane, (int)hid, parent);
    } else {
        if (!p_stopped) S.n_holes += 1;
        H.put(L, lane, -1, parent);
    }
}

// Rank-0 candidate of each seed to the output arrays, hit list unwound
// through the per-layer records.
template <int G>
__device__ __forceinline__ void finalize_lane(const Lane &S, const Params &P, CEvent &E, int lane,
                                              int seed, const Hist &H)
{
    const int gbase = (lane / G) * G;
    if (E.beam_par && lane < (kWave / G) * G && seed < E.n_seeds && lane - gbase < P.max_cands) {
        // every rank of the final beam: rank r sits in lane gbase + r
        const int r = lane - gbase;
        const size_t b = (size_t)seed * P.max_cands + r;
#pragma unroll
        for (int i = 0; i < 6; ++i) store_global(E.beam_par + 6 * b + i, S.live ? (double)S.p[i] : 0.0);
#pragma unroll
        for (int i = 0; i < 21; ++i) store_global(E.beam_cov + 21 * b + i, S.live ? (double)S.c[i] : 0.0);
        store_global(E.beam_chi2 + b, S.live ? (double)S.chi2 : 0.0);
        store_global(E.beam_nhits + b, S.live ? S.n_hits : 0);
        store_global(E.beam_nholes + b, S.live ? S.n_holes : 0);
        store_global(E.beam_status + b, S.live ? S.status : -1);
        int *bh = E.beam_hits + b * P.n_layers;
        for (int L = 0; L < P.n_seed_layers; ++L)
            store_global(bh + L, S.live ? load_global(E.seed_hits + (size_t)seed * P.n_seed_layers + L) : -1);
        int cur = r;
        for (int L = P.n_layers - 1; L >= P.n_seed_layers; --L) {
            store_global(bh + L, S.live ? H.hit(L, gbase + cur) : -1);
            if (S.live) cur = H.parent(L, gbase + cur);
        }
    }
    if (lane != gbase || seed >= E.n_seeds) return;
    const size_t s = (size_t)seed;
#pragma unroll
    for (int i = 0; i < 6; ++i) store_global(E.out_par + 6 * s + i, (double)S.p[i]);
#pragma unroll
    for (int i = 0; i < 21; ++i) store_global(E.out_cov + 21 * s + i, (double)S.c[i]);
    store_global(E.out_chi2 + s, (double)S.chi2);
    store_global(E.out_nhits + s, S.n_hits);
    store_global(E.out_nholes + s, S.n_holes);
    store_global(E.out_status + s, S.status);
    int *oh = E.out_hits + s * P.n_layers;
    for (int L = 0; L < P.n_seed_layers; ++L) store_global(oh + L, load_global(E.seed_hits + s * P.n_seed_layers + L));
    int cur = 0;
    for (int L = P.n_layers - 1; L >= P.n_seed_layers; --L) {
        store_global(oh + L, H.hit(L, gbase + cur));
        cur = H.parent(L, gbase + cur);
    }
}

template <bool kStats>
__device__ __forceinline__ void flush_counts(const Count &cnt, CEvent &E, int lane)
{
    if (!kStats) return;
    unsigned long long v[5] = {cnt.prop, cnt.chi2, cnt.acc, cnt.upd, cnt.scan};
#pragma unroll
    for (int j = 0; j < 5; ++j) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v[j] += shfl_xor_u64(v[j], o);
    }
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < 5; ++j) atomicAdd(&E.stats[j], v[j]);
    }
}

// Dynamic LDS of the batched builder: the per-layer records of every wave
// (an int per lane and layer), then one SearchLds per wave.
__host__ __device__ constexpr int search_lds_offset(int waves, int n_layers)
{
    return waves * n_layers * kWave;   // in ints (a multiple of 64: 16-byte aligned)
}

// Batched builder.  Each wavefront takes work items (event, group of 64/G
// seeds) - from a device counter when persistent, else from its block index -
// and runs every building layer of its seeds with the state in registers.
template <int G, bool kStats, int kGeo>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(geo_xyz(kGeo) ? 3 : 4))) k_build_batch(const Params P, const BatchArgs B, int persistent)
{
    extern __shared__ int s_dyn[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x >> 6;
    const int W = blockDim.x >> 6;
    Hist H{s_dyn + wave * P.n_layers * kWave, kWave};
    SearchLds<kGeo> &SL = reinterpret_cast<SearchLds<kGeo> *>(s_dyn + search_lds_offset(W, P.n_layers))[wave];
    int item = (persistent ? (int)blockIdx.x : xcd_contiguous(blockIdx.x, gridDim.x)) * W + wave;
    for (;;) {
        if (persistent) {
            unsigned v = 0;
            if (lane == 0) v = atomicAdd(B.queue, 1u);
            item = (int)__shfl(v, 0);
        }
        item = uniform(item);
        if (item >= B.total_items) break;
        const int e = uniform(upper_bound_i32(B.item_prefix, B.n_events + 1, item) - 1);
        CEvent &E = event_desc(B.events, e);
        // the item's seeds, taken in azimuth order
        const int k = (item - B.item_prefix[e]) * B.seeds_per_item + lane / G;
        const bool valid = lane < (kWave / G) * G && k < E.n_seeds;
        const int seed = valid ? load_global(E.seed_order + k) : E.n_seeds;
        Lane S;
        init_lane(S, E, P, valid ? seed : 0, valid && lane % G == 0);
        Count cnt;
        for (int L = P.n_seed_layers; L < P.n_layers; ++L) layer_step<G, kStats, kGeo>(S, L, P, E, lane, H, SL, cnt);
        finalize_lane<G>(S, P, E, lane, valid ? seed : E.n_seeds, H);
        flush_counts<kStats>(cnt, E, lane);
        if (!persistent) break;
    }
}

// Per-layer builder: one event, one layer per launch, candidate state in
// device memory (structure of arrays, slot = seed * G + rank) between layers.
template <int G, bool kStats, int kGeo>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(geo_xyz(kGeo) ? 3 : 4))) k_build_layer(const Params P, const DevEvent *__restrict__ Ep, int L)
{
    CEvent &E = event_desc(Ep, 0);
    const int lane = threadIdx.x & (kWave - 1);
    const int item = uniform(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    constexpr int kSeedsPerWave = kWave / G;
    const int first = item * kSeedsPerWave;
    if (first >= E.n_seeds) return;
    const int seed = first + lane / G;
    const bool valid = lane < kSeedsPerWave * G && seed < E.n_seeds;
    const int ns = E.st_slots;
    const int slot = item * kWave + lane;
    Hist H{E.st_hist + item * kWave, ns};
    Lane S;
    if (L == P.n_seed_layers) {
        init_lane(S, E, P, valid ? seed : 0, valid && lane % G == 0);
    } else {
        const int meta = load_global(E.st_meta + slot);
        S.live = meta & 1;
        S.stopped = (meta >> 1) & 1;
        S.status = (meta >> 2) & 3;
        S.n_hits = (meta >> 4) & 31;
        S.n_holes = (meta >> 9) & 15;
        S.chi2 = load_global(E.st_chi2 + slot);
#pragma unroll
        for (int i = 0; i < 6; ++i) S.p[i] = S.live ? load_global(E.st_par + i * ns + slot) : 0.f;
#pragma unroll
        for (int i = 0; i < 21; ++i) S.c[i] = S.live ? load_global(E.st_cov + i * ns + slot) : 0.f;
        S.tg = S.live ? Trig{load_global(E.st_trig + 0 * ns + slot), load_global(E.st_trig + 1 * ns + slot),
                             load_global(E.st_trig + 2 * ns + slot), load_global(E.st_trig + 3 * ns + slot)}
                      : Trig{0.f, 1.f, 1.f, 0.f};
    }
    extern __shared__ int s_dyn[];
    SearchLds<kGeo> &SL = reinterpret_cast<SearchLds<kGeo> *>(s_dyn)[threadIdx.x >> 6];
    Count cnt;
    layer_step<G, kStats, kGeo>(S, L, P, E, lane, H, SL, cnt);
    if (L == P.n_layers - 1) {
        finalize_lane<G>(S, P, E, lane, valid ? seed : E.n_seeds, H);
    } else {
        store_global(E.st_meta + slot, S.live | (S.stopped << 1) | (S.status << 2) | (S.n_hits << 4) | (S.n_holes << 9));
        store_global(E.st_chi2 + slot, S.chi2);
        if (S.live) {
#pragma unroll
            for (int i = 0; i < 6; ++i) store_global(E.st_par + i * ns + slot, S.p[i]);
#pragma unroll
            for (int i = 0; i < 21; ++i) store_global(E.st_cov + i * ns + slot, S.c[i]);
            store_global(E.st_trig + 0 * ns + slot, S.tg.sph);
            store_global(E.st_trig + 1 * ns + slot, S.tg.cph);
            store_global(E.st_trig + 2 * ns + slot, S.tg.sth);
            store_global(E.st_trig + 3 * ns + slot, S.tg.cth);
        }
    }
    flush_counts<kStats>(cnt, E, lane);
}

// Updates of a fit taken in Joseph form: three hits (six measured
// coordinates) determine the five track parameters.
constexpr int kJosephUpdates = 3;

// ---------------------------------------------------------------------------
// KF fit over a fixed hit list: from the prior (p, c) on layer 0, for each
// layer the scattering of the previous one, propagation, transport, and the
// update with that layer's hit if it has one (hit_of(L) >= 0).  (op, oc) is
// the state after the last update.
template <int kGeo, class HitOf>
__device__ __forceinline__ void fit_track(const Params &P, CEvent &E, float (&p)[6], float (&c)[21],
                                          HitOf hit_of, float (&op)[6], float (&oc)[21], float &chi2, int &nupd,
                                          int &status)
{
#pragma unroll
    for (int i = 0; i < 6; ++i) op[i] = p[i];
#pragma unroll
    for (int i = 0; i < 21; ++i) oc[i] = c[i];
    chi2 = 0.f;
    nupd = 0;
    status = 0;
    // bit 2 of kGeo: the 3x3 measurement (fit kernels only; the build kernels
    // test it at run time)
    constexpr bool kDisk = geo_disk(kGeo), kXyz = geo_xyz(kGeo), kFit3d = (kGeo & 4) != 0;
    Trig tg = trig_of(p);
    if constexpr (!kXyz) {
        // Thin layers: the hit of layer L + 1 is loaded while layer L is
        // updated and layer L + 1 propagated to, by every lane (no hit: any
        // hit of the event, or the first word of its input block when it has
        // none), so that its latency hides behind that arithmetic.  Two
        // layers per iteration in alternating registers keep the wait for a
        // hit next to its use.
        const int nh1 = max(E.n_hits - 1, 0);
        auto hit_at = [&](int L, int h) { return load_global(E.hits + min(E.layer_off[L] + max(h, 0), nh1)); };
        auto step = [&](const int L, const int h, const float4 hv, int &h_next, float4 &hv_next) -> bool {
            const bool more = L + 1 < P.n_layers;
            h_next = more ? hit_of(L + 1) : -1;
            if (L > 0) {
                float np[6], sn, cn;
                if (!predict<kDisk>(p, tg, kDisk ? P.layer[L].zplane : P.layer[L].r, P.w_per_qpt,
                                    P.layer[L - 1].x0, P.mass2, np, sn, cn, c)) {
                    status = 2;
                    return false;
                }
                tg.sph = sn;
                tg.cph = cn;
#pragma unroll
                for (int i = 0; i < 6; ++i) p[i] = np[i];
            }
            if (more) hv_next = hit_at(L + 1, h_next);
            if (h >= 0) {
                // Joseph form for the first updates, as below
                if (nupd < kJosephUpdates) {
                    if (kFit3d) chi2 += kf_update_3d<true>(p, c, tg, hv.x, hv.y, hv.z, P.var_u, P.var_r, P.var_z);
                    else chi2 += kf_update_joseph<kDisk>(p, c, tg, hv.x, hv.y, hv.z, P.var_u, kDisk ? P.var_r : P.var_z);
                } else {
                    if (kFit3d) chi2 += kf_update_3d<false>(p, c, tg, hv.x, hv.y, hv.z, P.var_u, P.var_r, P.var_z);
                    else chi2 += kf_update<kDisk>(p, c, tg, hv.x, hv.y, hv.z, P.var_u, kDisk ? P.var_r : P.var_z);
                }
                ++nupd;
#pragma unroll
                for (int i = 0; i < 6; ++i) op[i] = p[i];
#pragma unroll
                for (int i = 0; i < 21; ++i) oc[i] = c[i];
            }
            return true;
        };
        int ha = hit_of(0), hb = -1;
        float4 va = hit_at(0, ha), vb = va;
        for (int L = 0; L < P.n_layers; L += 2) {
            if (!step(L, ha, va, hb, vb) || L + 1 >= P.n_layers) break;
            if (!step(L + 1, hb, vb, ha, va)) break;
        }
        return;
    }
    for (int L = 0; L < P.n_layers; ++L) {
        const int h = hit_of(L);
        float4 hv = make_float4(1.f, 0.f, 0.f, 0.f);
        float where = kDisk ? P.layer[L].zplane : P.layer[L].r;
        if constexpr (kXyz) {
            // the hit carries (x, y, z): its own surface is the target (the
            // two steps composed)
            if (h >= 0) {
                hv = load_global(E.hits + E.layer_off[L] + h);
                where = kDisk ? hv.z : sqrtf(fmaf(hv.x, hv.x, hv.y * hv.y));
            }
        }
        if (L > 0) {
            float np[6], sn, cn;
            if (!predict<kDisk>(p, tg, where, P.w_per_qpt, P.layer[L - 1].x0, P.mass2, np, sn, cn, c)) {
                status = 2;
                break;
            }
            tg.sph = sn;
            tg.cph = cn;
#pragma unroll
            for (int i = 0; i < 6; ++i) p[i] = np[i];
        }
        if (h >= 0) {
            float ch, sh, g2h;
            if constexpr (kXyz) {
                hv = load_global(E.hits + E.layer_off[L] + h);   // again: short live range across the step
                const float rh = sqrtf(fmaf(hv.x, hv.x, hv.y * hv.y));
                const float irh = fast_rcp(rh);
                ch = hv.x * irh;
                sh = hv.y * irh;
                g2h = kDisk ? rh : hv.z;
            } else {
                hv = load_global(E.hits + E.layer_off[L] + h);
                ch = hv.x;
                sh = hv.y;
                g2h = hv.z;
            }
            // A fit starts from a wide prior: until a few hits have pinned
            // the five parameters, C - K H C subtracts nearly equal numbers
            // and would lose FP32 digits, so those updates take the Joseph
            // form; after them the prediction is about as precise as a hit
            // and the plain form keeps its digits.
            if (nupd < kJosephUpdates) {
                if (kFit3d) chi2 += kf_update_3d<true>(p, c, tg, hv.x, hv.y, hv.z, P.var_u, P.var_r, P.var_z);
                else chi2 += kf_update_joseph<kDisk>(p, c, tg, ch, sh, g2h, P.var_u, kDisk ? P.var_r : P.var_z);
            } else {
                if (kFit3d) chi2 += kf_update_3d<false>(p, c, tg, hv.x, hv.y, hv.z, P.var_u, P.var_r, P.var_z);
                else chi2 += kf_update<kDisk>(p, c, tg, ch, sh, g2h, P.var_u, kDisk ? P.var_r : P.var_z);
            }
            ++nupd;
#pragma unroll
            for (int i = 0; i < 6; ++i) op[i] = p[i];
#pragma unroll
            for (int i = 0; i < 21; ++i) oc[i] = c[i];
        }
    }
}

// One track of a fit with known hits, prior read and results written per
// lane.
template <int kGeo>
__device__ __forceinline__ void fit_known(const Params &P, CEvent &E, const size_t t)
{
    float p[6], c[21], op[6], oc[21], chi2;
    int nupd, status;
#pragma unroll
    for (int i = 0; i < 6; ++i) p[i] = load_global(E.track_par + 6 * t + i);
#pragma unroll
    for (int i = 0; i < 21; ++i) c[i] = load_global(E.track_cov + 21 * t + i);
    fit_track<kGeo>(P, E, p, c, [&](int L) { return load_global(E.track_hits + t * P.n_layers + L); }, op, oc,
                    chi2, nupd, status);
#pragma unroll
    for (int i = 0; i < 6; ++i) store_global(E.fit_par + 6 * t + i, (double)op[i]);
#pragma unroll
    for (int i = 0; i < 21; ++i) store_global(E.fit_cov + 21 * t + i, (double)oc[i]);
    store_global(E.fit_chi2 + t, (double)chi2);
    store_global(E.fit_nupd + t, nupd);
    store_global(E.fit_status + t, status);
}

// Dynamic LDS of the fit kernel per wavefront: 27 priors or results and the
// hit indices of 64 tracks.
__host__ __device__ constexpr int fit_lds_words(int n_layers) { return (27 + n_layers) * kWave; }

// Fit with known hits: one lane per track.  A wavefront whose 64 tracks lie
// in one batch moves their priors, hit lists and results through LDS, so
// that every global access of those transfers is one contiguous run (the
// arrays are track-major: a lane's own words lie 24 to 84 bytes apart from
// its neighbour's); a wavefront across a batch boundary, or at the end of
// the grid, takes one pass per batch with per-lane accesses instead.
template <int kGeo>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(geo_xyz(kGeo) ? 3 : 4))) k_fit(const Params P, const BatchArgs B)
{
    extern __shared__ int s_dyn[];
    const int lane = threadIdx.x & (kWave - 1);
    const int g0 = uniform(xcd_contiguous(blockIdx.x, gridDim.x) * blockDim.x + (threadIdx.x & ~(kWave - 1)));
    if (g0 >= B.total_tracks) return;
    const int g = g0 + lane;
    const int e0 = uniform(upper_bound_i32(B.track_prefix, B.n_events + 1, g0) - 1);
    if (g0 + kWave <= load_global(B.track_prefix + e0 + 1)) {
        CEvent &E = event_desc(B.events, e0);
        const size_t t0 = (size_t)(g0 - load_global(B.track_prefix + e0));
        const int nl = P.n_layers;
        float *sp = reinterpret_cast<float *>(s_dyn + (threadIdx.x >> 6) * fit_lds_words(nl));   // [64][6]
        float *sc = sp + 6 * kWave;                                                            // [64][21]
        int *sh = reinterpret_cast<int *>(sc + 21 * kWave);                                    // [64][nl]
        const float *gp = E.track_par + 6 * t0, *gc = E.track_cov + 21 * t0;
        const int *gh = E.track_hits + t0 * nl;
#pragma unroll
        for (int k = 0; k < 6; ++k) sp[k * kWave + lane] = load_global(gp + k * kWave + lane);
#pragma unroll
        for (int k = 0; k < 21; ++k) sc[k * kWave + lane] = load_global(gc + k * kWave + lane);
        for (int k = 0; k < nl; ++k) sh[k * kWave + lane] = load_global(gh + k * kWave + lane);
        wave_lds_sync();
        float p[6], c[21], op[6], oc[21], chi2;
        int nupd, status;
#pragma unroll
        for (int i = 0; i < 6; ++i) p[i] = sp[6 * lane + i];
#pragma unroll
        for (int i = 0; i < 21; ++i) c[i] = sc[21 * lane + i];
        fit_track<kGeo>(P, E, p, c, [&](int L) { return sh[nl * lane + L]; }, op, oc, chi2, nupd, status);
        wave_lds_sync();   // every prior read before the results take its place
#pragma unroll
        for (int i = 0; i < 6; ++i) sp[6 * lane + i] = op[i];
#pragma unroll
        for (int i = 0; i < 21; ++i) sc[21 * lane + i] = oc[i];
        wave_lds_sync();
        double *fp = E.fit_par + 6 * t0, *fc = E.fit_cov + 21 * t0;
#pragma unroll
        for (int k = 0; k < 6; ++k) store_global(fp + k * kWave + lane, (double)sp[k * kWave + lane]);
#pragma unroll
        for (int k = 0; k < 21; ++k) store_global(fc + k * kWave + lane, (double)sc[k * kWave + lane]);
        store_global(E.fit_chi2 + t0 + lane, (double)chi2);
        store_global(E.fit_nupd + t0 + lane, nupd);
        store_global(E.fit_status + t0 + lane, status);
        return;
    }
    if (g >= B.total_tracks) return;
    const int e_lane = upper_bound_i32(B.track_prefix, B.n_events + 1, g) - 1;
    // one pass per batch the wave's lanes cover (two where a batch boundary
    // falls inside the wave), each with a wave-uniform descriptor
    for (;;) {
        const int e = uniform(e_lane);
        if (e_lane != e) continue;
        CEvent &E = event_desc(B.events, e);
        fit_known<kGeo>(P, E, (size_t)(g - load_global(B.track_prefix + e)));
        break;
    }
}

// Prior of the final fit of a built track: the helix through its hits on
// layers 0, 1 and 2 (the transverse circle through the three points; z
// linear in the arc length), at the first hit, with a loose diagonal
// covariance in the frame (u, z, q/pT, phi, theta) of the layer tangent at
// that hit, (u, r, q/pT, phi, theta) on a disk: sigma = (1 cm, 10 cm,
// 1 / GeV, 0.1, 0.1).  FP32 from the event's packed hits; false without
// three usable points.
template <bool kDisk>
__device__ __forceinline__ bool final_fit_prior(CEvent &E, const Params &P, const int *hits, float (&p)[6],
                                                float (&c)[21])
{
    float q[3][3];
    for (int L = 0; L < 3; ++L) {
        const int h = hits[L];
        if (h < 0) return false;
        // the hit's position from its packed form: (x, y, z, -), or
        // (cos, sin, z, r) on a cylinder and (cos, sin, r, z) on a disk
        const float4 v = load_global(E.hits + E.layer_off[L] + h);
        if (geo_xyz(P.geo)) {
            q[L][0] = v.x;
            q[L][1] = v.y;
            q[L][2] = v.z;
        } else {
            const float r = kDisk ? v.z : v.w;
            q[L][0] = r * v.x;
            q[L][1] = r * v.y;
            q[L][2] = kDisk ? v.w : v.z;
        }
    }
    const float d1x = q[1][0] - q[0][0], d1y = q[1][1] - q[0][1];   // first to second
    const float d3x = q[2][0] - q[0][0], d3y = q[2][1] - q[0][1];   // first to third
    const float ex = q[2][0] - q[1][0], ey = q[2][1] - q[1][1];
    const float l1 = sqrtf(fmaf(d1x, d1x, d1y * d1y)), l3 = sqrtf(fmaf(d3x, d3x, d3y * d3y));
    const float l2 = sqrtf(fmaf(ex, ex, ey * ey));
    const float twice_area = fmaf(d1x, d3y, -d1y * d3x);
    if (!(l1 > 0.f && l2 > 0.f && l3 > 0.f) || twice_area == 0.f) return false;
    const float curv = 2.f * twice_area / (l1 * l2 * l3);           // > 0 turning counter-clockwise
    // tangent at the first point: the chord to the second point, turned back
    // by half the angle the arc between them sweeps
    const float half = asinf(fminf(1.f, fmaxf(-1.f, 0.5f * curv * l1)));
    const float phi = wrap_pi(atan2f(d1y, d1x) - half);
    const float u3 = 0.5f * curv * l3;
    const float arc3 = fabsf(u3) < 1e-4f ? l3 * fmaf(u3 * u3, 1.f / 6.f, 1.f)
                                         : 2.f * asinf(fminf(1.f, fmaxf(-1.f, u3))) / curv;
    const float theta = 0.5f * kPi - atanf((q[2][2] - q[0][2]) / arc3);
    p[0] = q[0][0];
    p[1] = q[0][1];
    p[2] = q[0][2];
    p[3] = curv / P.w_per_qpt;
    p[4] = phi;
    p[5] = theta;
    float sa, ca;
    sincosf(atan2f(q[0][1], q[0][0]), &sa, &ca);
#pragma unroll
    for (int i = 0; i < 21; ++i) c[i] = 0.f;
    if (!kDisk) {
        c[sym(0, 0)] = sa * sa;
        c[sym(0, 1)] = -sa * ca;
        c[sym(1, 1)] = ca * ca;
        c[sym(2, 2)] = 100.f;
    } else {
        c[sym(0, 0)] = fmaf(100.f * ca, ca, sa * sa);
        c[sym(0, 1)] = 99.f * sa * ca;
        c[sym(1, 1)] = fmaf(100.f * sa, sa, ca * ca);
    }
    c[sym(3, 3)] = 1.f;
    c[sym(4, 4)] = 0.01f;
    c[sym(5, 5)] = 0.01f;
    return true;
}

// Final fit of one built track, its hits from the build's output.
template <int kGeo>
__device__ __forceinline__ void refit_built(const Params &P, CEvent &E, const size_t t)
{
    const int *hits = E.out_hits + t * P.n_layers;
    float p[6], c[21], op[6], oc[21], chi2 = 0.f;
    int nupd = 0, status = 3;
    if (final_fit_prior<geo_disk(kGeo)>(E, P, hits, p, c))
        fit_track<kGeo>(P, E, p, c, [&](int L) { return load_global(hits + L); }, op, oc, chi2, nupd, status);
    else {
#pragma unroll
        for (int i = 0; i < 6; ++i) op[i] = 0.f;
#pragma unroll
        for (int i = 0; i < 21; ++i) oc[i] = 0.f;
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) store_global(E.rf_par + 6 * t + i, (double)op[i]);
#pragma unroll
    for (int i = 0; i < 21; ++i) store_global(E.rf_cov + 21 * t + i, (double)oc[i]);
    store_global(E.rf_chi2 + t, (double)chi2);
    store_global(E.rf_nupd + t, nupd);
    store_global(E.rf_status + t, status);
}

// Final fit of every built track of a batch (after the build): one lane per
// seed.  A wavefront whose 64 seeds lie in one event moves their hit lists in
// and their results out through LDS (as the fit does), so that each transfer
// is one contiguous run instead of 64 rows 40 to 168 bytes apart.
template <int kGeo>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(geo_xyz(kGeo) ? 3 : 4))) k_refit(const Params P, const BatchArgs B)
{
    extern __shared__ int s_dyn[];
    const int lane = threadIdx.x & (kWave - 1);
    const int g0 = uniform(xcd_contiguous(blockIdx.x, gridDim.x) * blockDim.x + (threadIdx.x & ~(kWave - 1)));
    if (g0 >= B.total_seeds) return;
    const int g = g0 + lane;
    const int e0 = uniform(upper_bound_i32(B.seed_prefix, B.n_events + 1, g0) - 1);
    if (g0 + kWave <= load_global(B.seed_prefix + e0 + 1)) {
        CEvent &E = event_desc(B.events, e0);
        const size_t t0 = (size_t)(g0 - load_global(B.seed_prefix + e0));
        const int nl = P.n_layers;
        float *sp = reinterpret_cast<float *>(s_dyn + (threadIdx.x >> 6) * fit_lds_words(nl));   // [64][6]
        float *sc = sp + 6 * kWave;                                                            // [64][21]
        int *sh = reinterpret_cast<int *>(sc + 21 * kWave);                                    // [64][nl]
        const int *gh = E.out_hits + t0 * nl;
        for (int k = 0; k < nl; ++k) sh[k * kWave + lane] = load_global(gh + k * kWave + lane);
        wave_lds_sync();
        const int *hits = sh + nl * lane;
        int h3[3];
#pragma unroll
        for (int L = 0; L < 3; ++L) h3[L] = hits[L];
        float p[6], c[21], op[6], oc[21], chi2 = 0.f;
        int nupd = 0, status = 3;
        if (final_fit_prior<geo_disk(kGeo)>(E, P, h3, p, c))
            fit_track<kGeo>(P, E, p, c, [&](int L) { return hits[L]; }, op, oc, chi2, nupd, status);
        else {
#pragma unroll
            for (int i = 0; i < 6; ++i) op[i] = 0.f;
#pragma unroll
            for (int i = 0; i < 21; ++i) oc[i] = 0.f;
        }
#pragma unroll
        for (int i = 0; i < 6; ++i) sp[6 * lane + i] = op[i];
#pragma unroll
        for (int i = 0; i < 21; ++i) sc[21 * lane + i] = oc[i];
        wave_lds_sync();
        double *fp = E.rf_par + 6 * t0, *fc = E.rf_cov + 21 * t0;
#pragma unroll
        for (int k = 0; k < 6; ++k) store_global(fp + k * kWave + lane, (double)sp[k * kWave + lane]);
#pragma unroll
        for (int k = 0; k < 21; ++k) store_global(fc + k * kWave + lane, (double)sc[k * kWave + lane]);
        store_global(E.rf_chi2 + t0 + lane, (double)chi2);
        store_global(E.rf_nupd + t0 + lane, nupd);
        store_global(E.rf_status + t0 + lane, status);
        return;
    }
    if (g >= B.total_seeds) return;
    const int e_lane = upper_bound_i32(B.seed_prefix, B.n_events + 1, g) - 1;
    // one pass per event the wave's lanes cover, as in k_fit
    for (;;) {
        const int e = uniform(e_lane);
        if (e_lane != e) continue;
        CEvent &E = event_desc(B.events, e);
        refit_built<kGeo>(P, E, (size_t)(g - load_global(B.seed_prefix + e)));
        break;
    }
}

// ---------------------------------------------------------------------------
// The no-allocation builder's batch descriptors: one fixed array in device
// memory per GPU, kept until the process ends.  Host code reaches it only
// through the address hipGetSymbolAddress returns for the current device.

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
static std::atomic<void *> g_scratch_addr[64];

hipError_t noalloc_scratch_init(int device)
{
    if (g_scratch_addr[device & 63].load()) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[device & 63].store(p);
    return hipSuccess;
}

void *noalloc_scratch(int device) { return g_scratch_addr[device & 63].load(); }

// ---------------------------------------------------------------------------
// launchers

static inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t launch_fill_i32(int *ptr, int value, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_fill_i32<<<blocks_for(n, 256), 256, 0, s>>>(ptr, value, n);
    return hipGetLastError();
}

hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s)
{
    const size_t n = bytes / 16;
    if (n == 0) return hipSuccess;
    const unsigned grid = (unsigned)std::min<size_t>((n + 255) / 256, 256 * 64);
    k_copy16<<<grid, 256, 0, s>>>(static_cast<const float4 *>(src), static_cast<float4 *>(dst), n);
    return hipGetLastError();
}

hipError_t launch_calib_fma(float *dst, int n_blocks, int iters, hipStream_t s)
{
    k_calib_fma<<<n_blocks, 256, 0, s>>>(dst, iters, 0.999999f, 1e-6f);
    return hipGetLastError();
}

int calib_fma_chains() { return kFmaChains; }

hipError_t launch_batch_zero(const BatchArgs &b, hipStream_t s)
{
    if (b.n_events <= 0) return hipSuccess;
    k_batch_zero<<<blocks_for(5 * b.n_events, 256), 256, 0, s>>>(b);
    return hipGetLastError();
}

// LDS one block may use on the current device (queried once per device;
// lowered to the 64 KB default if a larger launch is refused).
static std::atomic<int> g_lds_limit[64];

static std::atomic<int> g_cu_count[64];

static int compute_units()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    int v = g_cu_count[dev & 63].load();
    if (v <= 0) {
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
        g_cu_count[dev & 63].store(v);
    }
    return v;
}

static size_t lds_per_block()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536 - 1024;
    int v = g_lds_limit[dev & 63].load();
    if (v <= 0) {
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
            v = 65536;
        g_lds_limit[dev & 63].store(v);
    }
    return (size_t)v - 1024;   // room for the kernel's static LDS
}

static void lds_refused()
{
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) g_lds_limit[dev & 63].store(65536);
}

hipError_t launch_index(const Params &p, const BatchArgs &b, hipStream_t s)
{
    if (b.total_hits <= 0) return hipSuccess;
    const size_t nb = (size_t)b.max_bins;   // the batch's largest event grid
    const size_t lds = lds_per_block();
    const unsigned blocks = (unsigned)(b.n_events * p.n_layers);
    const int n_cu = compute_units();
    // chunks per (event, layer) of the per-hit kernels: about one hit per
    // thread for the largest layer, striding beyond that
    const dim3 grid(std::max(1u, std::min(4096u, blocks_for(b.max_layer_hits, 256))), blocks);
    // One block per (event, layer), binning included, from a quarter as many
    // pairs as compute units: measured on ten 20,000-track events, splitting
    // their 100 layers' bins over more blocks only adds re-reads of the bins.
    if ((int)blocks * 4 >= n_cu) {
        const size_t words = b.max_layer_hits <= 0xFFFF ? (nb + 1) / 2 : nb;
        if (words * 4 <= lds) {
            if (b.max_layer_hits <= 0xFFFF) k_index_layer<true><<<blocks, 1024, words * 4, s>>>(p, b);
            else k_index_layer<false><<<blocks, 1024, words * 4, s>>>(p, b);
            const hipError_t err = hipGetLastError();
            if (err == hipSuccess) return err;
            lds_refused();   // not launched: the split form below
        }
    }
    // else bin ranges per (event, layer): about one block per compute unit
    const int nsplit = (int)std::max<size_t>(1, std::min<size_t>({(size_t)64, (nb + 63) / 64,
                                                                  (size_t)(n_cu + blocks - 1) / blocks}));
    const size_t chunk = ((nb + nsplit - 1) / nsplit + 63) / 64 * 64;
    const bool fits = chunk * 4 <= lds || (chunk / 2 * 4 <= lds && b.max_layer_hits <= 0xFFFF);
    if (fits) {
        k_index_bin<<<grid, 256, 0, s>>>(p, b);
        const hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    if (fits && b.max_layer_hits <= 0xFFFF) {
        k_index_range<true><<<blocks * nsplit, 1024, (chunk + 1) / 2 * 4, s>>>(p, b, nsplit, (int)chunk);
        if (hipGetLastError() == hipSuccess) return hipSuccess;
        lds_refused();   // not launched: try a smaller form
    } else if (chunk * 4 <= lds) {
        k_index_range<false><<<blocks * nsplit, 1024, chunk * 4, s>>>(p, b, nsplit, (int)chunk);
        if (hipGetLastError() == hipSuccess) return hipSuccess;
        lds_refused();
    }
    // bins beyond one block's LDS: device-wide counting atomics
    k_index_prep<<<grid, 256, 0, s>>>(p, b);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    k_index_scan<<<(unsigned)(b.n_events * p.n_layers), 1024, 0, s>>>(p, b);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    k_index_scatter<<<grid, 256, 0, s>>>(p, b);
    return hipGetLastError();
}

size_t build_lds_bytes(int geo, int n_layers, int wpb)
{
    const size_t search = geo_xyz(geo) ? sizeof(SearchLds<2>) : sizeof(SearchLds<0>);
    return sizeof(int) * (size_t)search_lds_offset(wpb, n_layers) + (size_t)wpb * search;
}

template <int G, bool kStats>
static hipError_t launch_batch_t(const Params &p, const BatchArgs &b, int wpb, int persistent, int n_blocks,
                                 hipStream_t s)
{
    const unsigned grid = persistent ? (unsigned)n_blocks : blocks_for(b.total_items, wpb);
    if (grid == 0) return hipSuccess;
    const size_t hist = sizeof(int) * (size_t)search_lds_offset(wpb, p.n_layers);
    switch (p.geo) {
    case 0: k_build_batch<G, kStats, 0><<<grid, wpb * kWave, hist + wpb * sizeof(SearchLds<0>), s>>>(p, b, persistent); break;
    case 1: k_build_batch<G, kStats, 1><<<grid, wpb * kWave, hist + wpb * sizeof(SearchLds<1>), s>>>(p, b, persistent); break;
    case 2: k_build_batch<G, kStats, 2><<<grid, wpb * kWave, hist + wpb * sizeof(SearchLds<2>), s>>>(p, b, persistent); break;
    case 3: k_build_batch<G, kStats, 3><<<grid, wpb * kWave, hist + wpb * sizeof(SearchLds<3>), s>>>(p, b, persistent); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_build_batch(const Params &p, const BatchArgs &b, int G, int wpb, int persistent, int n_blocks,
                              bool stats, hipStream_t s)
{
#define MKF_BATCH_CASE(g)                                                                            \
    case g: return stats ? launch_batch_t<g, true>(p, b, wpb, persistent, n_blocks, s)              \
                         : launch_batch_t<g, false>(p, b, wpb, persistent, n_blocks, s);
    switch (G) {
        MKF_BATCH_CASE(1)
        MKF_BATCH_CASE(2)
        MKF_BATCH_CASE(4)
        MKF_BATCH_CASE(6)
        MKF_BATCH_CASE(8)
    default: return hipErrorInvalidValue;
    }
#undef MKF_BATCH_CASE
}

template <int G, bool kStats>
static hipError_t launch_layer_t(const Params &p, const DevEvent *ev_dev, int n_seeds, int L, int wpb,
                                 hipStream_t s)
{
    const int items = (n_seeds + kWave / G - 1) / (kWave / G);
    const unsigned grid = blocks_for(items, wpb);
    if (grid == 0) return hipSuccess;
    switch (p.geo) {
    case 0: k_build_layer<G, kStats, 0><<<grid, wpb * kWave, wpb * sizeof(SearchLds<0>), s>>>(p, ev_dev, L); break;
    case 1: k_build_layer<G, kStats, 1><<<grid, wpb * kWave, wpb * sizeof(SearchLds<1>), s>>>(p, ev_dev, L); break;
    case 2: k_build_layer<G, kStats, 2><<<grid, wpb * kWave, wpb * sizeof(SearchLds<2>), s>>>(p, ev_dev, L); break;
    case 3: k_build_layer<G, kStats, 3><<<grid, wpb * kWave, wpb * sizeof(SearchLds<3>), s>>>(p, ev_dev, L); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_build_layer(const Params &p, const DevEvent *ev_dev, const DevEvent &ev_host, int L, int G,
                              int wpb, bool stats, hipStream_t s)
{
    const int n = ev_host.n_seeds;
#define MKF_LAYER_CASE(g)                                                                            \
    case g: return stats ? launch_layer_t<g, true>(p, ev_dev, n, L, wpb, s)                          \
                         : launch_layer_t<g, false>(p, ev_dev, n, L, wpb, s);
    switch (G) {
        MKF_LAYER_CASE(1)
        MKF_LAYER_CASE(2)
        MKF_LAYER_CASE(4)
        MKF_LAYER_CASE(6)
        MKF_LAYER_CASE(8)
    default: return hipErrorInvalidValue;
    }
#undef MKF_LAYER_CASE
}

hipError_t launch_refit(const Params &p, const BatchArgs &b, hipStream_t s)
{
    if (b.total_seeds <= 0) return hipSuccess;
    const unsigned grid = blocks_for(b.total_seeds, 256);
    const size_t lds = 4 * sizeof(int) * (size_t)fit_lds_words(p.n_layers);
    switch (p.geo | (p.update3d ? 4 : 0)) {
    case 0: k_refit<0><<<grid, 256, lds, s>>>(p, b); break;
    case 1: k_refit<1><<<grid, 256, lds, s>>>(p, b); break;
    case 2: k_refit<2><<<grid, 256, lds, s>>>(p, b); break;
    case 3: k_refit<3><<<grid, 256, lds, s>>>(p, b); break;
    case 6: k_refit<6><<<grid, 256, lds, s>>>(p, b); break;
    case 7: k_refit<7><<<grid, 256, lds, s>>>(p, b); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fit(const Params &p, const BatchArgs &b, hipStream_t s)
{
    if (b.total_tracks <= 0) return hipSuccess;
    const unsigned grid = blocks_for(b.total_tracks, 256);
    const size_t lds = 4 * sizeof(int) * (size_t)fit_lds_words(p.n_layers);
    switch (p.geo | (p.update3d ? 4 : 0)) {
    case 0: k_fit<0><<<grid, 256, lds, s>>>(p, b); break;
    case 1: k_fit<1><<<grid, 256, lds, s>>>(p, b); break;
    case 2: k_fit<2><<<grid, 256, lds, s>>>(p, b); break;
    case 3: k_fit<3><<<grid, 256, lds, s>>>(p, b); break;
    case 6: k_fit<6><<<grid, 256, lds, s>>>(p, b); break;
    case 7: k_fit<7><<<grid, 256, lds, s>>>(p, b); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mkf
