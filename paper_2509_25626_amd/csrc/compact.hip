// Compaction of the visible splats (paper Section II-B(1): only splats that
// overlap some tile are replicated and sorted).  In one pass over the N
// Gaussians in index order:
//   - per 4096-Gaussian tile: the number of visible splats and their keys
//     (tiles touched), scanned to tile bases and to the totals n_vis and K,
//   - a stable compaction (index order kept) of the visible splats' depth
//     bits and of a 16-byte tile record (make_tile_rec), and
//   - the digit histograms of the depth sort over the compacted keys.
// K here is the sum of tiles touched, which does not depend on the order,
// so one host read-back of (n_vis, K) sizes everything that follows.
#include "device_utils.h"
#include "internal.h"

namespace cds {
namespace {

constexpr int kCT = 256;
constexpr int kCIPT = 16;
constexpr int64_t kCTile = (int64_t)kCT * kCIPT;
constexpr int kCWaves = kCT / kWave;

// Word ranges the counting kernel clears on the side: the depth histograms
// the scatter kernel then fills, and whatever the caller adds.
struct ZeroJobs {
    ZeroSpan s[1 + kZeroSpans];
};

// Per 4096-Gaussian tile: visible splats, keys and (with h_sums) the sum of
// the visible splats' rectangle heights.  The grid also clears the word
// ranges of z (grid-strided).
__global__ __launch_bounds__(kCT) void k_vis_count(int64_t n, const uint32_t* __restrict__ touched,
                                                   const uint2* __restrict__ rect,
                                                   uint64_t* __restrict__ vis_sums, uint64_t* __restrict__ key_sums,
                                                   uint64_t* __restrict__ h_sums, ZeroJobs z) {
    __shared__ unsigned long long s_v[kCWaves], s_k[kCWaves], s_h[kCWaves];
    const int64_t base = (int64_t)blockIdx.x * kCTile;
#pragma unroll
    for (int j = 0; j < 1 + kZeroSpans; ++j)
        for (int64_t k = (int64_t)blockIdx.x * kCT + threadIdx.x; k < z.s[j].n; k += (int64_t)gridDim.x * kCT)
            z.s[j].p[k] = 0u;
    uint32_t v = 0, hs = 0;
    unsigned long long k = 0;
    uint32_t c[kCIPT];
    uint2 rc[kCIPT];
    // all loads issued up front (one memory latency)
#pragma unroll
    for (int r = 0; r < kCIPT; ++r) {
        const int64_t i = base + (int64_t)r * kCT + threadIdx.x;
        c[r] = i < n ? touched[i] : 0u;
        rc[r] = h_sums && i < n ? rect[i] : make_uint2(0u, 0u);
    }
#pragma unroll
    for (int r = 0; r < kCIPT; ++r) {
        v += c[r] ? 1u : 0u;
        k += c[r];
        hs += c[r] ? (rc[r].y >> 16) - (rc[r].x >> 16) + 1u : 0u;
    }
    unsigned long long vv = v, hh = hs;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        vv += __shfl_xor(vv, o, kWave);
        k += __shfl_xor(k, o, kWave);
        hh += __shfl_xor(hh, o, kWave);
    }
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) {
        s_v[w] = vv;
        s_k[w] = k;
        s_h[w] = hh;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = 0, b = 0, c = 0;
#pragma unroll
        for (int q = 0; q < kCWaves; ++q) {
            a += s_v[q];
            b += s_k[q];
            c += s_h[q];
        }
        vis_sums[blockIdx.x] = a;
        key_sums[blockIdx.x] = b;
        if (h_sums) h_sums[blockIdx.x] = c;
    }
}

// Wave w of block b takes items [b*4096 + w*1024, +1024) in 16 rounds of 64
// consecutive items; a visible item's slot is the block base (scanned), the
// wave's base within the block, the round's base within the wave and its
// rank among the round's visible lanes (one ballot).
__global__ __launch_bounds__(kCT) void k_vis_scatter(int64_t n, const uint32_t* __restrict__ touched,
                                                     const uint2* __restrict__ rect,
                                                     const uint32_t* __restrict__ depth_bits,
                                                     const uint64_t* __restrict__ vis_base,
                                                     uint32_t* __restrict__ dkey, uint4* __restrict__ rec,
                                                     uint32_t* __restrict__ hist, uint32_t tiles_x,
                                                     const BatchItem* __restrict__ items, int nitems,
                                                     int hist_reps) {
    __shared__ uint32_t s_hist[4 * 256];
    __shared__ uint32_t s_wtot[kCWaves];
    const int t = threadIdx.x;
    const int w = t / kWave;
    const uint32_t lane = lane_id();
    for (int k = t; k < 4 * 256; k += kCT) s_hist[k] = 0;
    const int64_t wbase = (int64_t)blockIdx.x * kCTile + (int64_t)w * (kWave * kCIPT);
    // every round's inputs are loaded up front (one memory latency per wave,
    // not one per round; a line holds visible and culled items alike)
    uint32_t c[kCIPT], dv[kCIPT];
    uint2 rv[kCIPT];
#pragma unroll
    for (int r = 0; r < kCIPT; ++r) {
        const int64_t i = wbase + r * kWave + lane;
        const bool in = i < n;
        c[r] = in ? touched[i] : 0u;
        dv[r] = in ? depth_bits[i] : 0u;
        rv[r] = in ? rect[i] : make_uint2(0u, 0u);
    }
    uint32_t wtot = 0;
#pragma unroll
    for (int r = 0; r < kCIPT; ++r) wtot += (uint32_t)__popcll(ballot(c[r] != 0u));
    if (lane == 0) s_wtot[w] = wtot;
    __syncthreads();
    uint32_t slot = (uint32_t)vis_base[blockIdx.x];
    for (int q = 0; q < w; ++q) slot += s_wtot[q];
#pragma unroll
    for (int r = 0; r < kCIPT; ++r) {
        const int64_t i = wbase + r * kWave + lane;
        const uint64_t m = ballot(c[r] != 0u);
        if (c[r]) {
            const uint32_t pos = slot + count_below(m);
            const uint32_t d = dv[r];
            const uint2 rc = rv[r];
            uint32_t tx = tiles_x, tb = 0;
            if (items) {
                const int it = find_item_by_gaussian(items, nitems, i);
                const bool stacked = items[it].rec_stride > 0;
                tx = (uint32_t)(stacked ? items[it].rec_stride : items[it].P.tiles_x);
                tb = (uint32_t)(stacked ? items[it].rec_base : items[it].tile_base);
            }
            dkey[pos] = d;
            rec[pos] = make_tile_rec(rc, tx, tb, (uint32_t)i);
            // the three low depth bytes spread over their 256 values: plain
            // atomics; the top byte (sign and exponent) takes few values, so
            // its equal digits are merged first
#pragma unroll
            for (int p = 0; p < 3; ++p) atomicAdd(&s_hist[p * 256 + ((d >> (8 * p)) & 255u)], 1u);
            hist_add(s_hist + 3 * 256, d >> 24);
        }
        slot += (uint32_t)__popcll(m);
    }
    __syncthreads();
    uint32_t* const rep = hist + (size_t)(blockIdx.x % (uint32_t)hist_reps) * (4 * 256);
    for (int k = t; k < 4 * 256; k += kCT) {
        const uint32_t v = s_hist[k];
        if (v) atomicAdd(&rep[k], v);
    }
}

}  // namespace

int64_t compact_sums_size(int64_t n) { return (n + kCTile - 1) / kCTile + 1; }
int64_t compact_tiles(int64_t n) { return (n + kCTile - 1) / kCTile; }
int compact_tile_groups() { return (int)(kCTile / 256); }

hipError_t launch_compact_visible(int64_t n, const uint32_t* touched, const uint2* rect, const uint32_t* depth_bits,
                                  uint64_t* vis_sums, uint64_t* key_sums, uint64_t* totals, uint32_t* dkey,
                                  uint4* rec, uint32_t* depth_hist, hipStream_t stream, int tiles_x,
                                  const BatchItem* items, int nitems, uint64_t* h_sums, uint64_t* sum_h,
                                  const ZeroSpan* zero_spans, uint64_t* host_totals, hipEvent_t totals_ready) {
    const int64_t tiles = (n + kCTile - 1) / kCTile;
    if (sum_h && !h_sums) return hipErrorInvalidValue;
    ZeroJobs z;
    z.s[0].p = depth_hist;
    z.s[0].n = 4 * 256;
    for (int j = 0; j < kZeroSpans; ++j)
        if (zero_spans) z.s[1 + j] = zero_spans[j];
    hipError_t e = hipSuccess;
    if (tiles > 0) {
        hipLaunchKernelGGL(k_vis_count, dim3((unsigned)tiles), dim3(kCT), 0, stream, n, touched, rect, vis_sums,
                           key_sums, sum_h ? h_sums : nullptr, z);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    } else {
        for (int j = 0; j < 1 + kZeroSpans; ++j)
            if ((e = launch_fill_u32(z.s[j].p, z.s[j].n, 0u, stream)) != hipSuccess) return e;
    }
    if ((e = launch_scan_u64_pair(vis_sums, key_sums, tiles, totals, totals + 1, stream, sum_h ? h_sums : nullptr,
                                  sum_h, host_totals, host_totals ? host_totals + 1 : nullptr,
                                  host_totals ? host_totals + 3 : nullptr)) != hipSuccess)
        return e;
    if (totals_ready && (e = hipEventRecord(totals_ready, stream)) != hipSuccess) return e;
    if (tiles > 0) {
        hipLaunchKernelGGL(k_vis_scatter, dim3((unsigned)tiles), dim3(kCT), 0, stream, n, touched, rect, depth_bits,
                           vis_sums, dkey, rec, depth_hist, (uint32_t)tiles_x, items, nitems, 1);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_compact_counted(int64_t n, const PreCounts& c, const uint32_t* touched, const uint2* rect,
                                  const uint32_t* depth_bits, uint64_t* vis_sums, uint64_t* key_sums,
                                  uint64_t* h_sums, uint64_t* totals, uint64_t* sum_h, uint32_t* dkey, uint4* rec,
                                  uint32_t* depth_hist, hipStream_t stream, int tiles_x, uint64_t* host_totals) {
    static_assert(kCTile % 256 == 0, "a compaction tile spans whole preprocess workgroups");
    const int64_t tiles = (n + kCTile - 1) / kCTile;
    if ((sum_h != nullptr) != (h_sums != nullptr) || (sum_h && !c.h) || !c.vis || !c.keys ||
        c.group != (int)(kCTile / 256) || c.stride != tiles)
        return hipErrorInvalidValue;
    ScanGroups g;
    g.src_a = c.vis;
    g.src_b = c.keys;
    g.src_c = c.h;
    g.src_count = preprocess_blocks(n);
    g.group = (int)(kCTile / 256);
    hipError_t e = launch_scan_u64_pair(vis_sums, key_sums, tiles, totals, totals + 1, stream, h_sums, sum_h,
                                        host_totals, host_totals ? host_totals + 1 : nullptr,
                                        host_totals ? host_totals + 3 : nullptr, &g);
    if (e != hipSuccess) return e;
    if (tiles > 0) {
        hipLaunchKernelGGL(k_vis_scatter, dim3((unsigned)tiles), dim3(kCT), 0, stream, n, touched, rect, depth_bits,
                           vis_sums, dkey, rec, depth_hist, (uint32_t)tiles_x, nullptr, 0, kDepthHistReps);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace cds
