// Per-tile key counts straight from the splat rectangles, without touching
// the keys: every visible splat covers whole runs of consecutive tile ids
// (one run per rectangle row), so a difference array over the tile ids
// (+1 at a run's first tile, -1 past its last) integrates to the number of
// keys of every tile.  From those counts follow, before any key exists,
//  - the tile ranges of the sorted list (paper Section II-B(1): the start and
//    end of every tile's splats; empty tiles (0, 0)),
//  - the digit histograms of the tile-id radix passes (any digit layout), and
//  - the key count K.
// The runs of a batch of renders use the requests' global tile ids.
#include "device_utils.h"
#include "internal.h"

namespace cds {
namespace {

constexpr int kDiffThreads = 256;

struct DiffArgs {
    int64_t n;
    const uint32_t* touched;
    const uint2* rect;
    int tiles_x;
    int64_t ntiles;
    int* diff;  // [reps][ntiles + 1], zero on entry
    int reps;   // copies of diff the LDS counting kernel spreads its workgroups over
    const uint4* rec;  // tile records of the visible splats instead of touched/rect, or null
    const BatchItem* items;
    int nitems;
    const uint64_t* count_dev;  // when given, the number of splats (n is an upper bound)
};

// +1 / -1 at the ends of every rectangle row's run of tile ids.  Each thread
// loads four splats before adding any, so their loads overlap.
template <bool kLds>
__global__ __launch_bounds__(kDiffThreads) void k_tile_diff(DiffArgs a) {
    constexpr int kUnroll = 4;
    extern __shared__ int s_d[];
    int* d = kLds ? s_d : a.diff;
    if (kLds) {
        for (int64_t k = threadIdx.x; k <= a.ntiles; k += kDiffThreads) s_d[k] = 0;
        __syncthreads();
    }
    const int64_t n = a.count_dev ? (int64_t)*a.count_dev : a.n;
    const int64_t stride = (int64_t)gridDim.x * kDiffThreads;
    for (int64_t i0 = (int64_t)blockIdx.x * kDiffThreads + threadIdx.x; i0 < n; i0 += kUnroll * stride) {
        uint4 q[kUnroll];  // tile records (width | height << 16, stride, -, first tile)
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t i = i0 + u * stride;
            q[u] = make_uint4(0u, 0u, 0u, 0u);
            if (a.rec) {
                if (i < n) q[u] = a.rec[i];
            } else if (i < n && a.touched[i]) {
                uint32_t tx = (uint32_t)a.tiles_x, tb = 0;
                if (a.items) {
                    const int it = find_item_by_gaussian(a.items, a.nitems, i);
                    tx = (uint32_t)a.items[it].P.tiles_x;
                    tb = (uint32_t)a.items[it].tile_base;
                }
                q[u] = make_tile_rec(a.rect[i], tx, tb, 0u);
            }
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const uint32_t w = q[u].x & 0xFFFFu, h = q[u].x >> 16;
            uint32_t t0 = q[u].w;
            for (uint32_t y = 0; y < h; ++y, t0 += q[u].y) {
                atomicAdd(&d[t0], 1);
                atomicAdd(&d[t0 + w], -1);
            }
        }
    }
    if (kLds) {
        __syncthreads();
        int* const rep = a.diff + (int64_t)(blockIdx.x % (uint32_t)a.reps) * (a.ntiles + 1);
        for (int64_t k = threadIdx.x; k <= a.ntiles; k += kDiffThreads) {
            const int v = s_d[k];
            if (v) atomicAdd(&rep[k], v);
        }
    }
}

// Tile grids too large for one LDS array (batched renders, whose tile ids are
// global): a workgroup takes a contiguous chunk of records.  The chunk's
// records mostly belong to one or two requests, whose tile ids span a window
// that fits LDS: the rows are counted there and the window is added to the
// global array once.  A chunk whose window does not fit adds its rows with
// global atomics.  Chunks are large enough that the window flushes (one
// atomic per touched window entry) stay few: at most ~512 workgroups.
constexpr int64_t kDiffChunkMin = (int64_t)kDiffThreads * 32;  // records per workgroup, at least
constexpr int64_t kDiffChunkBlocks = 512;
__global__ __launch_bounds__(kDiffThreads) void k_tile_diff_chunk(DiffArgs a, int64_t chunk) {
    extern __shared__ int s_d[];  // kTileDiffLdsMaxTiles + 1 ints
    __shared__ uint32_t s_lo, s_hi;
    const int64_t n = a.count_dev ? (int64_t)*a.count_dev : a.n;
    const int64_t c0 = (int64_t)blockIdx.x * chunk;
    if (c0 >= n) return;  // uniform
    const int64_t c1 = c0 + chunk < n ? c0 + chunk : n;
    const int t = threadIdx.x;
    if (t == 0) {
        s_lo = 0xFFFFFFFFu;
        s_hi = 0u;
    }
    __syncthreads();
    // window [lo, hi]: every index a row of the chunk adds at
    uint32_t lo = 0xFFFFFFFFu, hi = 0u;
    for (int64_t i = c0 + t; i < c1; i += kDiffThreads) {
        const uint4 q = a.rec[i];  // (width | height << 16, row stride, -, first tile)
        const uint32_t w = q.x & 0xFFFFu, h = q.x >> 16;
        const uint32_t last = h > 0 ? q.w + (h - 1) * q.y + w : q.w;
        lo = q.w < lo ? q.w : lo;
        hi = last > hi ? last : hi;
    }
    atomicMin(&s_lo, lo);
    atomicMax(&s_hi, hi);
    __syncthreads();
    const uint32_t blo = s_lo, bhi = s_hi;
    const bool fits = bhi >= blo && bhi - blo <= (uint32_t)kTileDiffLdsMaxTiles;  // uniform
    if (fits) {
        for (uint32_t k = (uint32_t)t; k <= bhi - blo; k += kDiffThreads) s_d[k] = 0;
        __syncthreads();
    }
    for (int64_t i = c0 + t; i < c1; i += kDiffThreads) {
        const uint4 q = a.rec[i];
        const uint32_t w = q.x & 0xFFFFu, h = q.x >> 16;
        uint32_t t0 = q.w;
        for (uint32_t y = 0; y < h; ++y, t0 += q.y) {
            if (fits) {
                atomicAdd(&s_d[t0 - blo], 1);
                atomicAdd(&s_d[t0 + w - blo], -1);
            } else {
                atomicAdd(&a.diff[t0], 1);
                atomicAdd(&a.diff[t0 + w], -1);
            }
        }
    }
    if (fits) {
        __syncthreads();
        for (uint32_t k = (uint32_t)t; k <= bhi - blo; k += kDiffThreads) {
            const int v = s_d[k];
            if (v) atomicAdd(&a.diff[blo + k], v);
        }
    }
}

// One block: integrate the difference array to per-tile counts, scan them to
// tile starts, and build the tile-digit histograms and K.
constexpr int kRangeThreads = 1024;
__global__ __launch_bounds__(kRangeThreads) void k_tile_ranges(int64_t ntiles, const int* __restrict__ diff,
                                                               uint2* __restrict__ ranges, uint32_t* __restrict__ hist,
                                                               DigitPlan plan, uint64_t* __restrict__ total,
                                                               int reps) {
    const int tile_passes = plan.passes;
    __shared__ uint32_t s_hist[4 * 256];
    __shared__ unsigned long long s_wave[kRangeThreads / kWave];
    __shared__ int s_wcnt[kRangeThreads / kWave];
    __shared__ unsigned long long s_start;
    __shared__ int s_run;
    const int t = threadIdx.x;
    const int w = t / kWave;
    const uint32_t lane = lane_id();
    for (int k = t; k < 4 * 256; k += kRangeThreads) s_hist[k] = 0;
    if (t == 0) {
        s_start = 0;
        s_run = 0;
    }
    __syncthreads();
    for (int64_t base = 0; base < ntiles; base += kRangeThreads) {
        const int64_t i = base + t;
        // count = running sum of the difference array (int: entries may be
        // negative), summed over its copies (loads issued together)
        int x[kTileDiffMaxReps];
#pragma unroll
        for (int r = 0; r < kTileDiffMaxReps; ++r) x[r] = r < reps && i < ntiles ? diff[r * (ntiles + 1) + i] : 0;
        int v = 0;
#pragma unroll
        for (int r = 0; r < kTileDiffMaxReps; ++r) v += x[r];
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int u = __shfl_up(v, (unsigned)o, kWave);
            if (lane >= (uint32_t)o) v += u;
        }
        if (lane == kWave - 1) s_wcnt[w] = v;
        __syncthreads();
        int before = s_run, all = 0;
#pragma unroll
        for (int k = 0; k < kRangeThreads / kWave; ++k) {
            before += k < w ? s_wcnt[k] : 0;
            all += s_wcnt[k];
        }
        const uint32_t cnt = i < ntiles ? (uint32_t)(before + v) : 0u;
        // start = exclusive running sum of the counts (64-bit)
        unsigned long long inc = cnt;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const unsigned long long u = __shfl_up(inc, (unsigned)o, kWave);
            if (lane >= (uint32_t)o) inc += u;
        }
        if (lane == kWave - 1) s_wave[w] = inc;
        __syncthreads();
        unsigned long long sb = s_start, sall = 0;
#pragma unroll
        for (int k = 0; k < kRangeThreads / kWave; ++k) {
            sb += k < w ? s_wave[k] : 0ull;
            sall += s_wave[k];
        }
        if (i < ntiles) {
            const unsigned long long start = sb + inc - cnt;
            ranges[i] = cnt ? make_uint2((uint32_t)start, (uint32_t)(start + cnt)) : make_uint2(0u, 0u);
            if (cnt)
                for (int q = 0; q < tile_passes; ++q)
                    atomicAdd(&s_hist[q * 256 + (uint32_t)((i >> plan.shift[q]) & ((1 << plan.bits[q]) - 1))], cnt);
        }
        __syncthreads();
        if (t == 0) {
            s_run += all;
            s_start += sall;
        }
        __syncthreads();
    }
    if (hist)
        for (int k = t; k < tile_passes * 256; k += kRangeThreads) hist[k] = s_hist[k];
    if (t == 0 && total) *total = s_start;
}

}  // namespace

hipError_t launch_tile_counts(int64_t n, const uint32_t* touched, const uint2* rect, int tiles_x, int64_t ntiles,
                              int* diff, uint2* ranges, uint32_t* hist, const DigitPlan& plan, uint64_t* total,
                              int max_blocks, hipStream_t stream, const BatchItem* items, int nitems,
                              const uint4* rec, const uint64_t* count_dev, int reps) {
    if (ntiles <= 0) return hipSuccess;
    if (plan.passes > 4 || reps < 1 || reps > kTileDiffMaxReps) return hipErrorInvalidValue;
    if (ntiles > kTileDiffLdsMaxTiles) reps = 1;  // only the LDS kernel spreads its flushes
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(diff), reps * (ntiles + 1), 0u, stream);
    if (e != hipSuccess) return e;
    if (n > 0) {
        DiffArgs a;
        a.n = n;
        a.touched = touched;
        a.rect = rect;
        a.tiles_x = tiles_x;
        a.ntiles = ntiles;
        a.diff = diff;
        a.reps = reps;
        a.rec = rec;
        a.items = items;
        a.nitems = nitems;
        a.count_dev = count_dev;
        int64_t blocks = (n + kDiffThreads - 1) / kDiffThreads;
        if (blocks > max_blocks) blocks = max_blocks;
        if (ntiles <= kTileDiffLdsMaxTiles)
            hipLaunchKernelGGL(k_tile_diff<true>, dim3((unsigned)blocks), dim3(kDiffThreads),
                               sizeof(int) * (size_t)(ntiles + 1), stream, a);
        else if (rec) {
            int64_t chunk = (n + kDiffChunkBlocks - 1) / kDiffChunkBlocks;
            if (chunk < kDiffChunkMin) chunk = kDiffChunkMin;
            hipLaunchKernelGGL(k_tile_diff_chunk, dim3((unsigned)((n + chunk - 1) / chunk)), dim3(kDiffThreads),
                               sizeof(int) * (size_t)(kTileDiffLdsMaxTiles + 1), stream, a, chunk);
        }
        else
            hipLaunchKernelGGL(k_tile_diff<false>, dim3((unsigned)blocks), dim3(kDiffThreads), 0, stream, a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_tile_ranges, dim3(1), dim3(kRangeThreads), 0, stream, ntiles, diff, ranges, hist, plan,
                       total, reps);
    return hipGetLastError();
}

}  // namespace cds
