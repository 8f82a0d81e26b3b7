// Key duplication (paper Section II-B(1): each splat is replicated for every
// 16x16 tile it overlaps).  Key = (tile id << 32) | IEEE bits of the float32
// view depth; value = Gaussian index.  The keys of the j-th Gaussian visited
// occupy [offset[j], offset[j] + touched) in row-major tile order.
//
// Gaussians are visited either in index order or, when `order` is given, in
// the (depth, index) order produced by the per-Gaussian depth sort; in the
// latter case only the 32-bit tile ids are written (the depth digits are
// already sorted) and the 64-bit keys can be rebuilt from the values.
//
// Work split: each wave takes 64 consecutive visit positions and emits their
// Gaussians one after another, each Gaussian's keys spread over the 64 lanes
// (lane c writes keys c, c+64, ...), so stores are coalesced and a Gaussian
// covering thousands of tiles keeps the whole wave busy; the Gaussian's
// rectangle and offset are broadcast from its lane with readlane.
//
// The same pass builds the radix-sort digit histograms without touching each
// key: depth digits are per Gaussian (weight = tiles touched), and the tile
// digits of one rectangle row form a run of consecutive tile ids, added as a
// difference array (low byte) or as at most a few constant chunks (higher
// bytes).
#include "device_utils.h"
#include "internal.h"

namespace cds {
namespace {

constexpr int kNT = 256;
constexpr int kMaxPasses = 8;

struct DupArgs {
    int64_t n;
    const uint32_t* order;     // visit order (null: identity)
    const uint32_t* offsets;   // [n] per visit position
    const uint32_t* touched;   // [n] per Gaussian
    const uint2* rect;         // [n] per Gaussian
    const uint32_t* depth_bits;
    int tiles_x;
    uint64_t* keys64;          // 64-bit keys, or null
    uint32_t* tiles32;         // 32-bit tile ids, or null
    uint32_t* values;
    uint32_t* hist;            // [passes][256] or null
    int depth_passes;          // leading depth-digit passes in hist (0 or 4)
    int tile_passes;           // following tile-digit passes
    const BatchItem* items;    // batched render: per-scene tile layout (null: one scene)
    int nitems;
};

// +1 for every value v in [v0, v0 + len) on the histogram of (v >> shift) & 255.
__device__ __forceinline__ void add_run(uint32_t* s_hist, int* s_diff, uint32_t* s_all, int p, int shift,
                                        uint32_t v0, uint32_t len) {
    if (shift == 0) {
        const uint32_t full = len >> 8, rem = len & 255u;
        if (full) atomicAdd(&s_all[p], full);
        if (rem) {
            const uint32_t st = (v0 + (full << 8)) & 255u;
            int* d = s_diff + p * 257;
            atomicAdd(&d[st], 1);
            if (st + rem <= 256u) {
                atomicAdd(&d[st + rem], -1);
            } else {
                atomicAdd(&d[256], -1);
                atomicAdd(&d[0], 1);
                atomicAdd(&d[st + rem - 256u], -1);
            }
        }
    } else {
        uint32_t v = v0;
        const uint64_t end = (uint64_t)v0 + len;
        while (v < end) {
            const uint64_t next = ((uint64_t)(v >> shift) + 1) << shift;
            const uint32_t stop = (uint32_t)(next < end ? next : end);
            atomicAdd(&s_hist[p * 256 + ((v >> shift) & 255u)], stop - v);
            v = stop;
        }
    }
}

__global__ __launch_bounds__(kNT) void k_duplicate(DupArgs A) {
    __shared__ uint32_t s_hist[kMaxPasses * 256];
    __shared__ int s_diff[kMaxPasses * 257];
    __shared__ uint32_t s_all[kMaxPasses];
    const int t = threadIdx.x;
    const uint32_t lane = lane_id();
    const bool do_hist = A.hist != nullptr;
    const int passes = A.depth_passes + A.tile_passes;
    if (do_hist) {
        for (int k = t; k < passes * 256; k += kNT) s_hist[k] = 0;
        for (int k = t; k < passes * 257; k += kNT) s_diff[k] = 0;
        if (t < kMaxPasses) s_all[t] = 0;
        __syncthreads();
    }
    const int64_t n = A.n;
    const uint32_t tiles_x = (uint32_t)A.tiles_x;
    const int64_t wave = (int64_t)blockIdx.x * (kNT / kWave) + t / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * (kNT / kWave);
    for (int64_t base = wave * kWave; base < n; base += nwaves * kWave) {
        const int64_t j = base + lane;
        uint32_t off = 0, cnt = 0, gid = 0, depth = 0, tx_n = tiles_x, tbase = 0;
        uint2 r = make_uint2(0u, 0u);
        if (j < n) {
            gid = A.order ? A.order[j] : (uint32_t)j;
            off = A.offsets[j];
            cnt = A.touched[gid];
            if (cnt) {
                r = A.rect[gid];
                depth = A.depth_bits[gid];
                if (A.items) {
                    const int it = find_item_by_gaussian(A.items, A.nitems, gid);
                    tx_n = (uint32_t)A.items[it].P.tiles_x;
                    tbase = (uint32_t)A.items[it].tile_base;
                }
            }
        }
        uint64_t todo = ballot(cnt != 0);
        while (todo) {
            // one Gaussian at a time, its keys spread over the 64 lanes
            const int src = __builtin_ctzll(todo);
            todo &= todo - 1;
            const uint32_t g_off = __builtin_amdgcn_readlane(off, src);
            const uint32_t g_cnt = __builtin_amdgcn_readlane(cnt, src);
            const uint32_t g_id = __builtin_amdgcn_readlane(gid, src);
            const uint32_t g_depth = __builtin_amdgcn_readlane(depth, src);
            const uint32_t rx = __builtin_amdgcn_readlane(r.x, src);
            const uint32_t ry = __builtin_amdgcn_readlane(r.y, src);
            const uint32_t g_tx = __builtin_amdgcn_readlane(tx_n, src);
            const uint32_t g_tb = __builtin_amdgcn_readlane(tbase, src);
            const uint32_t x0 = rx & 0xFFFFu, y0 = rx >> 16, x1 = ry & 0xFFFFu, y1 = ry >> 16;
            const uint32_t w = x1 - x0 + 1;
            const float inv_w = __frcp_rn((float)w);
            for (uint32_t c = lane; c < g_cnt; c += kWave) {
                // c / w via a float estimate and an exact integer fix-up
                uint32_t q = (uint32_t)((float)c * inv_w);
                int32_t rem = (int32_t)c - (int32_t)(q * w);
                while (rem < 0) { --q; rem += (int32_t)w; }
                while (rem >= (int32_t)w) { ++q; rem -= (int32_t)w; }
                const uint32_t tile = g_tb + (y0 + q) * g_tx + (x0 + (uint32_t)rem);
                const uint32_t pos = g_off + c;
                if (A.keys64) A.keys64[pos] = ((uint64_t)tile << 32) | (uint64_t)g_depth;
                if (A.tiles32) A.tiles32[pos] = tile;
                A.values[pos] = g_id;
            }
            if (do_hist) {
                if (lane == 0)
                    for (int p = 0; p < A.depth_passes; ++p)
                        atomicAdd(&s_hist[p * 256 + ((g_depth >> (8 * p)) & 255u)], g_cnt);
                for (uint32_t ty = y0 + lane; ty <= y1; ty += kWave) {
                    const uint32_t t0 = g_tb + ty * g_tx + x0;
                    for (int q = 0; q < A.tile_passes; ++q)
                        add_run(s_hist, s_diff, s_all, A.depth_passes + q, 8 * q, t0, w);
                }
            }
        }
    }
    if (do_hist) {
        __syncthreads();
        // difference arrays of the low-byte tile digits -> counts
        if (t < kWave) {
            for (int q = 0; q < A.tile_passes; ++q) {
                const int p = A.depth_passes + q;
                int* d = s_diff + p * 257;
                int carry = 0;
                for (int c = 0; c < 4; ++c) {
                    const int b = c * kWave + t;
                    const int v = d[b];
                    int inc = (int)wave_incl_sum((uint32_t)v);
                    const int tot = __shfl(inc, kWave - 1, kWave);
                    s_hist[p * 256 + b] += (uint32_t)(carry + inc) + s_all[p];
                    carry += tot;
                }
            }
        }
        __syncthreads();
        for (int k = t; k < passes * 256; k += kNT) {
            const uint32_t c = s_hist[k];
            if (c) atomicAdd(&A.hist[k], c);
        }
    }
}

// 64-bit keys from sorted tile ids and values: key = tile << 32 | depth bits of the value.
__global__ __launch_bounds__(256) void k_make_keys(const uint32_t* __restrict__ tiles,
                                                   const uint32_t* __restrict__ values,
                                                   const uint32_t* __restrict__ depth_bits, int64_t count,
                                                   uint64_t* __restrict__ keys) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) keys[i] = ((uint64_t)tiles[i] << 32) | (uint64_t)depth_bits[values[i]];
}

}  // namespace

hipError_t launch_duplicate(int64_t n, const uint32_t* order, const uint32_t* offsets, const uint32_t* touched,
                            const uint2* rect, const uint32_t* depth_bits, int tiles_x, uint64_t* keys64,
                            uint32_t* tiles32, uint32_t* values, uint32_t* hist, int depth_passes,
                            int tile_passes, hipStream_t stream, const BatchItem* items, int nitems) {
    if (n == 0) return hipSuccess;
    if (depth_passes + tile_passes > kMaxPasses) return hipErrorInvalidValue;
    DupArgs A;
    A.n = n;
    A.order = order;
    A.offsets = offsets;
    A.touched = touched;
    A.rect = rect;
    A.depth_bits = depth_bits;
    A.tiles_x = tiles_x;
    A.keys64 = keys64;
    A.tiles32 = tiles32;
    A.values = values;
    A.hist = hist;
    A.depth_passes = depth_passes;
    A.tile_passes = tile_passes;
    A.items = items;
    A.nitems = nitems;
    const int64_t groups = (n + kNT - 1) / kNT;
    const int64_t grid = groups < 2048 ? groups : 2048;
    hipLaunchKernelGGL(k_duplicate, dim3((unsigned)grid), dim3(kNT), 0, stream, A);
    return hipGetLastError();
}

hipError_t launch_make_keys(const uint32_t* tiles, const uint32_t* values, const uint32_t* depth_bits,
                            int64_t count, uint64_t* keys, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_make_keys, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream, tiles,
                       values, depth_bits, count, keys);
    return hipGetLastError();
}

}  // namespace cds
