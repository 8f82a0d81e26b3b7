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
// Load balance: a workgroup takes 256 consecutive visit positions and spreads
// their combined output evenly over its 256 lanes (lane e writes outputs
// e, e+256, ...; the owner of an output is found by binary search over the
// group's offsets in LDS), so a Gaussian covering thousands of tiles costs
// the group the same as many small ones and every store is coalesced.
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
    __shared__ uint32_t s_start[kNT];
    __shared__ uint2 s_rect[kNT];
    __shared__ uint32_t s_depth[kNT];
    __shared__ uint32_t s_gid[kNT];
    __shared__ uint32_t s_hist[kMaxPasses * 256];
    __shared__ int s_diff[kMaxPasses * 257];
    __shared__ uint32_t s_all[kMaxPasses];
    __shared__ uint32_t s_range[2];
    const int t = threadIdx.x;
    const bool do_hist = A.hist != nullptr;
    const int passes = A.depth_passes + A.tile_passes;
    if (do_hist) {
        for (int k = t; k < passes * 256; k += kNT) s_hist[k] = 0;
        for (int k = t; k < passes * 257; k += kNT) s_diff[k] = 0;
        if (t < kMaxPasses) s_all[t] = 0;
    }
    const int64_t n = A.n;
    const int64_t groups = (n + kNT - 1) / kNT;
    for (int64_t g = blockIdx.x; g < groups; g += gridDim.x) {
        const int64_t j = g * kNT + t;
        // positions past the end get the largest start so the binary search
        // below never selects them
        uint32_t off = 0xFFFFFFFFu, cnt = 0, gid = 0;
        if (j < n) {
            gid = A.order ? A.order[j] : (uint32_t)j;
            off = A.offsets[j];
            cnt = A.touched[gid];
        }
        __syncthreads();  // the previous group finished reading the LDS arrays
        if (t == 0) s_range[0] = off;
        const int64_t last = (g * kNT + kNT - 1 < n) ? (g * kNT + kNT - 1) : (n - 1);
        if (j == last) s_range[1] = off + cnt;
        s_start[t] = off;
        if (cnt) {
            const uint2 r = A.rect[gid];
            const uint32_t depth = A.depth_bits[gid];
            s_rect[t] = r;
            s_depth[t] = depth;
            s_gid[t] = gid;
            if (do_hist) {
                for (int p = 0; p < A.depth_passes; ++p)
                    atomicAdd(&s_hist[p * 256 + ((depth >> (8 * p)) & 255u)], cnt);
                const uint32_t x0 = r.x & 0xFFFFu, y0 = r.x >> 16, x1 = r.y & 0xFFFFu, y1 = r.y >> 16;
                for (uint32_t ty = y0; ty <= y1; ++ty) {
                    const uint32_t t0 = ty * (uint32_t)A.tiles_x + x0;
                    for (int q = 0; q < A.tile_passes; ++q)
                        add_run(s_hist, s_diff, s_all, A.depth_passes + q, 8 * q, t0, x1 - x0 + 1);
                }
            }
        }
        __syncthreads();
        const uint32_t gbase = s_range[0];
        const uint32_t total = s_range[1] - gbase;
        for (uint32_t e = t; e < total; e += kNT) {
            const uint32_t pos = gbase + e;
            // owner: last lane with s_start <= pos (zero-count lanes share the
            // start of the next one and are skipped by taking the last)
            int lo = 0, hi = kNT - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_start[mid] <= pos) lo = mid; else hi = mid - 1;
            }
            const uint2 r = s_rect[lo];
            const uint32_t x0 = r.x & 0xFFFFu, y0 = r.x >> 16, x1 = r.y & 0xFFFFu;
            const uint32_t w = x1 - x0 + 1;
            const uint32_t local = pos - s_start[lo];
            // local / w via a float estimate and an exact integer fix-up
            uint32_t q = (uint32_t)((float)local * __frcp_rn((float)w));
            int32_t rem = (int32_t)local - (int32_t)(q * w);
            while (rem < 0) { --q; rem += (int32_t)w; }
            while (rem >= (int32_t)w) { ++q; rem -= (int32_t)w; }
            const uint32_t tile = (y0 + q) * (uint32_t)A.tiles_x + (x0 + (uint32_t)rem);
            if (A.keys64) A.keys64[pos] = ((uint64_t)tile << 32) | (uint64_t)s_depth[lo];
            if (A.tiles32) A.tiles32[pos] = tile;
            A.values[pos] = s_gid[lo];
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
                            int tile_passes, hipStream_t stream) {
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
