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
// Work split: a wave takes 64 consecutive visit positions.  Splats with at
// most kSmall tiles (most of them) are emitted lane-parallel, each lane
// walking its own rectangle; together the 64 lanes write one contiguous
// stretch of the key array per step.  Larger splats are emitted one after
// another with their keys spread over the 64 lanes (lane c writes keys c,
// c+64, ...), so a splat covering thousands of tiles keeps the whole wave
// busy; its rectangle and offset are broadcast from its lane with readlane.
#include "device_utils.h"
#include "internal.h"

namespace cds {
namespace {

constexpr int kNT = 256;
constexpr uint32_t kSmall = 8;

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
    const BatchItem* items;    // batched render: per-scene tile layout (null: one scene)
    int nitems;
    const uint4* rec;          // compacted visible records in visit order (rect, Gaussian index), or null
};

__device__ __forceinline__ void emit(const DupArgs& A, uint32_t pos, uint32_t tile, uint32_t depth, uint32_t gid) {
    if (A.keys64) A.keys64[pos] = ((uint64_t)tile << 32) | (uint64_t)depth;
    if (A.tiles32) A.tiles32[pos] = tile;
    A.values[pos] = gid;
}

__global__ __launch_bounds__(kNT) void k_duplicate(DupArgs A) {
    const uint32_t lane = lane_id();
    const int64_t n = A.n;
    const uint32_t tiles_x = (uint32_t)A.tiles_x;
    const int64_t wave = (int64_t)blockIdx.x * (kNT / kWave) + threadIdx.x / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * (kNT / kWave);
    for (int64_t base = wave * kWave; base < n; base += nwaves * kWave) {
        const int64_t j = base + lane;
        uint32_t off = 0, cnt = 0, gid = 0, depth = 0, tx_n = tiles_x, tbase = 0;
        uint2 r = make_uint2(0u, 0u);
        if (j < n && A.rec) {
            // the record's rectangle as (0, 0)..(width - 1, height - 1) on rows of
            // its stride, offset by its first tile
            const uint4 q = A.rec[j];
            gid = q.z;
            off = A.offsets[j];
            r = make_uint2(0u, ((q.x & 0xFFFFu) - 1u) | (((q.x >> 16) - 1u) << 16));
            cnt = tile_rec_area(q);
            tx_n = q.y;
            tbase = q.w;
            if (A.keys64) depth = A.depth_bits[gid];
        } else if (j < n) {
            gid = A.order ? A.order[j] : (uint32_t)j;
            off = A.offsets[j];
            cnt = A.touched[gid];
            if (cnt) {
                r = A.rect[gid];
                if (A.keys64) depth = A.depth_bits[gid];  // tile-id mode needs no depth
                if (A.items) {
                    const int it = find_item_by_gaussian(A.items, A.nitems, gid);
                    tx_n = (uint32_t)A.items[it].P.tiles_x;
                    tbase = (uint32_t)A.items[it].tile_base;
                }
            }
        }
        const uint32_t x0 = r.x & 0xFFFFu, y0 = r.x >> 16, x1 = r.y & 0xFFFFu;
        // small splats: each lane walks its own rectangle row by row
        if (cnt && cnt <= kSmall) {
            uint32_t x = x0, row = tbase + y0 * tx_n;
            for (uint32_t k = 0; k < cnt; ++k) {
                emit(A, off + k, row + x, depth, gid);
                if (++x > x1) {
                    x = x0;
                    row += tx_n;
                }
            }
        }
        uint64_t todo = ballot(cnt > kSmall);
        while (todo) {
            // one large splat at a time, its keys spread over the 64 lanes
            const int src = __builtin_ctzll(todo);
            todo &= todo - 1;
            const uint32_t g_off = __builtin_amdgcn_readlane(off, src);
            const uint32_t g_cnt = __builtin_amdgcn_readlane(cnt, src);
            const uint32_t g_id = __builtin_amdgcn_readlane(gid, src);
            const uint32_t g_depth = __builtin_amdgcn_readlane(depth, src);
            const uint32_t gx0 = __builtin_amdgcn_readlane(x0, src);
            const uint32_t gy0 = __builtin_amdgcn_readlane(y0, src);
            const uint32_t gx1 = __builtin_amdgcn_readlane(x1, src);
            const uint32_t g_tx = __builtin_amdgcn_readlane(tx_n, src);
            const uint32_t g_tb = __builtin_amdgcn_readlane(tbase, src);
            const uint32_t w = gx1 - gx0 + 1;
            const float inv_w = __frcp_rn((float)w);
            for (uint32_t c = lane; c < g_cnt; c += kWave) {
                // c / w via a float estimate and an exact integer fix-up
                uint32_t q = (uint32_t)((float)c * inv_w);
                int32_t rem = (int32_t)c - (int32_t)(q * w);
                while (rem < 0) { --q; rem += (int32_t)w; }
                while (rem >= (int32_t)w) { ++q; rem -= (int32_t)w; }
                emit(A, g_off + c, g_tb + (gy0 + q) * g_tx + (gx0 + (uint32_t)rem), g_depth, g_id);
            }
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
                            uint32_t* tiles32, uint32_t* values, hipStream_t stream, const BatchItem* items,
                            int nitems, const uint4* rec) {
    if (n == 0) return hipSuccess;
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
    A.items = items;
    A.nitems = nitems;
    A.rec = rec;
    const int64_t groups = (n + kNT - 1) / kNT;
    const int64_t grid = groups < 4096 ? groups : 4096;
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
