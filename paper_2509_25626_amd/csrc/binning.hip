// Tile binning: the tile-order pass of the key sort (paper Section II-B(1):
// splats replicated per overlapped tile, sorted by tile and depth) done as a
// stable counting sort whose single digit is the whole tile id, fused with
// key duplication.
//
// Once the Gaussians are in (depth bits, index) order -- the per-Gaussian
// depth sort -- the sorted (tile | depth) list is simply every tile's
// Gaussians in that visit order, so no per-key comparison is needed:
//
//  1. gather: the tile rectangles in visit order (empty for culled splats);
//  2. count: the visit order is cut into chunks and the tile grid into bands
//     of rows; for each (chunk, band) one wave adds the chunk's clipped
//     rectangles to a 2D difference array in LDS and integrates it, giving
//     how many of the chunk's Gaussians touch each tile of the band
//     (row M[chunk][tile] of a chunk-major count matrix);
//  3. scan: the exclusive scan of M down each tile's column, plus the tile's
//     start (exclusive scan of the column totals over tiles), is the list
//     position of each chunk's first key in each tile; the column totals are
//     the tile ranges and their sum the key count;
//  4. place: for each (chunk, band) one wave walks the chunk's Gaussians in
//     order, keeps the band's running list positions in LDS, and writes each
//     Gaussian's index at the positions of the tiles it covers.  A
//     Gaussian's tiles are distinct, so the lanes never collide, and walking
//     the chunk in order keeps each tile's list in visit order.
//
// The result (values and ranges) is the one the 64-bit (tile | depth) key
// sort produces; the keys themselves are rebuilt from it only on request.
#include <algorithm>

#include "device_utils.h"
#include "internal.h"

namespace cds {
namespace {

constexpr uint32_t kEmptyRect = 0xFFFFFFFFu;  // x0 = y0 = 0xFFFF > any x1, y1

__device__ __forceinline__ void unpack_rect(uint2 r, uint32_t& x0, uint32_t& y0, uint32_t& x1, uint32_t& y1) {
    x0 = r.x & 0xFFFFu;
    y0 = r.x >> 16;
    x1 = r.y & 0xFFFFu;
    y1 = r.y >> 16;
}

// (chunk, band) work item of a wave-sized block.  Each XCD takes a contiguous
// run of items: chunk-major for counting (the bands of a chunk read the same
// rectangles and write one row of M), band-major for placement (consecutive
// chunks of a band write neighbouring stretches of each tile's list).
template <bool kBandMajor>
__device__ __forceinline__ bool bin_item(const BinPlan& p, uint32_t per_xcd, int64_t& chunk, int& band) {
    const int64_t item = xcd_band(blockIdx.x, per_xcd);
    if (item >= p.chunks * p.bands) return false;
    if (kBandMajor) {
        band = (int)(item / p.chunks);
        chunk = item - (int64_t)band * p.chunks;
    } else {
        chunk = item / p.bands;
        band = (int)(item - chunk * p.bands);
    }
    return true;
}

__global__ __launch_bounds__(256) void k_bin_gather(int64_t n, const uint32_t* __restrict__ order,
                                                    const uint32_t* __restrict__ touched,
                                                    const uint2* __restrict__ rect, uint2* __restrict__ vrect) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const uint32_t g = order[j];
    vrect[j] = touched[g] ? rect[g] : make_uint2(kEmptyRect, 0u);
}

__global__ __launch_bounds__(kWave) void k_bin_count(BinPlan p, int64_t n, const uint2* __restrict__ vrect,
                                                     uint32_t* __restrict__ M, uint32_t per_xcd) {
    extern __shared__ int s_diff[];
    int64_t c;
    int b;
    if (!bin_item<false>(p, per_xcd, c, b)) return;
    const uint32_t lane = threadIdx.x;
    const int tx = p.tiles_x;
    const int by0 = b * p.band_rows;
    const int rows = min(p.band_rows, p.tiles_y - by0);
    const int stride = tx + 1;
    for (int k = lane; k < (rows + 1) * stride; k += kWave) s_diff[k] = 0;
    __syncthreads();
    const int64_t j0 = c * p.chunk;
    const int64_t j1 = min(n, j0 + p.chunk);
    for (int64_t j = j0 + lane; j < j1; j += kWave) {
        uint32_t x0, y0, x1, y1;
        unpack_rect(vrect[j], x0, y0, x1, y1);
        const int ya = max((int)y0, by0), yb = min((int)y1, by0 + rows - 1);
        if (x0 <= x1 && ya <= yb) {
            const int r0 = (ya - by0) * stride, r1 = (yb - by0 + 1) * stride;
            atomicAdd(&s_diff[r0 + x0], 1);
            atomicAdd(&s_diff[r0 + x1 + 1], -1);
            atomicAdd(&s_diff[r1 + x0], -1);
            atomicAdd(&s_diff[r1 + x1 + 1], 1);
        }
    }
    __syncthreads();
    // integrate along x (column tx and row `rows` only collect the closing edges)
    for (int y = 0; y < rows; ++y) {
        int carry = 0;
        for (int xc = 0; xc < tx; xc += kWave) {
            const int x = xc + (int)lane;
            const int v = x < tx ? s_diff[y * stride + x] : 0;
            const int inc = (int)wave_incl_sum((uint32_t)v) + carry;
            if (x < tx) s_diff[y * stride + x] = inc;
            carry = __shfl(inc, kWave - 1, kWave);
        }
    }
    __syncthreads();
    // integrate along y and store the band's counts
    uint32_t* out = M + c * p.ntiles + (int64_t)by0 * tx;
    for (int x = lane; x < tx; x += kWave) {
        int acc = 0;
        for (int y = 0; y < rows; ++y) {
            acc += s_diff[y * stride + x];
            out[(int64_t)y * tx + x] = (uint32_t)acc;
        }
    }
}

// P[g][t] = sum of M[c][t] over the chunks c of group g.
__global__ __launch_bounds__(256) void k_bin_reduce(BinPlan p, const uint32_t* __restrict__ M,
                                                    uint32_t* __restrict__ P) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= p.ntiles) return;
    const int64_t g = blockIdx.y;
    const int64_t c0 = g * kBinGroup, c1 = min(p.chunks, c0 + kBinGroup);
    uint32_t s = 0;
#pragma unroll 8
    for (int64_t c = c0; c < c1; ++c) s += M[c * p.ntiles + t];
    P[g * p.ntiles + t] = s;
}

// Exclusive scan of P down each tile's column; column totals to tsum.
__global__ __launch_bounds__(256) void k_bin_colscan(BinPlan p, uint32_t* __restrict__ P,
                                                     uint32_t* __restrict__ tsum) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= p.ntiles) return;
    uint32_t run = 0;
    for (int64_t g0 = 0; g0 < p.groups; g0 += 8) {
        uint32_t v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = g0 + k < p.groups ? P[(g0 + k) * p.ntiles + t] : 0u;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (g0 + k < p.groups) P[(g0 + k) * p.ntiles + t] = run;
            run += v[k];
        }
    }
    tsum[t] = run;
}

// One block: tile starts = exclusive scan of the column totals (in place),
// ranges (empty tiles (0, 0)), and the key count, summed in 64 bits so that
// a frame with too many keys is detected rather than wrapped.
constexpr int kStartThreads = 1024;
__global__ __launch_bounds__(kStartThreads) void k_bin_starts(int64_t ntiles, uint32_t* __restrict__ tsum,
                                                              uint2* __restrict__ ranges,
                                                              uint64_t* __restrict__ total) {
    __shared__ unsigned long long s_wave[kStartThreads / kWave];
    __shared__ unsigned long long s_carry;
    const int t = threadIdx.x;
    const int w = t / kWave;
    const uint32_t lane = lane_id();
    if (t == 0) s_carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < ntiles; base += kStartThreads) {
        const int64_t i = base + t;
        const uint32_t v = i < ntiles ? tsum[i] : 0u;
        unsigned long long inc = v;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const unsigned long long u = __shfl_up(inc, (unsigned)o, kWave);
            if (lane >= (uint32_t)o) inc += u;
        }
        if (lane == kWave - 1) s_wave[w] = inc;
        __syncthreads();
        unsigned long long before = s_carry, all = 0;
#pragma unroll
        for (int k = 0; k < kStartThreads / kWave; ++k) {
            const unsigned long long s = s_wave[k];
            before += k < w ? s : 0ull;
            all += s;
        }
        const unsigned long long start = before + inc - v;
        if (i < ntiles) {
            tsum[i] = (uint32_t)start;
            ranges[i] = v ? make_uint2((uint32_t)start, (uint32_t)(start + v)) : make_uint2(0u, 0u);
        }
        __syncthreads();
        if (t == 0) s_carry += all;
        __syncthreads();
    }
    if (t == 0) *total = s_carry;
}

// E[c][t] = tile start + keys of t in chunks before c, written over M.
__global__ __launch_bounds__(256) void k_bin_down(BinPlan p, uint32_t* __restrict__ M,
                                                  const uint32_t* __restrict__ P,
                                                  const uint32_t* __restrict__ tstart) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= p.ntiles) return;
    const int64_t g = blockIdx.y;
    const int64_t c0 = g * kBinGroup, c1 = min(p.chunks, c0 + kBinGroup);
    uint32_t run = tstart[t] + P[g * p.ntiles + t];
    for (int64_t c = c0; c < c1; ++c) {
        const uint32_t m = M[c * p.ntiles + t];
        M[c * p.ntiles + t] = run;
        run += m;
    }
}

__global__ __launch_bounds__(kWave) void k_bin_place(BinPlan p, int64_t n, const uint32_t* __restrict__ order,
                                                     const uint2* __restrict__ vrect,
                                                     const uint32_t* __restrict__ E, uint64_t count,
                                                     uint32_t* __restrict__ values, uint32_t* __restrict__ err,
                                                     uint32_t per_xcd) {
    extern __shared__ uint32_t s_run[];
    int64_t c;
    int b;
    if (!bin_item<true>(p, per_xcd, c, b)) return;
    const uint32_t lane = threadIdx.x;
    const uint32_t tx = (uint32_t)p.tiles_x;
    const int by0 = b * p.band_rows;
    const int rows = min(p.band_rows, p.tiles_y - by0);
    const uint32_t nt = (uint32_t)rows * tx;
    const uint32_t* e = E + c * p.ntiles + (int64_t)by0 * tx;
    for (uint32_t k = lane; k < nt; k += kWave) s_run[k] = e[k];
    __syncthreads();
    const int64_t j0 = c * p.chunk;
    const int64_t j1 = min(n, j0 + p.chunk);
    bool bad = false;
    for (int64_t base = j0; base < j1; base += kWave) {
        const int64_t j = base + lane;
        uint32_t gid = 0, x0 = 1, x1 = 0, ya = 1, yb = 0;
        if (j < j1) {
            uint32_t y0, y1;
            unpack_rect(vrect[j], x0, y0, x1, y1);
            ya = max(y0, (uint32_t)by0);
            yb = min(y1, (uint32_t)(by0 + rows - 1));
            gid = order[j];
        }
        uint64_t todo = ballot(x0 <= x1 && ya <= yb);
        while (todo) {
            // one Gaussian at a time, in visit order; its tiles spread over the lanes
            const int src = __builtin_ctzll(todo);
            todo &= todo - 1;
            const uint32_t g = __builtin_amdgcn_readlane(gid, src);
            const uint32_t gx0 = __builtin_amdgcn_readlane(x0, src);
            const uint32_t gx1 = __builtin_amdgcn_readlane(x1, src);
            const uint32_t gya = __builtin_amdgcn_readlane(ya, src);
            const uint32_t gyb = __builtin_amdgcn_readlane(yb, src);
            const uint32_t w = gx1 - gx0 + 1;
            const uint32_t nkeys = w * (gyb - gya + 1);
            const float inv_w = __frcp_rn((float)w);
            const uint32_t row0 = (gya - (uint32_t)by0) * tx + gx0;
            for (uint32_t k = lane; k < nkeys; k += kWave) {
                // k / w via a float estimate and an exact integer fix-up
                uint32_t q = (uint32_t)((float)k * inv_w);
                int32_t rem = (int32_t)k - (int32_t)(q * w);
                while (rem < 0) { --q; rem += (int32_t)w; }
                while (rem >= (int32_t)w) { ++q; rem -= (int32_t)w; }
                const uint32_t lt = row0 + q * tx + (uint32_t)rem;
                const uint32_t pos = s_run[lt];
                s_run[lt] = pos + 1;
                if ((uint64_t)pos < count) values[pos] = g;
                else bad = true;
            }
        }
    }
    // a position outside the list can only come from inconsistent counts
    if (bad) atomicOr(err, 4u);
}

// keys[i] = (tile << 32) | depth bits of values[i], one wave per tile.
__global__ __launch_bounds__(256) void k_keys_from_ranges(const uint2* __restrict__ ranges, int64_t ntiles,
                                                          const uint32_t* __restrict__ values,
                                                          const uint32_t* __restrict__ depth_bits,
                                                          uint64_t* __restrict__ keys) {
    const int64_t tile = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (tile >= ntiles) return;
    const uint2 r = ranges[tile];
    for (uint32_t i = r.x + lane_id(); i < r.y; i += kWave)
        keys[i] = ((uint64_t)tile << 32) | (uint64_t)depth_bits[values[i]];
}

uint32_t per_xcd_for(int64_t items) { return (uint32_t)((items + 7) / 8); }

}  // namespace

bool bin_supported(int tiles_x, int tiles_y) { return tiles_x >= 1 && tiles_y >= 1 && tiles_x <= kBinMaxRowTiles; }

BinPlan bin_plan(int64_t n, int tiles_x, int tiles_y) {
    BinPlan p;
    p.tiles_x = tiles_x;
    p.tiles_y = tiles_y;
    p.ntiles = (int64_t)tiles_x * tiles_y;
    p.band_rows = std::max(1, std::min(kBinMaxBandRows, kBinMaxRowTiles / std::max(tiles_x, 1)));
    p.bands = (tiles_y + p.band_rows - 1) / p.band_rows;
    // chunks of 2048 Gaussians, longer for large tile grids so the count
    // matrix stays near 4 bytes per Gaussian
    p.chunk = kBinChunk * (int)std::max<int64_t>(1, (p.ntiles + 8191) / 8192);
    p.chunks = std::max<int64_t>(1, (n + p.chunk - 1) / p.chunk);
    p.groups = (p.chunks + kBinGroup - 1) / kBinGroup;
    return p;
}

size_t bin_lds_bytes(const BinPlan& p) {
    return sizeof(int) * (size_t)(p.band_rows + 1) * (size_t)(p.tiles_x + 1);
}

hipError_t launch_bin_gather(int64_t n, const uint32_t* order, const uint32_t* touched, const uint2* rect,
                             uint2* vrect, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bin_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, n, order, touched,
                       rect, vrect);
    return hipGetLastError();
}

hipError_t launch_bin_count(const BinPlan& p, int64_t n, const uint2* vrect, uint32_t* M, hipStream_t stream) {
    const int64_t items = p.chunks * p.bands;
    const uint32_t per_xcd = per_xcd_for(items);
    hipLaunchKernelGGL(k_bin_count, dim3(8 * per_xcd), dim3(kWave), bin_lds_bytes(p), stream, p, n, vrect, M,
                       per_xcd);
    return hipGetLastError();
}

hipError_t launch_bin_scan(const BinPlan& p, uint32_t* M, uint32_t* P, uint32_t* tsum, uint2* ranges,
                           uint64_t* total, hipStream_t stream) {
    const unsigned tblocks = (unsigned)((p.ntiles + 255) / 256);
    hipLaunchKernelGGL(k_bin_reduce, dim3(tblocks, (unsigned)p.groups), dim3(256), 0, stream, p, M, P);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bin_colscan, dim3(tblocks), dim3(256), 0, stream, p, P, tsum);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_bin_starts, dim3(1), dim3(kStartThreads), 0, stream, p.ntiles, tsum, ranges, total);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_bin_down, dim3(tblocks, (unsigned)p.groups), dim3(256), 0, stream, p, M, P, tsum);
    return hipGetLastError();
}

hipError_t launch_bin_place(const BinPlan& p, int64_t n, const uint32_t* order, const uint2* vrect,
                            const uint32_t* E, uint64_t count, uint32_t* values, uint32_t* err,
                            hipStream_t stream) {
    if (count == 0) return hipSuccess;
    const int64_t items = p.chunks * p.bands;
    const uint32_t per_xcd = per_xcd_for(items);
    const size_t lds = sizeof(uint32_t) * (size_t)p.band_rows * (size_t)p.tiles_x;
    hipLaunchKernelGGL(k_bin_place, dim3(8 * per_xcd), dim3(kWave), lds, stream, p, n, order, vrect, E, count,
                       values, err, per_xcd);
    return hipGetLastError();
}

hipError_t launch_keys_from_ranges(const uint2* ranges, int64_t ntiles, const uint32_t* values,
                                   const uint32_t* depth_bits, uint64_t* keys, hipStream_t stream) {
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_keys_from_ranges, dim3((unsigned)((ntiles + 3) / 4)), dim3(256), 0, stream, ranges, ntiles,
                       values, depth_bits, keys);
    return hipGetLastError();
}

}  // namespace cds
