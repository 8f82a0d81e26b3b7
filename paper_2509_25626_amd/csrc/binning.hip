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
//     of rows; for each (chunk, band) a workgroup adds the chunk's clipped
//     rectangles to a 2D difference array in LDS and integrates it, giving
//     how many of the chunk's Gaussians touch each tile of the band
//     (row M[chunk][tile] of a chunk-major count matrix);
//  3. scan: the exclusive scan of M down each tile's column, plus the tile's
//     start (exclusive scan of the column totals over tiles), is the list
//     position of each chunk's first key in each tile; the column totals are
//     the tile ranges and their sum the key count;
//  4. place: for each (chunk, tile row) a workgroup transposes the chunk's
//     keys in that row from Gaussian-major to tile-major in LDS, then writes
//     every tile's stretch of the list as one contiguous run (about 55 keys
//     per tile and chunk at 3M Gaussians and 1 MP).  Its four waves take
//     consecutive quarters of the chunk: each first counts its keys per tile
//     (difference array), the counts fix every wave's start in every tile,
//     then each wave walks its Gaussians in order and drops their indices at
//     its running positions.  A Gaussian's tiles are distinct, so lanes never
//     collide, and the order (wave, then Gaussian) is the visit order.  A row
//     holding more keys than the staging buffer is done in several passes
//     over tile ranges.
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

constexpr int kCountThreads = 256;

__global__ __launch_bounds__(kCountThreads) void k_bin_count(BinPlan p, int64_t n, const uint2* __restrict__ vrect,
                                                             uint32_t* __restrict__ M, uint32_t per_xcd) {
    extern __shared__ int s_diff[];
    int64_t c;
    int b;
    if (!bin_item<false>(p, per_xcd, c, b)) return;
    const int t = threadIdx.x;
    const uint32_t lane = lane_id();
    const int tx = p.tiles_x;
    const int by0 = b * p.band_rows;
    const int rows = min(p.band_rows, p.tiles_y - by0);
    const int stride = tx + 1;
    for (int k = t; k < (rows + 1) * stride; k += kCountThreads) s_diff[k] = 0;
    __syncthreads();
    const int64_t j0 = c * p.chunk;
    const int64_t j1 = min(n, j0 + p.chunk);
    for (int64_t j = j0 + t; j < j1; j += kCountThreads) {
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
    // integrate along x, one row per wave (column tx and row `rows` only
    // collect the closing edges)
    for (int y = t / kWave; y < rows; y += kCountThreads / kWave) {
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
    for (int x = t; x < tx; x += kCountThreads) {
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

// E[c][t] = tile start + keys of t in chunks before c.
__global__ __launch_bounds__(256) void k_bin_down(BinPlan p, const uint32_t* __restrict__ M,
                                                  uint32_t* __restrict__ E, const uint32_t* __restrict__ P,
                                                  const uint32_t* __restrict__ tstart) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= p.ntiles) return;
    const int64_t g = blockIdx.y;
    const int64_t c0 = g * kBinGroup, c1 = min(p.chunks, c0 + kBinGroup);
    uint32_t run = tstart[t] + P[g * p.ntiles + t];
    for (int64_t c = c0; c < c1; ++c) {
        E[c * p.ntiles + t] = run;
        run += M[c * p.ntiles + t];
    }
}

constexpr int kPlaceThreads = 256;
constexpr int kPlaceWaves = kPlaceThreads / kWave;

__global__ __launch_bounds__(kPlaceThreads) void k_bin_place(BinPlan p, int64_t n, const uint32_t* __restrict__ order,
                                                             const uint2* __restrict__ vrect,
                                                             const uint32_t* __restrict__ M,
                                                             const uint32_t* __restrict__ E, uint64_t count,
                                                             uint32_t* __restrict__ values, uint32_t* __restrict__ err,
                                                             uint32_t per_xcd) {
    __shared__ uint32_t s_stage[kBinStage];          // Gaussian indices, tile-major
    __shared__ uint16_t s_tile[kBinStage];           // their tile (x - xa)
    __shared__ uint32_t s_pre[kBinMaxTilesX + 1];    // exclusive prefix of the row's counts
    __shared__ uint32_t s_base[kBinMaxTilesX];       // list position of the chunk's first key per tile
    __shared__ int s_w[kPlaceWaves][kBinMaxTilesX + 1];  // per-wave counts, then running positions
    __shared__ uint32_t s_scan[kPlaceThreads / kWave];
    __shared__ int s_xb;

    // item = (tile row, chunk), row-major: neighbouring chunks of a row write
    // neighbouring stretches of the same tile lists
    const int64_t item = xcd_band(blockIdx.x, per_xcd);
    if (item >= (int64_t)p.tiles_y * p.chunks) return;
    const int y = (int)(item / p.chunks);
    const int64_t c = item - (int64_t)y * p.chunks;
    const int t = threadIdx.x;
    const int w = t / kWave;
    const uint32_t lane = lane_id();
    const int tx = p.tiles_x;
    const uint32_t* Mrow = M + c * p.ntiles + (int64_t)y * tx;
    const uint32_t* Erow = E + c * p.ntiles + (int64_t)y * tx;

    // prefix of the row's per-tile counts (two tiles per thread: tx <= 512)
    static_assert(2 * kPlaceThreads >= kBinMaxTilesX, "two tiles per thread");
    const int xt = 2 * t;
    const uint32_t m0 = xt < tx ? Mrow[xt] : 0u, m1 = xt + 1 < tx ? Mrow[xt + 1] : 0u;
    uint32_t total = 0;
    const uint32_t ex = block_excl_sum<kPlaceThreads>(m0 + m1, s_scan, &total);
    if (xt < tx) {
        s_pre[xt] = ex;
        s_base[xt] = Erow[xt];
    }
    if (xt + 1 < tx) {
        s_pre[xt + 1] = ex + m0;
        s_base[xt + 1] = Erow[xt + 1];
    }
    if (t == 0) s_pre[tx] = total;
    __syncthreads();
    if (total == 0) return;  // uniform

    // the waves' consecutive quarters of the chunk
    const int64_t j0 = c * p.chunk, j1 = min(n, j0 + p.chunk);
    const int64_t q = (j1 - j0 + kPlaceWaves - 1) / kPlaceWaves;
    const int64_t wj0 = min(j1, j0 + w * q), wj1 = min(j1, wj0 + q);
    const uint32_t uy = (uint32_t)y;

    int xa = 0;
    while (xa < tx) {
        // tiles [xa, xb) whose keys fit the staging buffer (one tile always
        // fits: a chunk has at most kBinChunk <= kBinStage keys per tile)
        if (t == 0) {
            int lo = xa + 1, hi = tx;
            while (lo < hi) {
                const int mid = (lo + hi + 1) / 2;
                if (s_pre[mid] - s_pre[xa] <= (uint32_t)kBinStage) lo = mid;
                else hi = mid - 1;
            }
            s_xb = lo;
        }
        for (int k = lane; k <= tx; k += kWave) s_w[w][k] = 0;
        __syncthreads();
        const int xb = s_xb;
        const uint32_t ua = (uint32_t)xa, ub = (uint32_t)(xb - 1);
        const uint32_t pre_a = s_pre[xa];

        // 1. this wave's keys per tile of [xa, xb): difference array
        for (int64_t j = wj0 + lane; j < wj1; j += kWave) {
            uint32_t x0, y0, x1, y1;
            unpack_rect(vrect[j], x0, y0, x1, y1);
            const uint32_t lo = max(x0, ua), hi = min(x1, ub);
            if (y0 <= uy && uy <= y1 && lo <= hi) {
                atomicAdd(&s_w[w][lo - ua], 1);
                atomicAdd(&s_w[w][hi + 1 - ua], -1);
            }
        }
        __syncthreads();
        {
            int carry = 0;
            for (int xc = 0; xc < xb - xa; xc += kWave) {
                const int x = xc + (int)lane;
                const int v = x < xb - xa ? s_w[w][x] : 0;
                const int inc = (int)wave_incl_sum((uint32_t)v) + carry;
                if (x < xb - xa) s_w[w][x] = inc;
                carry = __shfl(inc, kWave - 1, kWave);
            }
        }
        __syncthreads();
        // 2. counts -> each wave's first staging slot in each tile
        for (int x = t; x < xb - xa; x += kPlaceThreads) {
            uint32_t run = s_pre[xa + x] - pre_a;
#pragma unroll
            for (int v = 0; v < kPlaceWaves; ++v) {
                const uint32_t cv = (uint32_t)s_w[v][x];
                s_w[v][x] = (int)run;
                run += cv;
            }
            if (run != s_pre[xa + x + 1] - pre_a) atomicOr(err, 8u);  // counts disagree with M
        }
        __syncthreads();
        // 3. each wave drops its Gaussians, in order, at its running positions
        for (int64_t base = wj0; base < wj1; base += kWave) {
            const int64_t j = base + lane;
            uint32_t lo = 1, hi = 0, gid = 0;
            if (j < wj1) {
                uint32_t x0, y0, x1, y1;
                unpack_rect(vrect[j], x0, y0, x1, y1);
                if (y0 <= uy && uy <= y1) {
                    lo = max(x0, ua);
                    hi = min(x1, ub);
                    gid = order[j];
                }
            }
            uint64_t todo = ballot(lo <= hi);
            while (todo) {
                const int src = __builtin_ctzll(todo);
                todo &= todo - 1;
                const uint32_t g = __builtin_amdgcn_readlane(gid, src);
                const uint32_t glo = __builtin_amdgcn_readlane(lo, src);
                const uint32_t ghi = __builtin_amdgcn_readlane(hi, src);
                for (uint32_t x = glo + lane; x <= ghi; x += kWave) {
                    const uint32_t lx = x - ua;
                    const int slot = s_w[w][lx];
                    s_w[w][lx] = slot + 1;
                    if ((uint32_t)slot < (uint32_t)kBinStage) {
                        s_stage[slot] = g;
                        s_tile[slot] = (uint16_t)lx;
                    }
                }
            }
        }
        __syncthreads();
        // 4. every tile's stretch as one contiguous run
        uint32_t npass = s_pre[xb] - pre_a;
        if (npass > (uint32_t)kBinStage) {  // only with inconsistent counts
            if (t == 0) atomicOr(err, 4u);
            npass = kBinStage;
        }
        for (uint32_t i = t; i < npass; i += kPlaceThreads) {
            const uint32_t lx = s_tile[i];
            if (lx >= (uint32_t)(xb - xa)) {
                atomicOr(err, 4u);
                continue;
            }
            const uint32_t pos = s_base[xa + lx] + (i - (s_pre[xa + lx] - pre_a));
            if ((uint64_t)pos < count) values[pos] = s_stage[i];
            else atomicOr(err, 4u);
        }
        __syncthreads();
        xa = xb;
    }
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

bool bin_supported(int tiles_x, int tiles_y) { return tiles_x >= 1 && tiles_y >= 1 && tiles_x <= kBinMaxTilesX; }

BinPlan bin_plan(int64_t n, int tiles_x, int tiles_y) {
    BinPlan p;
    p.tiles_x = tiles_x;
    p.tiles_y = tiles_y;
    p.ntiles = (int64_t)tiles_x * tiles_y;
    p.band_rows = std::max(1, std::min(kBinMaxBandRows, kBinMaxRowTiles / std::max(tiles_x, 1)));
    p.bands = (tiles_y + p.band_rows - 1) / p.band_rows;
    p.chunk = kBinChunk;
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
    hipLaunchKernelGGL(k_bin_count, dim3(8 * per_xcd), dim3(kCountThreads), bin_lds_bytes(p), stream, p, n, vrect,
                       M, per_xcd);
    return hipGetLastError();
}

hipError_t launch_bin_scan(const BinPlan& p, const uint32_t* M, uint32_t* E, uint32_t* P, uint32_t* tsum,
                           uint2* ranges, uint64_t* total, hipStream_t stream) {
    const unsigned tblocks = (unsigned)((p.ntiles + 255) / 256);
    hipLaunchKernelGGL(k_bin_reduce, dim3(tblocks, (unsigned)p.groups), dim3(256), 0, stream, p, M, P);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bin_colscan, dim3(tblocks), dim3(256), 0, stream, p, P, tsum);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_bin_starts, dim3(1), dim3(kStartThreads), 0, stream, p.ntiles, tsum, ranges, total);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_bin_down, dim3(tblocks, (unsigned)p.groups), dim3(256), 0, stream, p, M, E, P, tsum);
    return hipGetLastError();
}

hipError_t launch_bin_place(const BinPlan& p, int64_t n, const uint32_t* order, const uint2* vrect,
                            const uint32_t* M, const uint32_t* E, uint64_t count, uint32_t* values, uint32_t* err,
                            hipStream_t stream) {
    if (count == 0) return hipSuccess;
    const int64_t items = (int64_t)p.tiles_y * p.chunks;
    const uint32_t per_xcd = per_xcd_for(items);
    hipLaunchKernelGGL(k_bin_place, dim3(8 * per_xcd), dim3(kPlaceThreads), 0, stream, p, n, order, vrect, M, E,
                       count, values, err, per_xcd);
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
