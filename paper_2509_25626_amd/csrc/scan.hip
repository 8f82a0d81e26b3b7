// Exclusive prefix sum of per-Gaussian tile counts -> key offsets and the
// total number of keys ("bounds and ranges" preparation, paper Section II-B).
// The input may be read through a gather index (tile counts in depth order).
// Reduce-then-scan over 4096-element tiles: per-tile sums, a single-block
// scan of the sums, then a rescan that adds each tile's prefix.  Totals are
// kept in 64 bits so an overflow of the 32-bit key space is detected.
#include "device_utils.h"
#include "internal.h"

namespace cds {
namespace {

constexpr int kNT = 256;
constexpr int kIPT = 16;
constexpr int64_t kTileItems = (int64_t)kNT * kIPT;

// Scan input: the tile count of a splat's tile record when `rec` is given,
// else in[gather[i]] or in[i].
struct ScanSrc {
    const uint32_t* in;
    const uint32_t* gather;
    const uint4* rec;
};

__device__ __forceinline__ uint32_t scan_in(const ScanSrc& s, int64_t i) {
    if (s.rec) return tile_rec_area(s.rec[i]);
    return s.gather ? s.in[s.gather[i]] : s.in[i];
}

__global__ __launch_bounds__(kNT) void k_scan_reduce(ScanSrc src, int64_t n, uint64_t* __restrict__ sums,
                                                     const uint64_t* __restrict__ count_dev) {
    if (count_dev) n = (int64_t)*count_dev;  // tiles past it sum to 0
    __shared__ uint32_t scratch[kNT / kWave];
    const int64_t base = (int64_t)blockIdx.x * kTileItems;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kIPT; ++k) {
        const int64_t idx = base + (int64_t)k * kNT + threadIdx.x;
        if (idx < n) s += scan_in(src, idx);
    }
    uint32_t total;
    block_excl_sum<kNT>(s, scratch, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// One block scans the tile sums (exclusive, in place) and writes the total;
// a second and a third block, when launched, do the same for sums2 / total2
// and sums3 / total3.  A block whose host word (host_totals[block], pinned
// host memory) is given writes its total there too.
// With grouped sources (src[block] not null), value idx is instead the sum of
// src[j * count + idx] over j < group (at most 16), where entry (idx, j) is
// source item idx * group + j and items at or past src_count read as 0; the
// scan is written to sums.
struct HostTotals {
    uint64_t* p[3];
};
struct ScanSources {
    const uint64_t* src[3];
    int64_t src_count;
    int group;
};
__global__ __launch_bounds__(1024) void k_scan_sums(uint64_t* __restrict__ sums, int64_t count,
                                                    uint64_t* __restrict__ total, uint64_t* __restrict__ sums2,
                                                    uint64_t* __restrict__ total2, uint64_t* __restrict__ sums3,
                                                    uint64_t* __restrict__ total3, HostTotals host,
                                                    ScanSources srcs) {
    uint64_t* host_total = host.p[0];
    if (blockIdx.x == 1) {  // uniform
        sums = sums2;
        total = total2;
        host_total = host.p[1];
    } else if (blockIdx.x == 2) {
        sums = sums3;
        total = total3;
        host_total = host.p[2];
    }
    const uint64_t* src = srcs.src[blockIdx.x];
    __shared__ uint64_t wsum[1024 / kWave];
    __shared__ uint64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < count; base += 1024) {
        const int64_t idx = base + threadIdx.x;
        uint64_t v = 0;
        if (!src) {  // uniform
            v = idx < count ? sums[idx] : 0;
        } else if (idx < count) {
            // entry j of output idx's group is at j * count + idx: every load coalesced
            uint64_t x[16];
#pragma unroll
            for (int j = 0; j < 16; ++j)
                x[j] = j < srcs.group && idx * srcs.group + j < srcs.src_count ? src[j * count + idx] : 0;
#pragma unroll
            for (int j = 0; j < 16; ++j) v += x[j];
        }
        // inclusive wave scan in 64 bits
        uint64_t inc = v;
        const uint32_t l = lane_id();
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            uint64_t t = __shfl_up(inc, (unsigned)o, kWave);
            if (l >= (uint32_t)o) inc += t;
        }
        const int w = threadIdx.x / kWave;
        if (l == kWave - 1) wsum[w] = inc;
        __syncthreads();
        uint64_t before = 0, all = 0;
        for (int k = 0; k < 1024 / kWave; ++k) {
            before += (k < w) ? wsum[k] : 0;
            all += wsum[k];
        }
        const uint64_t c = carry;
        if (idx < count) sums[idx] = c + before + inc - v;
        __syncthreads();
        if (threadIdx.x == 0) carry = c + all;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *total = carry;
        if (host_total) *host_total = carry;
    }
}

__global__ __launch_bounds__(kNT) void k_scan_down(ScanSrc src, int64_t n, const uint64_t* __restrict__ sums,
                                                   uint32_t* __restrict__ out, uint32_t* __restrict__ owner,
                                                   const uint64_t* __restrict__ count_dev) {
    if (count_dev) n = (int64_t)*count_dev;
    __shared__ uint32_t scratch[kNT / kWave];
    // blocked arrangement: thread t owns items [t*kIPT, (t+1)*kIPT) of the tile
    const int64_t base = (int64_t)blockIdx.x * kTileItems + (int64_t)threadIdx.x * kIPT;
    uint32_t v[kIPT];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kIPT; ++k) {
        v[k] = (base + k < n) ? scan_in(src, base + k) : 0u;
        s += v[k];
    }
    uint32_t run = block_excl_sum<kNT>(s, scratch, nullptr) + (uint32_t)sums[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kIPT; ++k) {
        if (base + k < n) {
            out[base + k] = run;
            if (owner && v[k] > 0u) {
                // chunk starts inside [run, run + v[k])
                const uint32_t last = (run + v[k] - 1u) / (uint32_t)kKeyGenChunk;
                for (uint32_t q = (run + (uint32_t)kKeyGenChunk - 1u) / (uint32_t)kKeyGenChunk; q <= last; ++q)
                    owner[q] = (uint32_t)(base + k);
            }
        }
        run += v[k];
    }
}

}  // namespace

int64_t scan_block_sums_size(int64_t n) { return (n + kTileItems - 1) / kTileItems + 1; }

hipError_t launch_scan_u64_pair(uint64_t* a, uint64_t* b, int64_t count, uint64_t* total_a, uint64_t* total_b,
                                hipStream_t stream, uint64_t* c, uint64_t* total_c, uint64_t* host_a,
                                uint64_t* host_b, uint64_t* host_c, const ScanGroups* groups) {
    if ((c != nullptr) != (total_c != nullptr)) return hipErrorInvalidValue;
    const HostTotals host{{host_a, host_b, c ? host_c : nullptr}};
    ScanSources srcs{{nullptr, nullptr, nullptr}, 0, 1};
    if (groups) {
        srcs = ScanSources{{groups->src_a, groups->src_b, c ? groups->src_c : nullptr}, groups->src_count,
                           groups->group};
        if (srcs.group < 1 || srcs.group > 16 || !srcs.src[0] || !srcs.src[1] || (c && !srcs.src[2]))
            return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_scan_sums, dim3(c ? 3 : 2), dim3(1024), 0, stream, a, count, total_a, b, total_b, c,
                       total_c, host, srcs);
    return hipGetLastError();
}

hipError_t launch_exclusive_scan(const uint32_t* in, const uint32_t* gather, uint32_t* out, int64_t n,
                                 uint64_t* block_sums, uint64_t* total, hipStream_t stream, const uint4* rec,
                                 uint32_t* owner, const uint64_t* count_dev) {
    const int64_t tiles = (n + kTileItems - 1) / kTileItems;
    ScanSrc src;
    src.in = in;
    src.gather = gather;
    src.rec = rec;
    if (tiles > 0) {
        hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)tiles), dim3(kNT), 0, stream, src, n, block_sums,
                           count_dev);
    }
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, stream, block_sums, tiles, total, nullptr, nullptr,
                       nullptr, nullptr, HostTotals{{nullptr, nullptr, nullptr}},
                       ScanSources{{nullptr, nullptr, nullptr}, 0, 1});
    if (tiles > 0) {
        hipLaunchKernelGGL(k_scan_down, dim3((unsigned)tiles), dim3(kNT), 0, stream, src, n, block_sums, out, owner,
                           count_dev);
    }
    return hipGetLastError();
}

}  // namespace cds
