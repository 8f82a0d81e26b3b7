// Per-tile [start, end) ranges in the sorted key list (Algorithm 1, "load
// work range").  One lane per sorted key compares its tile with its
// neighbours'; ranges are zeroed first so empty tiles read (0, 0).  The tile
// of key i is the 32-bit word tile_words[i * stride] (stride 1 for tile ids,
// stride 2 offset by one word for the high halves of 64-bit keys).
#include "device_utils.h"
#include "internal.h"

namespace cds {
namespace {

__global__ __launch_bounds__(256) void k_ranges(const uint32_t* __restrict__ tw, int stride, int64_t count,
                                                uint2* __restrict__ ranges, int64_t ntiles) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const uint32_t tile = tw[i * stride];
    if (tile >= ntiles) return;  // cannot happen for keys made by the duplicate pass
    if (i == 0 || tw[(i - 1) * stride] != tile) ranges[tile].x = (uint32_t)i;
    if (i == count - 1 || tw[(i + 1) * stride] != tile) ranges[tile].y = (uint32_t)(i + 1);
}

// Contiguous 32-bit tile ids: four keys per lane through one 16-byte load.
__global__ __launch_bounds__(256) void k_ranges4(const uint32_t* __restrict__ tw, int64_t count,
                                                 uint2* __restrict__ ranges, int64_t ntiles) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i0 = q * 4;
    if (i0 >= count) return;
    uint32_t v[6];  // v[0] = key i0-1, v[1..4] = keys i0..i0+3, v[5] = key i0+4
    if (i0 + 4 <= count) {
        const uint4 x = *reinterpret_cast<const uint4*>(tw + i0);
        v[1] = x.x; v[2] = x.y; v[3] = x.z; v[4] = x.w;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) v[1 + k] = (i0 + k < count) ? tw[i0 + k] : 0xFFFFFFFFu;
    }
    v[0] = i0 > 0 ? tw[i0 - 1] : 0xFFFFFFFFu;
    v[5] = i0 + 4 < count ? tw[i0 + 4] : 0xFFFFFFFFu;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t i = i0 + k;
        const uint32_t tile = v[1 + k];
        if (i >= count || tile >= ntiles) continue;
        if (v[k] != tile) ranges[tile].x = (uint32_t)i;
        if (v[k + 2] != tile) ranges[tile].y = (uint32_t)(i + 1);
    }
}

}  // namespace

hipError_t launch_ranges(const uint32_t* tile_words, int stride, int64_t count, uint2* ranges,
                         int64_t ntiles, hipStream_t stream) {
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(ranges), 2 * ntiles, 0u, stream);
    if (e != hipSuccess || count <= 0) return e;
    if (stride == 1 && (reinterpret_cast<uintptr_t>(tile_words) & 15) == 0) {
        const int64_t blocks = ((count + 3) / 4 + 255) / 256;
        hipLaunchKernelGGL(k_ranges4, dim3((unsigned)blocks), dim3(256), 0, stream, tile_words, count, ranges,
                           ntiles);
    } else {
        const int64_t blocks = (count + 255) / 256;
        hipLaunchKernelGGL(k_ranges, dim3((unsigned)blocks), dim3(256), 0, stream, tile_words, stride, count,
                           ranges, ntiles);
    }
    return hipGetLastError();
}

}  // namespace cds
