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

}  // namespace

hipError_t launch_ranges(const uint32_t* tile_words, int stride, int64_t count, uint2* ranges,
                         int64_t ntiles, hipStream_t stream) {
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(ranges), 2 * ntiles, 0u, stream);
    if (e != hipSuccess || count <= 0) return e;
    const int64_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(k_ranges, dim3((unsigned)blocks), dim3(256), 0, stream, tile_words, stride, count,
                       ranges, ntiles);
    return hipGetLastError();
}

}  // namespace cds
