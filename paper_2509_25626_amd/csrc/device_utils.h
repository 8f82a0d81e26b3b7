// Device-side helpers for gfx950 (CDNA4, wave64): lane masks, wave and block
// scans, bounded-spin atomics.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cds {

constexpr int kWave = 64;
constexpr int kTile = 16;

__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Number of set bits of `mask` in lanes strictly below this lane.
__device__ __forceinline__ uint32_t count_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Inclusive prefix sum across the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t v) {
    const uint32_t l = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        uint32_t t = __shfl_up(v, (unsigned)o, kWave);
        if (l >= (uint32_t)o) v += t;
    }
    return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Cross-lane exchanges without the LDS crossbar.  DPP controls (gfx9
// encoding): quad permutations (1,0,3,2) and (2,3,0,1) are lane ^ 1 and
// lane ^ 2; a 16-lane row rotated by 8 is lane ^ 8; the half-row mirror maps
// lane i of each 8-lane group to 7 - i, the row mirror i of each row to 15 - i.
constexpr int kDppQuadXor1 = 0xB1;
constexpr int kDppQuadXor2 = 0x4E;
constexpr int kDppRowRor8 = 0x128;
constexpr int kDppRowHalfMirror = 0x141;
constexpr int kDppRowMirror = 0x140;

template <int kCtrl>
__device__ __forceinline__ float dpp_f32(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kCtrl, 0xF, 0xF, false));
}

// Lane pairs 32 apart (v_permlane32_swap: lanes 32-63 of the first operand
// trade places with lanes 0-31 of the second): lanes below 32 get the pair's
// sum of lo, lanes from 32 on the pair's sum of hi.
__device__ __forceinline__ float pair_sum32(float lo, float hi) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(lo), __float_as_uint(hi), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// The same for rows of 16 lanes 16 apart (v_permlane16_swap: odd rows of
// the first operand with even rows of the second): even rows get the pair's
// sum of lo, odd rows of hi.
__device__ __forceinline__ float pair_sum16(float lo, float hi) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(lo), __float_as_uint(hi), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Sum over the wave, in every lane (all lanes active).
__device__ __forceinline__ float wave_sum_dpp(float v) {
    v += dpp_f32<kDppQuadXor1>(v);
    v += dpp_f32<kDppQuadXor2>(v);
    v += dpp_f32<kDppRowHalfMirror>(v);
    v += dpp_f32<kDppRowMirror>(v);
    v = pair_sum16(v, v);
    return pair_sum32(v, v);
}

// Wave sums of eight per-lane values, scattered over the lanes: afterwards
// every lane holds the total of value index (lane >> 3) & 7 (all lanes
// active).  Each butterfly step sends half of the values still held and keeps
// the other half, so the eight sums cost 4 + 2 + 1 + 3 = 10 exchanges instead
// of 8 * 6, all of them permlane swaps and DPP (no LDS round trips).
__device__ __forceinline__ float wave_reduce_scatter8(const float (&v)[8]) {
    const uint32_t l = lane_id();
    float a[4], b[2];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = pair_sum32(v[i], v[4 + i]);  // lanes < 32: values 0-3; else 4-7
#pragma unroll
    for (int i = 0; i < 2; ++i) b[i] = pair_sum16(a[i], a[2 + i]);  // even rows: the lower two
    const bool h3 = (l & 8u) != 0;
    float c = (h3 ? b[1] : b[0]) + dpp_f32<kDppRowRor8>(h3 ? b[0] : b[1]);
    c += dpp_f32<kDppQuadXor1>(c);
    c += dpp_f32<kDppQuadXor2>(c);
    c += dpp_f32<kDppRowHalfMirror>(c);
    return c;
}

// Sum across the 64 lanes of a wave (every lane gets it).
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        uint32_t t = __shfl_xor(v, o, kWave);
        v = t > v ? t : v;
    }
    return v;
}

// Exclusive prefix sum over a block of NT threads (NT a multiple of 64).
// `scratch` holds NT/64 words of LDS.  Every thread of the block must call.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_sum(uint32_t v, uint32_t* scratch, uint32_t* total) {
    static_assert(NT % kWave == 0, "block must be whole waves");
    constexpr int NW = NT / kWave;
    const uint32_t inc = wave_incl_sum(v);
    const int w = threadIdx.x / kWave;
    if (lane_id() == kWave - 1) scratch[w] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        uint32_t s = scratch[k];
        before += (k < w) ? s : 0u;
        all += s;
    }
    __syncthreads();
    if (total) *total = all;
    return before + inc - v;
}

// h[d] += 1 for every active lane.  The first few distinct digits of the wave
// are merged into one atomic each (take the first remaining lane's digit,
// count the lanes sharing it), which removes the serialisation of skewed
// digits such as the exponent byte of a depth; the remaining lanes add one
// by one.
__device__ __forceinline__ void hist_add(uint32_t* h, uint32_t d) {
    uint64_t left = ballot(true);
    const uint32_t lane = lane_id();
#pragma unroll
    for (int it = 0; it < 3; ++it) {
        if (!left) break;
        const int src = __builtin_ctzll(left);
        const uint32_t v = __builtin_amdgcn_readlane(d, src);
        const uint64_t m = ballot(d == v) & left;
        if (lane == (uint32_t)src) atomicAdd(&h[v], (uint32_t)__popcll(m));
        left &= ~m;
    }
    if ((left >> lane) & 1ull) atomicAdd(&h[d], 1u);
}

// Lanes of one wave exchanging values through LDS: the hardware executes a
// wave's LDS operations in issue order, so only the compiler must keep the
// stores before the other lanes' loads (and earlier loads before later
// stores to the same slots).  Emits no instruction.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t atomic_load_agent(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void atomic_store_agent(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// XCD-aware block -> work-item map.  Consecutive workgroup ids are spread
// round-robin over the 8 XCDs of the chip; this sends a contiguous band of
// work items (neighbouring tiles) to each XCD so they share its L2.
// `grid` must be 8 * per_xcd; returns >= count for padding blocks.
__device__ __forceinline__ uint32_t xcd_band(uint32_t bid, uint32_t per_xcd) {
    return (bid & 7u) * per_xcd + (bid >> 3);
}

}  // namespace cds
