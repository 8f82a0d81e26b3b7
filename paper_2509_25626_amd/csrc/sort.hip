// Stable LSD radix sort of (32- or 64-bit key, 32-bit value) pairs: the
// per-tile depth order of paper Section II-B(1), done as a depth sort of the
// visible splats followed by a sort of their keys' tile ids.
//
// Every pass is a partitioned counting sort on a digit of up to 8 bits (the
// key bits are split evenly over the passes).  A workgroup (256 threads over
// 4096 keys, or 512 over 8192 for onesweep sorts of 2^23+ 32-bit keys) ranks
// its keys stably in LDS, reorders them by digit and writes each digit run as
// one contiguous, coalesced store (the 8192-key packed-word pass reorders wave
// by wave, so each wave writes its own runs and needs fewer registers).  Ranking is wave64
// native: keys are held "wave-striped" (round r of a wave covers 64
// consecutive input keys), lanes with the same digit are found with one
// ballot per digit bit, and a per-wave per-digit counter in LDS gives each key
// its rank; processing rounds in order keeps the sort stable.
//
// Two ways give a partition the global position of its digit runs:
//  - onesweep (default): each partition publishes its digit counts and sums
//    its predecessors' by decoupled look-back over a status word per
//    (partition, digit) (bits 31..30 = 0 not ready, 1 partition count, 2
//    inclusive prefix).  The status words are device-coherent, so every poll
//    is a memory round trip; with small digits the whole workgroup polls, a
//    window of predecessors per digit at once.  The wait is bounded: after
//    ~2^22 polls a workgroup records an error and proceeds, so a logic error
//    can corrupt the output but never hang the device.
//  - reduce-then-scan: an upsweep kernel counts the digits of every partition
//    into a digit-major [256][partitions] matrix, one exclusive scan of that
//    matrix yields every (digit, partition) base, and the pass kernel reads
//    its bases.  No workgroup ever waits for another.
//
// The first tile pass of a render can generate its keys from the splat
// records instead of reading them (generate_keys), and passes can carry key
// and value as one packed word once they fit (PassArgs::vbits).
#include <algorithm>

#include "device_utils.h"
#include "internal.h"

namespace cds {
namespace {

constexpr int kKPT = kSortKeysPerThread;
constexpr int kNTR = kSortThreads;  // reduce-then-scan workgroups
constexpr int kPR = kNTR * kKPT;
constexpr uint32_t kFlagAgg = 1u << 30;
constexpr uint32_t kFlagIncl = 2u << 30;
constexpr uint32_t kValueMask = (1u << 30) - 1;
constexpr uint32_t kSpinLimit = 1u << 22;
// status words a thread of a 256-thread workgroup reads per look-back poll
// (measured: 8 over 2, 4, 16, 32)
constexpr int kLookBack256 = 8;

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* __restrict__ p, int64_t count,
                                                  uint32_t value) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// Digit histograms of the plan's digits over all keys.
template <typename Key>
__global__ __launch_bounds__(256) void k_sort_histogram(const Key* __restrict__ keys, int64_t count, DigitPlan plan,
                                                        uint32_t* __restrict__ hist) {
    const int passes = plan.passes;
    __shared__ uint32_t s_hist[8 * 256];
    for (int k = threadIdx.x; k < passes * 256; k += blockDim.x) s_hist[k] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const Key key = keys[i];
        for (int p = 0; p < passes; ++p)
            hist_add(s_hist + p * 256, (uint32_t)(key >> plan.shift[p]) & ((1u << plan.bits[p]) - 1u));
    }
    __syncthreads();
    for (int k = threadIdx.x; k < passes * 256; k += blockDim.x) {
        const uint32_t c = s_hist[k];
        if (c) atomicAdd(&hist[k], c);
    }
}

// Lanes of the wave holding the same digit (restricted to `valid` lanes),
// from one ballot per digit bit.  x is all ones where the bit is set, so the
// lanes agreeing with this lane on the bit are ~(m ^ x); one three-input
// bitwise op per half keeps them: v_bitop3(m, p, x) = p & ~(m ^ x), whose
// truth table (true at (m, p, x) = (0, 1, 0) and (1, 1, 1): 0x84) reads the
// same whichever outer operand is the table's high bit.  The bit count is a
// compile-time constant: no branches, and the ballots of different bits are
// independent.
template <int kBits>
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, bool valid) {
    const uint64_t v = ballot(valid);
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
    for (int b = 0; b < kBits; ++b) {
        uint32_t x = (uint32_t)__builtin_amdgcn_sbfe((int)d, b, 1);
        asm("" : "+v"(x));  // compare x itself rather than a re-derived shift of d
        const uint64_t m = ballot(x != 0u);
        lo = __builtin_amdgcn_bitop3_b32((uint32_t)m, lo, x, 0x84);
        hi = __builtin_amdgcn_bitop3_b32((uint32_t)(m >> 32), hi, x, 0x84);
    }
    return ((uint64_t)hi << 32) | lo;
}

// Per-partition digit counts, digit-major: part_hist[d * parts + p].  Counts
// do not depend on order, so plain (skew-aware) LDS atomics suffice.
template <typename Key>
__global__ __launch_bounds__(kNTR) void k_rts_upsweep(const Key* __restrict__ keys, int64_t count, int shift,
                                                     int bits, uint32_t* __restrict__ part_hist, int64_t parts,
                                                     const uint64_t* __restrict__ count_dev) {
    if (count_dev) count = (int64_t)*count_dev;  // partitions past it count nothing
    __shared__ uint32_t s_h[256];
    const int t = threadIdx.x;
    s_h[t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kPR;
    Key k[kKPT];
#pragma unroll
    for (int r = 0; r < kKPT; ++r) {
        const int64_t idx = base + (int64_t)r * kNTR + t;
        k[r] = idx < count ? keys[idx] : (Key)0;
    }
#pragma unroll
    for (int r = 0; r < kKPT; ++r) {
        const int64_t idx = base + (int64_t)r * kNTR + t;
        if (idx < count) hist_add(s_h, (uint32_t)(k[r] >> shift) & ((1u << bits) - 1u));
    }
    __syncthreads();
    part_hist[(int64_t)t * parts + blockIdx.x] = s_h[t];
}

template <typename Key>
struct PassArgs {
    const Key* kin;
    const uint32_t* vin;  // null: the value of input position i is i
    Key* kout;            // null: only the values are written (a last pass whose keys are not needed)
    uint32_t* vout;
    int64_t count;
    int shift;
    int bits;               // digit bits of this pass (1..8): key bits [shift, shift + bits)
    uint32_t dmask;         // (1 << bits) - 1
    const uint32_t* hist;   // onesweep: [256] digit counts of all keys (summed over replicas)
    int hist_reps;          // replicas of the histogram, hist_rep_stride words apart
    int64_t hist_rep_stride;
    uint32_t* status;       // onesweep: [partitions][256]
    uint32_t* counter;      // onesweep: partition-id counter
    const uint32_t* bases;  // reduce-then-scan: [256][partitions] exclusive bases
    int64_t parts;
    uint32_t* err;
    KeyGen gen;  // generated first-pass keys (gen.off non-null): kin and vin unused
    // Packed words (32-bit keys, values of at most vbits bits): once the key
    // bits left for later passes and the value fit one word, a pass writes
    // ((key >> pack_shift) << vbits) | value to vout (and no keys), and the
    // passes after it read such words as their keys.
    uint32_t vbits;         // nonzero: pack the output
    uint32_t pack_shift;
    uint32_t unpack_mask;   // nonzero: keys are packed words, value = key & unpack_mask
    // last pass only: instead of value v, write gather_src[v] (16 B) to gather_dst
    const uint4* gather_src;
    uint4* gather_dst;
    // when given, the number of keys (at most `count`, which sized the grid
    // and the workspace) is read here on the device
    const uint64_t* count_dev;
};

// Digit t's count over all keys: the sum of the histogram's replicas (the
// counting kernel spreads its atomics over several copies of each counter).
template <typename Key>
__device__ __forceinline__ uint32_t hist_total(const PassArgs<Key>& a, int t) {
    uint32_t x[kDepthHistReps];  // the loads issued together (one latency)
#pragma unroll
    for (int r = 0; r < kDepthHistReps; ++r) x[r] = r < a.hist_reps ? a.hist[r * a.hist_rep_stride + t] : 0u;
    uint32_t v = 0;
#pragma unroll
    for (int r = 0; r < kDepthHistReps; ++r) v += x[r];
    return v;
}

// Generated keys (duplication fused into the first tile pass).  Key p
// belongs to the record j with off[j] <= p < off[j + 1]; its key is the
// tile, in row-major order within the record's rectangle, of its rank
// p - off[j] there, and its value the record's Gaussian index.  A wave
// generates its 16 rounds of 64 consecutive keys from the owner jb of its
// first key (owner table of the offset scan) and a window of the records
// from jb on (offsets and records in LDS).
//  - When the window holds every record starting among the wave's keys (the
//    usual case), each record after jb marks its start in a byte per key,
//    stored transposed (key 64 r + l at byte 16 l + r) so that a lane reads
//    the marks of its 16 rounds with one 16-byte load; the round's ballot
//    then gives every lane the number of records starting at or before it,
//    and the owner of its key is jb plus the marks before the round plus
//    that number.
//  - Otherwise the rounds run one after another: with jb the owner of the
//    key before the round, the at most 64 records after it that start
//    inside the round mark their start in a 64-slot array, one ballot gives
//    the owners, and the window moves when a round's candidates leave it.
constexpr int kGenWindow = 256;  // records per wave window

// key of rank c in a tile record's rectangle (make_tile_rec)
__device__ __forceinline__ uint32_t rect_key(uint4 q, uint32_t c) {
    const uint32_t w = q.x & 0xFFFFu;
    // c / w is a row of the rectangle, below 2^16; the estimate from the
    // hardware reciprocal (1 ulp) is within 2^16 * 2^-21 of it, so its
    // truncation is off by at most one, which one step each way corrects
    uint32_t qq = (uint32_t)((float)c * __builtin_amdgcn_rcpf((float)w));
    int32_t rem = (int32_t)c - (int32_t)(qq * w);
    const bool low = rem < 0;  // selects, not branches
    qq = low ? qq - 1u : qq;
    rem = low ? rem + (int32_t)w : rem;
    const bool high = rem >= (int32_t)w;
    qq = high ? qq + 1u : qq;
    rem = high ? rem - (int32_t)w : rem;
    return q.w + qq * q.y + (uint32_t)rem;
}

template <int kRounds>
__device__ __forceinline__ void generate_keys(const KeyGen& g, int64_t count, int64_t wbase, uint32_t* key,
                                              uint32_t* val, uint32_t* s_off, uint4* s_rec, uint32_t* s_mark,
                                              uint4* s_flag) {
    static_assert(kRounds == 16, "one 16-byte mark load per lane");
    const uint32_t l = lane_id();
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        key[r] = 0u;
        val[r] = 0u;
    }
    if (wbase >= count) return;  // uniform: past the last key
    const int64_t wend = wbase + kWave * kRounds;
    // owners of the wave's first key and of the first key after it: the
    // records the wave needs are jb .. jn (the owner table has an entry per
    // chunk start below count)
    int64_t jb = (int64_t)g.owner[wbase / kKeyGenChunk];
    const int64_t jn = wend < count ? (int64_t)g.owner[wend / kKeyGenChunk] : g.n - 1;
    int64_t jw = jb;  // window = records [jw, jw + kGenWindow)
    const int nrec = (int)min<int64_t>((int64_t)kGenWindow, jn - jb + 1);  // records loaded
    for (int k = (int)l; k < nrec; k += kWave) {
        const int64_t j = jw + k;
        if (j < g.n) {
            s_off[k] = g.off[j];
            s_rec[k] = g.rec[j];
        }
    }
    s_flag[l] = make_uint4(0u, 0u, 0u, 0u);
    wave_lds_sync();
    const bool covered = jn - jb < kGenWindow;  // uniform
    if (covered) {
        uint8_t* flag = reinterpret_cast<uint8_t*>(s_flag);
        for (int k = 1 + (int)l; k < nrec; k += kWave) {
            const int64_t sp = (int64_t)s_off[k] - wbase;  // >= 1: j starts after the owner of wbase
            if (sp < wend - wbase) flag[(sp & (kWave - 1)) * 16 + (sp >> 6)] = 1u;
        }
        wave_lds_sync();
        const uint4 mk = s_flag[l];
        const uint32_t mw[4] = {mk.x, mk.y, mk.z, mk.w};
        // 32-bit from here: keys and offsets are below 2^30, window slots below 256
        const uint32_t wb32 = (uint32_t)wbase + l;
        const int64_t left = count - wbase;  // keys of the wave that exist
        const uint32_t nkeys = left < (int64_t)(kWave * kRounds) ? (uint32_t)left : (uint32_t)(kWave * kRounds);
        int kr = (int)(jb - jw);           // window slot of the owner of the key before the round
        constexpr int kGroup = 4;          // rounds whose owner data are read together
#pragma unroll
        for (int g0 = 0; g0 < kRounds; g0 += kGroup) {
            uint4 q[kGroup];
            uint32_t c[kGroup];
#pragma unroll
            for (int i = 0; i < kGroup; ++i) {
                const int r = g0 + i;
                const uint64_t b = ballot(((mw[r >> 2] >> (8 * (r & 3))) & 0xFFu) != 0u);
                // starts at lanes 0..l: those of b >> 1 below the lane, plus lane 0's
                const int k = kr + (int)count_below(b >> 1) + (int)(b & 1u);
                q[i] = s_rec[k];
                c[i] = wb32 + (uint32_t)(r * kWave) - s_off[k];
                kr += __popcll(b);
            }
#pragma unroll
            for (int i = 0; i < kGroup; ++i) {
                if ((uint32_t)((g0 + i) * kWave) + l < nkeys) {
                    key[g0 + i] = rect_key(q[i], c[i]);
                    val[g0 + i] = q[i].z;
                }
            }
        }
        return;
    }
    s_mark[l] = 0u;
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int64_t R = wbase + r * kWave;
        if (R >= count) continue;  // uniform: past the last key
        if (jb + kWave + 1 > jw + kGenWindow) {  // candidates jb .. jb + 64
            jw = jb;
            wave_lds_sync();
            for (int k = (int)l; k < kGenWindow; k += kWave) {
                const int64_t j = jw + k;
                if (j < g.n) {
                    s_off[k] = g.off[j];
                    s_rec[k] = g.rec[j];
                }
            }
            wave_lds_sync();
        }
        const uint32_t stamp = (uint32_t)r + 1u;
        const int64_t jc = jb + 1 + (int64_t)l;
        if (jc < g.n) {
            const int64_t sc = (int64_t)s_off[jc - jw] - R;  // >= 0
            if (sc < kWave) s_mark[sc] = stamp;
        }
        wave_lds_sync();
        const uint64_t starts = ballot(s_mark[l] == stamp);
        wave_lds_sync();
        const uint32_t m = count_below(starts) + (uint32_t)((starts >> l) & 1ull);
        const int64_t p = R + l;
        if (p < count) {
            const int k = (int)(jb + m - jw);
            const uint4 q = s_rec[k];
            key[r] = rect_key(q, (uint32_t)(p - s_off[k]));
            val[r] = q.z;
        }
        jb += __builtin_amdgcn_readlane(m, kWave - 1);
    }
}

// Decoupled look-back of partition pid: the sum of the counts of digit t over
// all earlier partitions (threads t < 2^kBits), after which this partition's
// inclusive prefix is published.  s_tmp: 2 kNT + 512 words of LDS scratch,
// used when the look-back is block-cooperative (more threads than digits).
template <typename Key, int kBits, int kNT>
__device__ __forceinline__ uint32_t look_back(const PassArgs<Key>& a, uint32_t pid, uint32_t tot, uint32_t* st,
                                              uint32_t* s_tmp) {
    constexpr uint32_t kDig = 1u << kBits;
    constexpr int kSeg = kNT >> kBits;  // threads per digit in the look-back
    // status words per thread and poll: a window of kSeg * kLookBack * 256 / kNT
    // predecessors per digit (for 512 threads over 8-bit digits a 32-word window
    // measured slower than this 8)
    constexpr int kLookBack = kLookBack256 * 256 / kNT > 0 ? kLookBack256 * 256 / kNT : 1;
    const int t = threadIdx.x;
    uint32_t excl = 0;
    if (kSeg == 1 && pid > 0) {
        // one thread per digit: each polls on its own, without barriers
        if (t < (int)kDig) {
            int64_t p = (int64_t)pid - 1;
            uint32_t polls = 0;
            while (p >= 0) {
                uint32_t sw[kLookBack];
#pragma unroll
                for (int k = 0; k < kLookBack; ++k)
                    sw[k] = (p - k >= 0) ? atomic_load_agent(a.status + (size_t)(p - k) * 256 + t) : kFlagIncl;
                uint32_t state = 0;
                int consumed = 0;
#pragma unroll
                for (int k = 0; k < kLookBack; ++k) {
                    if (state) continue;
                    const uint32_t f = sw[k] & ~kValueMask;
                    if (f == 0u) {
                        state = 2;
                        continue;
                    }
                    excl += sw[k] & kValueMask;
                    ++consumed;
                    if (f == kFlagIncl) state = 1;
                }
                if (state == 1) break;
                p -= consumed;
                if (state == 2) {
                    if (++polls > kSpinLimit) {
                        atomicOr(a.err, 1u);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            atomic_store_agent(st + t, kFlagIncl | ((excl + tot) & kValueMask));
        }
    } else if (pid > 0) {
        uint32_t* s_sum = s_tmp;             // [kNT] per-thread sums
        uint32_t* s_cnt = s_sum + kNT;        // [kNT] state << 16 | words consumed
        uint32_t* s_dist = s_sum + 2 * kNT;   // [kDig] next distance, 0 = done
        uint32_t* s_acc = s_dist + 256;       // [kDig] sum so far
        const uint32_t d = (uint32_t)t & (kDig - 1u);
        const uint32_t seg = (uint32_t)t >> kBits;
        if (t < (int)kDig) {
            s_dist[t] = 1u;
            s_acc[t] = 0u;
        }
        __syncthreads();
        uint32_t polls = 0;
        for (;;) {
            const uint32_t dist0 = s_dist[d];
            uint32_t sum = 0, state = 0, cnt = 0;  // state: 1 inclusive found, 2 not ready
            if (dist0) {
                const int64_t q0 = (int64_t)pid - dist0 - (int64_t)seg * kLookBack;
                uint32_t sw[kLookBack];
#pragma unroll
                for (int k = 0; k < kLookBack; ++k)
                    sw[k] = (q0 - k >= 0) ? atomic_load_agent(a.status + (size_t)(q0 - k) * 256 + d) : kFlagIncl;
#pragma unroll
                for (int k = 0; k < kLookBack; ++k) {
                    if (state) continue;
                    const uint32_t f = sw[k] & ~kValueMask;
                    if (f == 0u) {
                        state = 2;
                        continue;
                    }
                    sum += sw[k] & kValueMask;
                    ++cnt;
                    if (f == kFlagIncl) state = 1;
                }
            }
            s_sum[t] = sum;
            s_cnt[t] = (state << 16) | cnt;
            __syncthreads();
            int pending = 0;
            if (t < (int)kDig && s_dist[t] != 0u) {
                uint32_t acc = s_acc[t], dist = s_dist[t], stop = 0;
#pragma unroll
                for (int sg = 0; sg < kSeg; ++sg) {
                    if (stop) continue;
                    const uint32_t sc = s_cnt[t + sg * (int)kDig];
                    acc += s_sum[t + sg * (int)kDig];
                    dist += sc & 0xFFFFu;
                    stop = sc >> 16;
                }
                s_acc[t] = acc;
                s_dist[t] = stop == 1u ? 0u : dist;
                pending = stop != 1u;
            }
            if (__syncthreads_count(pending) == 0) break;
            if (++polls > kSpinLimit) {  // uniform
                if (t == 0) atomicOr(a.err, 1u);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (t < (int)kDig) {
            excl = s_acc[t];
            atomic_store_agent(st + t, kFlagIncl | ((excl + tot) & kValueMask));
        }
    }
    return excl;
}

// One partition of one pass.  kFull: the partition has no tail (every key
// valid), compiled separately so the common case carries no bounds checks.
// kPacked: the keys are packed words that hold their values (value = key &
// unpack_mask), so no value is loaded, held or staged.
template <int kNT, typename Key, bool kOnesweep, int kBits, bool kFull, bool kGen, bool kPacked = false,
          bool kLeanRank = false, bool kWaveLocal = false>
__device__ __forceinline__ void sort_pass_body(const PassArgs<Key>& a, uint32_t pid, Key* s_keys, uint32_t* s_vals,
                                               uint32_t (*s_whist)[256], uint32_t* s_gbase, uint32_t* s_scan,
                                               uint32_t digit_info) {
    static_assert(!kPacked || (sizeof(Key) == 4 && !kGen), "packed words are 32-bit keys read from memory");
    constexpr uint32_t kMask = (1u << kBits) - 1u;
    constexpr int kP = kNT * kKPT;       // keys per partition
    constexpr int kWaves = kNT / kWave;
    const int t = threadIdx.x;
    const int w = t / kWave;
    const uint32_t l = lane_id();
    const int64_t base = (int64_t)pid * kP;
    const int64_t wbase = base + (int64_t)w * (kWave * kKPT);

    Key key[kKPT];
    uint32_t val[kKPT];
    if constexpr (kGen) {
        static_assert(sizeof(Key) == 4, "generated keys are 32-bit tile ids");
        static_assert(sizeof(Key) == 4, "generated keys are 32-bit tile ids");
        static_assert(kWave * kKPT == kKeyGenChunk, "a wave generates one owner-table chunk");
        // per-wave window in the reorder buffers, unused until after the ranking:
        // records in the wave's quarter of s_keys, offsets and marks in s_vals'
        static_assert(kGenWindow * sizeof(uint4) <= sizeof(Key) * kP / kWaves, "records fit");
        static_assert((kGenWindow + kWave + 256) * sizeof(uint32_t) <= sizeof(uint32_t) * kP / kWaves,
                      "offsets, slots and marks fit");
        uint4* s_rec = reinterpret_cast<uint4*>(s_keys + (size_t)w * (kP / kWaves));
        uint32_t* s_off = s_vals + (size_t)w * (kP / kWaves);
        generate_keys<kKPT>(a.gen, a.count, wbase, reinterpret_cast<uint32_t*>(key), val, s_off, s_rec,
                            s_off + kGenWindow, reinterpret_cast<uint4*>(s_off + kGenWindow + kWave));
    } else {
#pragma unroll
    for (int r = 0; r < kKPT; ++r) {
        const int64_t idx = wbase + r * kWave + l;
        key[r] = (kFull || idx < a.count) ? a.kin[idx] : (Key)0;
    }
    if constexpr (kPacked) {
        // values stay inside the keys
    } else if (a.unpack_mask) {  // uniform
#pragma unroll
        for (int r = 0; r < kKPT; ++r) val[r] = (uint32_t)key[r] & a.unpack_mask;
    } else if (a.vin) {  // uniform: one clean load loop either way
#pragma unroll
        for (int r = 0; r < kKPT; ++r) {
            const int64_t idx = wbase + r * kWave + l;
            val[r] = (kFull || idx < a.count) ? a.vin[idx] : 0u;
        }
    } else {
#pragma unroll
        for (int r = 0; r < kKPT; ++r) val[r] = (uint32_t)(wbase + r * kWave + l);
    }
    }

    // Stable wave-level ranking.  Per round, the first lane of every digit
    // group adds the group's size to the wave's counter with an LDS atomic;
    // the rounds' atomics do not wait on each other's results (LDS executes a
    // wave's operations in order), and the members then fetch the old count
    // from their group's first lane.
    uint32_t rank[kKPT];
    if constexpr (kLeanRank || kWaveLocal) {
        // each round's old count is fetched as soon as its atomic returns:
        // the LDS latency is exposed per round, but no per-round state is
        // held, which leaves room for more resident workgroups.  The count
        // travels from the group's first lane by ds_bpermute: a store by that
        // lane and loads by the others would be ordered only in the source
        // (the compiler may run the other lanes' loads first).
#pragma unroll
        for (int r = 0; r < kKPT; ++r) {
            const bool valid = kFull || (wbase + r * kWave + l) < a.count;
            const uint32_t d = (uint32_t)(key[r] >> a.shift) & kMask;
            const uint64_t peers = digit_peers<kBits>(d, valid);
            const uint32_t below = count_below(peers);
            const uint32_t first = valid ? (uint32_t)__builtin_ctzll(peers) : l;
            uint32_t pre = 0;
            if (valid && below == 0) pre = atomicAdd(&s_whist[w][d], (uint32_t)__popcll(peers));
            rank[r] = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(first << 2), (int)pre) + below;
        }
    } else {
        uint32_t pre[kKPT], info[kKPT];  // info: below | first lane << 8
#pragma unroll
        for (int r = 0; r < kKPT; ++r) {
            const bool valid = kFull || (wbase + r * kWave + l) < a.count;
            const uint32_t d = (uint32_t)(key[r] >> a.shift) & kMask;
            const uint64_t peers = digit_peers<kBits>(d, valid);
            const uint32_t below = count_below(peers);
            const uint32_t first = valid ? (uint32_t)__builtin_ctzll(peers) : l;
            pre[r] = 0;
            if (valid && below == 0) pre[r] = atomicAdd(&s_whist[w][d], (uint32_t)__popcll(peers));
            info[r] = below | (first << 8);
        }
#pragma unroll
        for (int r = 0; r < kKPT; ++r)
            rank[r] = (uint32_t)__builtin_amdgcn_ds_bpermute((int)((info[r] >> 8) << 2), (int)pre[r]) + (info[r] & 255u);
    }
    if constexpr (kWaveLocal) {
        // Wave-local reorder: each wave sorts its own keys by digit inside its
        // slice of the buffers right after its ranking, so that no key or rank
        // is held across the block scan and the look-back (fewer VGPRs, more
        // resident workgroups), and the scatter writes each wave's digit runs
        // at (wave, digit) offsets.
        static_assert(kOnesweep && kBits <= 6 && sizeof(Key) == 4, "one digit per lane, 32-bit keys");
        constexpr uint32_t kDigW = 1u << kBits;
        constexpr int kWK = kWave * kKPT;                       // keys per wave
        wave_lds_sync();  // the wave's ranking atomics (other lanes) before the reads
        const uint32_t cnt = l < kDigW ? s_whist[w][l] : 0u;
        const uint32_t wst = wave_incl_sum(cnt) - cnt;         // digit l's start inside the slice
        if (l < kDigW) s_whist[w][l] = (wst << 16) | cnt;
        Key* s_wk = s_keys + (size_t)w * kWK;
        uint32_t* s_wv = kPacked ? nullptr : s_vals + (size_t)w * kWK;
        // the digits are recomputed below rather than held through the ranking
#pragma unroll
        for (int r = 0; r < kKPT; ++r) asm volatile("" : "+v"(key[r]));
#pragma unroll
        for (int r = 0; r < kKPT; ++r) {
            const bool valid = kFull || (wbase + r * kWave + l) < a.count;
            const uint32_t d = (uint32_t)(key[r] >> a.shift) & kMask;
            const uint32_t pos = min((uint32_t)__shfl((int)wst, (int)d, kWave) + rank[r], (uint32_t)(kWK - 1));
            if (valid) {
                s_wk[pos] = key[r];
                if constexpr (!kPacked) s_wv[pos] = val[r];
            }
        }
        __syncthreads();
        // thread t < 2^kBits owns digit t: per wave, count (low half) and start in the slice (high half)
        uint32_t x[kWaves];
        uint32_t tot = 0;
#pragma unroll
        for (int v = 0; v < kWaves; ++v) {
            x[v] = t < (int)kDigW ? s_whist[v][t] : 0u;
            tot += x[v] & 0xFFFFu;
        }
        uint32_t* st = a.status + (size_t)pid * 256;
        if (t < (int)kDigW) atomic_store_agent(st + t, (pid == 0 ? kFlagIncl : kFlagAgg) | tot);
        const uint32_t gstart = block_excl_sum<kNT>(digit_info, s_scan, nullptr);  // barriers: counts read
        const uint32_t gb = gstart + look_back<Key, kBits, kNT>(a, pid, tot, st, &s_whist[0][0]);
        __syncthreads();  // the look-back's scratch is free
        if (t < (int)kDigW) {  // position of a slice's slot = its wave's offset for the digit + slot
            uint32_t run = gb;
#pragma unroll
            for (int v = 0; v < kWaves; ++v) {
                s_whist[v][t] = run - (x[v] >> 16);
                run += x[v] & 0xFFFFu;
            }
        }
        __syncthreads();
        const int64_t nw = kFull ? (int64_t)kWK : min((int64_t)kWK, max((int64_t)0, a.count - wbase));
        const uint32_t count32 = (uint32_t)a.count;  // counts are below 2^30
        bool bad = false;  // as in the block-wide scatter below
#pragma unroll
        for (int r = 0; r < kKPT; ++r) {
            const uint32_t i = (uint32_t)(r * kWave) + l;
            if (kFull || (int64_t)i < nw) {
                const Key k = s_wk[i];
                const uint32_t d = (uint32_t)(k >> a.shift) & kMask;
                const uint32_t g = s_whist[w][d] + i;
                if (g < count32) {
                    if (a.kout) a.kout[g] = k;
                    uint32_t v;
                    if constexpr (kPacked)
                        v = (uint32_t)k & a.unpack_mask;
                    else
                        v = s_wv[i];
                    if (a.gather_dst) {  // uniform; values are positions below count
                        if (v < count32)
                            a.gather_dst[g] = a.gather_src[v];
                        else
                            bad = true;
                    } else {
                        a.vout[g] = a.vbits ? ((uint32_t)(k >> a.pack_shift) << a.vbits) | v : v;
                    }
                } else {
                    bad = true;
                }
            }
        }
        if (bad) atomicOr(a.err, 2u);
        return;
    }
    __syncthreads();

    // thread t < 256 owns digit t
    uint32_t tot = 0;
    if (t < 256)
#pragma unroll
        for (int v = 0; v < kWaves; ++v) tot += s_whist[v][t];
    constexpr uint32_t kDig = 1u << kBits;  // digits of this pass
    uint32_t* st = a.status + (size_t)pid * 256;
    if constexpr (kOnesweep)  // publish this partition's counts first
        if (t < (int)kDig) atomic_store_agent(st + t, (pid == 0 ? kFlagIncl : kFlagAgg) | tot);
    const uint32_t bstart = block_excl_sum<kNT>(tot, s_scan, nullptr);
    if (t < 256) {
        uint32_t run = bstart;
#pragma unroll
        for (int v = 0; v < kWaves; ++v) {
            const uint32_t c = s_whist[v][t];
            s_whist[v][t] = run;
            run += c;
        }
    }
    __syncthreads();

    // reorder (key, value) pairs by digit in LDS; a slot can only fall outside
    // the partition with inconsistent counts, and is then clamped
#pragma unroll
    for (int r = 0; r < kKPT; ++r) {
        const bool valid = kFull || (wbase + r * kWave + l) < a.count;
        if (valid) {
            const uint32_t d = (uint32_t)(key[r] >> a.shift) & kMask;
            const uint32_t pos = min(s_whist[w][d] + rank[r], (uint32_t)(kP - 1));
            s_keys[pos] = key[r];
            if constexpr (!kPacked) s_vals[pos] = val[r];
        }
    }
    __syncthreads();  // s_whist is free from here on

    uint32_t gb;  // global position of this partition's first key with digit t
    if constexpr (kOnesweep) {
        const uint32_t gstart = block_excl_sum<kNT>(digit_info, s_scan, nullptr);
        // Look-back.  With 8-bit digits every thread polls for its own digit.
        // With smaller ones it is block-cooperative: every poll, thread t reads kLookBack
        // status words of digit t % kDig, segment t / kDig of the window of
        // kSeg * kLookBack predecessors (device-coherent loads, one memory round
        // trip for the whole window).  Each thread sums its words nearest first
        // up to an inclusive prefix or the first one not ready; the digit's
        // owner then combines its segments in order, and the digit is done at
        // an inclusive prefix, else the next poll starts after what was consumed.
        // The inclusive prefix thus moves kSeg * kLookBack partitions per round
        // trip, which with small digits keeps it ahead of the partitions.
        const uint32_t excl = look_back<Key, kBits, kNT>(a, pid, tot, st, &s_whist[0][0]);
        gb = gstart + excl;
    } else {
        gb = digit_info;
    }
    if (t < 256) s_gbase[t] = gb - bstart;
    __syncthreads();
    // each digit run goes out as a contiguous stretch
    const uint32_t nvalid = kFull ? (uint32_t)kP : (uint32_t)(a.count - base);
    const uint32_t count32 = (uint32_t)a.count;  // counts are below 2^30
    // a position outside the output can only come from inconsistent digit
    // counts: it is recorded, never written
    bool bad = false;
#pragma unroll
    for (int r = 0; r < kKPT; ++r) {
        const uint32_t i = (uint32_t)(r * kNT + t);
        if (kFull || i < nvalid) {
            const Key k = s_keys[i];
            const uint32_t d = (uint32_t)(k >> a.shift) & kMask;
            const uint32_t g = s_gbase[d] + i;
            if (g < count32) {
                if (a.kout) a.kout[g] = k;
                uint32_t v;
                if constexpr (kPacked)
                    v = (uint32_t)k & a.unpack_mask;
                else
                    v = s_vals[i];
                if (a.gather_dst) {  // uniform; values are positions below count
                    if (v < count32)
                        a.gather_dst[g] = a.gather_src[v];
                    else
                        bad = true;
                } else {
                    a.vout[g] = a.vbits ? ((uint32_t)(k >> a.pack_shift) << a.vbits) | v : v;
                }
            } else {
                bad = true;
            }
        }
    }
    if (bad) atomicOr(a.err, 2u);
}

template <int kNT, typename Key, bool kOnesweep, int kBits, bool kGen = false>
__device__ __forceinline__ void sort_pass_kernel(const PassArgs<Key>& a_in) {
    constexpr int kP = kNT * kKPT;
    constexpr int kWaves = kNT / kWave;
    PassArgs<Key> a = a_in;
    if (a.count_dev) a.count = (int64_t)*a.count_dev;
    __shared__ __align__(16) Key s_keys[kP];    // reorder buffer
    __shared__ __align__(16) uint32_t s_vals[kP];
    __shared__ uint32_t s_whist[kWaves][256];   // per-wave digit counters, then offsets
    __shared__ uint32_t s_gbase[256];
    __shared__ uint32_t s_scan[kWaves];
    __shared__ uint32_t s_pid;

    const int t = threadIdx.x;
    // a grid sized for a bound on the count (the count read on the device):
    // workgroups past the partitions the count needs leave before taking an
    // id, so the serialized id atomics are only the needed ones
    if ((int64_t)blockIdx.x * kP >= a.count) return;  // uniform
    if (t == 0) s_pid = kOnesweep ? atomicAdd(a.counter, 1u) : blockIdx.x;
    const uint32_t hist_t = (kOnesweep && t < 256) ? hist_total(a, t) : 0u;
    for (int k = t; k < kWaves * 256; k += kNT) (&s_whist[0][0])[k] = 0;
    __syncthreads();
    const uint32_t pid = s_pid;
    if ((int64_t)pid * kP >= a.count) return;  // uniform: past the keys (device-side count)
    // digit t's count over all keys (onesweep) or this partition's base for it
    // (reduce-then-scan), loaded before the ranking so its latency overlaps
    const uint32_t digit_info = (kOnesweep || t >= 256) ? hist_t : a.bases[(int64_t)t * a.parts + pid];
    if ((int64_t)(pid + 1) * kP <= a.count)
        sort_pass_body<kNT, Key, kOnesweep, kBits, true, kGen>(a, pid, s_keys, s_vals, s_whist, s_gbase, s_scan,
                                                          digit_info);
    else
        sort_pass_body<kNT, Key, kOnesweep, kBits, false, kGen>(a, pid, s_keys, s_vals, s_whist, s_gbase, s_scan,
                                                           digit_info);
}

// Workgroup shape of the onesweep kernels: 256 threads (4096-key partitions)
// or, for large sorts, 512 (8192-key partitions).  Every partition takes its
// id from one device-scope atomic counter, so that a partition only ever waits
// for partitions that are already running; those atomics are serialized
// (about 12 ns each measured), which bounds a pass over 20k partitions to
// ~0.23 ms.  Larger partitions halve that.  The second launch bound (waves
// per SIMD) keeps VGPRs at most 128: four 256-thread or two 512-thread
// workgroups per CU.
template <int kNT>
constexpr int kMinBlocks = 4;
// the packed-word pass over 8192-key partitions with small digits reorders
// wave by wave: few enough VGPRs for three workgroups per CU (LDS allows it)
template <int kNT, int kBits>
constexpr bool kPackedWaveLocal = kNT >= 512 && kBits <= 6;

// Onesweep passes (37 KB of LDS per 256 threads), so that partitions waiting
// in their look-back overlap with others' work.
template <typename Key, int kBits, int kNT>
__global__ __launch_bounds__(kNT, kMinBlocks<kNT>) void k_sort_pass_onesweep(PassArgs<Key> a) {
    sort_pass_kernel<kNT, Key, true, kBits>(a);
}

// Onesweep pass over packed words (value inside the key): one word per key
// in registers and in LDS, and the lean ranking (88 VGPRs: five 256-thread
// workgroups per CU against four).
template <int kBits, int kNT>
__global__ __launch_bounds__(kNT, kMinBlocks<kNT>) void k_sort_pass_packed(PassArgs<uint32_t> a) {
    constexpr int kP = kNT * kKPT;
    constexpr int kWaves = kNT / kWave;
    if (a.count_dev) a.count = (int64_t)*a.count_dev;
    __shared__ __align__(16) uint32_t s_keys[kP];
    __shared__ uint32_t s_whist[kWaves][256];
    __shared__ uint32_t s_gbase[256];
    __shared__ uint32_t s_scan[kWaves];
    __shared__ uint32_t s_pid;

    const int t = threadIdx.x;
    if ((int64_t)blockIdx.x * kP >= a.count) return;  // uniform: as in sort_pass_kernel
    if (t == 0) s_pid = atomicAdd(a.counter, 1u);
    const uint32_t hist_t = t < 256 ? hist_total(a, t) : 0u;
    for (int k = t; k < kWaves * 256; k += kNT) (&s_whist[0][0])[k] = 0;
    __syncthreads();
    const uint32_t pid = s_pid;
    if ((int64_t)pid * kP >= a.count) return;  // uniform: past the keys (device-side count)
    if ((int64_t)(pid + 1) * kP <= a.count)
        sort_pass_body<kNT, uint32_t, true, kBits, true, false, true, true, kPackedWaveLocal<kNT, kBits>>(a, pid, s_keys, nullptr, s_whist, s_gbase,
                                                                            s_scan, hist_t);
    else
        sort_pass_body<kNT, uint32_t, true, kBits, false, false, true, true, kPackedWaveLocal<kNT, kBits>>(a, pid, s_keys, nullptr, s_whist, s_gbase,
                                                                             s_scan, hist_t);
}

// The first tile pass with its keys generated from the splat records.
template <int kBits, int kNT>
__global__ __launch_bounds__(kNT, kMinBlocks<kNT>) void k_sort_pass_gen(PassArgs<uint32_t> a) {
    sort_pass_kernel<kNT, uint32_t, true, kBits, true>(a);
}

template <typename Key, int kBits>
__global__ __launch_bounds__(kNTR, 4) void k_sort_pass_rts(PassArgs<Key> a) {
    sort_pass_kernel<kNTR, Key, false, kBits>(a);
}

// kind: 0 plain onesweep, 1 packed words, 2 generated keys, 3 reduce-then-scan
template <typename Key, int kNT, int kBits>
void launch_kind(int kind, const PassArgs<Key>& a, dim3 grid, hipStream_t stream) {
    if constexpr (sizeof(Key) == 4) {
        if (kind == 1) {
            hipLaunchKernelGGL((k_sort_pass_packed<kBits, kNT>), grid, dim3(kNT), 0, stream, a);
            return;
        }
        if (kind == 2) {
            hipLaunchKernelGGL((k_sort_pass_gen<kBits, kNT>), grid, dim3(kNT), 0, stream, a);
            return;
        }
    }
    if (kind == 3)
        hipLaunchKernelGGL((k_sort_pass_rts<Key, kBits>), grid, dim3(kNTR), 0, stream, a);
    else
        hipLaunchKernelGGL((k_sort_pass_onesweep<Key, kBits, kNT>), grid, dim3(kNT), 0, stream, a);
}

template <typename Key, int kNT>
hipError_t launch_pass_nt(int kind, const PassArgs<Key>& a, int64_t parts, hipStream_t stream) {
    const dim3 grid((unsigned)parts);
    switch (a.bits) {
        case 1: launch_kind<Key, kNT, 1>(kind, a, grid, stream); break;
        case 2: launch_kind<Key, kNT, 2>(kind, a, grid, stream); break;
        case 3: launch_kind<Key, kNT, 3>(kind, a, grid, stream); break;
        case 4: launch_kind<Key, kNT, 4>(kind, a, grid, stream); break;
        case 5: launch_kind<Key, kNT, 5>(kind, a, grid, stream); break;
        case 6: launch_kind<Key, kNT, 6>(kind, a, grid, stream); break;
        case 7: launch_kind<Key, kNT, 7>(kind, a, grid, stream); break;
        case 8: launch_kind<Key, kNT, 8>(kind, a, grid, stream); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename Key>
hipError_t launch_pass(int kind, bool wide, const PassArgs<Key>& a, int64_t parts, hipStream_t stream) {
    if ((kind == 1 || kind == 2) && sizeof(Key) != 4) return hipErrorInvalidValue;
    if constexpr (sizeof(Key) == 4)  // 32-bit keys only: 64-bit ones would need 104 KB of LDS
        if (wide && kind != 3) return launch_pass_nt<Key, kSortThreadsWide>(kind, a, parts, stream);
    if (wide) return hipErrorInvalidValue;
    return launch_pass_nt<Key, kSortThreads>(kind, a, parts, stream);
}

template <typename Key>
hipError_t sort_histogram_impl(const Key* keys, int64_t count, int passes, int shift0, int end_bit, uint32_t* hist,
                               hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    const DigitPlan plan = digit_plan(passes, shift0, end_bit > 0 ? end_bit : shift0 + 8 * passes);
    hipLaunchKernelGGL(k_sort_histogram<Key>, dim3((unsigned)blocks), dim3(256), 0, stream, keys, count, plan, hist);
    return hipGetLastError();
}

template <typename Key>
hipError_t sort_passes_impl(const Key* kin, const uint32_t* vin, Key* ka, uint32_t* va, Key* kb,
                            uint32_t* vb, int64_t count, int passes, int shift0, int end_bit,
                            const SortWorkspace& ws, SortAlgo algo, hipStream_t stream, bool keep_keys,
                            const KeyGen* gen, int value_bits, hipEvent_t first_done, const uint4* gather_src,
                            uint4* gather_dst, const uint64_t* count_dev) {
    if (count <= 0 || passes <= 0) return hipSuccess;
    if (count > kSortMaxCount) return hipErrorInvalidValue;
    const bool onesweep = sort_uses_onesweep(count, algo);
    const bool wide = onesweep && sizeof(Key) == 4 && sort_uses_wide(count);
    const int64_t parts = wide ? sort_partitions_wide(count) : sort_partitions(count);
    if (passes > 8) return hipErrorInvalidValue;
    if (gen && (!onesweep || sizeof(Key) != 4 || !gen->off || !gen->rec || !gen->owner))
        return hipErrorInvalidValue;
    if ((gather_dst != nullptr) != (gather_src != nullptr) || (gather_dst && keep_keys)) return hipErrorInvalidValue;
    if (count_dev && gen) return hipErrorInvalidValue;
    const DigitPlan plan = digit_plan(passes, shift0, end_bit);
    const int pack_pass = sort_pack_pass(passes, shift0, end_bit, value_bits, keep_keys, sizeof(Key) == 8);
    const int packed_from = pack_pass < passes ? plan.shift[pack_pass] + plan.bits[pack_pass] : 0;
    for (int p = 0; p < passes; ++p) {
        PassArgs<Key> a;
        Key* kout = (p & 1) ? kb : ka;
        uint32_t* vout = (p & 1) ? vb : va;
        if (p == 0) {
            a.kin = kin;
            a.vin = vin;
        } else if (p > pack_pass) {  // packed words, written to the value buffer
            a.kin = reinterpret_cast<const Key*>((p & 1) ? va : vb);
            a.vin = nullptr;
        } else {
            a.kin = (p & 1) ? ka : kb;
            a.vin = (p & 1) ? va : vb;
        }
        a.kout = (p >= pack_pass || (p == passes - 1 && !keep_keys)) ? nullptr : kout;
        a.vout = vout;
        a.unpack_mask = p > pack_pass ? (uint32_t)((1ull << value_bits) - 1ull) : 0u;
        a.shift = p > pack_pass ? plan.shift[p] - packed_from + value_bits : plan.shift[p];
        a.vbits = (p >= pack_pass && p < passes - 1) ? (uint32_t)value_bits : 0u;
        a.pack_shift = p == pack_pass ? (uint32_t)packed_from : (uint32_t)value_bits;
        a.count = count;
        a.bits = plan.bits[p];
        a.dmask = (1u << a.bits) - 1u;
        a.hist = ws.hist + (size_t)p * 256;
        a.hist_reps = ws.hist_reps;
        a.hist_rep_stride = ws.hist_rep_stride;
        a.status = ws.status + (size_t)p * parts * 256;
        a.counter = ws.counters + p;
        a.bases = ws.bases;
        a.parts = parts;
        a.err = ws.err;
        a.gen = KeyGen{};
        a.count_dev = count_dev;
        a.gather_src = p == passes - 1 ? gather_src : nullptr;
        a.gather_dst = p == passes - 1 ? gather_dst : nullptr;
        hipError_t e;
        if (p == 0 && gen) {
            a.gen = *gen;
            if ((e = launch_pass<Key>(2, wide, a, parts, stream)) != hipSuccess) return e;
        } else if (onesweep && a.unpack_mask) {
            if ((e = launch_pass<Key>(1, wide, a, parts, stream)) != hipSuccess) return e;
        } else if (onesweep) {
            if ((e = launch_pass<Key>(0, wide, a, parts, stream)) != hipSuccess) return e;
        } else {
            hipLaunchKernelGGL(k_rts_upsweep<Key>, dim3((unsigned)parts), dim3(kNTR), 0, stream, a.kin, count,
                               a.shift, a.bits, ws.part_hist, parts, count_dev);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            e = launch_exclusive_scan(ws.part_hist, nullptr, ws.bases, 256 * parts, ws.scan_sums, ws.scan_total,
                                      stream);
            if (e != hipSuccess) return e;
            if ((e = launch_pass<Key>(3, false, a, parts, stream)) != hipSuccess) return e;
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (p == 0 && first_done && (e = hipEventRecord(first_done, stream)) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

int sort_pack_pass(int passes, int shift0, int end_bit, int value_bits, bool keep_keys, bool key64) {
    // 32-bit keys whose final keys are not kept, once the key bits left for
    // later passes and the value fit one word
    if (key64 || keep_keys || value_bits <= 0 || value_bits >= 32 || passes < 1 || passes > 8) return passes;
    const DigitPlan plan = digit_plan(passes, shift0, end_bit);
    for (int p = 0; p + 1 < passes; ++p)
        if (end_bit - (plan.shift[p] + plan.bits[p]) + value_bits <= 32) return p;
    return passes;
}

bool sort_uses_onesweep(int64_t count, SortAlgo algo) {
    return algo == SortAlgo::kOnesweep ||
           (algo == SortAlgo::kAuto && sort_partitions(count) < kSortRtsMinPartitions);
}

hipError_t launch_fill_u32(uint32_t* p, int64_t count, uint32_t value, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, stream, p, count, value);
    return hipGetLastError();
}

hipError_t launch_sort_histogram(const uint64_t* keys, int64_t count, int passes, int shift0, uint32_t* hist,
                                 hipStream_t stream, int end_bit) {
    return sort_histogram_impl<uint64_t>(keys, count, passes, shift0, end_bit, hist, stream);
}

hipError_t launch_sort_histogram(const uint32_t* keys, int64_t count, int passes, int shift0, uint32_t* hist,
                                 hipStream_t stream, int end_bit) {
    return sort_histogram_impl<uint32_t>(keys, count, passes, shift0, end_bit, hist, stream);
}

void sort_prepare_spans(const SortWorkspace& ws, int64_t count, int passes, int key_bytes, ZeroSpan spans[2]) {
    // the partitions the passes will use: 32-bit keys from 2^23 on run wide
    // (a reduce-then-scan sort uses no status words at all)
    const int64_t parts = key_bytes == 4 && sort_uses_wide(count) ? sort_partitions_wide(count) : sort_partitions(count);
    spans[0].p = ws.status;
    spans[0].n = (int64_t)passes * parts * 256;
    spans[1].p = ws.counters;
    spans[1].n = passes;
}

hipError_t launch_sort_prepare(const SortWorkspace& ws, int64_t count, int passes, bool clear_hist,
                               hipStream_t stream, int key_bytes) {
    ZeroSpan sp[2];
    sort_prepare_spans(ws, count, passes, key_bytes, sp);
    hipError_t e = launch_fill_u32(sp[0].p, sp[0].n, 0u, stream);
    if (e != hipSuccess) return e;
    e = launch_fill_u32(sp[1].p, sp[1].n, 0u, stream);
    if (e != hipSuccess) return e;
    if (clear_hist) e = launch_fill_u32(ws.hist, (int64_t)passes * 256, 0u, stream);
    return e;
}

hipError_t launch_sort_passes(const uint64_t* kin, const uint32_t* vin, uint64_t* ka, uint32_t* va,
                              uint64_t* kb, uint32_t* vb, int64_t count, int passes, int shift0,
                              const SortWorkspace& ws, SortAlgo algo, hipStream_t stream, int end_bit,
                              bool keep_keys, hipEvent_t first_done) {
    return sort_passes_impl<uint64_t>(kin, vin, ka, va, kb, vb, count, passes, shift0,
                                      end_bit > 0 ? end_bit : shift0 + 8 * passes, ws, algo, stream, keep_keys,
                                      nullptr, 0, first_done, nullptr, nullptr, nullptr);
}

hipError_t launch_sort_passes(const uint32_t* kin, const uint32_t* vin, uint32_t* ka, uint32_t* va,
                              uint32_t* kb, uint32_t* vb, int64_t count, int passes, int shift0,
                              const SortWorkspace& ws, SortAlgo algo, hipStream_t stream, int end_bit,
                              bool keep_keys, const KeyGen* gen, int value_bits, hipEvent_t first_done,
                              const uint4* gather_src, uint4* gather_dst, const uint64_t* count_dev) {
    return sort_passes_impl<uint32_t>(kin, vin, ka, va, kb, vb, count, passes, shift0,
                                      end_bit > 0 ? end_bit : shift0 + 8 * passes, ws, algo, stream, keep_keys,
                                      gen, value_bits, first_done, gather_src, gather_dst, count_dev);
}

}  // namespace cds
