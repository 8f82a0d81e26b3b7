// Tile lists by stable interval placement, row by row: the per-tile depth
// order of paper Section II-B(1) (every visible splat replicated into each
// tile it covers, each tile's splats in depth order) built without radix
// passes over the keys.
//
// The visible splats arrive as tile records in depth order (ties by Gaussian
// index).  A splat covers a rectangle of tiles: rows y0..y1, and in each of
// those rows the columns x0..x1.  Two stable placements of intervals give
// every tile's list:
//   A. row lists: each record goes, in depth order, into the list of every
//      tile row it spans (entries (x0 | x1 << 16, Gaussian index));
//   B. tile lists: each entry of row y's list goes, in list order, to every
//      tile (x, y) with x0 <= x <= x1, at that tile's slot of the sorted
//      value list (the tile ranges are known beforehand from the rectangles).
// Each placement cuts its input into chunks of consecutive intervals (one
// wave each, rounds of 64), counts per chunk how many intervals cover each
// bin (difference arrays in LDS), scans those counts over the chunks of a
// bin, and then places: for every bin b and round, the lanes whose interval
// covers b are found with one ballot; their rank among those lanes is the
// mask count below them, and the bin's write pointer advances by the count.
// A bin's entries of the whole chunk are gathered in LDS in that order and
// go out as full-wave stores of consecutive words.
//
// After each chunk every bin's write pointer must stand where the next chunk's
// part of the bin starts (or at the bin's end); anything else can only follow
// inconsistent counts and sets bit 32 of the device error word.  Slots are
// clamped to the output, so even then nothing outside it is written.
#include <algorithm>

#include <type_traits>

#include "device_utils.h"
#include "internal.h"

namespace cds {
namespace {

// A wave places a chunk of R rounds of 64 intervals: R = 4 for the records
// (more, smaller chunks: 1.5M records give 5.7k waves), 16 for the row-list
// entries (8M at 3M Gaussians).
constexpr int kRoundsA = 4;
constexpr int kRoundsB = 16;
constexpr int kChunkA = kWave * kRoundsA;
constexpr int kChunkB = kWave * kRoundsB;
constexpr int kRpWaves = 4;                  // waves (chunks) per workgroup
constexpr int kRpThreads = kRpWaves * kWave;
constexpr uint32_t kErrRowPlace = 32u;
// Output stores go through buffer resources sized to the output: a lane
// whose slot is not to be written gets this offset added, past any size the
// resource is given (at most 2^31 bytes), and the hardware range check drops
// its store; a slot past the output is dropped the same way.
constexpr uint32_t kDropOffset = 0x80000000u;
constexpr int kCachePolicyNt = 2;  // buffer store cache policy: non-temporal
constexpr uint32_t kBufferDword3 = 0x00020000u;  // raw 32-bit buffer access (gfx9 family)
typedef int int32x2_t __attribute__((ext_vector_type(2)));

// Interval of one visible splat's record: tile rows [y0, y1], columns [x0, x1]
// (clamped to the grid, which a record of the compaction never leaves).
struct RecSpan {
    uint32_t x0, x1, y0, y1, gid;
};
__device__ __forceinline__ RecSpan rec_span(uint4 q, uint32_t tiles_x, uint32_t tiles_y) {
    RecSpan s;
    const uint32_t w = q.x & 0xFFFFu, h = q.x >> 16;
    s.y0 = q.w / tiles_x;
    s.x0 = q.w - s.y0 * tiles_x;
    s.x1 = min(s.x0 + w - 1u, tiles_x - 1u);
    s.y1 = min(s.y0 + h - 1u, tiles_y - 1u);
    s.x0 = min(s.x0, s.x1);
    s.y0 = min(s.y0, s.y1);
    s.gid = q.z;
    return s;
}

// Per-chunk coverage counts: out[b * stride] = intervals of this chunk that
// cover bin b.  `diff` is this wave's nbins + 1 ints of LDS.
__device__ __forceinline__ void chunk_counts(uint32_t* diff, int nbins, uint32_t* out, int64_t stride) {
    wave_lds_sync();
    const uint32_t l = lane_id();
    uint32_t carry = 0;
    for (int b0 = 0; b0 < nbins; b0 += kWave) {
        const int b = b0 + (int)l;
        const uint32_t d = b < nbins ? diff[b] : 0u;
        const uint32_t inc = wave_incl_sum(d) + carry;
        if (b < nbins) out[b * stride] = inc;
        carry = (uint32_t)__builtin_amdgcn_readlane((int)inc, kWave - 1);
    }
}

struct RpArgs {
    const uint4* rec;       // [nvis] tile records in depth order
    const uint64_t* count;  // device: number of records (nvis)
    uint32_t tiles_x, tiles_y;
    uint32_t* ha;           // [rows][ha_stride]: per row and chunk, counts, then exclusive prefix
    int64_t ha_stride;      // chunks of records (bound)
    uint32_t* rowtot;       // [rows]
    uint32_t* rowstart;     // [rows + 1]
    uint32_t* cstart;       // [rows + 1]: first B chunk of each row; cstart[rows] = B chunks
    uint32_t* rowof;        // [cap_b] row of each B chunk
    uint32_t cap_b;         // bound on the B chunks (sizes rowof and hb)
    uint2* rowent;          // [sum_h] row-list entries (x0 | x1 << 16, Gaussian index)
    uint64_t sum_h;
    uint32_t* hb;           // [B chunks][tiles_x]: counts, then start slots
    const uint2* ranges;    // [tiles] ranges of the sorted list
    uint32_t* values;       // [K] output: Gaussian indices in (tile, depth) order
    uint64_t K;
    uint32_t* err;
};

// A1: per chunk of kChunkA records, how many cover each tile row.
__global__ __launch_bounds__(kRpThreads) void k_rp_count_rows(RpArgs a) {
    extern __shared__ uint32_t s_mem[];
    const int nbins = (int)a.tiles_y;
    const int w = threadIdx.x / kWave;
    const uint32_t l = lane_id();
    uint32_t* diff = s_mem + (size_t)w * (nbins + 1);
    const int64_t n = (int64_t)*a.count;
    const int64_t c = (int64_t)blockIdx.x * kRpWaves + w;
    const int64_t base = c * kChunkA;
    if (base >= n) return;  // uniform per wave; no barrier below
    for (int b = (int)l; b <= nbins; b += kWave) diff[b] = 0u;
    wave_lds_sync();
    uint4 q[kRoundsA];
#pragma unroll
    for (int r = 0; r < kRoundsA; ++r) {
        const int64_t i = base + r * kWave + l;
        q[r] = i < n ? a.rec[i] : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int r = 0; r < kRoundsA; ++r) {
        if (base + r * kWave + l < n) {
            const RecSpan s = rec_span(q[r], a.tiles_x, a.tiles_y);
            atomicAdd(&diff[s.y0], 1u);
            atomicSub(&diff[s.y1 + 1u], 1u);
        }
    }
    chunk_counts(diff, nbins, a.ha + c, a.ha_stride);
}

// A2: per row, the exclusive prefix of the chunk counts (in place) and the
// row total.  A thread takes kScanPer consecutive chunks, all loaded at once
// (one memory latency per kRpThreads * kScanPer chunks instead of one per
// kRpThreads), sums them, and one workgroup scan gives its start.
constexpr int kScanPer = 32;
__global__ __launch_bounds__(kRpThreads) void k_rp_scan_rows(RpArgs a) {
    __shared__ uint32_t s_scan[kRpWaves];
    const int y = blockIdx.x;
    const int64_t n = (int64_t)*a.count;
    const int64_t chunks = (n + kChunkA - 1) / kChunkA;
    uint32_t* col = a.ha + (size_t)y * a.ha_stride;
    uint32_t run = 0;
    for (int64_t k0 = 0; k0 < chunks; k0 += (int64_t)kRpThreads * kScanPer) {  // uniform
        const int64_t kb = k0 + (int64_t)threadIdx.x * kScanPer;
        uint32_t v[kScanPer], sum = 0;
#pragma unroll
        for (int u = 0; u < kScanPer; ++u) {
            v[u] = kb + u < chunks ? col[kb + u] : 0u;
            sum += v[u];
        }
        uint32_t tot;
        uint32_t ex = run + block_excl_sum<kRpThreads>(sum, s_scan, &tot);
#pragma unroll
        for (int u = 0; u < kScanPer; ++u) {
            if (kb + u < chunks) col[kb + u] = ex;
            ex += v[u];
        }
        run += tot;
    }
    if (threadIdx.x == 0) a.rowtot[y] = run;
}

// A3 (one workgroup): row starts of the row lists, the B chunks of every row
// and the row of every B chunk.
constexpr int kLayoutThreads = 1024;
__global__ __launch_bounds__(kLayoutThreads) void k_rp_layout(RpArgs a) {
    __shared__ uint32_t s_scan[kLayoutThreads / kWave];
    __shared__ uint32_t s_cs[kRowPlaceMaxBins + 1];
    const int rows = (int)a.tiles_y;
    constexpr int kPer = kRowPlaceMaxBins / kLayoutThreads;  // rows per thread
    const int y0 = threadIdx.x * kPer;
    uint32_t tot[kPer], nb[kPer], st = 0, sc = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        tot[k] = y0 + k < rows ? a.rowtot[y0 + k] : 0u;
        nb[k] = (tot[k] + kChunkB - 1) / kChunkB;
        st += tot[k];
        sc += nb[k];
    }
    uint32_t all_t, all_c;
    uint32_t rs = block_excl_sum<kLayoutThreads>(st, s_scan, &all_t);
    uint32_t cs = block_excl_sum<kLayoutThreads>(sc, s_scan, &all_c);
    all_c = all_c < a.cap_b ? all_c : a.cap_b;  // more only with inconsistent counts
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int y = y0 + k;
        if (y < rows) {
            a.rowstart[y] = rs;
            a.cstart[y] = cs;
            s_cs[y] = cs;
        }
        rs += tot[k];
        cs += nb[k];
    }
    if (threadIdx.x == 0) {
        a.rowstart[rows] = all_t;
        a.cstart[rows] = all_c;
        s_cs[rows] = all_c;
    }
    __syncthreads();
    // the row of every B chunk: the last row starting at or before it
    for (uint32_t cb = threadIdx.x; cb < all_c; cb += kLayoutThreads) {
        int lo = 0, hi = rows - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_cs[mid] <= cb) lo = mid; else hi = mid - 1;
        }
        a.rowof[cb] = (uint32_t)lo;
    }
}


// Row and entry range of B chunk cb (false past the last chunk).
__device__ __forceinline__ bool col_chunk(const RpArgs& a, int64_t cb, uint32_t& y, uint32_t& e0, uint32_t& e1) {
    if (cb >= (int64_t)a.cstart[a.tiles_y]) return false;
    y = a.rowof[cb];
    e0 = a.rowstart[y] + (uint32_t)(cb - a.cstart[y]) * (uint32_t)kChunkB;
    e1 = min(min(e0 + (uint32_t)kChunkB, a.rowstart[y + 1]), (uint32_t)a.sum_h);
    return true;
}

// B1: per chunk of a row list, how many entries cover each tile column.
__global__ __launch_bounds__(kRpThreads) void k_rp_count_cols(RpArgs a) {
    extern __shared__ uint32_t s_mem[];
    const int nbins = (int)a.tiles_x;
    const int w = threadIdx.x / kWave;
    const uint32_t l = lane_id();
    uint32_t* diff = s_mem + (size_t)w * (nbins + 1);
    const int64_t cb = (int64_t)blockIdx.x * kRpWaves + w;
    uint32_t y, e0, e1;
    if (!col_chunk(a, cb, y, e0, e1)) return;
    for (int b = (int)l; b <= nbins; b += kWave) diff[b] = 0u;
    wave_lds_sync();
    uint32_t xx[kRoundsB];
#pragma unroll
    for (int r = 0; r < kRoundsB; ++r) {
        const uint32_t e = e0 + (uint32_t)(r * kWave) + l;
        xx[r] = e < e1 ? a.rowent[e].x : 0xFFFFFFFFu;
    }
#pragma unroll
    for (int r = 0; r < kRoundsB; ++r) {
        if (xx[r] != 0xFFFFFFFFu) {
            // columns are below tiles_x; the clamp only keeps a corrupted
            // entry inside the array (its counts then fail the end check)
            const uint32_t x1 = min(xx[r] >> 16, (uint32_t)nbins - 1u);
            atomicAdd(&diff[min(xx[r] & 0xFFFFu, x1)], 1u);
            atomicSub(&diff[x1 + 1u], 1u);
        }
    }
    chunk_counts(diff, nbins, a.hb + (size_t)cb * nbins, 1);
}

// B2: per tile, the start slot of every chunk of its row: the tile's range
// start plus the counts of the row's earlier chunks.  Workgroup (row y,
// group of kScanCols columns): each column's chunks are cut into
// kRpThreads / kScanCols segments, one thread each; a thread sums its
// segment (kScanBatch loads in flight), the segment sums are scanned in LDS,
// and the thread writes its segment's starts (from registers when the
// segment fits one batch, else re-read).
constexpr int kScanCols = 16;
constexpr int kScanSegs = kRpThreads / kScanCols;
constexpr int kScanBatch = 16;
__global__ __launch_bounds__(kRpThreads) void k_rp_scan_cols(RpArgs a) {
    __shared__ uint32_t s_seg[kScanSegs][kScanCols];
    const uint32_t y = blockIdx.x;
    const uint32_t tx = a.tiles_x;
    const uint32_t xi = threadIdx.x % kScanCols, sg = threadIdx.x / kScanCols;
    const uint32_t x = blockIdx.y * kScanCols + xi;
    const uint32_t c1 = min(a.cstart[y + 1], a.cap_b), c0 = min(a.cstart[y], c1);
    const uint32_t len = (c1 - c0 + kScanSegs - 1) / kScanSegs;  // chunks per segment
    const uint32_t s0 = c0 + min(sg * len, c1 - c0), s1 = min(s0 + len, c1);
    const bool on = x < tx;
    uint32_t* col = a.hb + (on ? x : 0u);
    uint32_t h[kScanBatch], sum = 0;
    for (uint32_t cb = s0; cb < s1; cb += kScanBatch) {
#pragma unroll
        for (int u = 0; u < kScanBatch; ++u) {
            h[u] = on && cb + u < s1 ? col[(size_t)(cb + u) * tx] : 0u;
            sum += h[u];
        }
    }
    s_seg[sg][xi] = sum;
    __syncthreads();
    if (!on) return;
    uint32_t run = a.ranges[(size_t)y * tx + x].x;
    for (uint32_t q = 0; q < sg; ++q) run += s_seg[q][xi];
    if (s1 - s0 <= (uint32_t)kScanBatch) {  // the segment's counts are still in h
#pragma unroll
        for (int u = 0; u < kScanBatch; ++u) {
            if (s0 + u < s1) {
                col[(size_t)(s0 + u) * tx] = run;
                run += h[u];
            }
        }
    } else {
        for (uint32_t cb = s0; cb < s1; cb += kScanBatch) {
#pragma unroll
            for (int u = 0; u < kScanBatch; ++u) h[u] = cb + u < s1 ? col[(size_t)(cb + u) * tx] : 0u;
#pragma unroll
            for (int u = 0; u < kScanBatch; ++u) {
                if (cb + u < s1) {
                    col[(size_t)(cb + u) * tx] = run;
                    run += h[u];
                }
            }
        }
    }
}

// B3: each chunk of a row list into the tile lists.  One workgroup per
// chunk; its waves split the row's tile columns into blocks of kColBlock.  A
// wave loads the whole chunk, compacts in chunk order into LDS the entries
// that reach its block (their columns clipped to the block, as two 4-bit
// offsets), reads them back as a 16-bit column mask per entry, and places
// them bin by bin: per round one ballot, the run gathered in LDS, full-wave
// stores.  At 3M Gaussians a row entry covers about 10 of 78 columns, so a
// bin iterates over about a third of the chunk, and the five waves of a
// chunk run side by side.  Every bin ends where the next chunk's base (or
// the tile's range end) says, else error bit 32.
constexpr int kColBlock = 16;
constexpr int kColMaxWaves = 8;  // waves per workgroup (42 KB of LDS); more blocks are taken in turn
constexpr int kColBatch = kRoundsB / 2;  // rounds of compacted entries held in registers at once
static_assert(kColBatch == 8, "place_bins is instantiated for 1 to 8 rounds");
// per wave: compacted Gaussian indices (words), compacted offsets (bytes), a dump slot per lane
constexpr int kColWaveWords = kChunkB + kChunkB / 4 + kWave;
static_assert(kColBlock == 16, "compacted offsets are packed as 4-bit fields");

__host__ __device__ inline int col_blocks(int nbins) { return (nbins + kColBlock - 1) / kColBlock; }

// The bins of one block over R rounds of compacted entries (R known at
// compile time: no per-round checks).  Per bin and round one ballot; the
// covering lanes write their Gaussian index to the run in LDS, the others to
// a dump slot of their own (a select of the address, not a branch); then the run goes out in
// full-wave stores, lanes past its end given an offset the buffer drops.
template <int R, int W>
__device__ __forceinline__ void place_bins(const uint32_t (&cm)[kColBatch], const uint32_t (&cg)[kColBatch][W], int nb,
                                           uint32_t* stage, uint32_t* dump, uint32_t& vb,
                                           __amdgpu_buffer_rsrc_t out) {
    static_assert(W == 1 || W == 2, "payloads of one or two words");
    using u32x2 = uint32_t __attribute__((ext_vector_type(2)));
    using lds_w = __attribute__((address_space(3))) typename std::conditional<W == 1, uint32_t, u32x2>::type;
    const uint32_t l = lane_id();
    lds_w* const st = (lds_w*)stage;
    lds_w* const du = (lds_w*)dump;
    for (int j = 0; j < nb; ++j) {
        lds_w* wr = st;  // the run's end (one pointer add per round)
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const bool cov = (cm[q] >> j) & 1u;
            const uint64_t m = ballot(cov);
            // rank among the covering lanes below, computed in every lane (the
            // empty asm keeps the compiler from moving it under a branch)
            uint32_t rank = count_below(m);
            asm volatile("" : "+v"(rank));
            lds_w* dst = cov ? wr + rank : du + l;
            if constexpr (W == 1)
                *dst = cg[q][0];
            else
                *dst = u32x2{cg[q][0], cg[q][1]};
            wr += __popcll(m);
        }
        const uint32_t run = (uint32_t)(wr - st);
        wave_lds_sync();
        const uint32_t base = (uint32_t)__builtin_amdgcn_readlane((int)vb, j);
        // slots are below 2^29 (one word) or 2^28 (two), so a kept offset is
        // below 2^31 and the dropped lanes' 2^31 is past the buffer
        const uint32_t voff = (base + l) * (uint32_t)(4 * W);
        // one-word runs: every round's slots are read before the first store,
        // so the stores wait for LDS once per bin instead of once per round
        // (slots past the run hold stale words, whose offsets are dropped)
        uint32_t early[W == 1 ? R : 1];
        if constexpr (W == 1) {
#pragma unroll
            for (int t = 0; t < R; ++t) early[t] = st[t * kWave + l];
        }
#pragma unroll
        for (int t = 0; t < R; ++t) {
            if ((uint32_t)(t * kWave) < run) {  // uniform
                const uint32_t off =
                    l < run - (uint32_t)(t * kWave) ? voff + (uint32_t)(t * kWave * 4 * W) : kDropOffset;
                if constexpr (W == 1) {
                    // the tile lists: written once and, past each list's first
                    // few hundred entries, not read again this frame, so they
                    // go out non-temporal (cache policy bit 1: nt) rather than
                    // fill the last-level cache with dirty lines that the next
                    // frame's preprocessing would have to write back
                    __builtin_amdgcn_raw_buffer_store_b32((int)early[t], out, (int)off, 0, kCachePolicyNt);
                } else {
                    const u32x2 v = st[t * kWave + l];
                    __builtin_amdgcn_raw_buffer_store_b64(int32x2_t{(int)v.x, (int)v.y}, out, (int)off, 0, 0);
                }
            }
        }
        wave_lds_sync();  // the run is read before the next bin's gathers
        vb = l == (uint32_t)j ? base + run : vb;
    }
}

// six waves per SIMD: the register budget the early reads need (the
// kernel's LDS allows about that many anyway)
__global__ __launch_bounds__(kColMaxWaves * kWave) __attribute__((amdgpu_waves_per_eu(6)))
void k_rp_place_cols(RpArgs a) {
    extern __shared__ uint32_t s_mem[];
    const int nbins = (int)a.tiles_x;
    const int nblk = col_blocks(nbins);
    const int nw = (int)(blockDim.x / kWave);
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));  // uniform: LDS bases in SGPRs
    const uint32_t l = lane_id();
    uint32_t* s_cg = s_mem + (size_t)w * kColWaveWords;           // compacted Gaussian index; then the run stage
    uint8_t* s_cx = reinterpret_cast<uint8_t*>(s_cg + kChunkB);   // compacted offset | (last - offset) << 4
    uint32_t* s_dump = s_cg + kChunkB + kChunkB / 4;              // one slot per lane for uncovered writes
    const int64_t cb = blockIdx.x;
    uint32_t y, e0, e1;
    if (!col_chunk(a, cb, y, e0, e1)) return;
    uint32_t ex[kRoundsB], eg[kRoundsB];  // x0 | x1 << 16 (unused slot: x0 past every bin), Gaussian index
#pragma unroll
    for (int r = 0; r < kRoundsB; ++r) {
        const uint32_t e = e0 + (uint32_t)(r * kWave) + l;
        ex[r] = 0x0000FFFFu;
        eg[r] = 0u;
        if (e < e1) {
            const uint2 ent = a.rowent[e];
            // columns are below tiles_x; the clamp only keeps a corrupted
            // entry inside the row (its counts then fail the end check)
            const uint32_t x1 = min(ent.x >> 16, (uint32_t)nbins - 1u);
            ex[r] = min(ent.x & 0xFFFFu, x1) | (x1 << 16);
            eg[r] = ent.y;
        }
    }
    const bool last = cb + 1 >= (int64_t)min(a.cstart[y + 1], a.cap_b);
    const __amdgpu_buffer_rsrc_t out =
        __builtin_amdgcn_make_buffer_rsrc(a.values, 0, (int)(a.K * sizeof(uint32_t)), (int)kBufferDword3);
    bool bad = false;
    for (int blk = w; blk < nblk; blk += nw) {
        const int b0 = blk * kColBlock;
        const int nb = min(kColBlock, nbins - b0);
        const uint32_t bl = (uint32_t)b0, bh = (uint32_t)(b0 + nb - 1);
        // compaction: the entries reaching the block, in chunk order
        uint32_t cnt = 0;
#pragma unroll
        for (int r = 0; r < kRoundsB; ++r) {
            const uint32_t x0 = ex[r] & 0xFFFFu, x1 = ex[r] >> 16;
            // two ballots of plain compares: the mask comes straight from
            // them, where a ballot of the combined bool is rebuilt by two
            // more vector instructions
            const uint64_t m = ballot(x0 <= bh) & ballot(x1 >= bl);
            if (x0 <= bh && x1 >= bl) {
                const uint32_t k = cnt + count_below(m);
                const uint32_t o0 = (x0 > bl ? x0 : bl) - bl, o1 = (x1 < bh ? x1 : bh) - bl;
                s_cx[k] = (uint8_t)(o0 | ((o1 - o0) << 4));
                s_cg[k] = eg[r];
            }
            cnt += (uint32_t)__popcll(m);
        }
        // this block's bins start at the chunk's bases
        uint32_t vb = (int)l < nb ? a.hb[(size_t)cb * nbins + b0 + l] : 0u;
        // the compacted entries in batches of kColBatch rounds (one batch in
        // the common case); a batch's slots serve as its run stage once it
        // is in registers, and batch by batch keeps every bin in chunk order
        for (uint32_t h = 0; h < cnt; h += kColBatch * kWave) {  // uniform
            wave_lds_sync();
            const uint32_t hn = min(cnt - h, (uint32_t)(kColBatch * kWave));
            const uint32_t rounds = (hn + kWave - 1) / kWave;
            uint32_t* stage = s_cg + h;
            uint32_t cm[kColBatch], cg[kColBatch][1];  // columns of the block an entry covers (bit mask), Gaussian index
#pragma unroll
            for (int q = 0; q < kColBatch; ++q) {
                const uint32_t k = (uint32_t)(q * kWave) + l;
                cm[q] = 0u;
                cg[q][0] = 0u;
                if ((uint32_t)q < rounds && k < hn) {
                    const uint32_t c = s_cx[h + k];
                    cm[q] = ((2u << (c >> 4)) - 1u) << (c & 15u);
                    cg[q][0] = stage[k];
                }
            }
            wave_lds_sync();
            switch (rounds) {
                case 1: place_bins<1, 1>(cm, cg, nb, stage, s_dump, vb, out); break;
                case 2: place_bins<2, 1>(cm, cg, nb, stage, s_dump, vb, out); break;
                case 3: place_bins<3, 1>(cm, cg, nb, stage, s_dump, vb, out); break;
                case 4: place_bins<4, 1>(cm, cg, nb, stage, s_dump, vb, out); break;
                case 5: place_bins<5, 1>(cm, cg, nb, stage, s_dump, vb, out); break;
                case 6: place_bins<6, 1>(cm, cg, nb, stage, s_dump, vb, out); break;
                case 7: place_bins<7, 1>(cm, cg, nb, stage, s_dump, vb, out); break;
                default: place_bins<8, 1>(cm, cg, nb, stage, s_dump, vb, out); break;
            }
        }
        if ((int)l < nb) {
            const uint32_t b = (uint32_t)b0 + l;
            const uint32_t end = last ? a.ranges[(size_t)y * nbins + b].y : a.hb[(size_t)(cb + 1) * nbins + b];
            bad |= vb != end;
        }
    }
    if (bad) atomicOr(a.err, kErrRowPlace);
}


// A4: each chunk of kChunkA records into the row lists, the way B3 places
// row entries into tiles: one workgroup per chunk, one wave per block of
// kColBlock tile rows, the records reaching the block compacted in chunk
// order (rows clipped to the block as two 4-bit offsets), then placed row by
// row with their 8-byte entries (x0 | x1 << 16, Gaussian index) gathered in
// LDS and written as full-wave stores.  Afterwards every row's write pointer
// must stand where the next chunk's part of the row starts (or at the row's
// end), else error bit 32.
constexpr int kRowWaveWords = 2 * kChunkA + kChunkA / 4 + 2 * kWave;  // entries (2 words), offsets (bytes), dump
static_assert(kRoundsA <= kColBatch, "a chunk of records is one batch");

__global__ __launch_bounds__(kColMaxWaves * kWave) __attribute__((amdgpu_waves_per_eu(8)))
void k_rp_place_rows(RpArgs a) {
    extern __shared__ uint32_t s_mem[];
    const int nbins = (int)a.tiles_y;
    const int nblk = col_blocks(nbins);
    const int nw = (int)(blockDim.x / kWave);
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));  // uniform: LDS bases in SGPRs
    const uint32_t l = lane_id();
    uint32_t* s_cg = s_mem + (size_t)w * kRowWaveWords;              // compacted entries; then the run stage
    uint8_t* s_cx = reinterpret_cast<uint8_t*>(s_cg + 2 * kChunkA);  // compacted offset | (last - offset) << 4
    uint32_t* s_dump = s_cg + 2 * kChunkA + kChunkA / 4;            // two words per lane for uncovered writes
    const int64_t n = (int64_t)*a.count;
    const int64_t chunks = (n + kChunkA - 1) / kChunkA;
    const int64_t c = blockIdx.x;
    const int64_t base = c * kChunkA;
    if (base >= n) return;  // uniform over the workgroup
    uint32_t ey[kRoundsA], e0[kRoundsA], e1[kRoundsA];  // y0 | y1 << 16 (unused: y0 past every bin); the entry
#pragma unroll
    for (int r = 0; r < kRoundsA; ++r) {
        const int64_t i = base + r * kWave + l;
        ey[r] = 0x0000FFFFu;
        e0[r] = e1[r] = 0u;
        if (i < n) {
            const RecSpan sp = rec_span(a.rec[i], a.tiles_x, a.tiles_y);
            ey[r] = sp.y0 | (sp.y1 << 16);
            e0[r] = sp.x0 | (sp.x1 << 16);
            e1[r] = sp.gid;
        }
    }
    const uint32_t limit = min(a.rowstart[nbins], (uint32_t)a.sum_h);
    const __amdgpu_buffer_rsrc_t out =
        __builtin_amdgcn_make_buffer_rsrc(a.rowent, 0, (int)(limit * sizeof(uint2)), (int)kBufferDword3);
    bool bad = false;
    for (int blk = w; blk < nblk; blk += nw) {
        const int b0 = blk * kColBlock;
        const int nb = min(kColBlock, nbins - b0);
        const uint32_t bl = (uint32_t)b0, bh = (uint32_t)(b0 + nb - 1);
        uint32_t cnt = 0;
#pragma unroll
        for (int r = 0; r < kRoundsA; ++r) {
            const uint32_t y0 = ey[r] & 0xFFFFu, y1 = ey[r] >> 16;
            const uint64_t m = ballot(y0 <= bh) & ballot(y1 >= bl);
            if (y0 <= bh && y1 >= bl) {
                const uint32_t k = cnt + count_below(m);
                const uint32_t o0 = (y0 > bl ? y0 : bl) - bl, o1 = (y1 < bh ? y1 : bh) - bl;
                s_cx[k] = (uint8_t)(o0 | ((o1 - o0) << 4));
                s_cg[2 * k] = e0[r];
                s_cg[2 * k + 1] = e1[r];
            }
            cnt += (uint32_t)__popcll(m);
        }
        // this block's rows start at the chunk's part of each row list
        const uint32_t b = (uint32_t)b0 + l;
        uint32_t vb = (int)l < nb ? a.rowstart[b] + a.ha[(size_t)b * a.ha_stride + c] : 0u;
        if (cnt > 0) {  // uniform
            wave_lds_sync();
            const uint32_t rounds = (cnt + kWave - 1) / kWave;
            uint32_t cm[kColBatch], cg[kColBatch][2];  // rows of the block an entry covers (bit mask), the entry
#pragma unroll
            for (int q = 0; q < kColBatch; ++q) {
                const uint32_t k = (uint32_t)(q * kWave) + l;
                cm[q] = 0u;
                cg[q][0] = cg[q][1] = 0u;
                if (q < kRoundsA && (uint32_t)q < rounds && k < cnt) {
                    const uint32_t cx = s_cx[k];
                    cm[q] = ((2u << (cx >> 4)) - 1u) << (cx & 15u);
                    cg[q][0] = s_cg[2 * k];
                    cg[q][1] = s_cg[2 * k + 1];
                }
            }
            wave_lds_sync();  // the staged entries are the run stage from here
            switch (rounds) {
                case 1: place_bins<1, 2>(cm, cg, nb, s_cg, s_dump, vb, out); break;
                case 2: place_bins<2, 2>(cm, cg, nb, s_cg, s_dump, vb, out); break;
                case 3: place_bins<3, 2>(cm, cg, nb, s_cg, s_dump, vb, out); break;
                case 4: place_bins<4, 2>(cm, cg, nb, s_cg, s_dump, vb, out); break;
                case 5: place_bins<5, 2>(cm, cg, nb, s_cg, s_dump, vb, out); break;
                case 6: place_bins<6, 2>(cm, cg, nb, s_cg, s_dump, vb, out); break;
                case 7: place_bins<7, 2>(cm, cg, nb, s_cg, s_dump, vb, out); break;
                default: place_bins<8, 2>(cm, cg, nb, s_cg, s_dump, vb, out); break;
            }
        }
        if ((int)l < nb) {
            const uint32_t end = a.rowstart[b] + (c + 1 < chunks ? a.ha[(size_t)b * a.ha_stride + c + 1] : a.rowtot[b]);
            bad |= vb != end;
        }
    }
    if (bad) atomicOr(a.err, kErrRowPlace);
}

}  // namespace

bool row_place_supported(int tiles_x, int tiles_y) {
    return tiles_x >= 1 && tiles_y >= 1 && tiles_x <= kRowPlaceMaxBins && tiles_y <= kRowPlaceMaxBins;
}

RowPlaceSizes row_place_sizes(int64_t n_records, uint64_t sum_h, int tiles_x, int tiles_y) {
    RowPlaceSizes s;
    s.chunks_a = (n_records + kChunkA - 1) / kChunkA;
    s.chunks_b_max = (int64_t)((sum_h + kChunkB - 1) / kChunkB) + tiles_y;
    s.ha_words = std::max<int64_t>(s.chunks_a, 1) * tiles_y;
    s.hb_words = s.chunks_b_max * tiles_x;
    s.small_words = (int64_t)tiles_y + 2 * ((int64_t)tiles_y + 1) + s.chunks_b_max;
    return s;
}

hipError_t launch_row_place(const RowPlaceArgs& p, hipStream_t stream, hipEvent_t rows_done,
                            hipEvent_t cols_counted) {
    if (!row_place_supported(p.tiles_x, p.tiles_y)) return hipErrorInvalidValue;
    if (p.n_records_max <= 0 || p.K == 0 || p.sum_h == 0) return hipSuccess;
    // the output buffer resources hold at most 2^31 bytes
    if (p.sum_h > (uint64_t(1) << 28) || p.K > (uint64_t(1) << 29)) return hipErrorInvalidValue;
    const RowPlaceSizes sz = row_place_sizes(p.n_records_max, p.sum_h, p.tiles_x, p.tiles_y);
    RpArgs a;
    a.rec = p.rec;
    a.count = p.count_dev;
    a.tiles_x = (uint32_t)p.tiles_x;
    a.tiles_y = (uint32_t)p.tiles_y;
    a.ha = p.ha;
    a.ha_stride = std::max<int64_t>(sz.chunks_a, 1);
    a.rowtot = p.small;
    a.rowstart = p.small + p.tiles_y;
    a.cstart = a.rowstart + p.tiles_y + 1;
    a.rowof = a.cstart + p.tiles_y + 1;
    a.cap_b = (uint32_t)sz.chunks_b_max;
    a.rowent = p.rowent;
    a.sum_h = p.sum_h;
    a.hb = p.hb;
    a.ranges = p.ranges;
    a.values = p.values;
    a.K = p.K;
    a.err = p.err;
    const unsigned ga = (unsigned)((sz.chunks_a + kRpWaves - 1) / kRpWaves);
    const unsigned gb = (unsigned)((sz.chunks_b_max + kRpWaves - 1) / kRpWaves);
    // per wave: count kernels nbins + 1 words; place kernels nbins words of
    // pointers and a staging area
    const size_t lds_rows = sizeof(uint32_t) * kRpWaves * (size_t)(p.tiles_y + 1);
    const size_t lds_cols = sizeof(uint32_t) * kRpWaves * (size_t)(p.tiles_x + 1);
    const int row_waves = std::min(col_blocks((int)p.tiles_y), kColMaxWaves);
    const size_t lds_place_rows = sizeof(uint32_t) * row_waves * (size_t)kRowWaveWords;
    const int col_waves = std::min(col_blocks((int)p.tiles_x), kColMaxWaves);
    const size_t lds_place_cols = sizeof(uint32_t) * col_waves * (size_t)kColWaveWords;
    hipLaunchKernelGGL(k_rp_count_rows, dim3(ga), dim3(kRpThreads), lds_rows, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rp_scan_rows, dim3((unsigned)p.tiles_y), dim3(kRpThreads), 0, stream, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rp_layout, dim3(1), dim3(kLayoutThreads), 0, stream, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rp_place_rows, dim3((unsigned)sz.chunks_a), dim3(row_waves * kWave), lds_place_rows,
                       stream, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (rows_done && (e = hipEventRecord(rows_done, stream)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rp_count_cols, dim3(gb), dim3(kRpThreads), lds_cols, stream, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (p.ranges_ready) {
        e = hipStreamWaitEvent(stream, p.ranges_ready, 0);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_rp_scan_cols, dim3((unsigned)p.tiles_y, (unsigned)((p.tiles_x + kScanCols - 1) / kScanCols)),
                       dim3(kRpThreads), 0, stream, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (cols_counted && (e = hipEventRecord(cols_counted, stream)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rp_place_cols, dim3((unsigned)sz.chunks_b_max), dim3(col_waves * kWave), lds_place_cols,
                       stream, a);
    return hipGetLastError();
}

}  // namespace cds
