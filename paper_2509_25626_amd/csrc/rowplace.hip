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
// Each placement cuts its input into chunks of 1024 consecutive intervals
// (one wave each, 16 rounds of 64), counts per chunk how many intervals cover
// each bin (difference arrays in LDS), scans those counts over the chunks of
// a bin, and then places: per round, for every bin b the lanes whose interval
// covers b are found with one ballot; their rank among those lanes is the
// mask count below them, and the bin's write pointer advances by the count.
// The lanes of one bin write consecutive words, so each ballot becomes one
// contiguous store.  Bins are held in blocks of 64, one per lane: a bin's pointer is read
// with readlane and its lane updated with a select.
//
// After each chunk every bin's write pointer must stand where the next chunk's
// part of the bin starts (or at the bin's end); anything else can only follow
// inconsistent counts and sets bit 32 of the device error word.  Slots are
// clamped to the output, so even then nothing outside it is written.
#include <algorithm>

#include "device_utils.h"
#include "internal.h"

namespace cds {
namespace {

constexpr int kRpRounds = 16;
constexpr int kRpChunk = kWave * kRpRounds;  // intervals per wave chunk
constexpr int kRpWaves = 4;                  // waves (chunks) per workgroup
constexpr int kRpThreads = kRpWaves * kWave;
constexpr uint32_t kErrRowPlace = 32u;

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

// Per-chunk coverage counts: out[c * nbins + b] = intervals of chunk c that
// cover bin b.  `diff` is this wave's nbins + 1 ints of LDS.
__device__ __forceinline__ void chunk_counts(uint32_t* diff, int nbins, uint32_t* out) {
    wave_lds_sync();
    const uint32_t l = lane_id();
    uint32_t carry = 0;
    for (int b0 = 0; b0 < nbins; b0 += kWave) {
        const int b = b0 + (int)l;
        const uint32_t d = b < nbins ? diff[b] : 0u;
        const uint32_t inc = wave_incl_sum(d) + carry;
        if (b < nbins) out[b] = inc;
        carry = (uint32_t)__builtin_amdgcn_readlane((int)inc, kWave - 1);
    }
}

// Stable placement of one round of intervals [lo, hi] (lanes with `valid`)
// over nbins bins: for every bin, the covering lanes in lane order get
// consecutive slots from the bin's write pointer (s_base, this wave's nbins
// words of LDS), which then advances past them.  emit(slot) is called by each
// covering lane with its slot.  Per block of 64 bins the pointers sit one per
// lane; a bin's pointer is read with readlane, and after the block the
// pointers advance by the round's coverage counts, which a difference array
// (s_diff, 65 words of this wave's LDS) and a wave prefix sum give.
template <typename Emit>
__device__ __forceinline__ void place_round(bool valid, uint32_t lo, uint32_t hi, int nbins, uint32_t* s_base,
                                            uint32_t* s_diff, Emit emit) {
    const uint32_t l = lane_id();
    if (!ballot(valid)) return;  // uniform
    // bin b is covered iff b - lo <= span (unsigned); an invalid lane gets an
    // interval no bin falls in (lo past every bin, span 0)
    if (!valid) {
        lo = 0xFFFF0000u;
        hi = lo;
    }
    const uint32_t span = hi - lo;
    for (int b0 = 0; b0 < nbins; b0 += kWave) {
        const uint32_t bl = (uint32_t)b0, bh = (uint32_t)b0 + kWave - 1u;
        const bool meets = valid && lo <= bh && hi >= bl;
        if (!ballot(meets)) continue;  // uniform: no lane covers this block
        const int nb = __builtin_amdgcn_readfirstlane(min(kWave, nbins - b0));
        uint32_t vb = (int)l < nb ? s_base[b0 + l] : 0u;
        s_diff[l] = 0u;
        if (l == 0) s_diff[kWave] = 0u;
        for (int j = 0; j < nb; ++j) {
            const bool cov = (uint32_t)(b0 + j) - lo <= span;
            const uint64_t m = ballot(cov);
            const uint32_t base = (uint32_t)__builtin_amdgcn_readlane((int)vb, j);
            if (cov) emit(base + count_below(m));
        }
        wave_lds_sync();
        if (meets) {
            atomicAdd(&s_diff[(lo > bl ? lo : bl) - bl], 1u);
            atomicSub(&s_diff[(hi < bh ? hi : bh) + 1u - bl], 1u);
        }
        wave_lds_sync();
        vb += wave_incl_sum(s_diff[l]);
        if ((int)l < nb) s_base[b0 + l] = vb;
        wave_lds_sync();
    }
}

struct RpArgs {
    const uint4* rec;       // [nvis] tile records in depth order
    const uint64_t* count;  // device: number of records (nvis)
    uint32_t tiles_x, tiles_y;
    uint32_t* ha;           // [chunks_a][rows]: counts, then exclusive prefix within the row
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

// A1: per chunk of 1024 records, how many cover each tile row.
__global__ __launch_bounds__(kRpThreads) void k_rp_count_rows(RpArgs a) {
    extern __shared__ uint32_t s_mem[];
    const int nbins = (int)a.tiles_y;
    const int w = threadIdx.x / kWave;
    const uint32_t l = lane_id();
    uint32_t* diff = s_mem + (size_t)w * (nbins + 1);
    const int64_t n = (int64_t)*a.count;
    const int64_t c = (int64_t)blockIdx.x * kRpWaves + w;
    const int64_t base = c * kRpChunk;
    if (base >= n) return;  // uniform per wave; no barrier below
    for (int b = (int)l; b <= nbins; b += kWave) diff[b] = 0u;
    wave_lds_sync();
#pragma unroll 4
    for (int r = 0; r < kRpRounds; ++r) {
        const int64_t i = base + r * kWave + l;
        if (i < n) {
            const RecSpan s = rec_span(a.rec[i], a.tiles_x, a.tiles_y);
            atomicAdd(&diff[s.y0], 1u);
            atomicSub(&diff[s.y1 + 1u], 1u);
        }
    }
    chunk_counts(diff, nbins, a.ha + (size_t)c * nbins);
}

// Exclusive prefix over the chunks of one bin column, in place, in
// workgroup-wide tiles of 256 chunks: col[k * stride] for k < count; the
// column total is returned to every thread.
__device__ __forceinline__ uint32_t column_excl_scan(uint32_t* col, int64_t count, int64_t stride, uint32_t base,
                                                     uint32_t* s_scan) {
    uint32_t run = base;
    for (int64_t k0 = 0; k0 < count; k0 += kRpThreads) {
        const int64_t k = k0 + threadIdx.x;
        const uint32_t v = k < count ? col[k * stride] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_sum<kRpThreads>(v, s_scan, &tot);
        if (k < count) col[k * stride] = run + ex;
        run += tot;
    }
    return run - base;
}

// A2: per row, the exclusive prefix of the chunk counts and the row total.
__global__ __launch_bounds__(kRpThreads) void k_rp_scan_rows(RpArgs a) {
    __shared__ uint32_t s_scan[kRpWaves];
    const int y = blockIdx.x;
    const int64_t n = (int64_t)*a.count;
    const int64_t chunks = (n + kRpChunk - 1) / kRpChunk;
    const uint32_t tot = column_excl_scan(a.ha + y, chunks, a.tiles_y, 0u, s_scan);
    if (threadIdx.x == 0) a.rowtot[y] = tot;
}

// A3 (one workgroup): row starts of the row lists, the B chunks of every row
// and the row of every B chunk.
constexpr int kLayoutThreads = 1024;
__global__ __launch_bounds__(kLayoutThreads) void k_rp_layout(RpArgs a) {
    __shared__ uint32_t s_scan[kLayoutThreads / kWave];
    const int rows = (int)a.tiles_y;
    constexpr int kPer = 4;  // rows per thread (rows <= 4096)
    const int y0 = threadIdx.x * kPer;
    uint32_t tot[kPer], nb[kPer], st = 0, sc = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        tot[k] = y0 + k < rows ? a.rowtot[y0 + k] : 0u;
        nb[k] = (tot[k] + kRpChunk - 1) / kRpChunk;
        st += tot[k];
        sc += nb[k];
    }
    uint32_t all_t, all_c;
    uint32_t rs = block_excl_sum<kLayoutThreads>(st, s_scan, &all_t);
    uint32_t cs = block_excl_sum<kLayoutThreads>(sc, s_scan, &all_c);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int y = y0 + k;
        if (y < rows) {
            a.rowstart[y] = rs;
            a.cstart[y] = cs;
            for (uint32_t q = 0; q < nb[k] && cs + q < a.cap_b; ++q) a.rowof[cs + q] = (uint32_t)y;
        }
        rs += tot[k];
        cs += nb[k];
    }
    if (threadIdx.x == 0) {
        a.rowstart[rows] = all_t;
        a.cstart[rows] = all_c < a.cap_b ? all_c : a.cap_b;  // more only with inconsistent counts
    }
}

// A4: each chunk of records into the row lists.  Afterwards every row's
// write pointer must stand where the next chunk's part of the row starts (or
// at the row's end); otherwise the counts were inconsistent (error bit).
__global__ __launch_bounds__(kRpThreads) void k_rp_place_rows(RpArgs a) {
    extern __shared__ uint32_t s_mem[];
    const int nbins = (int)a.tiles_y;
    const int w = threadIdx.x / kWave;
    const uint32_t l = lane_id();
    uint32_t* s_base = s_mem + (size_t)w * (nbins + kWave + 1);
    uint32_t* s_diff = s_base + nbins;
    const int64_t n = (int64_t)*a.count;
    const int64_t chunks = (n + kRpChunk - 1) / kRpChunk;
    const int64_t c = (int64_t)blockIdx.x * kRpWaves + w;
    const int64_t base = c * kRpChunk;
    if (base >= n) return;
    for (int b = (int)l; b < nbins; b += kWave) s_base[b] = a.rowstart[b] + a.ha[(size_t)c * nbins + b];
    wave_lds_sync();
    const uint32_t limit = min(a.rowstart[nbins], (uint32_t)a.sum_h);  // >= 1: launched only when sum_h > 0
    for (int r = 0; r < kRpRounds; ++r) {
        const int64_t i = base + r * kWave + l;
        const bool valid = i < n;
        RecSpan s{0u, 0u, 1u, 0u, 0u};
        if (valid) s = rec_span(a.rec[i], a.tiles_x, a.tiles_y);
        const uint2 ent = make_uint2(s.x0 | (s.x1 << 16), s.gid);
        // a slot past the row lists (inconsistent counts) is clamped to the
        // last one, so nothing outside the buffer is written; the end check
        // below reports it
        place_round(valid, s.y0, s.y1, nbins, s_base, s_diff,
                    [&](uint32_t pos) { a.rowent[min(pos, limit - 1u)] = ent; });
    }
    bool bad = false;
    for (int b = (int)l; b < nbins; b += kWave) {
        const uint32_t end = a.rowstart[b] + (c + 1 < chunks ? a.ha[(size_t)(c + 1) * nbins + b] : a.rowtot[b]);
        bad |= s_base[b] != end;
    }
    if (bad) atomicOr(a.err, kErrRowPlace);
}

// Row and entry range of B chunk cb (false past the last chunk).
__device__ __forceinline__ bool col_chunk(const RpArgs& a, int64_t cb, uint32_t& y, uint32_t& e0, uint32_t& e1) {
    if (cb >= (int64_t)a.cstart[a.tiles_y]) return false;
    y = a.rowof[cb];
    e0 = a.rowstart[y] + (uint32_t)(cb - a.cstart[y]) * (uint32_t)kRpChunk;
    e1 = min(min(e0 + (uint32_t)kRpChunk, a.rowstart[y + 1]), (uint32_t)a.sum_h);
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
#pragma unroll 4
    for (int r = 0; r < kRpRounds; ++r) {
        const uint32_t e = e0 + (uint32_t)(r * kWave) + l;
        if (e < e1) {
            // columns are below tiles_x; the clamp only keeps a corrupted
            // entry inside the array (its counts then fail the end check)
            const uint32_t xx = a.rowent[e].x;
            const uint32_t x1 = min(xx >> 16, (uint32_t)nbins - 1u);
            atomicAdd(&diff[min(xx & 0xFFFFu, x1)], 1u);
            atomicSub(&diff[x1 + 1u], 1u);
        }
    }
    chunk_counts(diff, nbins, a.hb + (size_t)cb * nbins);
}

// B2: per tile, the start slot of every chunk of its row: the tile's range
// start plus the counts of the row's earlier chunks.
__global__ __launch_bounds__(kRpThreads) void k_rp_scan_cols(RpArgs a) {
    const uint32_t y = blockIdx.x;
    const uint32_t tx = a.tiles_x;
    const uint32_t c1 = min(a.cstart[y + 1], a.cap_b), c0 = min(a.cstart[y], c1);
    // one thread per tile column, 16 chunk loads in flight
    for (uint32_t x = threadIdx.x; x < tx; x += kRpThreads) {
        uint32_t run = a.ranges[(size_t)y * tx + x].x;
        uint32_t* col = a.hb + x;
        for (uint32_t cb = c0; cb < c1; cb += 16) {
            uint32_t h[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) h[u] = cb + u < c1 ? col[(size_t)(cb + u) * tx] : 0u;
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                if (cb + u < c1) {
                    col[(size_t)(cb + u) * tx] = run;
                    run += h[u];
                }
            }
        }
    }
}

// B3: each chunk of a row list into the tile lists; the same end check.
__global__ __launch_bounds__(kRpThreads) void k_rp_place_cols(RpArgs a) {
    extern __shared__ uint32_t s_mem[];
    const int nbins = (int)a.tiles_x;
    const int w = threadIdx.x / kWave;
    const uint32_t l = lane_id();
    uint32_t* s_base = s_mem + (size_t)w * (nbins + kWave + 1);
    uint32_t* s_diff = s_base + nbins;
    const int64_t cb = (int64_t)blockIdx.x * kRpWaves + w;
    uint32_t y, e0, e1;
    if (!col_chunk(a, cb, y, e0, e1)) return;
    for (int b = (int)l; b < nbins; b += kWave) s_base[b] = a.hb[(size_t)cb * nbins + b];
    wave_lds_sync();
    const uint32_t limit = (uint32_t)a.K;
    for (int r = 0; r < kRpRounds; ++r) {
        const uint32_t e = e0 + (uint32_t)(r * kWave) + l;
        const bool valid = e < e1;
        const uint2 ent = valid ? a.rowent[e] : make_uint2(1u, 0u);
        const uint32_t x1 = min(ent.x >> 16, (uint32_t)nbins - 1u);
        place_round(valid, min(ent.x & 0xFFFFu, x1), x1, nbins, s_base, s_diff,
                    [&](uint32_t pos) { a.values[min(pos, limit - 1u)] = ent.y; });
    }
    const bool last = cb + 1 >= (int64_t)min(a.cstart[y + 1], a.cap_b);
    bool bad = false;
    for (int b = (int)l; b < nbins; b += kWave) {
        const uint32_t end = last ? a.ranges[(size_t)y * nbins + b].y : a.hb[(size_t)(cb + 1) * nbins + b];
        bad |= s_base[b] != end;
    }
    if (bad) atomicOr(a.err, kErrRowPlace);
}

}  // namespace

bool row_place_supported(int tiles_x, int tiles_y) {
    return tiles_x >= 1 && tiles_y >= 1 && tiles_x <= kRowPlaceMaxBins && tiles_y <= kRowPlaceMaxBins;
}

RowPlaceSizes row_place_sizes(int64_t n_records, uint64_t sum_h, int tiles_x, int tiles_y) {
    RowPlaceSizes s;
    s.chunks_a = (n_records + kRpChunk - 1) / kRpChunk;
    s.chunks_b_max = (int64_t)((sum_h + kRpChunk - 1) / kRpChunk) + tiles_y;
    s.ha_words = std::max<int64_t>(s.chunks_a, 1) * tiles_y;
    s.hb_words = s.chunks_b_max * tiles_x;
    s.small_words = (int64_t)tiles_y + 2 * ((int64_t)tiles_y + 1) + s.chunks_b_max;
    return s;
}

hipError_t launch_row_place(const RowPlaceArgs& p, hipStream_t stream, hipEvent_t rows_done) {
    if (!row_place_supported(p.tiles_x, p.tiles_y)) return hipErrorInvalidValue;
    if (p.n_records_max <= 0 || p.K == 0 || p.sum_h == 0) return hipSuccess;
    if (p.sum_h > (uint64_t)kSortMaxCount || p.K > (uint64_t)kSortMaxCount) return hipErrorInvalidValue;
    const RowPlaceSizes sz = row_place_sizes(p.n_records_max, p.sum_h, p.tiles_x, p.tiles_y);
    RpArgs a;
    a.rec = p.rec;
    a.count = p.count_dev;
    a.tiles_x = (uint32_t)p.tiles_x;
    a.tiles_y = (uint32_t)p.tiles_y;
    a.ha = p.ha;
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
    // count kernels: nbins + 1 words per wave; place kernels: nbins + 65
    const size_t lds_rows = sizeof(uint32_t) * kRpWaves * (size_t)(p.tiles_y + kWave + 1);
    const size_t lds_cols = sizeof(uint32_t) * kRpWaves * (size_t)(p.tiles_x + kWave + 1);
    hipLaunchKernelGGL(k_rp_count_rows, dim3(ga), dim3(kRpThreads), lds_rows, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rp_scan_rows, dim3((unsigned)p.tiles_y), dim3(kRpThreads), 0, stream, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rp_layout, dim3(1), dim3(kLayoutThreads), 0, stream, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rp_place_rows, dim3(ga), dim3(kRpThreads), lds_rows, stream, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (rows_done && (e = hipEventRecord(rows_done, stream)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rp_count_cols, dim3(gb), dim3(kRpThreads), lds_cols, stream, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (p.ranges_ready) {
        e = hipStreamWaitEvent(stream, p.ranges_ready, 0);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_rp_scan_cols, dim3((unsigned)p.tiles_y), dim3(kRpThreads), 0, stream, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rp_place_cols, dim3(gb), dim3(kRpThreads), lds_cols, stream, a);
    return hipGetLastError();
}

}  // namespace cds
