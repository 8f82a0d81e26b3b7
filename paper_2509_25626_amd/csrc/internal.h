// Internal interface between the host runtime and the kernel translation
// units.  Each launcher enqueues its kernels on `stream` and returns the HIP
// status of the launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cds {

// Camera and per-frame constants of the projection (double precision: the
// projection decides tile coverage and depth keys in float64).
struct ProjParams {
    int64_t n;
    int32_t sh_degree;
    int32_t width, height, tiles_x, tiles_y;
    int32_t pad;
    double R[9];        // world -> camera rotation, row-major
    double t[3];        // world -> camera translation
    double campos[3];   // camera centre in world space, -R^T t
    double fx, fy, cx, cy;
    double near_plane;
    double limx, limy;  // 1.3 x half field of view tangents (Jacobian guard band)
};

struct SceneParams {
    const float* means;
    const float* log_scales;
    const float* quats;
    const float* opacity_logits;
    const float* sh;
};

// Per-Gaussian projected state (the paper's points_xy_image, conic_opacity,
// features and depths, plus tile bookkeeping).
struct SplatBuffers {
    float2* mean2d;
    float4* conic_opacity;
    float4* rgb;
    uint32_t* depth_bits;
    int32_t* radius;
    uint2* rect;
    uint32_t* touched;
    uint8_t* clamp_flags;
    // [9][n] or null: d rgb_ch / d dir_c at 3 ch + c (dir = unit view
    // direction), written for renders kept for the backward pass (SH degree > 0)
    float* jac = nullptr;
};

struct GradBuffers2D {  // [9][n]: mean x, mean y, conic A, B, C, opacity, r, g, b
    float* g;
};

hipError_t launch_preprocess(const ProjParams& p, const SceneParams& s, const SplatBuffers& out,
                             hipStream_t stream);

// One request of a batched render: a scene, its camera, and where its
// Gaussians and tiles sit in the batch's concatenated index spaces.
struct BatchItem {
    ProjParams P;
    SceneParams S;
    int64_t gauss_base;  // first global Gaussian index of this item
    int64_t tile_base;   // first global tile id of this item
    float bg[3];
    float* out_rgb;
    float* out_T;            // may be null
    uint32_t* out_ncontrib;  // may be null
    // With rec_stride > 0 the batch's tiles also live on a stacked grid for
    // the row-wise placement: the requests' tile rows one below the other,
    // every row rec_stride tiles wide; tile (x, y) of this item is stacked
    // tile rec_base + y * rec_stride + x (its tile records and ranges use it).
    int64_t rec_base;
    int32_t rec_stride;
};

// Item owning global Gaussian g / global tile t (items sorted by base).
__device__ __forceinline__ int find_item_by_gaussian(const BatchItem* items, int nitems, int64_t g) {
    int lo = 0, hi = nitems - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].gauss_base <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}
__device__ __forceinline__ int find_item_by_tile(const BatchItem* items, int nitems, int64_t t) {
    int lo = 0, hi = nitems - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].tile_base <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

hipError_t launch_preprocess_batch(const BatchItem* items, int nitems, int64_t total, const SplatBuffers& out,
                                   hipStream_t stream);

// Two (or, with c, three) exclusive in-place scans of `count` uint64 values
// each (one workgroup per array, one launch); the totals go to *total_a,
// *total_b (and *total_c).  With `groups` (group <= 16), value i of a (b, c)
// is instead the sum of src_a (src_b, src_c) items i * group + j below
// src_count, item i * group + j stored at index j * count + i, and the scans
// are written to a (b, c).
struct ScanGroups {
    const uint64_t* src_a = nullptr;
    const uint64_t* src_b = nullptr;
    const uint64_t* src_c = nullptr;
    int64_t src_count = 0;
    int group = 1;
};
hipError_t launch_scan_u64_pair(uint64_t* a, uint64_t* b, int64_t count, uint64_t* total_a, uint64_t* total_b,
                                hipStream_t stream, uint64_t* c = nullptr, uint64_t* total_c = nullptr,
                                uint64_t* host_a = nullptr, uint64_t* host_b = nullptr, uint64_t* host_c = nullptr,
                                const ScanGroups* groups = nullptr);

// Tile record of a visible splat (16 B): its rectangle of tiles as runs of
// tile ids, (width | height << 16, row stride, Gaussian index, id of the first
// tile).  Key c of the splat, in row-major order over the rectangle, is tile
// first + (c / width) * stride + c % width.  Batched renders store global
// tile ids (the request's tile base added), single renders their own.
__host__ __device__ inline uint4 make_tile_rec(uint2 rect, uint32_t tiles_x, uint32_t tile_base, uint32_t gid) {
    const uint32_t x0 = rect.x & 0xFFFFu, y0 = rect.x >> 16, x1 = rect.y & 0xFFFFu, y1 = rect.y >> 16;
    return make_uint4((x1 - x0 + 1u) | ((y1 - y0 + 1u) << 16), tiles_x, gid, tile_base + y0 * tiles_x + x0);
}
__host__ __device__ inline uint32_t tile_rec_area(uint4 q) { return (q.x & 0xFFFFu) * (q.x >> 16); }

struct BatchItem;

// Compaction of the visible splats (tiles touched > 0) in index order:
// dkey[n_vis] depth bits, rec[n_vis] tile records (make_tile_rec; `items`
// give the per-request grids of a batched render, else tiles_x and tile base
// 0), depth_hist [4][256] digit histograms of dkey, totals[0] = n_vis,
// totals[1] = K.  vis_sums, key_sums: compact_sums_size(n) uint64 each.
// With sum_h (and h_sums, compact_sums_size(n) more uint64 of workspace),
// *sum_h = the sum of the visible splats' rectangle heights.
// zero_spans: up to kZeroSpans more word ranges cleared by the counting
// kernel (so the caller needs no fill launches of its own before the sort).
// host_totals (4 words of fine-grained pinned host memory, device address):
// totals[0], totals[1] and *sum_h are written there too; totals_ready, if
// given, is recorded once they are, before the scatter kernel runs (else the
// caller records its own event after the compaction).
int64_t compact_sums_size(int64_t n);
int64_t compact_tiles(int64_t n);  // compaction tiles over n Gaussians
int compact_tile_groups();         // preprocess workgroups per compaction tile
struct ZeroSpan {
    uint32_t* p = nullptr;
    int64_t n = 0;
};
constexpr int kZeroSpans = 2;

// Per-workgroup counts of the single-render preprocess (one per 256
// Gaussians): visible splats, their tiles touched and (h, when not null)
// their rectangle heights in tiles.  Workgroup b's counts are stored at
// (b % group) * stride + b / group, with group = the workgroups per
// compaction tile and stride = the number of compaction tiles (so the scan
// reads them coalesced).  The kernel also clears the word ranges in `clear`
// (the visible compaction's depth histograms and whatever the caller adds).
struct PreCounts {
    uint64_t* vis = nullptr;
    uint64_t* keys = nullptr;
    uint64_t* h = nullptr;
    int64_t stride = 0;
    int group = 1;
    ZeroSpan clear[1 + kZeroSpans];
};
inline int64_t preprocess_blocks(int64_t n) { return (n + 255) / 256; }
hipError_t launch_preprocess_counted(const ProjParams& p, const SceneParams& s, const SplatBuffers& out,
                                     const PreCounts& c, hipStream_t stream);
// The visible compaction after launch_preprocess_counted: its per-256 counts
// (c.vis, c.keys, c.h) are summed per compaction tile and scanned into
// vis_sums / key_sums (compact_sums_size(n) each), then the splats are
// compacted as by launch_compact_visible (which this replaces, counting pass
// included), with the depth histograms in kDepthHistReps replicas
// (depth_hist [kDepthHistReps][4][256], cleared by c.clear).
hipError_t launch_compact_counted(int64_t n, const PreCounts& c, const uint32_t* touched, const uint2* rect,
                                  const uint32_t* depth_bits, uint64_t* vis_sums, uint64_t* key_sums,
                                  uint64_t* h_sums, uint64_t* totals, uint64_t* sum_h, uint32_t* dkey, uint4* rec,
                                  uint32_t* depth_hist, hipStream_t stream, int tiles_x, uint64_t* host_totals);
hipError_t launch_compact_visible(int64_t n, const uint32_t* touched, const uint2* rect, const uint32_t* depth_bits,
                                  uint64_t* vis_sums, uint64_t* key_sums, uint64_t* totals, uint32_t* dkey,
                                  uint4* rec, uint32_t* depth_hist, hipStream_t stream, int tiles_x,
                                  const BatchItem* items = nullptr, int nitems = 0, uint64_t* h_sums = nullptr,
                                  uint64_t* sum_h = nullptr, const ZeroSpan* zero_spans = nullptr,
                                  uint64_t* host_totals = nullptr, hipEvent_t totals_ready = nullptr);

// Exclusive scan of n uint32 values (read as in[gather[i]] when gather is
// not null); the total (uint64, device) is written too.  `block_sums` needs
// scan_block_sums_size(n) uint64 elements.
int64_t scan_block_sums_size(int64_t n);
// Key offsets of splat records.  With `owner`, also the record owning every
// kKeyGenChunk-th key (owner[q] = the record whose keys include key
// q * kKeyGenChunk; K / kKeyGenChunk + 1 words).  With count_dev, the
// number of items is read on the device (`n` is an upper bound).
constexpr int64_t kKeyGenChunk = 1024;
hipError_t launch_exclusive_scan(const uint32_t* in, const uint32_t* gather, uint32_t* out, int64_t n,
                                 uint64_t* block_sums, uint64_t* total, hipStream_t stream,
                                 const uint4* rec = nullptr, uint32_t* owner = nullptr,
                                 const uint64_t* count_dev = nullptr);

// Key duplication over the visit order `order` (identity when null): writes
// Digit layout of an LSD sort of key bits [shift0, end_bit) in `passes`
// passes: the bits are split as evenly as possible (at most 8 per pass, the
// lower passes taking the remainder), so that e.g. 12-bit tile ids sort in
// two 6-bit passes whose digit runs are four times longer than 8 + 4.
struct DigitPlan {
    int passes = 0;
    int shift[8] = {};
    int bits[8] = {};
};
inline DigitPlan digit_plan(int passes, int shift0, int end_bit) {
    DigitPlan d;
    d.passes = passes;
    const int total = end_bit - shift0;
    int sh = shift0;
    for (int p = 0; p < passes && p < 8; ++p) {
        int b = total / passes + (p < total % passes ? 1 : 0);
        if (b < 1) b = 1;
        if (b > 8) b = 8;
        d.shift[p] = sh;
        d.bits[p] = b;
        sh += b;
    }
    return d;
}

// 64-bit keys and/or 32-bit tile ids plus values.
hipError_t launch_duplicate(int64_t n, const uint32_t* order, const uint32_t* offsets, const uint32_t* touched,
                            const uint2* rect, const uint32_t* depth_bits, int tiles_x, uint64_t* keys64,
                            uint32_t* tiles32, uint32_t* values, hipStream_t stream, const BatchItem* items = nullptr,
                            int nitems = 0, const uint4* rec = nullptr);
// Per-tile key counts from the rectangles: ranges [ntiles] of the sorted
// list, the tile-digit histograms hist [plan.passes][256] (written, not
// accumulated; may be null) and *total = K (may be null).  diff: reps *
// (ntiles + 1) ints of workspace: with reps > 1 the workgroups of the LDS
// counting kernel add into copy (workgroup % reps), so that fewer of them
// meet on one counter, and the ranges kernel sums the copies (reps <=
// kTileDiffMaxReps).  Batched renders pass their items (global tile ids).
constexpr int kTileCountBlocks = 512;
constexpr int64_t kTileDiffLdsMaxTiles = 16383;  // ntiles + 1 ints fit 64 KiB of LDS
constexpr int kTileDiffMaxReps = 4;
hipError_t launch_tile_counts(int64_t n, const uint32_t* touched, const uint2* rect, int tiles_x, int64_t ntiles,
                              int* diff, uint2* ranges, uint32_t* hist, const DigitPlan& plan, uint64_t* total,
                              int max_blocks, hipStream_t stream, const BatchItem* items = nullptr, int nitems = 0,
                              const uint4* rec = nullptr, const uint64_t* count_dev = nullptr, int reps = 1);
hipError_t launch_make_keys(const uint32_t* tiles, const uint32_t* values, const uint32_t* depth_bits,
                            int64_t count, uint64_t* keys, hipStream_t stream);

// Stable LSD radix sort, 8-bit digits from bit shift0.  Pass 0 reads (kin,
// vin) -- vin null means value = input position -- and the passes ping-pong
// between (ka, va) and (kb, vb): the result is in (ka, va) after an odd
// number of passes, in (kb, vb) after an even number.  kin may alias kb.
enum class SortAlgo { kAuto, kOnesweep, kReduceScan };
// Replicas of the depth sort's digit histograms: the compaction adds each
// workgroup's counts into copy (workgroup % kDepthHistReps), so that fewer
// workgroups' atomics meet on one counter; the passes sum the copies.
constexpr int kDepthHistReps = 4;
struct SortWorkspace {
    uint32_t* hist;       // onesweep: [passes][256] digit counts of all keys (replica 0)
    int hist_reps = 1;    // replicas of hist, hist_rep_stride words apart
    int64_t hist_rep_stride = 0;
    uint32_t* status;     // onesweep: [passes][partitions][256]
    uint32_t* counters;   // onesweep: [passes]
    uint32_t* part_hist;  // reduce-then-scan: [256][partitions]
    uint32_t* bases;      // reduce-then-scan: [256][partitions]
    uint64_t* scan_sums;  // reduce-then-scan: scan_block_sums_size(256 * partitions)
    uint64_t* scan_total;
    uint32_t* err;        // device error word
};
constexpr int kSortThreads = 256;
constexpr int kSortKeysPerThread = 16;
constexpr int64_t kSortPartition = (int64_t)kSortThreads * kSortKeysPerThread;
constexpr int64_t kSortMaxCount = (int64_t(1) << 30) - 1;
constexpr int64_t kSortRtsMinPartitions = int64_t(1) << 40;  // auto: onesweep (measured faster at 80M keys)
inline int64_t sort_partitions(int64_t count) { return (count + kSortPartition - 1) / kSortPartition; }
// Large onesweep sorts run 512-thread workgroups over 8192-key partitions:
// half the partitions, hence half the partition-id atomics.  Workspaces are
// sized with sort_partitions, the larger count.
constexpr int kSortThreadsWide = 512;
constexpr int64_t kSortWideMinCount = int64_t(1) << 23;
inline bool sort_uses_wide(int64_t count) { return count >= kSortWideMinCount; }
inline int64_t sort_partitions_wide(int64_t count) {
    const int64_t part = (int64_t)kSortThreadsWide * kSortKeysPerThread;
    return (count + part - 1) / part;
}
bool sort_uses_onesweep(int64_t count, SortAlgo algo);
hipError_t launch_sort_histogram(const uint64_t* keys, int64_t count, int passes, int shift0, uint32_t* hist,
                                 hipStream_t stream, int end_bit = 0);
hipError_t launch_sort_histogram(const uint32_t* keys, int64_t count, int passes, int shift0, uint32_t* hist,
                                 hipStream_t stream, int end_bit = 0);
// key_bytes: 4 when the sort's keys are 32-bit (its status words then cover
// wide partitions from 2^23 keys on); the default clears for narrow ones, a superset
hipError_t launch_sort_prepare(const SortWorkspace& ws, int64_t count, int passes, bool clear_hist,
                               hipStream_t stream, int key_bytes = 8);
// The words launch_sort_prepare (clear_hist false) clears, as two spans
// (look-back status, pass counters), for a kernel that clears them instead.
void sort_prepare_spans(const SortWorkspace& ws, int64_t count, int passes, int key_bytes, ZeroSpan spans[2]);
// The sort covers key bits [shift0, end_bit) (end_bit 0: shift0 + 8 * passes)
// split over the passes by digit_plan.  keep_keys false: the last pass
// writes only the values (its keys are left unwritten).
// `first_done`, when given, is recorded on `stream` after the first pass.
hipError_t launch_sort_passes(const uint64_t* kin, const uint32_t* vin, uint64_t* ka, uint32_t* va,
                              uint64_t* kb, uint32_t* vb, int64_t count, int passes, int shift0,
                              const SortWorkspace& ws, SortAlgo algo, hipStream_t stream, int end_bit = 0,
                              bool keep_keys = true, hipEvent_t first_done = nullptr);
// Bits needed for the values 0 .. v (at least 1).
inline int value_bits_for(int64_t v) {
    int b = 1;
    while (b < 63 && (v >> b) > 0) ++b;
    return b;
}
// First pass of launch_sort_passes whose output is packed words (see there),
// or `passes` when none is.
int sort_pack_pass(int passes, int shift0, int end_bit, int value_bits, bool keep_keys, bool key64);
// Whether launch_sort_passes with key generation in its first pass reads or
// writes the key buffers (ka, kb) at all; when not, they may be null.
inline bool sort_gen_needs_key_buffers(int passes, int end_bit, int value_bits) {
    return passes > 1 && sort_pack_pass(passes, 0, end_bit, value_bits, false, false) > 0;
}

// Keys of the tile sort generated inside its first pass instead of read:
// key p is the tile of the record owning it (row-major order within the
// record's rectangle), its value the record's Gaussian index, which is what
// launch_duplicate writes in record mode.
struct KeyGen {
    const uint32_t* off;    // [n] first key of each record
    const uint4* rec;       // [n] tile records (make_tile_rec)
    const uint32_t* owner;  // [count / kKeyGenChunk + 1] from launch_exclusive_scan
    int64_t n;
};
// With `gen`, kin and vin are ignored and the first pass generates the keys;
// it needs the onesweep passes (hipErrorInvalidValue otherwise).
// With gather_src/gather_dst (keep_keys false), the last pass writes
// gather_src[value] to gather_dst instead of the value to its value buffer.
// With count_dev (not with gen), the number of keys is read on the device
// from *count_dev; `count` is then an upper bound that sizes the grids.
// value_bits > 0 promises every value is below 2^value_bits: without
// keep_keys, the passes after the first one whose remaining key bits and
// value fit 32 bits then move one packed word per key instead of two
// (intermediate keys are not written; the result is the same).
hipError_t launch_sort_passes(const uint32_t* kin, const uint32_t* vin, uint32_t* ka, uint32_t* va,
                              uint32_t* kb, uint32_t* vb, int64_t count, int passes, int shift0,
                              const SortWorkspace& ws, SortAlgo algo, hipStream_t stream, int end_bit = 0,
                              bool keep_keys = true, const KeyGen* gen = nullptr, int value_bits = 0,
                              hipEvent_t first_done = nullptr, const uint4* gather_src = nullptr,
                              uint4* gather_dst = nullptr, const uint64_t* count_dev = nullptr);

hipError_t launch_fill_u32(uint32_t* p, int64_t count, uint32_t value, hipStream_t stream);

// Tile binning (stable counting sort by tile of Gaussians already in depth
// order, fused with duplication).  The visit order is cut into chunks of
// `chunk` Gaussians and the tile grid into bands of `band_rows` rows; one
// wave handles one (chunk, band) item.
struct BinPlan {
    int tiles_x = 0, tiles_y = 0;
    int band_rows = 0, bands = 0;
    int chunk = 0;        // Gaussians per chunk
    int64_t chunks = 0;
    int64_t groups = 0;   // chunk groups of the column scan
    int64_t ntiles = 0;
};
constexpr int kBinChunk = 8192;      // Gaussians per chunk
constexpr int kBinStage = 8192;      // keys staged per placement pass (>= kBinChunk)
constexpr int kBinGroup = 32;        // chunks per group of the column scan
constexpr int kBinMaxBandRows = 16;  // tile rows per counting band
constexpr int kBinMaxRowTiles = 4096;  // band_rows * tiles_x <= this
constexpr int kBinMaxTilesX = 512;   // tiles per row (8192 px)
static_assert(kBinStage >= kBinChunk, "one tile's keys of a chunk must fit one placement pass");
bool bin_supported(int tiles_x, int tiles_y);
BinPlan bin_plan(int64_t n, int tiles_x, int tiles_y);
// rectangles in visit order, culled splats as empty rectangles: vrect [n]
hipError_t launch_bin_gather(int64_t n, const uint32_t* order, const uint32_t* touched, const uint2* rect,
                             uint2* vrect, hipStream_t stream);
// M [chunks][ntiles]: keys of each chunk in each tile
hipError_t launch_bin_count(const BinPlan& p, int64_t n, const uint2* vrect, uint32_t* M, hipStream_t stream);
// E (first list position of each chunk's keys in each tile), from M;
// P [groups][ntiles] and tsum [ntiles] are workspace; ranges [ntiles]; *total = K
hipError_t launch_bin_scan(const BinPlan& p, const uint32_t* M, uint32_t* E, uint32_t* P, uint32_t* tsum,
                           uint2* ranges, uint64_t* total, hipStream_t stream);
// values [count]: Gaussian indices in (tile, visit order); M is the count
// matrix, E the positions; err |= 4 / 8 on inconsistent counts
hipError_t launch_bin_place(const BinPlan& p, int64_t n, const uint32_t* order, const uint2* vrect,
                            const uint32_t* M, const uint32_t* E, uint64_t count, uint32_t* values, uint32_t* err,
                            hipStream_t stream);
hipError_t launch_keys_from_ranges(const uint2* ranges, int64_t ntiles, const uint32_t* values,
                                   const uint32_t* depth_bits, uint64_t* keys, hipStream_t stream);

// Tile lists by stable interval placement, row by row (sort variant 4): the
// visible splats' tile records in depth order go into per-tile-row lists,
// then each row list into the tile lists at the tile ranges, without radix
// passes over the keys.  Images of at most kRowPlaceMaxBins tiles per axis.
constexpr int kRowPlaceMaxBins = 4096;
bool row_place_supported(int tiles_x, int tiles_y);
struct RowPlaceSizes {
    int64_t chunks_a = 0;      // chunks of 1024 records
    int64_t chunks_b_max = 0;  // bound on the chunks of the row lists
    int64_t ha_words = 0;      // uint32 words of RowPlaceArgs::ha
    int64_t hb_words = 0;      // uint32 words of RowPlaceArgs::hb
    int64_t small_words = 0;   // uint32 words of RowPlaceArgs::small
};
// n_records: the number of records (or a bound on it); sum_h: the sum of the
// records' rectangle heights (the number of row-list entries).
RowPlaceSizes row_place_sizes(int64_t n_records, uint64_t sum_h, int tiles_x, int tiles_y);
struct RowPlaceArgs {
    const uint4* rec;            // [n] tile records in depth order (single render: tile base 0)
    const uint64_t* count_dev;   // device: number of records
    int64_t n_records_max;       // bound on it (sizes the grids)
    int tiles_x = 0, tiles_y = 0;
    uint64_t sum_h = 0;          // row-list entries
    uint64_t K = 0;              // keys
    const uint2* ranges;         // [tiles] ranges of the sorted list
    hipEvent_t ranges_ready;     // recorded where the ranges are complete, or null
    uint32_t* ha;                // workspace, row_place_sizes words each
    uint32_t* hb;
    uint32_t* small;
    uint2* rowent;               // [sum_h] workspace
    uint32_t* values;            // [K] output
    uint32_t* err;               // device error word (bit 32: inconsistent counts)
};
// `rows_done` and `cols_counted`, when given, are recorded on `stream` once
// the row lists are complete and right before the last kernel (the placement
// into the tile lists).
hipError_t launch_row_place(const RowPlaceArgs& a, hipStream_t stream, hipEvent_t rows_done = nullptr,
                            hipEvent_t cols_counted = nullptr);

hipError_t launch_ranges(const uint32_t* tile_words, int stride, int64_t count, uint2* ranges,
                         int64_t ntiles, hipStream_t stream);

struct BlendArgs {
    const uint2* ranges;
    const uint32_t* point_list;
    const float2* mean2d;
    const float4* conic_opacity;
    const float4* rgb;
    int32_t width, height, tiles_x, tiles_y;
    float bg[3];
    float* out_rgb;
    float* out_T;
    uint32_t* out_ncontrib;
    const uint32_t* depth_bits;  // float32 bits of each Gaussian's depth (read with out_invdepth)
    float* out_invdepth;         // [H][W] expected inverse depth, or null
    uint32_t* counter;           // work counter of the work-stealing variant (3)
    int64_t n;                   // number of splats: a list entry at or past it is never read
    uint32_t* err;               // device error word: bit 16 set on a list entry at or past n
};
// variant: 1, 2, 4 = pixels per thread of the per-tile kernel; 3 = work-stealing half tiles
hipError_t launch_blend(const BlendArgs& a, int variant, hipStream_t stream);

// Persistent blend over the tiles of a batch: workgroups pull global tile
// ids from `counter` (zero on entry) until all `total_tiles` are done.
hipError_t launch_blend_batch(const BatchItem* items, int nitems, int64_t total_tiles, const uint2* ranges,
                              const uint32_t* point_list, int64_t n, const float2* mean2d,
                              const float4* conic_opacity, const float4* rgb, uint32_t* counter, int grid,
                              uint32_t* err, hipStream_t stream);

// Per-Gaussian 2D gradient sums of the backward pass, one row per Gaussian:
// the sums over its pixels of dL/dpower times dx, dy, dx^2, dx dy and dy^2
// (dx, dy = 2D mean - pixel; power = the exponent of G), from which the
// backward preprocessing forms the 2D mean and conic gradients; then
// dL/dopacity, dL/d(r, g, b) and dL/d(1 / depth).
constexpr int kGrad2d = 10;

struct BlendBwdArgs {
    const uint2* ranges;
    const uint32_t* point_list;
    const float2* mean2d;
    const float4* conic_opacity;
    const float4* rgb;
    int32_t width, height, tiles_x, tiles_y;
    float bg[3];
    const float* final_T;
    const uint32_t* ncontrib;
    const float* dL_drgb;
    const uint32_t* depth_bits;  // float32 bits of each Gaussian's depth (read with dL_dinvdepth)
    const float* dL_dinvdepth;   // [H][W] gradient w.r.t. the expected inverse depth, or null
    int64_t n;
    float* grad2d;  // [n][kGrad2d], zero on entry
    uint32_t* err;  // device error word: bit 16 set on a list entry at or past n
};
hipError_t launch_blend_backward(const BlendBwdArgs& a, hipStream_t stream);

struct PreBwdArgs {
    const int32_t* radius;
    const uint8_t* clamp_flags;
    const float* grad2d;  // [n][kGrad2d]
    const float* jac = nullptr;  // SplatBuffers::jac of the forward render, or null (read the SH)
    float* g_means;
    float* g_log_scales;
    float* g_quats;
    float* g_opacity_logits;
    float* g_sh;
};
hipError_t launch_preprocess_backward(const ProjParams& p, const SceneParams& s, const PreBwdArgs& a,
                                      hipStream_t stream);

// partial: 1024 floats of device workspace
hipError_t launch_l1_loss_grad(const float* rgb, const float* target, int64_t count, float* grad,
                               float* loss, float* partial, hipStream_t stream);

}  // namespace cds
