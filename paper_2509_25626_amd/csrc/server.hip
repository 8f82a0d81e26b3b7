// Continuous-batching render server over resident scenes.
//
// Requests (scene, camera, output image) are queued by any host thread.  A
// scheduler thread admits queued requests in arrival order whenever a batch
// workspace is free, the number of requests in flight is below the slot
// limit, and the estimated workspace of the admitted requests fits the HBM
// budget.  A batch takes at most max_batch requests and at most its share of
// the queue over the free workspaces (a short queue runs as batches side by
// side), and stops before its global tile ids pass 14 bits or its Gaussian
// indices 25, so that it sorts like a single render.  Each admitted batch
// runs as one pass of batched kernels:
// preprocess over the concatenated Gaussians of all its scenes, compaction
// of the visible splats into tile records in global tile ids (request tile
// bases) and the key-count read-back, one depth sort, the key offsets, the
// ranges from the records, one tile sort whose first pass generates the
// keys, and a persistent blend whose workgroups pull tiles of every request
// from one work counter.  Two
// workspaces on two streams let the next batch's preprocessing overlap the
// current batch's sort and blend; requests that arrive meanwhile join the
// next batch.
//
// The per-Gaussian and per-tile work are the same device functions as the
// single render, and the sorted (global tile, depth, index) order restricted
// to one request equals its own (tile, depth, index) order, so a request's
// image is bit-identical alone or in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "runtime_internal.h"

using namespace cds;

namespace {

constexpr int kMaxSlots = 64;
constexpr int kWorkspaces = 2;

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct SrvRequest {
    uint64_t ticket = 0;
    int32_t scene = 0;
    cds_camera cam{};
    float* out_rgb = nullptr;
    double t_submit = 0, t_done = 0;
    int64_t est_bytes = 0;
    bool done = false;
    cds_status status = CDS_OK;
    std::string error;
};

struct Workspace {
    cds_frame* frame = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    BatchItem* items_host = nullptr;  // pinned
    BatchItem* items_dev = nullptr;
    uint32_t* counter = nullptr;      // persistent-blend work counter
    uint64_t* pinned = nullptr;       // key-count read-back
    bool busy = false;
    std::vector<SrvRequest*> reqs;
    int64_t reserved = 0;
    int64_t held = 0;  // device bytes its frame buffers hold (measured after each batch is enqueued)
};

}  // namespace

struct cds_server {
    cds_ctx* ctx = nullptr;
    cds_server_opts opts{};
    int cus = 256;
    std::vector<cds_scene> scenes;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<SrvRequest*> pending;
    std::unordered_map<uint64_t, SrvRequest*> tickets;
    uint64_t next_ticket = 1;
    std::thread worker;
    bool stop = false;
    Workspace ws[kWorkspaces];
    int64_t budget = 0, reserved = 0;
    int64_t held = 0;  // sum of the workspaces' held bytes
    int inflight = 0;
    double key_scale = 1.0;  // learned ratio of actual to estimated keys
    cds_server_stats stats{};
};

namespace {

#define SRV_HIP(expr, what)                              \
    do {                                                 \
        hipError_t _e = (expr);                          \
        if (_e != hipSuccess) return hip_fail(_e, what); \
    } while (0)
#define SRV_TRY(expr)                \
    do {                             \
        cds_status _s = (expr);      \
        if (_s != CDS_OK) return _s; \
    } while (0)

// Workspace estimate of one request: ~120 B per Gaussian of frame state,
// visible-splat records and depth sort, ~9 B per key (packed words and
// values, sort status), keys estimated at 64 per Gaussian per megapixel,
// scaled by what earlier batches measured.
constexpr int64_t kBatchMaxTiles = kTileDiffLdsMaxTiles;     // 14-bit global tile ids
constexpr int64_t kBatchMaxGaussians = int64_t(1) << 25;      // 25-bit Gaussian indices

int64_t estimate_bytes(const cds_server* s, const cds_scene& sc, const cds_camera& cam) {
    const double mp = (double)cam.width * cam.height / 1.0e6;
    const double keys = s->key_scale * 64.0 * (double)sc.n * std::max(mp, 0.05);
    const int64_t tiles = (int64_t)((cam.width + CDS_TILE - 1) / CDS_TILE) * ((cam.height + CDS_TILE - 1) / CDS_TILE);
    return (int64_t)(120.0 * (double)sc.n + 9.0 * keys) + 12 * tiles + 4096;
}

cds_status run_batch(cds_server* s, Workspace& w) {
    cds_ctx* ctx = s->ctx;
    cds_frame* f = w.frame;
    hipStream_t stream = w.stream;
    const int nitems = (int)w.reqs.size();
    int64_t N = 0, T = 0;
    for (int k = 0; k < nitems; ++k) {
        const SrvRequest* r = w.reqs[k];
        const cds_scene& sc = s->scenes[r->scene];
        BatchItem& it = w.items_host[k];
        std::memset(&it, 0, sizeof(it));
        it.P = make_proj(&sc, &r->cam);
        it.S = make_scene(&sc);
        it.gauss_base = N;
        it.tile_base = T;
        for (int c = 0; c < 3; ++c) it.bg[c] = r->cam.bg[c];
        it.out_rgb = r->out_rgb;
        N += sc.n;
        T += (int64_t)it.P.tiles_x * it.P.tiles_y;
    }
    if (N > (int64_t)0x7FFFFFFF || T > (int64_t)0x7FFFFFFF) return fail(CDS_ERR_CAPACITY, "batch too large");
    // The stacked tile grid of the row-wise placement: every request's tile
    // rows one below the other, all as wide as the widest request.  Its tile
    // order restricted to the real tiles is the global tile order, so the
    // sorted list is the same; records, ranges and the blend use its ids.
    int64_t W = 0, Rows = 0;
    for (int k = 0; k < nitems; ++k) W = std::max<int64_t>(W, w.items_host[k].P.tiles_x);
    for (int k = 0; k < nitems; ++k) Rows += w.items_host[k].P.tiles_y;
    const bool stacked = row_place_supported((int)std::min<int64_t>(W, INT32_MAX),
                                             (int)std::min<int64_t>(Rows, INT32_MAX));
    int64_t row_base = 0;
    for (int k = 0; k < nitems && stacked; ++k) {
        BatchItem& it = w.items_host[k];
        it.rec_stride = (int32_t)W;
        it.rec_base = row_base * W;
        row_base += it.P.tiles_y;
    }
    const int64_t Tg = stacked ? W * Rows : T;  // tile ids of the records, the ranges and the blend
    const int tile_passes = (tile_bits_for(Tg) + 7) / 8;
    SRV_HIP(hipMemcpyAsync(w.items_dev, w.items_host, sizeof(BatchItem) * nitems, hipMemcpyHostToDevice, stream),
            "hipMemcpyAsync(batch items)");
    const size_t nn = (size_t)std::max<int64_t>(N, 1);
    SRV_TRY(ensure(ctx, f->mean2d, sizeof(float2) * nn, 1.25));
    SRV_TRY(ensure(ctx, f->conic, sizeof(float4) * nn, 1.25));
    SRV_TRY(ensure(ctx, f->rgb, sizeof(float4) * nn, 1.25));
    SRV_TRY(ensure(ctx, f->depth, sizeof(uint32_t) * nn, 1.25));
    SRV_TRY(ensure(ctx, f->radius, sizeof(int32_t) * nn, 1.25));
    SRV_TRY(ensure(ctx, f->rect, sizeof(uint2) * nn, 1.25));
    SRV_TRY(ensure(ctx, f->touched, sizeof(uint32_t) * nn, 1.25));
    SRV_TRY(ensure(ctx, f->offsets, sizeof(uint32_t) * nn, 1.25));
    SRV_TRY(ensure(ctx, f->clampf, nn, 1.25));
    SRV_TRY(ensure(ctx, f->blocksums, sizeof(uint64_t) * scan_block_sums_size(N), 1.25));
    SRV_TRY(ensure(ctx, f->total, 256));
    SRV_TRY(ensure(ctx, f->order0, sizeof(uint32_t) * nn, 1.25));
    SRV_TRY(ensure(ctx, f->order1, sizeof(uint32_t) * nn, 1.25));
    SRV_TRY(ensure(ctx, f->dkey0, sizeof(uint32_t) * nn, 1.25));
    SRV_TRY(ensure(ctx, f->dkey1, sizeof(uint32_t) * nn, 1.25));
    SRV_TRY(ensure(ctx, f->dkeyc, sizeof(uint32_t) * nn, 1.25));
    SRV_TRY(ensure(ctx, f->recc, sizeof(uint4) * nn, 1.25));
    SRV_TRY(ensure(ctx, f->recv, sizeof(uint4) * nn, 1.25));
    SRV_TRY(ensure(ctx, f->vsums, sizeof(uint64_t) * compact_sums_size(N), 1.25));
    SRV_TRY(ensure(ctx, f->ksums, sizeof(uint64_t) * compact_sums_size(N), 1.25));
    SRV_TRY(ensure(ctx, f->ranges, sizeof(uint2) * (size_t)std::max<int64_t>(Tg, 1), 1.25));
    SRV_TRY(ensure(ctx, f->tdiff, sizeof(int) * (size_t)(Tg + 1), 1.25));
    if (stacked) SRV_TRY(ensure(ctx, f->hsums, sizeof(uint64_t) * compact_sums_size(N), 1.25));
    SRV_TRY(ensure(ctx, f->thist, sizeof(uint32_t) * 4 * 256));
    SRV_TRY(ensure_sort_workspace(ctx, f->sort_d, N, 4));

    SplatBuffers sb;
    sb.mean2d = (float2*)f->mean2d.p;
    sb.conic_opacity = (float4*)f->conic.p;
    sb.rgb = (float4*)f->rgb.p;
    sb.depth_bits = (uint32_t*)f->depth.p;
    sb.radius = (int32_t*)f->radius.p;
    sb.rect = (uint2*)f->rect.p;
    sb.touched = (uint32_t*)f->touched.p;
    sb.clamp_flags = (uint8_t*)f->clampf.p;
    SRV_HIP(launch_preprocess_batch(w.items_dev, nitems, N, sb, stream), "batched preprocess");
    const SortAlgo algo = SortAlgo::kAuto;
    SortWorkspace wd = sort_ws(ctx, f->sort_d);
    uint64_t* d_total = (uint64_t*)f->total.p;  // [0] = visible splats, [1] = K
    // visible splats compacted with tile records in global tile ids, the
    // depth histograms, n_vis and K
    SRV_HIP(launch_compact_visible(N, sb.touched, sb.rect, sb.depth_bits, (uint64_t*)f->vsums.p,
                                   (uint64_t*)f->ksums.p, d_total, (uint32_t*)f->dkeyc.p, (uint4*)f->recc.p,
                                   wd.hist, stream, 0, w.items_dev, nitems,
                                   stacked ? (uint64_t*)f->hsums.p : nullptr, stacked ? d_total + 3 : nullptr),
            "batched compaction");
    SRV_HIP(hipMemcpyAsync(w.pinned, d_total, 4 * sizeof(uint64_t), hipMemcpyDeviceToHost, stream),
            "hipMemcpyAsync(key count)");
    SRV_HIP(hipStreamSynchronize(stream), "hipStreamSynchronize(key count)");
    const int64_t nvis = (int64_t)w.pinned[0];
    const uint64_t K = w.pinned[1];
    const uint64_t sum_h = stacked ? w.pinned[3] : 0;
    // the row-wise placement's limits (buffer offsets below 2^31 bytes)
    const bool rowplace = stacked && s->opts.sort_variant != 2 && K > 0 && K <= (uint64_t(1) << 29) &&
                          sum_h <= (uint64_t(1) << 28);
    if (K > (uint64_t)kSortMaxCount) return fail(CDS_ERR_CAPACITY, "batch needs more than 2^30-1 tile keys");
    int64_t est = 0;
    for (const SrvRequest* r : w.reqs) {
        const double mp = (double)r->cam.width * r->cam.height / 1.0e6;
        est += (int64_t)(s->key_scale * 64.0 * (double)s->scenes[r->scene].n * std::max(mp, 0.05));
    }
    if (est > 0) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->key_scale = std::max(0.05, 0.7 * s->key_scale + 0.3 * s->key_scale * (double)K / (double)est);
    }
    const uint4* recv = (const uint4*)f->recv.p;
    if (nvis > 0) {
        // depth order of the visible splats, their records in that order, key
        // offsets and the owner of every 1024th key
        if (sort_uses_onesweep(nvis, algo)) SRV_HIP(launch_sort_prepare(wd, nvis, 4, false, stream, 4), "depth prepare");
        SRV_HIP(launch_sort_passes((const uint32_t*)f->dkeyc.p, nullptr, (uint32_t*)f->dkey0.p, (uint32_t*)f->order0.p,
                                   (uint32_t*)f->dkey1.p, (uint32_t*)f->order1.p, nvis, 4, 0, wd, algo, stream, 32,
                                   false, nullptr, value_bits_for(nvis - 1), nullptr, (const uint4*)f->recc.p,
                                   (uint4*)f->recv.p),
                "depth sort (records in depth order)");
        if (!rowplace) {
            SRV_TRY(ensure(ctx, f->kowner, sizeof(uint32_t) * (size_t)(K / kKeyGenChunk + 1), 1.25));
            SRV_HIP(launch_exclusive_scan(nullptr, nullptr, (uint32_t*)f->offsets.p, nvis,
                                          (uint64_t*)f->blocksums.p, d_total + 2, stream, recv,
                                          (uint32_t*)f->kowner.p),
                    "offset scan");
        }
    }
    // ranges and tile-digit histograms from the records (global or stacked tile ids)
    const int tile_bits = tile_bits_for(Tg);
    SRV_HIP(launch_tile_counts(nvis, nullptr, nullptr, 0, Tg, (int*)f->tdiff.p, (uint2*)f->ranges.p,
                               (uint32_t*)f->thist.p, digit_plan(tile_passes, 0, tile_bits), nullptr, kTileCountBlocks,
                               stream, nullptr, 0, (const uint4*)f->recc.p),  // index order: chunks stay in one request
            "batched tile counts");
    if (rowplace) {
        // tile lists by stable placement over the stacked tile rows, then columns
        const RowPlaceSizes rs = row_place_sizes(nvis, sum_h, (int)W, (int)Rows);
        SRV_TRY(ensure(ctx, f->rp_ha, sizeof(uint32_t) * (size_t)rs.ha_words, 1.25));
        SRV_TRY(ensure(ctx, f->rp_hb, sizeof(uint32_t) * (size_t)std::max<int64_t>(rs.hb_words, 1), 1.25));
        SRV_TRY(ensure(ctx, f->rp_small, sizeof(uint32_t) * (size_t)rs.small_words, 1.25));
        SRV_TRY(ensure(ctx, f->rp_rowent, sizeof(uint2) * (size_t)std::max<uint64_t>(sum_h, 1), 1.25));
        SRV_TRY(ensure(ctx, f->vals0, sizeof(uint32_t) * (size_t)K, 1.25));
        RowPlaceArgs ra;
        ra.rec = recv;
        ra.count_dev = d_total;
        ra.n_records_max = nvis;
        ra.tiles_x = (int)W;
        ra.tiles_y = (int)Rows;
        ra.sum_h = sum_h;
        ra.K = K;
        ra.ranges = (const uint2*)f->ranges.p;
        ra.ranges_ready = nullptr;  // same stream
        ra.ha = (uint32_t*)f->rp_ha.p;
        ra.hb = (uint32_t*)f->rp_hb.p;
        ra.small = (uint32_t*)f->rp_small.p;
        ra.rowent = (uint2*)f->rp_rowent.p;
        ra.values = (uint32_t*)f->vals0.p;
        ra.err = ctx->d_err;
        SRV_HIP(launch_row_place(ra, stream), "batched row-wise tile placement");
        const int64_t grid = std::min<int64_t>(T, (int64_t)s->cus * 8);
        SRV_HIP(launch_blend_batch(w.items_dev, nitems, T, (const uint2*)f->ranges.p, (const uint32_t*)f->vals0.p, N,
                                   sb.mean2d, sb.conic_opacity, sb.rgb, w.counter, (int)grid, ctx->d_err, stream),
                "batched blend");
        SRV_HIP(hipEventRecord(w.done, stream), "hipEventRecord");
        return CDS_OK;
    }
    const size_t kk = (size_t)std::max<uint64_t>(K, 1);
    const bool fused = sort_uses_onesweep((int64_t)K, algo) && tile_passes > 0;
    const int vbits = value_bits_for(N - 1);
    if (!fused || sort_gen_needs_key_buffers(tile_passes, tile_bits, vbits)) {
        SRV_TRY(ensure(ctx, f->tk0, sizeof(uint32_t) * kk, 1.25));
        SRV_TRY(ensure(ctx, f->tk1, sizeof(uint32_t) * kk, 1.25));
    }
    SRV_TRY(ensure(ctx, f->vals0, sizeof(uint32_t) * kk, 1.25));
    SRV_TRY(ensure(ctx, f->vals1, sizeof(uint32_t) * kk, 1.25));
    SRV_TRY(ensure_sort_workspace(ctx, f->sort, (int64_t)K, std::max(tile_passes, 1)));
    SortWorkspace ws = sort_ws(ctx, f->sort);
    if (K > 0) {
        if (sort_uses_onesweep((int64_t)K, algo) && tile_passes > 0)
            SRV_HIP(launch_sort_prepare(ws, (int64_t)K, tile_passes, false, stream, 4), "sort prepare");
        ws.hist = (uint32_t*)f->thist.p;
        KeyGen gen;
        gen.off = (const uint32_t*)f->offsets.p;
        gen.rec = recv;
        gen.owner = (const uint32_t*)f->kowner.p;
        gen.n = nvis;
        if (!fused)
            SRV_HIP(launch_duplicate(nvis, nullptr, (const uint32_t*)f->offsets.p, nullptr, nullptr, nullptr, 0,
                                     nullptr, (uint32_t*)f->tk0.p, (uint32_t*)f->vals0.p, stream, nullptr, 0, recv),
                    "batched duplicate");
        SRV_HIP(launch_sort_passes((const uint32_t*)f->tk0.p, (const uint32_t*)f->vals0.p, (uint32_t*)f->tk1.p,
                                   (uint32_t*)f->vals1.p, (uint32_t*)f->tk0.p, (uint32_t*)f->vals0.p, (int64_t)K,
                                   tile_passes, 0, ws, algo, stream, tile_bits, false, fused ? &gen : nullptr, vbits),
                "tile sort");
    }
    const bool odd = (tile_passes & 1) != 0;
    const uint32_t* values = (const uint32_t*)(odd ? f->vals1.p : f->vals0.p);
    const int64_t grid = std::min<int64_t>(T, (int64_t)s->cus * 8);
    SRV_HIP(launch_blend_batch(w.items_dev, nitems, T, (const uint2*)f->ranges.p, values, N, sb.mean2d,
                               sb.conic_opacity, sb.rgb, w.counter, (int)grid, ctx->d_err, stream),
            "batched blend");
    SRV_HIP(hipEventRecord(w.done, stream), "hipEventRecord");
    return CDS_OK;
}

// Frees an idle workspace's frame buffers (the next batch there allocates again).
void release_workspace(cds_server* s, Workspace& w) {
    (void)hipStreamSynchronize(w.stream);  // idle already; the buffers must not be in use
    release_frame_buffers(w.frame);
    s->held -= w.held;
    w.held = 0;
    s->stats.held_bytes = s->held;
}

void finish(cds_server* s, Workspace& w, cds_status st, const std::string& err) {
    const double t = now_ms();
    for (SrvRequest* r : w.reqs) {
        r->done = true;
        r->t_done = t;
        r->status = st;
        r->error = err;
    }
    s->stats.completed += (int64_t)w.reqs.size();
    if (st != CDS_OK) s->stats.rejected += (int64_t)w.reqs.size();
    s->inflight -= (int)w.reqs.size();
    s->reserved -= w.reserved;
    s->stats.workspace_bytes = s->reserved;
    w.reqs.clear();
    w.reserved = 0;
    w.busy = false;
    // buffers grown past the workspace's share of the budget (an oversized
    // batch) are given back once its work is done
    if (w.held > s->budget / kWorkspaces) release_workspace(s, w);
}

void worker_main(cds_server* s) {
    (void)hipSetDevice(s->ctx->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // retire finished batches
        for (Workspace& w : s->ws) {
            if (!w.busy || w.reqs.empty() || !w.done) continue;
            lk.unlock();
            const hipError_t q = hipEventQuery(w.done);
            lk.lock();
            if (q == hipSuccess) finish(s, w, CDS_OK, "");
            else if (q != hipErrorNotReady) finish(s, w, CDS_ERR_DEVICE, hipGetErrorString(q));
        }
        s->cv.notify_all();
        int nbusy = 0;
        Workspace* free_ws = nullptr;
        int nfree = 0;
        for (Workspace& w : s->ws) {
            if (w.busy) ++nbusy;
            else {
                ++nfree;
                if (!free_ws) free_ws = &w;
            }
        }
        if (s->stop && s->pending.empty() && nbusy == 0) break;
        // admit: arrival order, slot limit, batch limit, HBM budget
        if (free_ws && !s->pending.empty()) {
            std::vector<SrvRequest*> batch;
            int64_t bytes = 0, tiles = 0, gaussians = 0;
            // a short queue is spread over the free workspaces (their batches
            // run side by side) rather than packed into one batch that all of
            // its requests wait for; a long one still fills batches
            const int share = (int)((s->pending.size() + (size_t)nfree - 1) / (size_t)nfree);
            const int limit = std::min(s->opts.max_batch, std::max(1, share));
            // the device memory the batch would leave held: the other
            // workspaces' buffers plus this one's grown to the estimate (with
            // the allocator's 1.25 growth); idle workspaces give theirs back
            // when that is what keeps it within the budget
            const auto projected = [&](int64_t est) {
                const int64_t need = est + est / 4;
                return s->held - free_ws->held + std::max(free_ws->held, need);
            };
            while (!s->pending.empty() && (int)batch.size() < limit &&
                   s->inflight + (int)batch.size() < s->opts.max_slots) {
                SrvRequest* r = s->pending.front();
                const bool alone = batch.empty() && s->reserved == 0;
                if (projected(bytes + r->est_bytes) > s->budget)
                    for (Workspace& o : s->ws)
                        if (&o != free_ws && !o.busy && o.held > 0) release_workspace(s, o);
                if (!alone && (s->reserved + bytes + r->est_bytes > s->budget ||
                               projected(bytes + r->est_bytes) > s->budget))
                    break;
                // a batch's global tile ids and Gaussian indices stay small enough
                // for the single render's sort shape: tile counts in one LDS array,
                // two tile passes of at most 7-bit digits, and the second pass's
                // key bits with the index in one packed word
                const int64_t rt = (int64_t)((r->cam.width + CDS_TILE - 1) / CDS_TILE) * ((r->cam.height + CDS_TILE - 1) / CDS_TILE);
                const int64_t rg = s->scenes[r->scene].n;
                if (!batch.empty() && (tiles + rt > kBatchMaxTiles || gaussians + rg > kBatchMaxGaussians)) break;
                batch.push_back(r);
                bytes += r->est_bytes;
                tiles += rt;
                gaussians += rg;
                s->pending.pop_front();
            }
            if (!batch.empty()) {
                Workspace& w = *free_ws;
                w.busy = true;
                w.reqs = batch;
                w.reserved = bytes;
                s->reserved += bytes;
                s->inflight += (int)batch.size();
                s->stats.batches += 1;
                s->stats.workspace_bytes = s->reserved;
                s->stats.peak_workspace_bytes = std::max(s->stats.peak_workspace_bytes, s->reserved);
                lk.unlock();
                const cds_status st = run_batch(s, w);
                const std::string err = st == CDS_OK ? "" : g_last_error;
                const int64_t held = frame_held_bytes(w.frame);
                lk.lock();
                s->held += held - w.held;
                w.held = held;
                s->stats.held_bytes = s->held;
                s->stats.peak_held_bytes = std::max(s->stats.peak_held_bytes, s->held);
                if (st != CDS_OK) finish(s, w, st, err);
                continue;
            }
        }
        // wait for work: a completion if anything is in flight, else a submission
        Workspace* oldest = nullptr;
        for (Workspace& w : s->ws)
            if (w.busy && (!oldest)) oldest = &w;
        if (oldest && (nbusy == kWorkspaces || !s->pending.empty())) {
            hipEvent_t ev = oldest->done;
            lk.unlock();
            (void)hipEventSynchronize(ev);
            lk.lock();
        } else if (oldest) {
            s->cv.wait_for(lk, std::chrono::microseconds(50));
        } else {
            s->cv.wait(lk, [&] { return s->stop || !s->pending.empty(); });
        }
    }
}

void destroy_workspaces(cds_server* s) {
    for (Workspace& w : s->ws) {
        if (w.frame) {
            w.frame->release_all();
            delete w.frame;
            w.frame = nullptr;
        }
        if (w.stream) (void)hipStreamDestroy(w.stream);
        if (w.done) (void)hipEventDestroy(w.done);
        if (w.items_host) (void)hipHostFree(w.items_host);
        if (w.pinned) (void)hipHostFree(w.pinned);
        if (w.items_dev) ctx_free(s->ctx, w.items_dev);
        if (w.counter) ctx_free(s->ctx, w.counter);
        w = Workspace();
    }
}

}  // namespace

extern "C" {

cds_status cds_server_create(cds_ctx* ctx, const cds_server_opts* opts, cds_server** out) {
    if (out) *out = nullptr;
    if (!ctx || !opts || !out) return fail(CDS_ERR_INVALID_ARG, "NULL argument");
    if (opts->max_slots < 1 || opts->max_slots > kMaxSlots) return fail(CDS_ERR_INVALID_ARG, "max_slots must be 1..64");
    if (opts->sort_variant != 0 && opts->sort_variant != 2 && opts->sort_variant != 4)
        return fail(CDS_ERR_INVALID_ARG, "server sort_variant must be 0, 2 or 4");
    if (opts->max_batch < 1 || opts->max_batch > opts->max_slots)
        return fail(CDS_ERR_INVALID_ARG, "max_batch must be 1..max_slots");
    if (opts->hbm_budget_bytes < 0) return fail(CDS_ERR_INVALID_ARG, "hbm_budget_bytes < 0");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    cds_server* s = new cds_server();
    s->ctx = ctx;
    s->opts = *opts;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess && prop.multiProcessorCount > 0)
        s->cus = prop.multiProcessorCount;
    if (opts->hbm_budget_bytes > 0) {
        s->budget = opts->hbm_budget_bytes;
    } else {
        size_t freeb = 0, total = 0;
        if ((e = hipMemGetInfo(&freeb, &total)) != hipSuccess) {
            delete s;
            return hip_fail(e, "hipMemGetInfo");
        }
        s->budget = (int64_t)(0.5 * (double)freeb);
    }
    cds_status st = CDS_OK;
    for (Workspace& w : s->ws) {
        w.frame = new cds_frame();
        w.frame->ctx = ctx;
        if ((e = hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&w.done, hipEventDisableTiming)) != hipSuccess ||
            (e = hipHostMalloc((void**)&w.items_host, sizeof(BatchItem) * kMaxSlots, hipHostMallocDefault)) !=
                hipSuccess ||
            (e = hipHostMalloc((void**)&w.pinned, 4096, hipHostMallocDefault)) != hipSuccess) {
            st = hip_fail(e, "server stream/event/pinned allocation");
            break;
        }
        w.items_dev = (BatchItem*)ctx_alloc(ctx, sizeof(BatchItem) * kMaxSlots);
        w.counter = (uint32_t*)ctx_alloc(ctx, 256);
        if (!w.items_dev || !w.counter) {
            st = fail(CDS_ERR_OOM, "server workspace allocation failed");
            break;
        }
    }
    if (st != CDS_OK) {
        destroy_workspaces(s);
        delete s;
        return st;
    }
    s->worker = std::thread(worker_main, s);
    *out = s;
    return CDS_OK;
}

cds_status cds_server_add_scene(cds_server* s, const cds_scene* scene, int32_t* scene_id) {
    if (!s || !scene_id) return fail(CDS_ERR_INVALID_ARG, "NULL argument");
    cds_status st = validate_scene(scene);
    if (st != CDS_OK) return st;
    std::lock_guard<std::mutex> lk(s->mu);
    s->scenes.push_back(*scene);
    *scene_id = (int32_t)s->scenes.size() - 1;
    return CDS_OK;
}

cds_status cds_server_submit(cds_server* s, int32_t scene_id, const cds_camera* cam, float* out_rgb,
                             uint64_t* ticket) {
    if (!s || !ticket || !out_rgb) return fail(CDS_ERR_INVALID_ARG, "NULL argument");
    cds_status st = validate_camera(cam);
    if (st != CDS_OK) return st;
    SrvRequest* r = new SrvRequest();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (scene_id < 0 || scene_id >= (int32_t)s->scenes.size()) {
            delete r;
            return fail(CDS_ERR_INVALID_ARG, "no such scene");
        }
        r->scene = scene_id;
        r->cam = *cam;
        r->out_rgb = out_rgb;
        r->est_bytes = estimate_bytes(s, s->scenes[scene_id], *cam);
        if (r->est_bytes > s->budget) {
            s->stats.rejected += 1;
            delete r;
            return fail(CDS_ERR_BUSY, "request workspace estimate exceeds the server's HBM budget");
        }
        r->ticket = s->next_ticket++;
        r->t_submit = now_ms();
        s->tickets[r->ticket] = r;
        s->pending.push_back(r);
        s->stats.submitted += 1;
        *ticket = r->ticket;
    }
    s->cv.notify_all();
    return CDS_OK;
}

cds_status cds_server_poll(cds_server* s, uint64_t ticket, int32_t* done, double* latency_ms) {
    if (!s || !done) return fail(CDS_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return fail(CDS_ERR_INVALID_ARG, "unknown or already collected ticket");
    SrvRequest* r = it->second;
    *done = r->done ? 1 : 0;
    if (!r->done) return CDS_OK;
    if (latency_ms) *latency_ms = r->t_done - r->t_submit;
    const cds_status st = r->status;
    const std::string err = r->error;
    s->tickets.erase(it);
    delete r;
    if (st != CDS_OK) return fail(st, "request failed: " + err);
    return CDS_OK;
}

cds_status cds_server_drain(cds_server* s) {
    if (!s) return fail(CDS_ERR_INVALID_ARG, "NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv.notify_all();
    s->cv.wait(lk, [&] {
        if (!s->pending.empty()) return false;
        for (const Workspace& w : s->ws)
            if (w.busy) return false;
        return true;
    });
    return CDS_OK;
}

cds_status cds_server_get_stats(cds_server* s, cds_server_stats* out) {
    if (!s || !out) return fail(CDS_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    return CDS_OK;
}

void cds_server_destroy(cds_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    (void)hipSetDevice(s->ctx->device);
    for (Workspace& w : s->ws)
        if (w.stream) (void)hipStreamSynchronize(w.stream);
    destroy_workspaces(s);
    for (auto& kv : s->tickets) delete kv.second;
    delete s;
}

}  // extern "C"
