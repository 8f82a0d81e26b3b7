// The stream-ordered launch sequence of one forward render and one backward
// pass (paper Section II-B: preprocessing -> duplication -> sort -> ranges ->
// alpha blending).  The only host wait is the read-back of the key count K
// after the prefix sum; every other step is enqueued on the caller's stream.
#include <cstring>

#include "runtime_internal.h"

namespace cds {

void release_frame_events(cds_frame* f) {
    for (hipEvent_t& e : f->ev)
        if (e) {
            (void)hipEventDestroy(e);
            e = nullptr;
        }
    for (hipEvent_t* e : {&f->fork, &f->join, &f->copied})
        if (*e) {
            (void)hipEventDestroy(*e);
            *e = nullptr;
        }
    if (f->side) {
        (void)hipStreamDestroy(f->side);  // waits for its work
        f->side = nullptr;
    }
}

// Every device buffer a frame may hold.
template <typename F>
void for_each_frame_buffer(cds_frame* f, F&& fn) {
    DevBuf* bufs[] = {&f->mean2d, &f->conic, &f->rgb, &f->depth, &f->radius, &f->rect, &f->touched,
                      &f->offsets, &f->kowner, &f->clampf, &f->blocksums, &f->total, &f->order0, &f->order1,
                      &f->dkey0, &f->dkey1, &f->sort_d.hist, &f->sort_d.status, &f->sort_d.counters,
                      &f->sort_d.part_hist, &f->sort_d.bases, &f->sort_d.scan_sums, &f->sort_d.scan_total,
                      &f->vrect, &f->binM, &f->binE, &f->binP, &f->tsum, &f->tdiff, &f->thist,
                      &f->dkeyc, &f->recc, &f->recv, &f->vsums, &f->ksums, &f->hsums, &f->rp_ha, &f->rp_hb,
                      &f->rp_small, &f->rp_rowent,
                      &f->keys0, &f->keys1, &f->tk0, &f->tk1, &f->vals0, &f->vals1, &f->sort.hist,
                      &f->sort.status, &f->sort.counters, &f->sort.part_hist, &f->sort.bases,
                      &f->sort.scan_sums, &f->sort.scan_total, &f->ranges, &f->grad2d, &f->jac,
                      &f->pvis, &f->pkeys, &f->ph};
    for (DevBuf* b : bufs) fn(*b);
}

void release_frame_buffers(cds_frame* f) {
    cds_ctx* c = f->ctx;
    for_each_frame_buffer(f, [c](DevBuf& b) { release(c, b); });
    f->valid = false;
}

int64_t frame_held_bytes(cds_frame* f) {
    int64_t held = 0;
    for_each_frame_buffer(f, [&held](DevBuf& b) { held += b.p ? (int64_t)b.bytes : 0; });
    return held;
}

#define CDS_HIP(expr, what)                          \
    do {                                             \
        hipError_t _e = (expr);                      \
        if (_e != hipSuccess) return hip_fail(_e, what); \
    } while (0)
#define CDS_TRY(expr)                   \
    do {                                \
        cds_status _s = (expr);         \
        if (_s != CDS_OK) return _s;    \
    } while (0)

int tile_bits_for(int64_t ntiles) {
    int bits = 0;
    while (bits < 32 && (int64_t(1) << bits) < ntiles) ++bits;
    return bits;
}

/*
 * Sort variants.  Every variant yields the same sorted (tile | depth, index)
 * list and tile ranges.
 *  1: the 64-bit keys are generated per (Gaussian, tile) in index order and
 *     radix-sorted on all their digits.
 *  2: the visible splats are compacted (index order kept) and their 32 depth
 *     bits -- shared by all keys of a splat -- are sorted once per splat
 *     (four LSD passes over n_vis, stable, ties by index); keys are generated
 *     in that order, exactly the sequence the depth passes would have
 *     produced, and only the tile-digit passes run over the keys, as 32-bit
 *     tile ids.  Ranges and the tile-digit histograms come from the
 *     rectangles (per-tile counts), so the last pass writes only the values.
 *  3: a per-splat depth sort as in 2 (over all N), then the tile-order pass as
 *     a counting sort on the whole tile id fused with duplication (binning).
 *  0: 2 (the fastest at every size measured so far).
 * Stage events: start, preprocess, key count read back, depth order, keys
 * generated, tile sort, ranges, blend (see cds_stage_times).
 */
cds_status render_forward_impl(cds_ctx* ctx, cds_frame* f, const cds_scene* scene, const cds_camera* cam,
                               int blend_variant, int sort_variant, SortAlgo algo, float* out_rgb, float* out_T,
                               uint32_t* out_ncontrib, float* out_invdepth, hipStream_t stream) {
    const int64_t n = scene->n;
    f->timed_backward = false;
    CDS_TRY(f->record(kEvStart, stream));
    const ProjParams P = make_proj(scene, cam);
    const int64_t ntiles = (int64_t)P.tiles_x * P.tiles_y;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    const int tile_bits = tile_bits_for(ntiles);
    const int tile_passes = (tile_bits + 7) / 8;
    const bool can_bin = bin_supported(P.tiles_x, P.tiles_y);
    // default: row-wise placement where the grid allows it, else radix-sorted tile digits
    if (sort_variant == 0) sort_variant = row_place_supported(P.tiles_x, P.tiles_y) ? 4 : 2;
    if (sort_variant == 3 && !can_bin)
        return fail(CDS_ERR_INVALID_ARG, "tile binning needs at most 512 tiles per row");
    if (sort_variant == 4 && !row_place_supported(P.tiles_x, P.tiles_y))
        return fail(CDS_ERR_INVALID_ARG, "row-wise tile placement needs at most 4096 tiles per axis");
    // variants 2 and 4 both start from the compacted visible splats in depth order
    const bool compact = sort_variant == 2 || sort_variant == 4;
    const bool rowplace = sort_variant == 4;
    const bool binned = sort_variant == 3;

    CDS_TRY(ensure(ctx, f->mean2d, sizeof(float2) * nn, 1.1));
    CDS_TRY(ensure(ctx, f->conic, sizeof(float4) * nn, 1.1));
    CDS_TRY(ensure(ctx, f->rgb, sizeof(float4) * nn, 1.1));
    CDS_TRY(ensure(ctx, f->depth, sizeof(uint32_t) * nn, 1.1));
    CDS_TRY(ensure(ctx, f->radius, sizeof(int32_t) * nn, 1.1));
    CDS_TRY(ensure(ctx, f->rect, sizeof(uint2) * nn, 1.1));
    CDS_TRY(ensure(ctx, f->touched, sizeof(uint32_t) * nn, 1.1));
    CDS_TRY(ensure(ctx, f->clampf, nn, 1.1));
    CDS_TRY(ensure(ctx, f->total, 256));
    CDS_TRY(ensure(ctx, f->ranges, sizeof(uint2) * (size_t)ntiles, 1.1));
    if (!binned) {
        CDS_TRY(ensure(ctx, f->offsets, sizeof(uint32_t) * nn, 1.1));
        CDS_TRY(ensure(ctx, f->blocksums, sizeof(uint64_t) * scan_block_sums_size(n), 1.1));
    }
    if (compact) {
        CDS_TRY(ensure(ctx, f->tdiff, sizeof(int) * kTileDiffMaxReps * (size_t)(ntiles + 1), 1.1));
        CDS_TRY(ensure(ctx, f->thist, sizeof(uint32_t) * 4 * 256));
        CDS_TRY(ensure(ctx, f->dkeyc, sizeof(uint32_t) * nn, 1.1));
        CDS_TRY(ensure(ctx, f->recc, sizeof(uint4) * nn, 1.1));
        CDS_TRY(ensure(ctx, f->recv, sizeof(uint4) * nn, 1.1));
        CDS_TRY(ensure(ctx, f->vsums, sizeof(uint64_t) * compact_sums_size(n), 1.1));
        CDS_TRY(ensure(ctx, f->ksums, sizeof(uint64_t) * compact_sums_size(n), 1.1));
        if (rowplace) CDS_TRY(ensure(ctx, f->hsums, sizeof(uint64_t) * compact_sums_size(n), 1.1));
    }
    if (compact || binned) {
        CDS_TRY(ensure(ctx, f->order0, sizeof(uint32_t) * nn, 1.1));
        CDS_TRY(ensure(ctx, f->order1, sizeof(uint32_t) * nn, 1.1));
        CDS_TRY(ensure(ctx, f->dkey0, sizeof(uint32_t) * nn, 1.1));
        CDS_TRY(ensure(ctx, f->dkey1, sizeof(uint32_t) * nn, 1.1));
        CDS_TRY(ensure_sort_workspace(ctx, f->sort_d, n, 4));
    }
    BinPlan bp;
    if (binned) {
        bp = bin_plan(n, P.tiles_x, P.tiles_y);
        CDS_TRY(ensure(ctx, f->vrect, sizeof(uint2) * nn, 1.1));
        CDS_TRY(ensure(ctx, f->binM, sizeof(uint32_t) * (size_t)(bp.chunks * bp.ntiles), 1.1));
        CDS_TRY(ensure(ctx, f->binE, sizeof(uint32_t) * (size_t)(bp.chunks * bp.ntiles), 1.1));
        CDS_TRY(ensure(ctx, f->binP, sizeof(uint32_t) * (size_t)(bp.groups * bp.ntiles), 1.1));
        CDS_TRY(ensure(ctx, f->tsum, sizeof(uint32_t) * (size_t)ntiles, 1.1));
    }

    SplatBuffers sb;
    sb.mean2d = (float2*)f->mean2d.p;
    sb.conic_opacity = (float4*)f->conic.p;
    sb.rgb = (float4*)f->rgb.p;
    sb.depth_bits = (uint32_t*)f->depth.p;
    sb.radius = (int32_t*)f->radius.p;
    sb.rect = (uint2*)f->rect.p;
    sb.touched = (uint32_t*)f->touched.p;
    sb.clamp_flags = (uint8_t*)f->clampf.p;
    // a render kept for the backward pass stores the colour's direction
    // derivative, which the backward then reads instead of the SH coefficients
    f->jac_valid = false;
    if (f->keep_jac && scene->sh_degree > 0) {
        CDS_TRY(ensure(ctx, f->jac, sizeof(float) * 9 * nn, 1.1));
        sb.jac = (float*)f->jac.p;
    }
    SortWorkspace wd = (compact || binned) ? sort_ws(ctx, f->sort_d) : SortWorkspace{};
    PreCounts pc;
    if (compact) {
        // the preprocess also counts the visible splats per workgroup (the
        // compaction's scan input) and clears the depth histograms and the
        // depth sort's look-back status and id counters
        pc.group = compact_tile_groups();
        pc.stride = compact_tiles(n);
        const size_t nblk = (size_t)std::max<int64_t>(pc.stride * pc.group, 1);
        CDS_TRY(ensure(ctx, f->pvis, sizeof(uint64_t) * nblk, 1.1));
        CDS_TRY(ensure(ctx, f->pkeys, sizeof(uint64_t) * nblk, 1.1));
        if (rowplace) CDS_TRY(ensure(ctx, f->ph, sizeof(uint64_t) * nblk, 1.1));
        pc.vis = (uint64_t*)f->pvis.p;
        pc.keys = (uint64_t*)f->pkeys.p;
        pc.h = rowplace ? (uint64_t*)f->ph.p : nullptr;
        pc.clear[0].p = wd.hist;
        pc.clear[0].n = 4 * 256 * kDepthHistReps;
        wd.hist_reps = kDepthHistReps;  // as the compaction fills them
        wd.hist_rep_stride = 4 * 256;
        if (n > 0 && sort_uses_onesweep(n, algo)) sort_prepare_spans(wd, n, 4, 4, pc.clear + 1);
        CDS_HIP(launch_preprocess_counted(P, make_scene(scene), sb, pc, stream), "preprocess kernel");
    } else {
        CDS_HIP(launch_preprocess(P, make_scene(scene), sb, stream), "preprocess kernel");
    }
    f->jac_valid = sb.jac != nullptr;
    CDS_TRY(f->record(kEvPreprocess, stream));

    uint64_t* d_total = (uint64_t*)f->total.p;  // [0] = n_vis (variant 2), [1] = K
    // When the render returns early (an allocation failing after the side
    // stream was forked), the render stream still waits for the side stream's
    // work, so buffers freed after the error are no longer in use by it.
    struct JoinOnExit {
        hipStream_t stream;
        hipEvent_t join;
        bool armed;
        ~JoinOnExit() {
            if (armed) (void)hipStreamWaitEvent(stream, join, 0);
        }
    } side_join{stream, nullptr, false};
    const uint32_t* order = nullptr;
    if (compact) {
        // visible splats compacted in index order, with the depth histograms; n_vis and K
        // (row-wise placement: also the sum of the rectangle heights, d_total[3]) from the
        // preprocess's per-workgroup counts
        CDS_TRY(f->side_stream());  // its events too: f->copied is recorded after the compaction
        CDS_HIP(launch_compact_counted(n, pc, sb.touched, sb.rect, sb.depth_bits, (uint64_t*)f->vsums.p,
                                       (uint64_t*)f->ksums.p, rowplace ? (uint64_t*)f->hsums.p : nullptr, d_total,
                                       rowplace ? d_total + 3 : nullptr, (uint32_t*)f->dkeyc.p, (uint4*)f->recc.p,
                                       wd.hist, stream, P.tiles_x, ctx->host_pinned_dev),
                "visible compaction");
    } else if (binned) {
        // depth order of all N Gaussians: 4 passes, result in (dkey1, order1)
        if (n > 0) {
            if (sort_uses_onesweep(n, algo)) {
                CDS_HIP(launch_sort_prepare(wd, n, 4, true, stream), "depth sort prepare");
                CDS_HIP(launch_sort_histogram(sb.depth_bits, n, 4, 0, wd.hist, stream), "depth sort histogram");
            }
            CDS_HIP(launch_sort_passes(sb.depth_bits, nullptr, (uint32_t*)f->dkey0.p, (uint32_t*)f->order0.p,
                                       (uint32_t*)f->dkey1.p, (uint32_t*)f->order1.p, n, 4, 0, wd, algo, stream),
                    "depth sort");
            order = (const uint32_t*)f->order1.p;
        }
        CDS_HIP(launch_bin_gather(n, order, sb.touched, sb.rect, (uint2*)f->vrect.p, stream), "bin gather");
        CDS_HIP(launch_bin_count(bp, n, (const uint2*)f->vrect.p, (uint32_t*)f->binM.p, stream), "bin count");
        CDS_HIP(launch_bin_scan(bp, (const uint32_t*)f->binM.p, (uint32_t*)f->binE.p, (uint32_t*)f->binP.p,
                                (uint32_t*)f->tsum.p, (uint2*)f->ranges.p, d_total + 1, stream),
                "bin scan");
    } else {
        CDS_HIP(launch_exclusive_scan(sb.touched, nullptr, (uint32_t*)f->offsets.p, n, (uint64_t*)f->blocksums.p,
                                      d_total + 1, stream),
                "scan kernels");
    }
    // the compacting path's scan wrote the counts into the pinned host words
    // itself (the host waits for f->copied, recorded after the compaction
    // below); the others copy them
    if (!compact)
        CDS_HIP(hipMemcpyAsync(ctx->host_pinned, d_total, 4 * sizeof(uint64_t), hipMemcpyDeviceToHost, stream),
                "hipMemcpyAsync(key count)");
    CDS_TRY(f->record(kEvCount, stream));
    if (compact) {
        // Enqueued before the host waits for the counts, so the device is not idle
        // meanwhile: these kernels are sized for all n Gaussians and read the
        // number of visible splats (d_total[0]) on the device.
        side_join.join = f->join;
        // ranges and tile-digit histograms from the records (their order does not
        // matter), on the side stream while the depth sort runs; one event marks
        // both the records complete (the fork) and the counts in the host words
        CDS_HIP(hipEventRecord(f->copied, stream), "hipEventRecord(copied)");
        CDS_HIP(hipStreamWaitEvent(f->side, f->copied, 0), "hipStreamWaitEvent(fork)");
        CDS_HIP(launch_tile_counts(n, nullptr, nullptr, P.tiles_x, ntiles, (int*)f->tdiff.p, (uint2*)f->ranges.p,
                                   (uint32_t*)f->thist.p, digit_plan(tile_passes, 0, tile_bits), nullptr,
                                   kTileCountBlocks, f->side, nullptr, 0, (const uint4*)f->recc.p, d_total,
                                   kTileDiffMaxReps),
                "tile counts");
        CDS_HIP(hipEventRecord(f->join, f->side), "hipEventRecord(join)");
        side_join.armed = true;
        if (n > 0) {
            // depth sort of the compacted keys (values: compacted positions); the
            // last pass writes the records in depth order (recv) instead
            CDS_HIP(launch_sort_passes((const uint32_t*)f->dkeyc.p, nullptr, (uint32_t*)f->dkey0.p,
                                       (uint32_t*)f->order0.p, (uint32_t*)f->dkey1.p, (uint32_t*)f->order1.p, n, 4,
                                       0, wd, algo, stream, 32, false, nullptr, value_bits_for(n - 1), nullptr,
                                       (const uint4*)f->recc.p, (uint4*)f->recv.p, d_total),
                    "depth sort");
        }
        CDS_HIP(hipEventSynchronize(f->copied), "hipEventSynchronize(key count)");
    } else {
        CDS_HIP(hipStreamSynchronize(stream), "hipStreamSynchronize(key count)");
    }
    const int64_t nvis = compact ? (int64_t)ctx->host_pinned[0] : n;
    const uint64_t K = ctx->host_pinned[1];
    if (K > (uint64_t)kSortMaxCount)
        return fail(CDS_ERR_CAPACITY, "render needs " + std::to_string(K) +
                                          " tile keys; the sorted list supports at most 2^30-1");
    const size_t kk = (size_t)(K > 0 ? K : 1);
    CDS_TRY(ensure(ctx, f->vals0, sizeof(uint32_t) * kk, 1.25));
    f->n = n;
    f->n_vis = nvis;
    f->row_entries = rowplace ? (int64_t)ctx->host_pinned[3] : 0;
    f->K = (int64_t)K;
    f->width = cam->width;
    f->height = cam->height;
    f->tiles_x = P.tiles_x;
    f->tiles_y = P.tiles_y;
    f->sort_variant = sort_variant;

    if (rowplace) {
        // tile lists by interval placement over tile rows, then tile columns
        const uint64_t sum_h = ctx->host_pinned[3];
        const RowPlaceSizes rs = row_place_sizes(nvis, sum_h, P.tiles_x, P.tiles_y);
        CDS_TRY(ensure(ctx, f->rp_ha, sizeof(uint32_t) * (size_t)rs.ha_words, 1.25));
        CDS_TRY(ensure(ctx, f->rp_hb, sizeof(uint32_t) * (size_t)std::max<int64_t>(rs.hb_words, 1), 1.25));
        CDS_TRY(ensure(ctx, f->rp_small, sizeof(uint32_t) * (size_t)rs.small_words, 1.25));
        CDS_TRY(ensure(ctx, f->rp_rowent, sizeof(uint2) * (size_t)std::max<uint64_t>(sum_h, 1), 1.25));
        side_join.armed = false;
        CDS_HIP(hipStreamWaitEvent(stream, f->join, 0), "hipStreamWaitEvent(join)");
        // events: depth order done; row lists (kEvKeys); column counts and starts
        // (kEvSortFirst); tile lists (kEvSort)
        CDS_TRY(f->record(kEvDepth, stream));
        RowPlaceArgs ra;
        ra.rec = (const uint4*)f->recv.p;
        ra.count_dev = d_total;
        ra.n_records_max = nvis;
        ra.tiles_x = P.tiles_x;
        ra.tiles_y = P.tiles_y;
        ra.sum_h = sum_h;
        ra.K = K;
        ra.ranges = (const uint2*)f->ranges.p;
        ra.ranges_ready = nullptr;  // the stream waited for the tile counts above
        ra.ha = (uint32_t*)f->rp_ha.p;
        ra.hb = (uint32_t*)f->rp_hb.p;
        ra.small = (uint32_t*)f->rp_small.p;
        ra.rowent = (uint2*)f->rp_rowent.p;
        ra.values = (uint32_t*)f->vals0.p;
        ra.err = ctx->d_err;
        CDS_HIP(launch_row_place(ra, stream, f->event(kEvKeys), f->event(kEvSortFirst)), "row-wise tile placement");
        if (K == 0 || nvis == 0 || sum_h == 0) {  // nothing was placed
            CDS_TRY(f->record(kEvKeys, stream));
            CDS_TRY(f->record(kEvSortFirst, stream));
        }
        CDS_TRY(f->record(kEvSort, stream));
        CDS_TRY(f->record(kEvRanges, stream));
        f->res_values = (const uint32_t*)f->vals0.p;
        f->res_tiles = nullptr;
        f->res_tile_stride = 1;
        f->res_keys = nullptr;
        f->passes = 4;
    } else if (binned) {
        CDS_TRY(f->record(kEvDepth, stream));
        CDS_HIP(launch_bin_place(bp, n, order, (const uint2*)f->vrect.p, (const uint32_t*)f->binM.p,
                                 (const uint32_t*)f->binE.p, K, (uint32_t*)f->vals0.p, ctx->d_err, stream),
                "bin place");
        CDS_TRY(f->record(kEvKeys, stream));
        CDS_TRY(f->record(kEvSortFirst, stream));
        CDS_TRY(f->record(kEvSort, stream));
        CDS_TRY(f->record(kEvRanges, stream));
        f->res_values = (const uint32_t*)f->vals0.p;
        f->res_tiles = nullptr;
        f->res_tile_stride = 1;
        f->res_keys = nullptr;
        f->passes = 4;
    } else {
        const uint4* recv = (const uint4*)f->recv.p;
        if (compact && nvis > 0) {
            // key offsets of the records in depth order and the owner of every 1024th key
            CDS_TRY(ensure(ctx, f->kowner, sizeof(uint32_t) * (size_t)(K / kKeyGenChunk + 1), 1.25));
            CDS_HIP(launch_exclusive_scan(nullptr, nullptr, (uint32_t*)f->offsets.p, n, (uint64_t*)f->blocksums.p,
                                          d_total + 2, stream, recv, (uint32_t*)f->kowner.p, d_total),
                    "offset scan");
        }
        if (compact) {
            side_join.armed = false;
            CDS_HIP(hipStreamWaitEvent(stream, f->join, 0), "hipStreamWaitEvent(join)");
        }
        CDS_TRY(f->record(kEvDepth, stream));
        const int passes = compact ? tile_passes : 4 + tile_passes;
        // variant 2 with onesweep passes: the first tile pass generates the keys
        const bool fused = compact && sort_uses_onesweep((int64_t)K, algo) && passes > 0;
        CDS_TRY(ensure(ctx, f->vals1, sizeof(uint32_t) * kk, 1.25));
        if (compact) {
            // generated keys packed with their values need no tile-id buffers
            if (!fused || sort_gen_needs_key_buffers(passes, tile_bits, value_bits_for(n - 1))) {
                CDS_TRY(ensure(ctx, f->tk0, sizeof(uint32_t) * kk, 1.25));
                CDS_TRY(ensure(ctx, f->tk1, sizeof(uint32_t) * kk, 1.25));
            }
        } else {
            CDS_TRY(ensure(ctx, f->keys0, sizeof(uint64_t) * kk, 1.25));
            CDS_TRY(ensure(ctx, f->keys1, sizeof(uint64_t) * kk, 1.25));
        }
        CDS_TRY(ensure_sort_workspace(ctx, f->sort, (int64_t)K, passes > 0 ? passes : 1));
        SortWorkspace ws = sort_ws(ctx, f->sort);
        const bool onesweep = sort_uses_onesweep((int64_t)K, algo) && passes > 0;
        KeyGen gen;
        gen.off = (const uint32_t*)f->offsets.p;
        gen.rec = recv;
        gen.owner = (const uint32_t*)f->kowner.p;
        gen.n = nvis;
        if (K > 0) {
            if (compact) {
                // the onesweep passes take the tile-digit histograms made from the rectangles
                if (onesweep) CDS_HIP(launch_sort_prepare(ws, (int64_t)K, passes, false, stream, 4), "sort prepare");
                ws.hist = (uint32_t*)f->thist.p;
                if (!fused)
                    CDS_HIP(launch_duplicate(nvis, nullptr, (const uint32_t*)f->offsets.p, nullptr, nullptr,
                                             sb.depth_bits, P.tiles_x, nullptr, (uint32_t*)f->tk0.p,
                                             (uint32_t*)f->vals0.p, stream, nullptr, 0, recv),
                            "duplicate kernel");
            } else {
                CDS_HIP(launch_duplicate(n, nullptr, (const uint32_t*)f->offsets.p, sb.touched, sb.rect,
                                         sb.depth_bits, P.tiles_x, (uint64_t*)f->keys0.p, nullptr,
                                         (uint32_t*)f->vals0.p, stream),
                        "duplicate kernel");
                if (onesweep) {
                    CDS_HIP(launch_sort_prepare(ws, (int64_t)K, passes, true, stream), "sort prepare");
                    CDS_HIP(launch_sort_histogram((const uint64_t*)f->keys0.p, (int64_t)K, passes, 0, ws.hist,
                                                  stream, 32 + tile_bits),
                            "key histogram");
                }
            }
        }
        CDS_TRY(f->record(kEvKeys, stream));
        const bool odd = (passes & 1) != 0;
        if (compact) {
            if (K > 0)
                // the ranges come from the tile counts and the blend needs only the
                // values, so the last pass does not write the tile ids
                CDS_HIP(launch_sort_passes((const uint32_t*)f->tk0.p, (const uint32_t*)f->vals0.p,
                                           (uint32_t*)f->tk1.p, (uint32_t*)f->vals1.p, (uint32_t*)f->tk0.p,
                                           (uint32_t*)f->vals0.p, (int64_t)K, passes, 0, ws, algo, stream, tile_bits,
                                           false, fused ? &gen : nullptr, value_bits_for(n - 1),
                                           f->event(kEvSortFirst)),
                        "tile sort");
            f->res_tiles = passes > 0 ? nullptr : (const uint32_t*)f->tk0.p;
            f->res_tile_stride = 1;
            f->res_keys = nullptr;
        } else {
            if (K > 0)
                CDS_HIP(launch_sort_passes((const uint64_t*)f->keys0.p, (const uint32_t*)f->vals0.p,
                                           (uint64_t*)f->keys1.p, (uint32_t*)f->vals1.p, (uint64_t*)f->keys0.p,
                                           (uint32_t*)f->vals0.p, (int64_t)K, passes, 0, ws, algo, stream,
                                           32 + tile_bits, true, f->event(kEvSortFirst)),
                        "key sort");
            f->res_keys = (const uint64_t*)(odd ? f->keys1.p : f->keys0.p);
            f->res_tiles = reinterpret_cast<const uint32_t*>(f->res_keys) + 1;  // high words
            f->res_tile_stride = 2;
        }
        f->res_values = (const uint32_t*)(odd ? f->vals1.p : f->vals0.p);
        if (K == 0 || passes == 0) CDS_TRY(f->record(kEvSortFirst, stream));  // no pass ran
        CDS_TRY(f->record(kEvSort, stream));
        f->passes = compact ? 4 + tile_passes : passes;
        if (!compact)  // variant 2 has its ranges from the tile counts
            CDS_HIP(launch_ranges(f->res_tiles, f->res_tile_stride, (int64_t)K, (uint2*)f->ranges.p, ntiles,
                                  stream),
                    "ranges kernel");
        CDS_TRY(f->record(kEvRanges, stream));
    }

    BlendArgs ba;
    ba.ranges = (const uint2*)f->ranges.p;
    ba.point_list = f->res_values;
    ba.mean2d = sb.mean2d;
    ba.conic_opacity = sb.conic_opacity;
    ba.rgb = sb.rgb;
    ba.width = cam->width;
    ba.height = cam->height;
    ba.tiles_x = P.tiles_x;
    ba.tiles_y = P.tiles_y;
    for (int k = 0; k < 3; ++k) ba.bg[k] = cam->bg[k];
    ba.out_rgb = out_rgb;
    ba.out_T = out_T;
    ba.out_ncontrib = out_ncontrib;
    ba.depth_bits = sb.depth_bits;
    ba.out_invdepth = out_invdepth;
    ba.counter = reinterpret_cast<uint32_t*>(d_total + 8);  // a free word of the frame's totals
    ba.n = n;
    ba.err = ctx->d_err;
    CDS_HIP(launch_blend(ba, blend_variant, stream), "blend kernel");
    CDS_TRY(f->record(kEvBlend, stream));
    f->valid = true;
    return CDS_OK;
}

// Build the 64-bit sorted keys of a render that did not sort them (for inspection).
cds_status frame_build_keys(cds_frame* f) {
    if (f->res_keys || f->K == 0) return CDS_OK;
    CDS_TRY(ensure(f->ctx, f->keys0, sizeof(uint64_t) * (size_t)f->K, 1.25));
    if (f->res_tiles)
        CDS_HIP(launch_make_keys(f->res_tiles, f->res_values, (const uint32_t*)f->depth.p, f->K,
                                 (uint64_t*)f->keys0.p, nullptr),
                "make keys");
    else
        CDS_HIP(launch_keys_from_ranges((const uint2*)f->ranges.p, (int64_t)f->tiles_x * f->tiles_y, f->res_values,
                                        (const uint32_t*)f->depth.p, (uint64_t*)f->keys0.p, nullptr),
                "keys from ranges");
    CDS_HIP(hipStreamSynchronize(nullptr), "hipStreamSynchronize");
    f->res_keys = (const uint64_t*)f->keys0.p;
    return CDS_OK;
}

cds_status render_backward_impl(cds_ctx* ctx, cds_frame* f, const cds_scene* scene, const cds_camera* cam,
                                const float* out_T, const uint32_t* out_ncontrib, const float* dL_drgb,
                                const float* dL_dinvdepth, const cds_scene_grad* g, hipStream_t stream) {
    const int64_t n = scene->n;
    if (n == 0) return CDS_OK;
    const ProjParams P = make_proj(scene, cam);
    CDS_TRY(ensure(ctx, f->grad2d, sizeof(float) * kGrad2d * (size_t)n, 1.1));
    CDS_TRY(f->record(kEvBwdStart, stream));
    CDS_HIP(launch_fill_u32((uint32_t*)f->grad2d.p, kGrad2d * n, 0u, stream), "fill");
    BlendBwdArgs b;
    b.ranges = (const uint2*)f->ranges.p;
    b.point_list = f->res_values;
    b.mean2d = (const float2*)f->mean2d.p;
    b.conic_opacity = (const float4*)f->conic.p;
    b.rgb = (const float4*)f->rgb.p;
    b.width = f->width;
    b.height = f->height;
    b.tiles_x = f->tiles_x;
    b.tiles_y = f->tiles_y;
    for (int k = 0; k < 3; ++k) b.bg[k] = cam->bg[k];
    b.final_T = out_T;
    b.ncontrib = out_ncontrib;
    b.dL_drgb = dL_drgb;
    b.depth_bits = (const uint32_t*)f->depth.p;
    b.dL_dinvdepth = dL_dinvdepth;
    b.n = n;
    b.grad2d = (float*)f->grad2d.p;
    b.err = ctx->d_err;
    CDS_HIP(launch_blend_backward(b, stream), "blend backward kernel");
    CDS_TRY(f->record(kEvBwdBlend, stream));
    PreBwdArgs pa;
    pa.radius = (const int32_t*)f->radius.p;
    pa.clamp_flags = (const uint8_t*)f->clampf.p;
    pa.grad2d = (const float*)f->grad2d.p;
    pa.jac = f->jac_valid ? (const float*)f->jac.p : nullptr;
    pa.g_means = g->means;
    pa.g_log_scales = g->log_scales;
    pa.g_quats = g->quats;
    pa.g_opacity_logits = g->opacity_logits;
    pa.g_sh = g->sh;
    CDS_HIP(launch_preprocess_backward(P, make_scene(scene), pa, stream), "preprocess backward kernel");
    CDS_TRY(f->record(kEvBwdPre, stream));
    f->timed_backward = f->timing;
    return CDS_OK;
}

}  // namespace cds

void cds_frame::release_all() {
    cds::release_frame_buffers(this);
    cds::release_frame_events(this);
}

cds_status cds_frame::side_stream() {
    hipError_t e;
    if (!side && (e = hipStreamCreateWithFlags(&side, hipStreamNonBlocking)) != hipSuccess)
        return cds::hip_fail(e, "hipStreamCreate(side)");
    if (!fork && (e = hipEventCreateWithFlags(&fork, hipEventDisableTiming)) != hipSuccess)
        return cds::hip_fail(e, "hipEventCreate(fork)");
    if (!join && (e = hipEventCreateWithFlags(&join, hipEventDisableTiming)) != hipSuccess)
        return cds::hip_fail(e, "hipEventCreate(join)");
    if (!copied && (e = hipEventCreateWithFlags(&copied, hipEventDisableTiming)) != hipSuccess)
        return cds::hip_fail(e, "hipEventCreate(copied)");
    return CDS_OK;
}

hipEvent_t cds_frame::event(int i) {
    if (!timing) return nullptr;
    if (!ev[i] && hipEventCreate(&ev[i]) != hipSuccess) return nullptr;
    return ev[i];
}

cds_status cds_frame::record(int i, hipStream_t s) {
    if (!timing) return CDS_OK;
    hipError_t e;
    if (!ev[i] && (e = hipEventCreate(&ev[i])) != hipSuccess) return cds::hip_fail(e, "hipEventCreate");
    if ((e = hipEventRecord(ev[i], s)) != hipSuccess) return cds::hip_fail(e, "hipEventRecord");
    return CDS_OK;
}

extern "C" cds_status cds_frame_stage_times(cds_frame* f, cds_stage_times* out) {
    using namespace cds;
    if (!f || !out) return cds::fail(CDS_ERR_INVALID_ARG, "NULL argument");
    if (!f->valid || !f->timing) return cds::fail(CDS_ERR_INVALID_ARG, "frame has no timed render");
    hipError_t e = hipSetDevice(f->ctx->device);
    if (e != hipSuccess) return cds::hip_fail(e, "hipSetDevice");
    const int last = f->timed_backward ? kEvBwdPre : kEvBlend;
    if ((e = hipEventSynchronize(f->ev[last])) != hipSuccess) return cds::hip_fail(e, "hipEventSynchronize");
    auto span = [&](int a, int b, float* out) -> hipError_t { return hipEventElapsedTime(out, f->ev[a], f->ev[b]); };
    std::memset(out, 0, sizeof(*out));
    if ((e = span(kEvStart, kEvPreprocess, &out->preprocess_ms)) != hipSuccess ||
        (e = span(kEvPreprocess, kEvCount, &out->scan_ms)) != hipSuccess ||
        (e = span(kEvCount, kEvDepth, &out->depth_order_ms)) != hipSuccess ||
        (e = span(kEvDepth, kEvKeys, &out->duplicate_ms)) != hipSuccess ||
        (e = span(kEvKeys, kEvSort, &out->sort_ms)) != hipSuccess ||
        (e = span(kEvKeys, kEvSortFirst, &out->sort_first_pass_ms)) != hipSuccess ||
        (e = span(kEvSort, kEvRanges, &out->ranges_ms)) != hipSuccess ||
        (e = span(kEvRanges, kEvBlend, &out->blend_ms)) != hipSuccess)
        return cds::hip_fail(e, "hipEventElapsedTime");
    if (f->timed_backward &&
        ((e = span(kEvBwdStart, kEvBwdBlend, &out->blend_backward_ms)) != hipSuccess ||
         (e = span(kEvBwdBlend, kEvBwdPre, &out->preprocess_backward_ms)) != hipSuccess))
        return cds::hip_fail(e, "hipEventElapsedTime");
    return CDS_OK;
}
