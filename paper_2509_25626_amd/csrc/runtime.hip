// Host runtime behind the C ABI declared in include/cdnasplat.h: contexts,
// frames (grow-only device buffers reused across renders), argument
// validation, and the stream-ordered launch sequence of a render.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "cdnasplat.h"
#include "internal.h"
#include "runtime_internal.h"

using namespace cds;

namespace cds {

thread_local std::string g_last_error;

cds_status fail(cds_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

cds_status hip_fail(hipError_t e, const char* what) {
    return fail(CDS_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void* ctx_alloc(cds_ctx* c, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    if (c->has_alloc) return c->alloc.alloc(bytes, c->alloc.user);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void ctx_free(cds_ctx* c, void* p) {
    if (!p) return;
    if (c->has_alloc) c->alloc.free(p, c->alloc.user);
    else (void)hipFree(p);
}

cds_status ensure(cds_ctx* c, DevBuf& b, size_t bytes, double grow) {
    if (bytes == 0) bytes = 256;
    if (b.p && bytes <= b.bytes) return CDS_OK;
    if (b.p) {
        ctx_free(c, b.p);
        b.p = nullptr;
        b.bytes = 0;
    }
    size_t want = (size_t)((double)bytes * grow);
    if (want < bytes) want = bytes;
    want = (want + 255) & ~size_t(255);
    void* p = ctx_alloc(c, want);
    if (!p) return fail(CDS_ERR_OOM, "device allocation of " + std::to_string(want) + " bytes failed");
    b.p = p;
    b.bytes = want;
    return CDS_OK;
}

void release(cds_ctx* c, DevBuf& b) {
    ctx_free(c, b.p);
    b.p = nullptr;
    b.bytes = 0;
}

cds_status validate_scene(const cds_scene* s) {
    if (!s) return fail(CDS_ERR_INVALID_ARG, "scene is NULL");
    if (s->n < 0) return fail(CDS_ERR_INVALID_ARG, "scene n < 0");
    if (s->n > (int64_t)0x7FFFFFFF) return fail(CDS_ERR_CAPACITY, "more than 2^31-1 Gaussians");
    if (s->sh_degree < 0 || s->sh_degree > CDS_MAX_SH_DEGREE)
        return fail(CDS_ERR_INVALID_ARG, "sh_degree must be in [0, 3]");
    if (s->n > 0 && (!s->means || !s->log_scales || !s->quats || !s->opacity_logits || !s->sh))
        return fail(CDS_ERR_INVALID_ARG, "scene array pointer is NULL");
    return CDS_OK;
}

cds_status validate_camera(const cds_camera* c) {
    if (!c) return fail(CDS_ERR_INVALID_ARG, "camera is NULL");
    if (c->width <= 0 || c->height <= 0) return fail(CDS_ERR_INVALID_ARG, "image size must be positive");
    if ((int64_t)((c->width + CDS_TILE - 1) / CDS_TILE) > 65535 ||
        (int64_t)((c->height + CDS_TILE - 1) / CDS_TILE) > 65535)
        return fail(CDS_ERR_INVALID_ARG, "image too large (more than 65535 tiles per axis)");
    if (!(c->near_plane > 0.0f)) return fail(CDS_ERR_INVALID_ARG, "near_plane must be > 0");
    if (!(c->fx > 0.0f) || !(c->fy > 0.0f)) return fail(CDS_ERR_INVALID_ARG, "focal lengths must be > 0");
    for (int i = 0; i < 12; ++i)
        if (!std::isfinite(c->view[i])) return fail(CDS_ERR_INVALID_ARG, "view matrix not finite");
    if (!std::isfinite(c->cx) || !std::isfinite(c->cy))
        return fail(CDS_ERR_INVALID_ARG, "principal point not finite");
    return CDS_OK;
}

ProjParams make_proj(const cds_scene* s, const cds_camera* c) {
    ProjParams p;
    std::memset(&p, 0, sizeof(p));
    p.n = s->n;
    p.sh_degree = s->sh_degree;
    p.width = c->width;
    p.height = c->height;
    p.tiles_x = (c->width + CDS_TILE - 1) / CDS_TILE;
    p.tiles_y = (c->height + CDS_TILE - 1) / CDS_TILE;
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) p.R[3 * r + k] = c->view[4 * r + k];
        p.t[r] = c->view[4 * r + 3];
    }
    for (int k = 0; k < 3; ++k)
        p.campos[k] = -(p.R[k] * p.t[0] + p.R[3 + k] * p.t[1] + p.R[6 + k] * p.t[2]);
    p.fx = c->fx;
    p.fy = c->fy;
    p.cx = c->cx;
    p.cy = c->cy;
    p.near_plane = c->near_plane;
    p.limx = 1.3 * (0.5 * (double)c->width / p.fx);
    p.limy = 1.3 * (0.5 * (double)c->height / p.fy);
    return p;
}

SceneParams make_scene(const cds_scene* s) {
    SceneParams sp;
    sp.means = s->means;
    sp.log_scales = s->log_scales;
    sp.quats = s->quats;
    sp.opacity_logits = s->opacity_logits;
    sp.sh = s->sh;
    return sp;
}

cds_status ensure_sort_workspace(cds_ctx* ctx, SortState& s, int64_t count, int passes) {
    const int64_t parts = std::max<int64_t>(sort_partitions(count), 1);
    cds_status st;
    if ((st = ensure(ctx, s.hist, sizeof(uint32_t) * 256 * 8 * kDepthHistReps)) != CDS_OK) return st;
    if ((st = ensure(ctx, s.counters, sizeof(uint32_t) * 8)) != CDS_OK) return st;
    if ((st = ensure(ctx, s.status, sizeof(uint32_t) * 256 * (size_t)parts * passes, 1.25)) != CDS_OK) return st;
    if ((st = ensure(ctx, s.part_hist, sizeof(uint32_t) * 256 * (size_t)parts, 1.25)) != CDS_OK) return st;
    if ((st = ensure(ctx, s.bases, sizeof(uint32_t) * 256 * (size_t)parts, 1.25)) != CDS_OK) return st;
    if ((st = ensure(ctx, s.scan_sums, sizeof(uint64_t) * (size_t)scan_block_sums_size(256 * parts), 1.25)) !=
        CDS_OK)
        return st;
    if ((st = ensure(ctx, s.scan_total, 256)) != CDS_OK) return st;
    return CDS_OK;
}

SortWorkspace sort_ws(cds_ctx* ctx, SortState& s) {
    SortWorkspace ws;
    ws.hist = (uint32_t*)s.hist.p;
    ws.status = (uint32_t*)s.status.p;
    ws.counters = (uint32_t*)s.counters.p;
    ws.part_hist = (uint32_t*)s.part_hist.p;
    ws.bases = (uint32_t*)s.bases.p;
    ws.scan_sums = (uint64_t*)s.scan_sums.p;
    ws.scan_total = (uint64_t*)s.scan_total.p;
    ws.err = ctx->d_err;
    return ws;
}

SortAlgo sort_algo_from_flags(uint32_t flags) {
    if (flags & CDS_OPT_SORT_ONESWEEP) return SortAlgo::kOnesweep;
    if (flags & CDS_OPT_SORT_REDUCE_SCAN) return SortAlgo::kReduceScan;
    return SortAlgo::kAuto;
}

}  // namespace cds

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* cds_version(void) { return "cdnasplat 0.1.0 (gfx950)"; }

const char* cds_last_error(void) { return g_last_error.c_str(); }

cds_status cds_create(cds_ctx** out, int device, const cds_allocator* alloc) {
    if (!out) return fail(CDS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= count) return fail(CDS_ERR_INVALID_ARG, "no such device");
    if (alloc && (!alloc->alloc || !alloc->free))
        return fail(CDS_ERR_INVALID_ARG, "allocator needs both alloc and free");
    if ((e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    cds_ctx* c = new cds_ctx();
    c->device = device;
    c->has_alloc = alloc != nullptr;
    if (alloc) c->alloc = *alloc;
    // fine-grained (coherent) pinned words: kernels write the per-render
    // counts straight into them, visible to the host once the kernel is done
    if ((e = hipHostMalloc((void**)&c->host_pinned, 4096, hipHostMallocCoherent)) != hipSuccess) {
        delete c;
        return hip_fail(e, "hipHostMalloc");
    }
    if ((e = hipHostGetDevicePointer((void**)&c->host_pinned_dev, c->host_pinned, 0)) != hipSuccess) {
        (void)hipHostFree(c->host_pinned);
        delete c;
        return hip_fail(e, "hipHostGetDevicePointer");
    }
    // one allocation: the error word (256 B) and the loss partial sums (4 KiB)
    c->d_err = (uint32_t*)ctx_alloc(c, 256 + 4096);
    if (!c->d_err) {
        (void)hipHostFree(c->host_pinned);
        delete c;
        return fail(CDS_ERR_OOM, "device allocation failed");
    }
    if ((e = hipMemset(c->d_err, 0, 256)) != hipSuccess) {
        ctx_free(c, c->d_err);
        (void)hipHostFree(c->host_pinned);
        delete c;
        return hip_fail(e, "hipMemset");
    }
    c->d_partial = reinterpret_cast<float*>(reinterpret_cast<char*>(c->d_err) + 256);
    // the allocation-free sort's scratch array on this device (looked up once
    // per device; a failure is reported by that entry point only)
    (void)noalloc_init_device(device);
    c->scratch = new cds_frame();
    c->scratch->ctx = c;
    *out = c;
    return CDS_OK;
}

void cds_destroy(cds_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    if (c->scratch) {
        c->scratch->release_all();
        delete c->scratch;
    }
    ctx_free(c, c->d_err);
    (void)hipHostFree(c->host_pinned);
    delete c;
}

cds_status cds_frame_create(cds_ctx* ctx, cds_frame** out) {
    if (!ctx || !out) return fail(CDS_ERR_INVALID_ARG, "NULL argument");
    cds_frame* f = new cds_frame();
    f->ctx = ctx;
    *out = f;
    return CDS_OK;
}

void cds_frame_release(cds_frame* f) {
    if (!f) return;
    (void)hipSetDevice(f->ctx->device);
    f->release_all();
    delete f;
}

cds_status cds_render_forward_ex(cds_ctx* ctx, cds_frame* f, const cds_scene* scene, const cds_camera* cam,
                                 const cds_render_opts* opts, float* out_rgb, float* out_T,
                                 uint32_t* out_ncontrib, float* out_invdepth, void* stream_) {
    if (!ctx || !f) return fail(CDS_ERR_INVALID_ARG, "context or frame is NULL");
    if (f->ctx != ctx) return fail(CDS_ERR_INVALID_ARG, "frame belongs to another context");
    cds_status st;
    if ((st = validate_scene(scene)) != CDS_OK) return st;
    if ((st = validate_camera(cam)) != CDS_OK) return st;
    if (!out_rgb || !out_T || !out_ncontrib) return fail(CDS_ERR_INVALID_ARG, "output pointer is NULL");
    int variant = 0, sort_variant = 0;
    bool timing = false;
    SortAlgo algo = SortAlgo::kAuto;
    if (opts) {
        if (opts->flags &
            ~(CDS_OPT_STAGE_TIMING | CDS_OPT_SORT_ONESWEEP | CDS_OPT_SORT_REDUCE_SCAN | CDS_OPT_KEEP_FOR_BACKWARD))
            return fail(CDS_ERR_INVALID_ARG, "unknown option flags");
        if ((opts->flags & CDS_OPT_SORT_ONESWEEP) && (opts->flags & CDS_OPT_SORT_REDUCE_SCAN))
            return fail(CDS_ERR_INVALID_ARG, "choose one radix-sort pass algorithm");
        timing = (opts->flags & CDS_OPT_STAGE_TIMING) != 0;
        algo = sort_algo_from_flags(opts->flags);
        variant = opts->blend_variant;
        if (variant < 0 || variant > 5)
            return fail(CDS_ERR_INVALID_ARG, "blend_variant must be 0 to 5");
        if (opts->sort_variant < 0 || opts->sort_variant > 4)
            return fail(CDS_ERR_INVALID_ARG, "sort_variant must be 0 to 4");
        sort_variant = opts->sort_variant;
    }
    hipStream_t stream = (hipStream_t)stream_;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    f->valid = false;
    f->timing = timing;
    f->keep_jac = opts && (opts->flags & CDS_OPT_KEEP_FOR_BACKWARD) != 0;
    return render_forward_impl(ctx, f, scene, cam, variant, sort_variant, algo, out_rgb, out_T, out_ncontrib,
                               out_invdepth, stream);
}

cds_status cds_render_forward(cds_ctx* ctx, cds_frame* f, const cds_scene* scene, const cds_camera* cam,
                              const cds_render_opts* opts, float* out_rgb, float* out_T,
                              uint32_t* out_ncontrib, void* stream) {
    return cds_render_forward_ex(ctx, f, scene, cam, opts, out_rgb, out_T, out_ncontrib, nullptr, stream);
}

cds_status cds_render_backward_ex(cds_ctx* ctx, cds_frame* f, const cds_scene* scene, const cds_camera* cam,
                                  const float* out_T, const uint32_t* out_ncontrib, const float* dL_drgb,
                                  const float* dL_dinvdepth, const cds_scene_grad* g, void* stream_) {
    if (!ctx || !f || f->ctx != ctx) return fail(CDS_ERR_INVALID_ARG, "bad context or frame");
    cds_status st;
    if ((st = validate_scene(scene)) != CDS_OK) return st;
    if ((st = validate_camera(cam)) != CDS_OK) return st;
    if (!f->valid) return fail(CDS_ERR_INVALID_ARG, "frame holds no forward render");
    if (scene->n != f->n || cam->width != f->width || cam->height != f->height)
        return fail(CDS_ERR_INVALID_ARG, "scene/camera differ from the frame's forward render");
    if (!out_T || !out_ncontrib || !dL_drgb || !g) return fail(CDS_ERR_INVALID_ARG, "NULL pointer");
    if (scene->n > 0 && (!g->means || !g->log_scales || !g->quats || !g->opacity_logits || !g->sh))
        return fail(CDS_ERR_INVALID_ARG, "gradient pointer is NULL");
    hipStream_t stream = (hipStream_t)stream_;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    return render_backward_impl(ctx, f, scene, cam, out_T, out_ncontrib, dL_drgb, dL_dinvdepth, g, stream);
}

cds_status cds_render_backward(cds_ctx* ctx, cds_frame* f, const cds_scene* scene, const cds_camera* cam,
                               const float* out_T, const uint32_t* out_ncontrib, const float* dL_drgb,
                               const cds_scene_grad* g, void* stream) {
    return cds_render_backward_ex(ctx, f, scene, cam, out_T, out_ncontrib, dL_drgb, nullptr, g, stream);
}

cds_status cds_l1_loss_grad(cds_ctx* ctx, const float* rgb, const float* target, int64_t count,
                            float* dL_drgb, float* loss_out, void* stream) {
    if (!ctx || !rgb || !target || !dL_drgb || count < 0) return fail(CDS_ERR_INVALID_ARG, "bad argument");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    e = launch_l1_loss_grad(rgb, target, count, dL_drgb, loss_out, ctx->d_partial, (hipStream_t)stream);
    return e == hipSuccess ? CDS_OK : hip_fail(e, "l1 loss kernel");
}

cds_status cds_frame_get_info(cds_frame* f, cds_frame_info* o) {
    if (!f || !o) return fail(CDS_ERR_INVALID_ARG, "NULL argument");
    if (!f->valid) return fail(CDS_ERR_INVALID_ARG, "frame holds no forward render");
    hipError_t e = hipSetDevice(f->ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    cds_status st = frame_build_keys(f);
    if (st != CDS_OK) return st;
    std::memset(o, 0, sizeof(*o));
    o->n = f->n;
    o->num_keys = f->K;
    o->width = f->width;
    o->height = f->height;
    o->tiles_x = f->tiles_x;
    o->tiles_y = f->tiles_y;
    o->sort_passes = f->passes;
    o->num_visible = (int32_t)f->n_vis;
    o->mean2d = (const float*)f->mean2d.p;
    o->conic_opacity = (const float*)f->conic.p;
    o->rgb = (const float*)f->rgb.p;
    o->depth_bits = (const uint32_t*)f->depth.p;
    o->radius = (const int32_t*)f->radius.p;
    o->tile_rect = (const uint32_t*)f->rect.p;
    o->tiles_touched = (const uint32_t*)f->touched.p;
    o->offsets = (f->sort_variant == 3 || f->sort_variant == 4) ? nullptr : (const uint32_t*)f->offsets.p;
    o->keys = f->res_keys;
    o->values = f->res_values;
    o->ranges = (const uint32_t*)f->ranges.p;
    o->clamp_flags = (const uint8_t*)f->clampf.p;
    o->num_row_entries = f->row_entries;
    return CDS_OK;
}

cds_status cds_sort_pairs(cds_ctx* ctx, const uint64_t* keys_in, const uint32_t* values_in, int64_t count,
                          int32_t end_bit, uint64_t* keys_out, uint32_t* values_out, uint32_t flags,
                          void* stream_) {
    if (!ctx) return fail(CDS_ERR_INVALID_ARG, "context is NULL");
    if (flags & ~(CDS_OPT_SORT_ONESWEEP | CDS_OPT_SORT_REDUCE_SCAN) ||
        ((flags & CDS_OPT_SORT_ONESWEEP) && (flags & CDS_OPT_SORT_REDUCE_SCAN)))
        return fail(CDS_ERR_INVALID_ARG, "bad sort flags");
    const SortAlgo algo = sort_algo_from_flags(flags);
    if (count < 0 || end_bit < 1 || end_bit > 64) return fail(CDS_ERR_INVALID_ARG, "bad count or end_bit");
    if (count > kSortMaxCount) return fail(CDS_ERR_CAPACITY, "sort supports at most 2^30-1 pairs");
    if (count > 0 && (!keys_in || !values_in || !keys_out || !values_out))
        return fail(CDS_ERR_INVALID_ARG, "NULL array");
    if (count > 0 && ((const void*)keys_out == (const void*)keys_in ||
                      (const void*)values_out == (const void*)values_in))
        return fail(CDS_ERR_INVALID_ARG, "outputs may not alias inputs");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    if (count == 0) return CDS_OK;
    hipStream_t stream = (hipStream_t)stream_;
    const int passes = (end_bit + 7) / 8;
    cds_frame* s = ctx->scratch;
    cds_status st;
    if ((st = ensure(ctx, s->keys1, sizeof(uint64_t) * (size_t)count)) != CDS_OK) return st;
    if ((st = ensure(ctx, s->vals1, sizeof(uint32_t) * (size_t)count)) != CDS_OK) return st;
    if ((st = ensure_sort_workspace(ctx, s->sort, count, passes)) != CDS_OK) return st;
    // ping-pong so the last pass writes the caller's output buffers and the input is never written
    uint64_t* tmpk = (uint64_t*)s->keys1.p;
    uint32_t* tmpv = (uint32_t*)s->vals1.p;
    uint64_t *ka, *kb;
    uint32_t *va, *vb;
    if (passes & 1) { ka = keys_out; va = values_out; kb = tmpk; vb = tmpv; }
    else            { ka = tmpk; va = tmpv; kb = keys_out; vb = values_out; }
    SortWorkspace ws = sort_ws(ctx, s->sort);
    if ((e = launch_sort_prepare(ws, count, passes, true, stream)) != hipSuccess) return hip_fail(e, "sort prepare");
    if (sort_uses_onesweep(count, algo) &&
        (e = launch_sort_histogram(keys_in, count, passes, 0, ws.hist, stream, end_bit)) != hipSuccess)
        return hip_fail(e, "sort histogram");
    if ((e = launch_sort_passes(keys_in, values_in, ka, va, kb, vb, count, passes, 0, ws, algo, stream,
                                end_bit)) !=
        hipSuccess)
        return hip_fail(e, "sort passes");
    return CDS_OK;
}

cds_status cds_exclusive_scan_u32(cds_ctx* ctx, const uint32_t* in, int64_t count, uint32_t* out,
                                  uint64_t* total, void* stream) {
    if (!ctx || count < 0 || !total || (count > 0 && (!in || !out)))
        return fail(CDS_ERR_INVALID_ARG, "bad argument");
    if (count > 0 && (const void*)in == (const void*)out) return fail(CDS_ERR_INVALID_ARG, "out aliases in");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    cds_status st;
    if ((st = ensure(ctx, ctx->scratch->blocksums, sizeof(uint64_t) * scan_block_sums_size(count))) != CDS_OK)
        return st;
    e = launch_exclusive_scan(in, nullptr, out, count, (uint64_t*)ctx->scratch->blocksums.p, total,
                              (hipStream_t)stream);
    return e == hipSuccess ? CDS_OK : hip_fail(e, "scan");
}

cds_status cds_check_device(cds_ctx* ctx, void* stream) {
    if (!ctx) return fail(CDS_ERR_INVALID_ARG, "context is NULL");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    if ((e = hipStreamSynchronize((hipStream_t)stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    uint32_t err = 0;
    if ((e = hipMemcpy(&err, ctx->d_err, 4, hipMemcpyDeviceToHost)) != hipSuccess) return hip_fail(e, "hipMemcpy");
    if (err) {
        (void)hipMemset(ctx->d_err, 0, 4);
        return fail(CDS_ERR_DEVICE, "device-side check failed (code " + std::to_string(err) +
                                        "): 1 = a bounded wait in the radix sort gave up, "
                                        "2 = a radix-sort scatter or gather index was out of range, "
                                        "4 or 8 = tile binning counts were inconsistent, "
                                        "16 = a blend met a tile-list entry at or past the splat count");
    }
    return CDS_OK;
}

}  // extern "C"
