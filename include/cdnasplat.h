/*
 * cdnasplat.h -- C ABI of the MI355X (gfx950) 3D Gaussian-splatting rasterizer.
 *
 * The library renders a set of 3D Gaussians for a pinhole camera with the
 * pipeline the paper describes in Section II-B ("Structure of Gaussian
 * Splatting Rendering Pipeline") and Algorithm 1:
 *
 *   preprocess  per Gaussian: visibility, projection to a 2D splat (mean,
 *               conic, screen radius), colour from spherical harmonics, depth
 *   duplicate   one (tile | depth) key per covered 16x16 tile
 *   sort        stable radix sort of the 64-bit keys (ties by Gaussian index)
 *   ranges      [start, end) of every tile in the sorted list
 *   blend       per pixel, front to back alpha blending with early stop when
 *               the transmittance falls below 1e-4 (Eq. (1), Algorithm 1)
 *
 * plus the exact backward pass of all of it (gradients for every raw
 * parameter) and a continuous-batching server for many resident scenes.
 *
 * Conventions shared by every call:
 *  - Device pointers are plain HIP device addresses on the context's device;
 *    host pointers are ordinary process memory.  Every pointer argument says
 *    which it is.
 *  - Work is enqueued on the caller's HIP stream (`stream`, a hipStream_t
 *    passed as void*; NULL is the legacy default stream).  Calls return once
 *    the work is enqueued unless stated otherwise.
 *  - No call throws or aborts.  Every fallible call returns a cds_status;
 *    cds_last_error() gives a human-readable message for the calling thread.
 *  - Arguments are validated before any device work is enqueued; an invalid
 *    argument returns CDS_ERR_INVALID_ARG and changes nothing.
 *  - A context (and every frame or server made from it) may be used by one
 *    host thread at a time.
 *  - A frame owns all of a render's device state, so renders into different
 *    frames (and different outputs) may be in flight on different streams at
 *    once: the next frame's projection then runs beside the previous one's
 *    sort and blend.  Successive calls on one frame must be stream-ordered
 *    (the same stream, or ordered by the caller).
 */
#ifndef CDNASPLAT_H
#define CDNASPLAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CDS_TILE 16          /* tile edge in pixels (Section II-B: 16 x 16 tiles) */
#define CDS_MAX_SH_DEGREE 3  /* spherical-harmonics degree 0..3 (16 coefficients) */

typedef enum cds_status {
    CDS_OK = 0,
    CDS_ERR_INVALID_ARG = 1, /* bad pointer, size or option; nothing was enqueued */
    CDS_ERR_OOM = 2,         /* the allocator returned NULL; outputs unspecified, no leak */
    CDS_ERR_CAPACITY = 3,    /* a size limit of the library was exceeded (more than 2^31-1
                                Gaussians or 2^30-1 tile keys) */
    CDS_ERR_DEVICE = 4,      /* a HIP call or a device-side check failed (message has details) */
    CDS_ERR_BUSY = 5         /* the server has no free slot / budget for the request right now */
} cds_status;

/* Device-memory allocator.  alloc returns a device pointer aligned to at least
 * 256 bytes, or NULL on failure; free releases it.  Memory may be reused by
 * the library for later stream-ordered work only through these calls.  Pass
 * NULL to cds_create to use hipMalloc / hipFree. */
typedef struct cds_allocator {
    void* (*alloc)(size_t bytes, void* user);
    void (*free)(void* ptr, void* user);
    void* user;
} cds_allocator;

/* A scene: n Gaussians (0 <= n <= 2^31-1) as structure-of-arrays float32
 * planes in DEVICE memory, owned by the caller and only read by the library.
 *   means          [3][n]              world-space centres
 *   log_scales     [3][n]              log of the per-axis standard deviation
 *   quats          [4][n]              rotation (w, x, y, z); need not be normalised
 *   opacity_logits [n]                 opacity = 1 / (1 + exp(-logit))
 *   sh             [(deg+1)^2][3][n]   spherical-harmonics coefficients,
 *                                      coefficient-major, then colour channel */
typedef struct cds_scene {
    int64_t n;
    int32_t sh_degree;
    int32_t reserved;
    const float* means;
    const float* log_scales;
    const float* quats;
    const float* opacity_logits;
    const float* sh;
} cds_scene;

/* Gradients with the same layouts as cds_scene, DEVICE memory, caller-owned.
 * Every element is overwritten by cds_render_backward. */
typedef struct cds_scene_grad {
    float* means;
    float* log_scales;
    float* quats;
    float* opacity_logits;
    float* sh;
} cds_scene_grad;

/* Pinhole camera (HOST struct, copied by value).  `view` is the world->camera
 * transform [R | t], row-major 3 x 4; the camera looks down +z, image x to
 * the right and y down; pixel (x, y) is sampled at integer coordinates.
 * Gaussians with camera-space z <= near_plane are culled.  bg is the
 * background colour composited behind the splats. */
typedef struct cds_camera {
    int32_t width, height;
    float fx, fy, cx, cy;
    float view[12];
    float near_plane;
    float bg[3];
} cds_camera;

/* Render options (HOST struct; NULL means all defaults). */
#define CDS_OPT_DEFAULT 0u
#define CDS_OPT_STAGE_TIMING 1u      /* record HIP events around every stage (forward and backward) */
#define CDS_OPT_SORT_ONESWEEP 2u      /* radix-sort passes by decoupled look-back (default: by size) */
#define CDS_OPT_SORT_REDUCE_SCAN 4u   /* radix-sort passes by reduce-then-scan (default: by size) */
#define CDS_OPT_KEEP_FOR_BACKWARD 8u  /* the render will be differentiated: with SH degree > 0 the forward
                                         also stores per Gaussian the colour's derivative with respect to
                                         the view direction (36 bytes, in the frame), which the backward
                                         then reads instead of the SH coefficients (up to 192 bytes);
                                         the gradients are the same either way, up to rounding */
typedef struct cds_render_opts {
    uint32_t flags;         /* CDS_OPT_* bits */
    int32_t blend_variant;  /* 0 = default (2 pixels per thread; 1 below ten tiles per compute unit);
                               1, 2, 4 = pixels per thread of the blend kernel */
    int32_t sort_variant;   /* how the (tile | depth) list is ordered; every variant gives the same
                               sorted keys, values and ranges:
                               1 = 64-bit keys radix-sorted on all their digits;
                               2 = depth digits sorted once per Gaussian, then the tile digits of
                                   32-bit tile ids radix-sorted per key;
                               3 = depth digits per Gaussian, then a counting sort on the whole tile id
                                   fused with duplication (needs at most 512 tiles per row, i.e.
                                   images up to 8192 pixels wide; wider ones are rejected);
                               4 = depth digits per Gaussian, then the tile lists by stable
                                   placement of each splat's rectangle, first into per-tile-row
                                   lists, then into the tiles (at most 4096 tiles per axis);
                               0 = default: 4 where the grid allows it, else 2. */
    int32_t reserved;
} cds_render_opts;

typedef struct cds_ctx cds_ctx;
typedef struct cds_frame cds_frame;
typedef struct cds_server cds_server;

/* Library version string (static storage). */
const char* cds_version(void);

/* Message describing the last non-OK status returned to this thread. */
const char* cds_last_error(void);

/* Create a context on HIP device `device`.  `alloc` (HOST struct, copied) may
 * be NULL for hipMalloc/hipFree.  *out receives the context. */
cds_status cds_create(cds_ctx** out, int device, const cds_allocator* alloc);

/* Destroy a context; frames and servers made from it must be released first.
 * Waits for the context's outstanding work.  NULL is ignored. */
void cds_destroy(cds_ctx* ctx);

/* Per-render state: the per-Gaussian projected splats, the keys and tile
 * lists of the last forward render, kept for the backward pass and for
 * inspection.  A frame grows its buffers as needed and reuses them; it must
 * not be used by two renders in flight at once. */
cds_status cds_frame_create(cds_ctx* ctx, cds_frame** out);
void cds_frame_release(cds_frame* frame);

/*
 * Forward render (Section II-B, Algorithm 1).
 *   out_rgb      DEVICE float [3][H][W]  colour, planar, C + T * bg
 *   out_T        DEVICE float [H][W]     final transmittance T
 *   out_ncontrib DEVICE u32   [H][W]     1-based position, in the pixel's tile
 *                                        list, of the last Gaussian blended
 *                                        (0 if none); skipped entries count
 * All three outputs are caller-owned and fully overwritten.  The call
 * synchronises the stream once to learn the number of keys (the only host
 * wait of a render).  Returns CDS_ERR_CAPACITY when the number of keys
 * exceeds 2^30 - 1.
 */
cds_status cds_render_forward(cds_ctx* ctx, cds_frame* frame, const cds_scene* scene,
                              const cds_camera* cam, const cds_render_opts* opts,
                              float* out_rgb, float* out_T, uint32_t* out_ncontrib,
                              void* stream);

/*
 * cds_render_forward with the optional expected inverse depth of the
 * Appendix B blend kernels (their `invdepth` output):
 *   out_invdepth DEVICE float [H][W]  sum over the blended Gaussians of
 *                                     alpha * T / depth (no background
 *                                     term), or NULL for none
 * Everything else as cds_render_forward.
 */
cds_status cds_render_forward_ex(cds_ctx* ctx, cds_frame* frame, const cds_scene* scene,
                                 const cds_camera* cam, const cds_render_opts* opts,
                                 float* out_rgb, float* out_T, uint32_t* out_ncontrib,
                                 float* out_invdepth, void* stream);

/*
 * Backward pass of the last forward render of `frame`: the exact derivative
 * of the forward with every discrete decision (culls, tile lists, skipped and
 * terminated blending steps, colour and alpha clamps, Jacobian guard band)
 * held fixed.  The transmittance of each step is recomputed by division from
 * the final T, walking each pixel's list backwards.
 *   out_T, out_ncontrib  DEVICE, the forward's outputs (unchanged since)
 *   dL_drgb              DEVICE float [3][H][W]  gradient of the loss w.r.t. out_rgb
 *   grads                DEVICE, caller-owned, cds_scene layouts, overwritten
 * `scene` and `cam` must be those of the forward.
 */
cds_status cds_render_backward(cds_ctx* ctx, cds_frame* frame, const cds_scene* scene,
                               const cds_camera* cam, const float* out_T,
                               const uint32_t* out_ncontrib, const float* dL_drgb,
                               const cds_scene_grad* grads, void* stream);

/*
 * cds_render_backward with a gradient for the expected inverse depth too:
 *   dL_dinvdepth DEVICE float [H][W]  gradient of the loss w.r.t. the
 *                                     out_invdepth of cds_render_forward_ex,
 *                                     or NULL (then the same as
 *                                     cds_render_backward)
 * The inverse depth flows back through alpha (as a colour channel with no
 * background) and through 1 / depth to the means.
 */
cds_status cds_render_backward_ex(cds_ctx* ctx, cds_frame* frame, const cds_scene* scene,
                                  const cds_camera* cam, const float* out_T,
                                  const uint32_t* out_ncontrib, const float* dL_drgb,
                                  const float* dL_dinvdepth, const cds_scene_grad* grads,
                                  void* stream);

/* L1 image loss helper: dL_drgb[i] = sign(rgb[i] - target[i]) / count and,
 * if loss_out is not NULL, loss_out[0] = mean |rgb - target| (DEVICE float,
 * overwritten; summed in a fixed order, so repeated calls agree bit for bit).
 * All pointers DEVICE, count elements.  Calls on one context share a small
 * reduction workspace: do not overlap them on different streams. */
cds_status cds_l1_loss_grad(cds_ctx* ctx, const float* rgb, const float* target, int64_t count,
                            float* dL_drgb, float* loss_out, void* stream);

/* Device pointers into a frame's state after cds_render_forward (read-only,
 * owned by the frame, valid until the frame's next render or release).  The
 * caller must have synchronised with the render; building the 64-bit sorted
 * keys on first request synchronises the device. */
typedef struct cds_frame_info {
    int64_t n;                     /* Gaussians of the last render */
    int64_t num_keys;              /* K: duplicated (tile | depth) keys */
    int32_t width, height, tiles_x, tiles_y;
    int32_t sort_passes;           /* radix passes over the key's digits (depth + tile) */
    int32_t num_visible;           /* splats with at least one tile (visit positions of offsets, variant 2) */
    const float* mean2d;           /* [n] float2 (x, y), pixels */
    const float* conic_opacity;    /* [n] float4 (A, B, C, opacity): power = -A dx^2/2 - B dx dy - C dy^2/2 */
    const float* rgb;              /* [n] float4 (r, g, b, 0) after the clamp at 0 */
    const uint32_t* depth_bits;    /* [n] IEEE bits of the float32 view depth (0 if culled) */
    const int32_t* radius;         /* [n] screen radius in pixels, 0 if culled */
    const uint32_t* tile_rect;     /* [n] uint2: (tx0 | ty0 << 16, tx1 | ty1 << 16), inclusive */
    const uint32_t* tiles_touched; /* [n] number of covered tiles */
    const uint32_t* offsets;       /* exclusive prefix sum of tiles_touched in visit order: [n] in
                                      index order (sort variant 1); [num_visible] over the visible
                                      splats in (depth, index) order (variant 2); NULL for variant 3,
                                      which does not form it */
    const uint64_t* keys;          /* [K] sorted (tile << 32 | depth bits) */
    const uint32_t* values;        /* [K] Gaussian index of each sorted key */
    const uint32_t* ranges;        /* [tiles_x * tiles_y] uint2 [start, end), (0, 0) if empty */
    const uint8_t* clamp_flags;    /* [n] bit 0..2 colour channel clamped, 3/4 Jacobian x/y clamped */
    int64_t num_row_entries;       /* variant 4: entries of the per-tile-row lists (the visible
                                      splats' rectangle heights summed); 0 otherwise */
} cds_frame_info;

cds_status cds_frame_get_info(cds_frame* frame, cds_frame_info* out);

/* Per-stage device time of the frame's last forward (and backward) render,
 * in milliseconds, from HIP events recorded on the render's stream when the
 * forward ran with CDS_OPT_STAGE_TIMING.  Waits for those events.
 *   preprocess_ms   projection and colour (a1, a2)
 *   scan_ms         up to the host read-back of the key count, included:
 *                   the visible-splat compaction (sort variants 2 and 4), the
 *                   prefix sum of tiles_touched (variant 1), or the depth sort
 *                   and tile counts of binning (variant 3)
 *   depth_order_ms  variants 2 and 4: depth sort of the visible splats (with
 *                   variant 2 also their key offsets), the per-tile counts and
 *                   ranges; 0 otherwise
 *   duplicate_ms    key generation as its own kernel (variant 1, variant 2
 *                   with reduce-then-scan passes; variant 3: the fused
 *                   placement; variant 4: the per-tile-row lists); about 0
 *                   when the first radix pass generates the keys
 *   sort_ms         the per-key radix passes (0 for variant 3); with variant 2
 *                   and onesweep passes the first of them generates the keys;
 *                   variant 4: the placement of the row lists into the tiles
 *   sort_first_pass_ms  the part of sort_ms taken by the first pass (variant
 *                   4: by the column counts and start slots, before the last
 *                   kernel)
 *   ranges_ms       ranges from the sorted keys (variant 1 only)
 *   blend_ms        the per-pixel blend
 * Backward fields are 0 until a backward pass has run. */
typedef struct cds_stage_times {
    float preprocess_ms, scan_ms, depth_order_ms, duplicate_ms, sort_ms, ranges_ms, blend_ms;
    float blend_backward_ms, preprocess_backward_ms;
    float sort_first_pass_ms;
} cds_stage_times;

cds_status cds_frame_stage_times(cds_frame* frame, cds_stage_times* out);

/*
 * Stand-alone stable LSD radix sort of (key, value) pairs on key bits
 * [0, end_bit), the sort the forward render uses.  All arrays DEVICE,
 * `count` elements; the inputs are not modified; outputs may not alias
 * inputs.  Equal keys keep their input order.  `flags`: 0 or one of
 * CDS_OPT_SORT_ONESWEEP / CDS_OPT_SORT_REDUCE_SCAN.
 */
cds_status cds_sort_pairs(cds_ctx* ctx, const uint64_t* keys_in, const uint32_t* values_in,
                          int64_t count, int32_t end_bit, uint64_t* keys_out,
                          uint32_t* values_out, uint32_t flags, void* stream);

/*
 * The same sort without any allocation, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation.  Arguments, results and errors as
 * cds_sort_pairs, except:
 *   - count may be at most CDS_NOALLOC_MAX_PAIRS (larger: CDS_ERR_CAPACITY,
 *     no device work);
 *   - every buffer beyond the inputs and outputs comes from one fixed device
 *     array of CDS_NOALLOC_SCRATCH_BYTES, held by each GPU the library runs
 *     on until the process ends; the call makes no allocation, through the
 *     context's allocator or otherwise;
 *   - all calls on one GPU share that array: calls that overlap on one GPU
 *     (on different streams or from different threads) race and must be
 *     ordered by the caller.
 */
#define CDS_NOALLOC_MAX_PAIRS 1048576
#define CDS_NOALLOC_SCRATCH_BYTES 15217152
cds_status cds_sort_pairs_noalloc(cds_ctx* ctx, const uint64_t* keys_in, const uint32_t* values_in,
                                  int64_t count, int32_t end_bit, uint64_t* keys_out,
                                  uint32_t* values_out, uint32_t flags, void* stream);

/*
 * Stand-alone exclusive prefix sum of `count` uint32 (DEVICE in/out, may not
 * alias); the total is written to DEVICE *total (uint64).  Used by the
 * forward render for key offsets.
 */
cds_status cds_exclusive_scan_u32(cds_ctx* ctx, const uint32_t* in, int64_t count, uint32_t* out,
                                  uint64_t* total, void* stream);

/* Synchronise `stream` and report device-side errors raised since the last
 * check, then clear them: CDS_OK or CDS_ERR_DEVICE with a message naming the
 * bits of the device error word.  Bits: 1 a sort's bounded look-back gave up
 * waiting; 2 a sort's record gather met an index at or past the key count;
 * 4 / 8 tile binning found counts that disagree; 16 a blend (forward,
 * backward or batched) met a tile-list entry at or past the splat count.
 * Each of these can only follow a logic error or corrupted input; the kernel
 * that detects it substitutes an in-bounds value, so outputs are then wrong
 * but no memory outside the buffers is touched. */
cds_status cds_check_device(cds_ctx* ctx, void* stream);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of render requests over resident scenes.    */
/* ------------------------------------------------------------------------ */

typedef struct cds_server_opts {
    int32_t max_slots;          /* requests in flight at once (1..64) */
    int32_t max_batch;          /* at most this many requests fused into one batched launch (1..max_slots);
                                   fewer when the queue is short or the batch reaches 16,383 tiles or 2^25 Gaussians */
    int64_t hbm_budget_bytes;   /* workspace budget for admitted requests; 0 = free HBM at create */
    int32_t sort_variant;       /* how a batch's tile lists are ordered: 0 = default (4: row-wise placement
                                   over the stacked tile grid; 2 for batches past its limits);
                                   2 = radix-sorted tile keys (sort variant 2); the lists are the same */
    int32_t reserved;
} cds_server_opts;

typedef struct cds_server_stats {
    int64_t submitted, completed, rejected;
    int64_t batches;            /* batched launches issued */
    int64_t workspace_bytes;    /* workspace currently reserved by admitted requests (estimate) */
    int64_t peak_workspace_bytes;
    int64_t held_bytes;         /* device memory the workspaces' buffers hold now (measured) */
    int64_t peak_held_bytes;    /* its maximum; admission keeps it within the HBM budget
                                   except for a request that runs alone */
} cds_server_stats;

/* Create a server on a context.  The server owns one HIP stream pair and a
 * host scheduler thread. */
cds_status cds_server_create(cds_ctx* ctx, const cds_server_opts* opts, cds_server** out);

/* Register a resident scene (DEVICE arrays, caller-owned; they must stay
 * valid and unchanged until the server is destroyed).  *scene_id (HOST)
 * receives its id. */
cds_status cds_server_add_scene(cds_server* srv, const cds_scene* scene, int32_t* scene_id);

/* Queue a render of `scene_id` for `cam`.  out_rgb (DEVICE, caller-owned,
 * [3][H][W]) becomes valid when cds_server_poll reports the ticket done.
 * Returns CDS_ERR_BUSY if the request could never fit the budget. */
cds_status cds_server_submit(cds_server* srv, int32_t scene_id, const cds_camera* cam,
                             float* out_rgb, uint64_t* ticket);

/* *done (HOST) = 1 when the ticket's image is complete on the device, else 0.
 * If latency_ms is not NULL it receives submit-to-completion time in ms
 * (valid when done). */
cds_status cds_server_poll(cds_server* srv, uint64_t ticket, int32_t* done, double* latency_ms);

/* Block until every queued request is complete. */
cds_status cds_server_drain(cds_server* srv);

cds_status cds_server_get_stats(cds_server* srv, cds_server_stats* out);

/* Drain and destroy the server.  NULL is ignored. */
void cds_server_destroy(cds_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* CDNASPLAT_H */
