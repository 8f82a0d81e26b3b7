// Host-side state shared by the runtime translation units.
#pragma once
#include <string>

#include "cdnasplat.h"
#include "internal.h"

namespace cds {

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct SortState {
    DevBuf hist, status, counters, part_hist, bases, scan_sums, scan_total;
};

// stage boundaries of a timed render
enum StageEvent {
    kEvStart = 0,
    kEvPreprocess,  // preprocess done
    kEvCount,       // key count read back (compaction / scans)
    kEvDepth,       // depth order, key offsets and tile counts ready
    kEvKeys,        // keys generated
    kEvSortFirst,   // first radix pass over the keys done
    kEvSort,        // tile sort done
    kEvRanges,      // ranges done
    kEvBlend,       // blend done
    kEvBwdStart,
    kEvBwdBlend,
    kEvBwdPre,
    kEvCount_
};

}  // namespace cds

struct cds_ctx {
    int device = 0;
    cds_allocator alloc{};
    bool has_alloc = false;
    uint64_t* host_pinned = nullptr;  // pinned host words for the per-render key count
    uint64_t* host_pinned_dev = nullptr;  // the same words as kernels address them (fine-grained)
    uint32_t* d_err = nullptr;        // device-side error word
    float* d_partial = nullptr;       // 1024 floats: per-block partial sums of the loss
    cds_frame* scratch = nullptr;     // buffers of the stand-alone sort / scan calls
};

struct cds_frame {
    cds_ctx* ctx = nullptr;
    // per Gaussian
    cds::DevBuf mean2d, conic, rgb, depth, radius, rect, touched, offsets, clampf;
    cds::DevBuf blocksums, total;
    cds::DevBuf order0, order1, dkey0, dkey1;  // per-Gaussian depth sort (sort variants 2, 3)
    cds::DevBuf vrect, binM, binE, binP, tsum;  // tile binning (sort variant 3)
    cds::DevBuf tdiff, thist;                  // per-tile counts and tile-digit histograms (variant 2)
    cds::DevBuf dkeyc, recc, recv, vsums, ksums;  // compacted visible splats (variant 2)
    cds::DevBuf kowner;                        // record owning every 1024th key (variant 2)
    cds::DevBuf hsums;                         // per-tile rectangle-height sums (variant 4)
    cds::DevBuf pvis, pkeys, ph;               // per-preprocess-workgroup counts (compacting variants)
    cds::DevBuf rp_ha, rp_hb, rp_small, rp_rowent;  // row-wise tile placement (variant 4)
    cds::SortState sort_d;
    // per key
    cds::DevBuf keys0, keys1;                  // 64-bit keys (variant 1; others: rebuilt on request)
    cds::DevBuf tk0, tk1;                      // 32-bit tile ids (variant 2)
    cds::DevBuf vals0, vals1;
    cds::SortState sort;
    // per tile
    cds::DevBuf ranges;
    // backward
    cds::DevBuf grad2d;
    cds::DevBuf jac;  // [9][n] colour direction derivative (renders kept for the backward pass)
    bool keep_jac = false, jac_valid = false;
    int64_t n = 0, n_vis = 0, K = 0;
    int64_t row_entries = 0;  // variant 4: entries of the per-tile-row lists
    int32_t width = 0, height = 0, tiles_x = 0, tiles_y = 0, passes = 0, sort_variant = 0;
    bool valid = false;
    // where the last render left its sorted list
    const uint32_t* res_values = nullptr;
    const uint32_t* res_tiles = nullptr;  // tile id words, stride res_tile_stride (null: binned)
    int res_tile_stride = 1;
    const uint64_t* res_keys = nullptr;   // 64-bit keys, null until built (variants 2, 3)
    // stage timing: HIP events at the stage boundaries (kEv*)
    bool timing = false, timed_backward = false;
    hipEvent_t ev[cds::kEvCount_] = {};
    // a second stream (default priority) for work that overlaps the depth
    // sort, forked from and joined back into the render stream
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    hipEvent_t copied = nullptr;  // the key-count read-back has landed
    cds_status side_stream();
    cds_status record(int i, hipStream_t s);
    hipEvent_t event(int i);  // the stage event, created on demand; null without timing
    void release_all();
};

namespace cds {

extern thread_local std::string g_last_error;
cds_status fail(cds_status s, const std::string& msg);
// Looks up `device`'s copy of the allocation-free sort's scratch array (with
// that device current); once per device.
hipError_t noalloc_init_device(int device);
cds_status hip_fail(hipError_t e, const char* what);
void* ctx_alloc(cds_ctx* c, size_t bytes);
void ctx_free(cds_ctx* c, void* p);
cds_status ensure(cds_ctx* c, DevBuf& b, size_t bytes, double grow = 1.0);
void release(cds_ctx* c, DevBuf& b);
cds_status validate_scene(const cds_scene* s);
cds_status validate_camera(const cds_camera* c);
ProjParams make_proj(const cds_scene* s, const cds_camera* c);
SceneParams make_scene(const cds_scene* s);
cds_status ensure_sort_workspace(cds_ctx* ctx, SortState& s, int64_t count, int passes);
SortWorkspace sort_ws(cds_ctx* ctx, SortState& s);

void release_frame_buffers(cds_frame* f);
int64_t frame_held_bytes(cds_frame* f);  // device bytes the frame's buffers hold now

cds_status render_forward_impl(cds_ctx* ctx, cds_frame* f, const cds_scene* scene, const cds_camera* cam,
                               int blend_variant, int sort_variant, SortAlgo algo, float* out_rgb, float* out_T,
                               uint32_t* out_ncontrib, float* out_invdepth, hipStream_t stream);
SortAlgo sort_algo_from_flags(uint32_t flags);
int tile_bits_for(int64_t ntiles);
cds_status frame_build_keys(cds_frame* f);
cds_status render_backward_impl(cds_ctx* ctx, cds_frame* f, const cds_scene* scene, const cds_camera* cam,
                                const float* out_T, const uint32_t* out_ncontrib, const float* dL_drgb,
                                const float* dL_dinvdepth, const cds_scene_grad* g, hipStream_t stream);

}  // namespace cds
