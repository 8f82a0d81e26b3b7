// Per-pixel front-to-back alpha blending (paper Section II-B(2), Eq. (1) with
// the splat alpha, Algorithm 1) and its backward pass.
//
// One workgroup per 16x16 tile.  The tile's sorted splats are staged through
// LDS in batches (the shared-memory staging the paper measures at
// +11.3%), the colour included (the coalesced-RGB point).  Each lane blends
// PPT vertically adjacent pixels (PPT = 1, 2, 4), so every LDS read of a splat
// serves PPT pixel evaluations and the column-dependent terms of the
// quadratic form are computed once per lane.  The conic is pre-scaled by
// -log2(e)/2, -log2(e), -log2(e)/2 when staged so the hot loop needs one
// hardware exp2 (v_exp_f32, the gfx950 counterpart of the paper's __expf).
// The loop has no data-dependent trip count (per-pixel "done" masks only),
// an early exit is voted block-wide once per batch, and a wave whose pixels
// are all done leaves the batch early.
//
// Each staged splat also carries a pixel box outside which its alpha is
// below 1/255 for certain (the ellipse of power >= -ln(255 o), widened by a
// margin that covers the rounding of the alpha test).  A wave evaluates only
// the splats whose box meets its pixels, found with four ballots per batch;
// every pair it skips is one the alpha test would skip, so the result is the
// same as evaluating all of them.
//
// Tiles are assigned in XCD-contiguous bands so neighbouring tiles, which
// share most of their splats, hit the same L2.
//
// Optional expected inverse depth (the inverse-depth output of the paper's
// Appendix B kernels): 1 / depth of every splat composited like one more
// colour channel with no background (kDepth, staged per splat in s_d).
#include <algorithm>

#include <atomic>

#include "device_utils.h"
#include "internal.h"

namespace cds {
namespace {

// splats staged per batch: the forward keeps its registers under 64 and its
// LDS at 8 KB with 128 (eight waves per SIMD); the backward, heavier per
// splat, is faster with fewer, larger batches
constexpr int kBatch = 128;
constexpr int kBwdBatch = 256;
constexpr float kLn2 = 0.69314718055994531f;
constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTMin = 0.0001f;

// Staged splat, one LDS slot per splat:
//   s_q  double4 (mean x, mean y, A', B')   s_c double C'   s_f float4 (opacity, r, g, b)
//   s_b  the tile pixels its alpha can reach: 5-bit fields (x min, x max,
//        y min, y max) + 1, relative to the tile origin and clamped to
//        [-1, 16], and from bit 20 a mask of the tile's 4-row groups the
//        alpha >= 1/255 ellipse itself can meet
// with A' = -log2(e)/2 A, B' = -log2(e) B, C' = -log2(e)/2 C, so that
// A' dx^2 + B' dx dy + C' dy^2 = log2(e) * power.
//
// Box: alpha >= 1/255 needs o exp(power) >= 1/255, i.e. d^T M d <= 2 ln(255 o)
// with d = mean - pixel and M = [[A, B], [B, C]]; that ellipse lies within
// |dx| <= sqrt(2 t C / det), |dy| <= sqrt(2 t A / det).  t is ln(255 o) plus
// 1e-3 (+1e-5 relative): the float32 rounding of power, of exp2, of the
// product and of the log2 that gives t move the test by far less.  Splats with o < 1/255 reach no pixel
// (alpha <= o); when M is not positive definite or anything is not finite,
// the box is unbounded.
//
// Row groups: for each group of four tile rows (all 16 columns), the least
// value of d^T M d over that rectangle of pixel centres, against 2t.  The
// form is convex with its minimum at d = 0, so when d = 0 lies outside the
// rectangle the least value is on an edge, at the edge's stationary point
// clamped to the edge; a group is dropped only when that value exceeds 2t
// by more than the float32 rounding of the form can account for.
// For a thin splat at an angle this drops about half of the (splat, wave)
// pairs its box admits.
__device__ __forceinline__ void stage_splat(const float2* __restrict__ mean2d,
                                            const float4* __restrict__ conic_opacity,
                                            const float4* __restrict__ rgb, uint32_t id, double4* s_q,
                                            double* s_c, float4* s_f, uint32_t* s_b, int k, int tx0, int ty0) {
    const double L = 1.4426950408889634;  // log2(e)
    const float2 m = mean2d[id];
    const float4 co = conic_opacity[id];
    const float4 c = rgb[id];
    s_q[k] = make_double4((double)m.x, (double)m.y, -0.5 * L * (double)co.x, -L * (double)co.y);
    s_c[k] = -0.5 * L * (double)co.z;
    s_f[k] = make_float4(co.w, c.x, c.y, c.z);
    // box relative to the tile origin, in whole pixels, clamped to [-1, 16]
    int x0 = -1, x1 = kTile, y0 = -1, y1 = kTile;  // unbounded
    uint32_t rows = 0xFu;                          // every row group
    if (co.w < kAlphaMin) {
        x0 = kTile;  // empty
        x1 = -1;
    } else {
        const double a = (double)co.x, b = (double)co.y, cc = (double)co.z;
        const double det = a * cc - b * b;
        // ln(255 o) from the hardware log2 (error ~1e-7 relative), widened
        const double t = (double)(__builtin_amdgcn_logf(255.0f * co.w) * kLn2) * (1.0 + 1e-5) + 1e-3;
        if (a > 0.0 && cc > 0.0 && det > 0.0 && t > 0.0 && t < 1e30) {
            const double ex = sqrt(2.0 * t * cc / det) * (1.0 + 1e-6) + 0.01;
            const double ey = sqrt(2.0 * t * a / det) * (1.0 + 1e-6) + 0.01;
            const double mx = (double)m.x - tx0, my = (double)m.y - ty0;
            // comparisons are false for NaN, which keeps the unbounded box
            if (mx - ex > -1.0) x0 = mx - ex < (double)kTile ? (int)floor(mx - ex) : kTile;
            if (mx + ex < (double)kTile) x1 = mx + ex > -1.0 ? (int)ceil(mx + ex) : -1;
            if (my - ey > -1.0) y0 = my - ey < (double)kTile ? (int)floor(my - ey) : kTile;
            if (my + ey < (double)kTile) y1 = my + ey > -1.0 ? (int)ceil(my + ey) : -1;
            if (fabs(mx) < 1e30 && fabs(my) < 1e30) {  // finite: the edge minima below
                // float32: a group is dropped only when the least value exceeds
                // 2t by more than 1e-6 of the terms' magnitude (the float32
                // rounding of the form is below 3e-7 of it) plus what the
                // rounding of the offsets to float32 (at most e per axis) can
                // move it: |2 e^T M d| <= 2 e (|a u| + |b| (|u| + |v|) + |c v|)
                const float af = co.x, bf = co.y, cf = co.z, t2 = (float)(2.0 * t);
                const float mxf = (float)mx, myf = (float)my;
                const float ua = mxf - (float)(kTile - 1), ub = mxf;
                const float e2 = 2.4e-7f * (fabsf(mxf) + fabsf(myf) + (float)(2 * kTile));
                const float ue = fmaxf(fabsf(ua), fabsf(ub));
                const float sv = -bf / cf, su = -bf / af;
                const auto form = [&](float u, float v, float& mag) {
                    mag = fmaxf(mag, fabsf(af) * u * u + 2.0f * fabsf(bf * u * v) + fabsf(cf) * v * v);
                    return (af * u + 2.0f * bf * v) * u + cf * v * v;
                };
                const bool in_u = ua <= 0.0f && ub >= 0.0f;
#pragma unroll 1
                for (int g = 0; g < 4; ++g) {
                    const float va = myf - (float)(4 * g + 3), vb = myf - (float)(4 * g);
                    const float v0 = fminf(fmaxf(sv * ua, va), vb), v1 = fminf(fmaxf(sv * ub, va), vb);
                    const float u0 = fminf(fmaxf(su * va, ua), ub), u1 = fminf(fmaxf(su * vb, ua), ub);
                    float mag = 0.0f;
                    const float q = fminf(fminf(form(ua, v0, mag), form(ub, v1, mag)),
                                          fminf(form(u0, va, mag), form(u1, vb, mag)));
                    const float ve = fmaxf(fabsf(va), fabsf(vb));
                    const float shift = e2 * (fabsf(af) * ue + fabsf(bf) * (ue + ve) + fabsf(cf) * ve);
                    if (!(in_u && va <= 0.0f && vb >= 0.0f) && q > t2 + 1e-6f * mag + shift) rows &= ~(1u << g);
                }
            }
        }
    }
    s_b[k] = (uint32_t)(x0 + 1) | ((uint32_t)(x1 + 1) << 5) | ((uint32_t)(y0 + 1) << 10) |
             ((uint32_t)(y1 + 1) << 15) | (rows << 20);
}

// Whether a staged splat (see stage_splat) can reach the tile pixel rows
// [r0, r1] (all 16 columns; r0 a multiple of 4): its box meets them and so
// does its ellipse in one of their row groups.
__device__ __forceinline__ bool box_meets_rows(uint32_t box, int r0, int r1) {
    const int x0 = (int)(box & 31u) - 1, x1 = (int)((box >> 5) & 31u) - 1;
    const int y0 = (int)((box >> 10) & 31u) - 1, y1 = (int)((box >> 15) & 31u) - 1;
    const uint32_t groups = (box >> (20 + (r0 >> 2))) & ((2u << ((r1 >> 2) - (r0 >> 2))) - 1u);
    return x1 >= 0 && x0 <= kTile - 1 && y1 >= r0 && y0 <= r1 && groups != 0u;
}

// The blending decision of one (pixel, splat) pair, shared by the forward
// and the backward pass so both take bit-identical decisions.
//   adx2 = A' dx^2, bdx = B' dx (column terms), dy = mean_y - pixel_y.
// The quadratic form is evaluated in float64: for thin splats its terms
// cancel and float32 would lose the digits that decide alpha.  Float64 FMA
// runs at the float32 (non-packed) rate on CDNA4, so this costs one
// conversion per pair.  Returns false when the splat is skipped
// (power > 0 or alpha < 1/255); alpha and G are computed either way (the
// callers select), and are only meaningful when it returns true.
__device__ __forceinline__ bool splat_alpha(double adx2, double bdx, double c2, double dy, float opacity,
                                            float& alpha, float& G) {
    const double power = fma(dy, fma(c2, dy, bdx), adx2);  // log2(e) * power
    G = __builtin_amdgcn_exp2f((float)power);
    alpha = fminf(kAlphaMax, opacity * G);
    return !(power > 0.0) && !(alpha < kAlphaMin);
}

// A list entry is a splat index below n; one at or past n can only come from
// a corrupted list: it is replaced by splat 0 rather than read out of bounds,
// and bit 16 of the device error word is set so the corruption is reported.
constexpr uint32_t kErrBadListEntry = 16u;
__device__ __forceinline__ uint32_t splat_id(uint32_t id, int64_t n, uint32_t* err) {
    if ((int64_t)id < n) return id;
    atomicOr(err, kErrBadListEntry);
    return 0u;
}

// One 16x16 tile: stage its sorted splats through LDS in batches and blend
// each pixel front to back.  Shared by the single-render kernel and the
// persistent batched kernel so a request renders bit-identically in both.
// Every thread of the workgroup must call it (it contains barriers).  kU
// candidate splats are taken per step: their alphas do not depend on each
// other (only the accumulation is sequential), which shortens the chain of
// dependent instructions a wave walks through a long list; the accumulation
// order, and so every result bit, does not depend on kU.
template <int PPT, bool kDepth = false, int kU = 2>
__device__ __forceinline__ void blend_tile(int tx, int ty, int width, int height, uint2 range,
                                           const uint32_t* __restrict__ point_list, int64_t n, uint32_t* err,
                                           const float2* __restrict__ mean2d,
                                           const float4* __restrict__ conic_opacity,
                                           const float4* __restrict__ rgb, float bg0, float bg1, float bg2,
                                           float* out_rgb, float* out_T, uint32_t* out_ncontrib, double4* s_q,
                                           double* s_c, float4* s_f, uint32_t* s_b,
                                           const uint32_t* __restrict__ depth_bits = nullptr,
                                           float* out_invdepth = nullptr, float* s_d = nullptr) {
    constexpr int NT = 256 / PPT;
    constexpr int kRowsPerWave = kWave / kTile * PPT;
    const int t = threadIdx.x;
    const int px = tx * kTile + (t & 15);
    const int py0 = ty * kTile + (t >> 4) * PPT;
    const double fpx = (double)px;
    const uint32_t lane = lane_id();
    // this wave's pixels: 16 columns, tile rows [wr0, wr0 + kRowsPerWave)
    const int wr0 = (t / kWave) * kRowsPerWave;

    float T[PPT], C0[PPT], C1[PPT], C2[PPT], D[PPT];
    double fpy[PPT];
    uint32_t last[PPT];
    bool done[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        T[p] = 1.0f;
        C0[p] = C1[p] = C2[p] = D[p] = 0.0f;
        last[p] = 0;
        fpy[p] = (double)(py0 + p);
        done[p] = !(px < width && py0 + p < height);
    }

    const int todo = (int)(range.y - range.x);
    for (int base = 0; base < todo; base += kBatch) {
        int alive = 0;
#pragma unroll
        for (int p = 0; p < PPT; ++p) alive |= done[p] ? 0 : 1;
        if (__syncthreads_count(alive) == 0) break;
        for (int k = t; k < kBatch; k += NT) {
            const int idx = base + k;
            if (idx < todo) {
                const uint32_t id = splat_id(point_list[range.x + idx], n, err);
                stage_splat(mean2d, conic_opacity, rgb, id, s_q, s_c, s_f, s_b, k, tx * kTile, ty * kTile);
                if constexpr (kDepth) s_d[k] = 1.0f / __uint_as_float(depth_bits[id]);
            }
        }
        __syncthreads();
        const int cnt = min(kBatch, todo - base);
        // the batch's splats whose box meets this wave's pixels, in list order
        uint64_t cand[kBatch / kWave];
#pragma unroll
        for (int q = 0; q < kBatch / kWave; ++q) {
            const int k = q * kWave + (int)lane;
            cand[q] = ballot(k < cnt && box_meets_rows(s_b[k], wr0, wr0 + kRowsPerWave - 1));
        }
        int visited = 0;
        bool wave_done = false;
        // the accumulation of one splat into a pixel (front to back, in list order)
        const auto accumulate = [&](int p, int j, float alpha, const float4& f) {
            const float test_T = T[p] * (1.0f - alpha);
            if (test_T < kTMin) {
                done[p] = true;
            } else {
                const float wgt = alpha * T[p];
                C0[p] = fmaf(f.y, wgt, C0[p]);
                C1[p] = fmaf(f.z, wgt, C1[p]);
                C2[p] = fmaf(f.w, wgt, C2[p]);
                if constexpr (kDepth) D[p] = fmaf(s_d[j], wgt, D[p]);
                T[p] = test_T;
                last[p] = (uint32_t)(base + j + 1);
            }
        };
        for (int q = 0; q < kBatch / kWave && !wave_done; ++q) {
            uint64_t m = cand[q];
            while (m) {
            int js[kU];
            bool has[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                has[u] = m != 0;  // uniform
                js[u] = has[u] ? q * kWave + __builtin_ctzll(m) : js[0];
                if (has[u]) m &= m - 1;
            }
            if ((visited++ & 15) == 0) {
                int live = 0;
#pragma unroll
                for (int p = 0; p < PPT; ++p) live |= done[p] ? 0 : 1;
                if (!__any(live)) {  // wave-uniform: this wave's pixels are all done
                    wave_done = true;
                    break;
                }
            }
            double adx2[kU], bdx[kU], cc[kU], qy[kU];
            float4 fs[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const double4 qq = s_q[js[u]];
                cc[u] = s_c[js[u]];
                fs[u] = s_f[js[u]];
                const double dx = qq.x - fpx;
                adx2[u] = (qq.z * dx) * dx;
                bdx[u] = qq.w * dx;
                qy[u] = qq.y;
            }
            // alpha and the skip test without branches; one branch around the
            // (mostly skipped) accumulation
#pragma unroll
            for (int p = 0; p < PPT; ++p) {
                float alpha[kU], G[kU];
                bool ok[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) ok[u] = splat_alpha(adx2[u], bdx[u], cc[u], qy[u] - fpy[p], fs[u].x, alpha[u], G[u]);
#pragma unroll
                for (int u = 0; u < kU; ++u)
                    if (has[u] && ok[u] && !done[p]) accumulate(p, js[u], alpha[u], fs[u]);
            }
            }
        }
    }

    const int64_t npix = (int64_t)width * height;
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const int py = py0 + p;
        if (px < width && py < height) {
            const int64_t pix = (int64_t)py * width + px;
            if (out_T) out_T[pix] = T[p];
            if (out_ncontrib) out_ncontrib[pix] = last[p];
            out_rgb[pix] = fmaf(T[p], bg0, C0[p]);
            out_rgb[npix + pix] = fmaf(T[p], bg1, C1[p]);
            out_rgb[2 * npix + pix] = fmaf(T[p], bg2, C2[p]);
            if constexpr (kDepth) out_invdepth[pix] = D[p];
        }
    }
}

template <int PPT, bool kDepth, int kU = 2>
__global__ __launch_bounds__(256 / PPT) void k_blend(BlendArgs a, uint32_t per_xcd) {
    __shared__ double4 s_q[kBatch];
    __shared__ double s_c[kBatch];
    __shared__ float4 s_f[kBatch];
    __shared__ uint32_t s_b[kBatch];
    __shared__ float s_d[kDepth ? kBatch : 1];
    const uint32_t tile = xcd_band(blockIdx.x, per_xcd);
    if (tile >= (uint32_t)(a.tiles_x * a.tiles_y)) return;  // whole block: padding
    const int tx = (int)(tile % (uint32_t)a.tiles_x), ty = (int)(tile / (uint32_t)a.tiles_x);
    blend_tile<PPT, kDepth, kU>(tx, ty, a.width, a.height, a.ranges[tile], a.point_list, a.n, a.err, a.mean2d,
                            a.conic_opacity,
                            a.rgb, a.bg[0], a.bg[1], a.bg[2], a.out_rgb, a.out_T, a.out_ncontrib, s_q, s_c, s_f,
                            s_b, a.depth_bits, a.out_invdepth, s_d);
}

// Work-stealing blend (the load-balanced variant): one tile's time is
// nearly the same everywhere, but 4096 tiles fill a chip of ~2300 resident
// workgroups about 1.8 times, so a per-tile grid leaves much of the chip idle
// in its last wave.  Here every wave takes half tiles (16 x 8 pixels, two
// vertically adjacent pixels per lane, as a wave of the PPT = 2 tile kernel)
// from one counter until none is left, with its own LDS staging area and no
// workgroup barrier.  Each pixel sees the same splats in the same order
// through the same arithmetic as in the tile kernels, so the output is the
// same bit for bit.
constexpr int kWaveBatch = 128;  // splats staged per wave and batch

template <int PPT, bool kDepth>
__device__ __forceinline__ void blend_half_tile(const BlendArgs& a, uint32_t tile, uint32_t half, double4* s_q,
                                                double* s_c, float4* s_f, uint32_t* s_b, float* s_d) {
    constexpr int kRows = kWave / kTile * PPT;  // rows of the tile this wave blends
    const uint32_t lane = lane_id();
    const int tx = (int)(tile % (uint32_t)a.tiles_x), ty = (int)(tile / (uint32_t)a.tiles_x);
    const int wr0 = (int)half * kRows;  // first tile row of this half
    const int px = tx * kTile + (int)(lane & 15u);
    const int py0 = ty * kTile + wr0 + (int)(lane >> 4) * PPT;
    const double fpx = (double)px;
    const uint2 range = a.ranges[tile];

    float T[PPT], C0[PPT], C1[PPT], C2[PPT], D[PPT];
    double fpy[PPT];
    uint32_t last[PPT];
    bool done[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        T[p] = 1.0f;
        C0[p] = C1[p] = C2[p] = D[p] = 0.0f;
        last[p] = 0;
        fpy[p] = (double)(py0 + p);
        done[p] = !(px < a.width && py0 + p < a.height);
    }
    const int todo = (int)(range.y - range.x);
    for (int base = 0; base < todo; base += kWaveBatch) {
        int alive = 0;
#pragma unroll
        for (int p = 0; p < PPT; ++p) alive |= done[p] ? 0 : 1;
        if (!__any(alive)) break;  // wave-uniform
        wave_lds_sync();           // the previous batch has been read
        for (int k = (int)lane; k < kWaveBatch; k += kWave) {
            const int idx = base + k;
            if (idx < todo) {
                const uint32_t id = splat_id(a.point_list[range.x + idx], a.n, a.err);
                stage_splat(a.mean2d, a.conic_opacity, a.rgb, id, s_q, s_c, s_f, s_b, k, tx * kTile, ty * kTile);
                if constexpr (kDepth) s_d[k] = 1.0f / __uint_as_float(a.depth_bits[id]);
            }
        }
        wave_lds_sync();
        const int cnt = min(kWaveBatch, todo - base);
        uint64_t cand[kWaveBatch / kWave];
#pragma unroll
        for (int q = 0; q < kWaveBatch / kWave; ++q) {
            const int k = q * kWave + (int)lane;
            cand[q] = ballot(k < cnt && box_meets_rows(s_b[k], wr0, wr0 + kRows - 1));
        }
        int visited = 0;
        bool wave_done = false;
        for (int q = 0; q < kWaveBatch / kWave && !wave_done; ++q) {
            uint64_t m = cand[q];
            while (m) {
                const int j = q * kWave + __builtin_ctzll(m);
                m &= m - 1;
                if ((visited++ & 31) == 0) {
                    int live = 0;
#pragma unroll
                    for (int p = 0; p < PPT; ++p) live |= done[p] ? 0 : 1;
                    if (!__any(live)) {
                        wave_done = true;
                        break;
                    }
                }
                const double4 qq = s_q[j];
                const double c2 = s_c[j];
                const float4 f = s_f[j];
                const double dx = qq.x - fpx;
                const double adx2 = (qq.z * dx) * dx;
                const double bdx = qq.w * dx;
#pragma unroll
                for (int p = 0; p < PPT; ++p) {
                    float alpha, G;
                    const bool hit = splat_alpha(adx2, bdx, c2, qq.y - fpy[p], f.x, alpha, G) && !done[p];
                    if (hit) {
                        const float test_T = T[p] * (1.0f - alpha);
                        if (test_T < kTMin) {
                            done[p] = true;
                        } else {
                            const float wgt = alpha * T[p];
                            C0[p] = fmaf(f.y, wgt, C0[p]);
                            C1[p] = fmaf(f.z, wgt, C1[p]);
                            C2[p] = fmaf(f.w, wgt, C2[p]);
                            if constexpr (kDepth) D[p] = fmaf(s_d[j], wgt, D[p]);
                            T[p] = test_T;
                            last[p] = (uint32_t)(base + j + 1);
                        }
                    }
                }
            }
        }
    }
    const int64_t npix = (int64_t)a.width * a.height;
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const int py = py0 + p;
        if (px < a.width && py < a.height) {
            const int64_t pix = (int64_t)py * a.width + px;
            if (a.out_T) a.out_T[pix] = T[p];
            if (a.out_ncontrib) a.out_ncontrib[pix] = last[p];
            a.out_rgb[pix] = fmaf(T[p], a.bg[0], C0[p]);
            a.out_rgb[npix + pix] = fmaf(T[p], a.bg[1], C1[p]);
            a.out_rgb[2 * npix + pix] = fmaf(T[p], a.bg[2], C2[p]);
            if constexpr (kDepth) a.out_invdepth[pix] = D[p];
        }
    }
}

template <int PPT, bool kDepth>
__global__ __launch_bounds__(128) void k_blend_steal(BlendArgs a, uint32_t* counter, uint32_t units) {
    constexpr uint32_t kParts = kTile / (kWave / kTile * PPT);  // wave units per tile
    constexpr int kW = 128 / kWave;
    __shared__ double4 s_q[kW][kWaveBatch];
    __shared__ double s_c[kW][kWaveBatch];
    __shared__ float4 s_f[kW][kWaveBatch];
    __shared__ uint32_t s_b[kW][kWaveBatch];
    __shared__ float s_d[kW][kDepth ? kWaveBatch : 1];
    const int w = threadIdx.x / kWave;
    for (;;) {  // every wave leaves once the counter passes the last half tile
        uint32_t u = 0;
        if (lane_id() == 0) u = atomicAdd(counter, 1u);
        u = (uint32_t)__builtin_amdgcn_readfirstlane((int)u);
        if (u >= units) break;
        blend_half_tile<PPT, kDepth>(a, u / kParts, u % kParts, s_q[w], s_c[w], s_f[w], s_b[w], s_d[w]);
    }
}

// Persistent blend over every tile of a batch of renders: each workgroup
// takes the next global tile id from an atomic counter until none is left
// (every wave reaches the exit), finds the owning request by binary search
// over the tile bases, and blends that tile (its range found by global or
// stacked tile id, as the item says).
template <int PPT>
__global__ __launch_bounds__(256 / PPT) void k_blend_batch(const BatchItem* __restrict__ items, int nitems,
                                                           int64_t total_tiles, const uint2* __restrict__ ranges,
                                                           const uint32_t* __restrict__ point_list, int64_t n,
                                                           const float2* __restrict__ mean2d,
                                                           const float4* __restrict__ conic_opacity,
                                                           const float4* __restrict__ rgb, uint32_t* counter,
                                                           uint32_t* err) {
    __shared__ double4 s_q[kBatch];
    __shared__ double s_c[kBatch];
    __shared__ float4 s_f[kBatch];
    __shared__ uint32_t s_b[kBatch];
    __shared__ uint32_t s_tile;
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t g = s_tile;
        __syncthreads();  // every thread has read s_tile before it is overwritten
        if ((int64_t)g >= total_tiles) break;
        const int r = find_item_by_tile(items, nitems, g);
        const BatchItem& it = items[r];
        const uint32_t local = g - (uint32_t)it.tile_base;
        const int tx = (int)(local % (uint32_t)it.P.tiles_x), ty = (int)(local / (uint32_t)it.P.tiles_x);
        // ranges by global tile id, or by stacked tile id (row-wise placement)
        const int64_t rt = it.rec_stride > 0 ? it.rec_base + (int64_t)ty * it.rec_stride + tx : (int64_t)g;
        blend_tile<PPT>(tx, ty, it.P.width, it.P.height, ranges[rt], point_list, n, err, mean2d, conic_opacity, rgb,
                        it.bg[0], it.bg[1], it.bg[2], it.out_rgb, it.out_T, it.out_ncontrib, s_q, s_c, s_f, s_b);
    }
}

// Backward: each pixel walks its list from its last blended splat down to
// the first, recovering the transmittance before each splat by division
// (T_i = T_{i+1} / (1 - alpha_i)) from the stored final T, and carrying the
// colour S_i composited behind splat i (background included):
//   dL/drgb_i  = alpha_i T_i dL/dC
//   dL/dalpha_i = T_i (rgb_i - S_i) . dL/dC,   S_{i-1} = alpha_i rgb_i + (1 - alpha_i) S_i
// alpha = min(0.99, o G): when unclamped dalpha/do = G and dalpha/dpower = alpha.
// Per-splat sums over the wave are reduced with cross-lane shuffles and
// added to the per-Gaussian 2D gradient sums ([n][kGrad2d]) with atomics.  A wave
// visits only the splats whose box meets its pixels (as in the forward
// pass): the others contribute nothing.
template <int PPT, bool kDepth>
__global__ __launch_bounds__(256 / PPT) void k_blend_bwd(BlendBwdArgs a, uint32_t per_xcd) {
    constexpr int NT = 256 / PPT;
    constexpr int kRowsPerWave = kWave / kTile * PPT;
    __shared__ double4 s_q[kBwdBatch];
    __shared__ double s_c[kBwdBatch];
    __shared__ float4 s_f[kBwdBatch];
    __shared__ uint32_t s_b[kBwdBatch];
    __shared__ uint32_t s_id[kBwdBatch];
    __shared__ float s_d[kDepth ? kBwdBatch : 1];
    __shared__ uint32_t s_max;

    const uint32_t tile = xcd_band(blockIdx.x, per_xcd);
    if (tile >= (uint32_t)(a.tiles_x * a.tiles_y)) return;
    const int t = threadIdx.x;
    const int tx = (int)(tile % (uint32_t)a.tiles_x), ty = (int)(tile / (uint32_t)a.tiles_x);
    const int px = tx * kTile + (t & 15);
    const int py0 = ty * kTile + (t >> 4) * PPT;
    const double fpx = (double)px;
    const int64_t npix = (int64_t)a.width * a.height;
    const int wr0 = (t / kWave) * kRowsPerWave;  // this wave's first tile row

    float T[PPT], S0[PPT], S1[PPT], S2[PPT], D0[PPT], D1[PPT], D2[PPT], Sd[PPT], Dd[PPT];
    double fpy[PPT];
    uint32_t last[PPT];
    uint32_t mylast = 0;
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const int py = py0 + p;
        fpy[p] = (double)py;
        S0[p] = a.bg[0];
        S1[p] = a.bg[1];
        S2[p] = a.bg[2];
        Sd[p] = 0.0f;  // inverse depth behind: no background term
        if (px < a.width && py < a.height) {
            const int64_t pix = (int64_t)py * a.width + px;
            T[p] = a.final_T[pix];
            last[p] = a.ncontrib[pix];
            D0[p] = a.dL_drgb[pix];
            D1[p] = a.dL_drgb[npix + pix];
            D2[p] = a.dL_drgb[2 * npix + pix];
            Dd[p] = kDepth ? a.dL_dinvdepth[pix] : 0.0f;
        } else {
            T[p] = 1.0f;
            last[p] = 0;
            D0[p] = D1[p] = D2[p] = Dd[p] = 0.0f;
        }
        mylast = last[p] > mylast ? last[p] : mylast;
    }
    if (t == 0) s_max = 0;
    __syncthreads();
    mylast = wave_max(mylast);
    if (lane_id() == 0) atomicMax(&s_max, mylast);
    __syncthreads();
    const uint2 range = a.ranges[tile];
    // n_contrib can never exceed the tile's list length; clamp so a stale or
    // foreign n_contrib cannot walk past the list
    const uint32_t len = range.y - range.x;
    const int maxlast = (int)(s_max < len ? s_max : len);
    const int64_t n = a.n;
    for (int end = maxlast; end > 0; end -= kBwdBatch) {
        const int begin = end - kBwdBatch > 0 ? end - kBwdBatch : 0;
        __syncthreads();  // the previous batch is fully consumed
        for (int k = t; k < end - begin; k += NT) {
            const uint32_t id = splat_id(a.point_list[range.x + begin + k], a.n, a.err);
            s_id[k] = id;
            stage_splat(a.mean2d, a.conic_opacity, a.rgb, id, s_q, s_c, s_f, s_b, k, tx * kTile, ty * kTile);
            if constexpr (kDepth) s_d[k] = 1.0f / __uint_as_float(a.depth_bits[id]);
        }
        __syncthreads();
        const int cnt = end - begin;
        uint64_t cand[kBwdBatch / kWave];
#pragma unroll
        for (int qd = 0; qd < kBwdBatch / kWave; ++qd) {
            const int k = qd * kWave + (int)lane_id();
            // past this wave's last contributor no pixel of the wave can hit
            cand[qd] = ballot(k < cnt && (uint32_t)(begin + k) < mylast &&
                              box_meets_rows(s_b[k], wr0, wr0 + kRowsPerWave - 1));
        }
        for (int qd = kBwdBatch / kWave - 1; qd >= 0; --qd) {
            uint64_t m = cand[qd];
            while (m) {  // back to front
            const int bit = 63 - __builtin_clzll(m);
            m &= ~(1ull << bit);
            const int k = qd * kWave + bit;
            const int j = begin + k;
            const double4 q = s_q[k];
            const double c2 = s_c[k];
            const float4 f = s_f[k];
            const double dx = q.x - fpx;
            const double adx2 = (q.z * dx) * dx;
            const double bdx = q.w * dx;
            const float invd = kDepth ? s_d[k] : 0.0f;
            // Per-lane sums over the lane's pixels (one column, so dx is
            // common): sp = sum dL/dpower, spy and spyy its dy and dy^2
            // moments; the mean and conic gradients are linear in these and
            // dx (kGrad2d).  A pixel the splat does not
            // reach takes alpha = 0, which leaves T and the colours behind it
            // unchanged and makes every term zero, so no pixel branches.
            float sp = 0.f, spy = 0.f, spyy = 0.f, go = 0.f, gr = 0.f, gg = 0.f, gb = 0.f, gd = 0.f;
            bool any = false;
#pragma unroll
            for (int p = 0; p < PPT; ++p) {
                const double dy = q.y - fpy[p];
                float alpha, G;
                const bool hit = splat_alpha(adx2, bdx, c2, dy, f.x, alpha, G) && (uint32_t)j < last[p];
                any |= hit;
                const float al = hit ? alpha : 0.0f;
                const float one_m = 1.0f - al;
                const float Tr = T[p] * __builtin_amdgcn_rcpf(one_m);  // 1 ulp; alpha <= 0.99
                T[p] = hit ? Tr : T[p];
                const float Tp = T[p];
                float dLda = Tp * ((f.y - S0[p]) * D0[p] + (f.z - S1[p]) * D1[p] +
                                   (f.w - S2[p]) * D2[p]);
                S0[p] = al * f.y + one_m * S0[p];
                S1[p] = al * f.z + one_m * S1[p];
                S2[p] = al * f.w + one_m * S2[p];
                const float wgt = al * Tp;
                // the first pixel starts each sum (no addition to zero)
                auto acc = [p](float& s, float v) { s = p == 0 ? v : s + v; };
                acc(gr, wgt * D0[p]);
                acc(gg, wgt * D1[p]);
                acc(gb, wgt * D2[p]);
                if constexpr (kDepth) {
                    dLda += Tp * (invd - Sd[p]) * Dd[p];
                    Sd[p] = al * invd + one_m * Sd[p];
                    acc(gd, wgt * Dd[p]);
                }
                const bool unclamped = hit && !(f.x * G > kAlphaMax);
                acc(go, unclamped ? dLda * G : 0.0f);
                const float dLdp = unclamped ? dLda * alpha : 0.0f;
                const float dyf = (float)dy;
                const float e = dLdp * dyf;
                acc(sp, dLdp);
                acc(spy, e);
                acc(spyy, e * dyf);
            }
            if (__any(any)) {
                // nine (ten) wave sums: eight scattered over lane groups, the
                // rest full; each Gaussian's sums are contiguous, so a single
                // atomic instruction adds them all (lanes 8i: sum i, lane 1:
                // sum 8, lane 2: sum 9).  One instruction rather than two per
                // visit matters: the second, single-lane one cost 0.2 of the
                // kernel's time.
                const float dxf = (float)dx;
                const float spx = sp * dxf;
                const float v8[8] = {spx, spy, spx * dxf, spy * dxf, spyy, go, gr, gg};
                const float s8 = wave_reduce_scatter8(v8);
                const float sb = wave_sum_dpp(gb);
                const uint32_t l = lane_id();
                float v = s8;
                uint32_t slot = l >> 3;
                if (l == 1) {
                    v = sb;
                    slot = 8;
                }
                if constexpr (kDepth) {
                    const float sd = wave_sum_dpp(gd);
                    if (l == 2) {
                        v = sd;
                        slot = 9;
                    }
                }
                if ((l & 7u) == 0 || l == 1 || (kDepth && l == 2))
                    atomicAdd(a.grad2d + (size_t)s_id[k] * kGrad2d + slot, v);
            }
            }
        }
    }
}

constexpr int kLossBlocks = 1024;

// dL/drgb of the mean absolute error, and per-block partial sums of |rgb - target|.
__global__ __launch_bounds__(256) void k_l1_loss_grad(const float* __restrict__ rgb,
                                                      const float* __restrict__ target, int64_t count,
                                                      float* __restrict__ grad, float* __restrict__ partial) {
    __shared__ float s_w[256 / kWave];
    float acc = 0.0f;
    const float inv = 1.0f / (float)count;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float d = rgb[i] - target[i];
        grad[i] = d > 0.0f ? inv : (d < 0.0f ? -inv : 0.0f);
        acc += fabsf(d);
    }
    if (partial) {
        acc = wave_sum(acc);
        if (lane_id() == 0) s_w[threadIdx.x / kWave] = acc;
        __syncthreads();
        if (threadIdx.x == 0) partial[blockIdx.x] = (s_w[0] + s_w[1]) + (s_w[2] + s_w[3]);
    }
}

// loss = (sum of the partials, in a fixed order) / count: deterministic.
__global__ __launch_bounds__(kLossBlocks) void k_l1_loss_finish(const float* __restrict__ partial, int nparts,
                                                                int64_t count, float* __restrict__ loss) {
    __shared__ float s_w[kLossBlocks / kWave];
    float v = (int)threadIdx.x < nparts ? partial[threadIdx.x] : 0.0f;
    v = wave_sum(v);
    if (lane_id() == 0) s_w[threadIdx.x / kWave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.0f;
        for (int k = 0; k < kLossBlocks / kWave; ++k) t += s_w[k];
        *loss = t / (float)count;
    }
}

}  // namespace

static uint32_t xcd_per(int64_t tiles) { return (uint32_t)((tiles + 7) / 8); }

// Compute units of the current device (cached per device).
int device_cus() {
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int c = cache[dev].load(std::memory_order_relaxed);
    if (c <= 0) {
        c = 256;
        (void)hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev);
        cache[dev].store(c, std::memory_order_relaxed);
    }
    return c;
}

hipError_t launch_blend(const BlendArgs& a, int variant, hipStream_t stream) {
    const int64_t tiles = (int64_t)a.tiles_x * a.tiles_y;
    if (tiles == 0) return hipSuccess;
    if (!a.err) return hipErrorInvalidValue;
    // default: two pixels per lane (two waves per tile) once the tiles give
    // every SIMD several waves; fewer tiles (below ten per CU) run one pixel
    // per lane, four waves per tile
    if (variant == 0) variant = tiles < 10 * (int64_t)device_cus() ? 1 : 2;
    const uint32_t per = xcd_per(tiles);
    const dim3 grid(8 * per);
    const bool depth = a.out_invdepth != nullptr;
    if (depth && !a.depth_bits) return hipErrorInvalidValue;
    if (variant == 3 || variant == 5) {
        if (!a.counter) return hipErrorInvalidValue;
        hipError_t e = launch_fill_u32(a.counter, 1, 0u, stream);
        if (e != hipSuccess) return e;
        const uint32_t units = (uint32_t)((variant == 3 ? 2 : 1) * tiles);
        const int cus = device_cus();
        // at most as many workgroups (two waves each) as fit, all of them busy
        const int64_t g = std::min<int64_t>((int64_t)(units + 1) / 2, (int64_t)cus * 12);
        if (variant == 3) {
            if (depth)
                hipLaunchKernelGGL((k_blend_steal<2, true>), dim3((unsigned)g), dim3(128), 0, stream, a, a.counter,
                                   units);
            else
                hipLaunchKernelGGL((k_blend_steal<2, false>), dim3((unsigned)g), dim3(128), 0, stream, a, a.counter,
                                   units);
        } else {
            if (depth)
                hipLaunchKernelGGL((k_blend_steal<4, true>), dim3((unsigned)g), dim3(128), 0, stream, a, a.counter,
                                   units);
            else
                hipLaunchKernelGGL((k_blend_steal<4, false>), dim3((unsigned)g), dim3(128), 0, stream, a, a.counter,
                                   units);
        }
        return hipGetLastError();
    }
    switch (variant) {
        case 1:
            // with fewer tiles than four per compute unit a wave has its SIMD
            // to itself: four candidates per step hide more of its latency
            if (tiles < 4 * (int64_t)device_cus()) {
                if (depth) hipLaunchKernelGGL((k_blend<1, true, 4>), grid, dim3(256), 0, stream, a, per);
                else hipLaunchKernelGGL((k_blend<1, false, 4>), grid, dim3(256), 0, stream, a, per);
            } else {
                if (depth) hipLaunchKernelGGL((k_blend<1, true>), grid, dim3(256), 0, stream, a, per);
                else hipLaunchKernelGGL((k_blend<1, false>), grid, dim3(256), 0, stream, a, per);
            }
            break;
        case 4:
            if (depth) hipLaunchKernelGGL((k_blend<4, true>), grid, dim3(64), 0, stream, a, per);
            else hipLaunchKernelGGL((k_blend<4, false>), grid, dim3(64), 0, stream, a, per);
            break;
        default:
            if (depth) hipLaunchKernelGGL((k_blend<2, true>), grid, dim3(128), 0, stream, a, per);
            else hipLaunchKernelGGL((k_blend<2, false>), grid, dim3(128), 0, stream, a, per);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_blend_batch(const BatchItem* items, int nitems, int64_t total_tiles, const uint2* ranges,
                              const uint32_t* point_list, int64_t n, const float2* mean2d,
                              const float4* conic_opacity, const float4* rgb, uint32_t* counter, int grid,
                              uint32_t* err, hipStream_t stream) {
    if (total_tiles == 0) return hipSuccess;
    if (!err) return hipErrorInvalidValue;
    hipError_t e = launch_fill_u32(counter, 1, 0u, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_blend_batch<2>, dim3((unsigned)grid), dim3(128), 0, stream, items, nitems, total_tiles,
                       ranges, point_list, n, mean2d, conic_opacity, rgb, counter, err);
    return hipGetLastError();
}

hipError_t launch_blend_backward(const BlendBwdArgs& a, hipStream_t stream) {
    const int64_t tiles = (int64_t)a.tiles_x * a.tiles_y;
    if (tiles == 0) return hipSuccess;
    if (!a.err) return hipErrorInvalidValue;
    const uint32_t per = xcd_per(tiles);
    if (a.dL_dinvdepth) {
        if (!a.depth_bits) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_blend_bwd<2, true>), dim3(8 * per), dim3(128), 0, stream, a, per);
    } else {
        hipLaunchKernelGGL((k_blend_bwd<2, false>), dim3(8 * per), dim3(128), 0, stream, a, per);
    }
    return hipGetLastError();
}

hipError_t launch_l1_loss_grad(const float* rgb, const float* target, int64_t count, float* grad,
                               float* loss, float* partial, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > kLossBlocks) blocks = kLossBlocks;
    hipLaunchKernelGGL(k_l1_loss_grad, dim3((unsigned)blocks), dim3(256), 0, stream, rgb, target, count, grad,
                       loss ? partial : nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !loss) return e;
    hipLaunchKernelGGL(k_l1_loss_finish, dim3(1), dim3(kLossBlocks), 0, stream, partial, (int)blocks, count, loss);
    return hipGetLastError();
}

}  // namespace cds
