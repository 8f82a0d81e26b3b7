// Per-Gaussian preprocessing (paper Section II-B(1)): visibility, projection
// of each 3D Gaussian to a 2D splat (mean, conic, screen radius, covered tile
// rectangle), depth, and colour from spherical harmonics (degree <= 3).
//
// The geometry runs in float64: it decides the discrete outputs (near cull,
// radius, covered tiles, depth-key bits), and float64 is what makes those
// decisions reproducible by an independent implementation.  The kernel reads
// ~236 B and writes ~61 B per Gaussian, so the float64 arithmetic (full rate
// on CDNA4 vector units) stays below the HBM time.  Colour is float32.
//
// Loads are coalesced structure-of-arrays planes, one Gaussian per lane.
#include "device_utils.h"
#include "internal.h"

namespace cds {
namespace {

// Real spherical-harmonics normalisation constants (orthonormal basis with
// the Condon-Shortley phase), written from their closed forms:
// 1/(2 sqrt(pi)), sqrt(3/(4 pi)), sqrt(15/(4 pi)), sqrt(5/(16 pi)),
// sqrt(15/(16 pi)), sqrt(35/(32 pi)), sqrt(105/(4 pi)), sqrt(21/(32 pi)),
// sqrt(7/(16 pi)), sqrt(105/(16 pi)).
constexpr float kY00 = 0.28209479177387814f;
constexpr float kY1 = 0.48860251190291992f;
constexpr float kY2a = 1.0925484305920792f;
constexpr float kY2b = 0.31539156525252005f;
constexpr float kY2c = 0.54627421529603959f;
constexpr float kY3a = 0.59004358992664352f;
constexpr float kY3b = 2.8906114426405538f;
constexpr float kY3c = 0.45704579946446572f;
constexpr float kY3d = 0.3731763325901154f;
constexpr float kY3e = 1.4453057213202769f;

__device__ __forceinline__ void sh_basis_f32(float x, float y, float z, int degree, float b[16]) {
    b[0] = kY00;
    if (degree < 1) return;
    b[1] = -kY1 * y;
    b[2] = kY1 * z;
    b[3] = -kY1 * x;
    if (degree < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    b[4] = kY2a * (x * y);
    b[5] = -kY2a * (y * z);
    b[6] = kY2b * (2.0f * zz - xx - yy);
    b[7] = -kY2a * (x * z);
    b[8] = kY2c * (xx - yy);
    if (degree < 3) return;
    b[9] = -kY3a * y * (3.0f * xx - yy);
    b[10] = kY3b * (x * y) * z;
    b[11] = -kY3c * y * (4.0f * zz - xx - yy);
    b[12] = kY3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
    b[13] = -kY3c * x * (4.0f * zz - xx - yy);
    b[14] = kY3e * z * (xx - yy);
    b[15] = -kY3a * x * (xx - 3.0f * yy);
}

// colour = sum_k basis[k] sh[k] over the kNB coefficients, each channel
// accumulated in coefficient order; all coefficient loads are issued before
// the first product.  With J (a render kept for the backward pass), also the
// colour's derivative with respect to the unit view direction (x, y, z):
// J[3 ch + c] = sum_k sh[k][ch] dY_k/ddir_c, from the derivatives of the
// basis polynomials above.
template <int kNB, bool kJac>
__device__ __forceinline__ void sh_colour(const float* __restrict__ sh, int64_t n, int64_t i, const float* basis,
                                          float col[3], float x, float y, float z, float (&J)[9]) {
    float v[kNB][3];
#pragma unroll
    for (int k = 0; k < kNB; ++k)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) v[k][ch] = __builtin_nontemporal_load(&sh[((int64_t)k * 3 + ch) * n + i]);
#pragma unroll
    for (int e = 0; e < 9; ++e) J[e] = 0.0f;
    const float xx = x * x, yy = y * y, zz = z * z;
    // coefficient k's term d * dY_k/ddir_c, every channel
    const auto add = [&](int k, int c, float d) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) J[3 * ch + c] += v[k][ch] * d;
    };
    // one pass over the coefficients, each used once for the colour and
    // once for the derivative, so none has to stay live (or be loaded again)
#pragma unroll
    for (int k = 0; k < kNB; ++k) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) col[ch] += basis[k] * v[k][ch];
        if constexpr (!kJac) continue;
        switch (k) {
            case 1: add(1, 1, -kY1); break;
            case 2: add(2, 2, kY1); break;
            case 3: add(3, 0, -kY1); break;
            case 4: add(4, 0, kY2a * y); add(4, 1, kY2a * x); break;
            case 5: add(5, 1, -kY2a * z); add(5, 2, -kY2a * y); break;
            case 6:
                add(6, 0, -2.0f * kY2b * x); add(6, 1, -2.0f * kY2b * y); add(6, 2, 4.0f * kY2b * z);
                break;
            case 7: add(7, 0, -kY2a * z); add(7, 2, -kY2a * x); break;
            case 8: add(8, 0, 2.0f * kY2c * x); add(8, 1, -2.0f * kY2c * y); break;
            case 9: add(9, 0, -6.0f * kY3a * x * y); add(9, 1, -3.0f * kY3a * (xx - yy)); break;
            case 10: add(10, 0, kY3b * y * z); add(10, 1, kY3b * x * z); add(10, 2, kY3b * x * y); break;
            case 11:
                add(11, 0, 2.0f * kY3c * x * y); add(11, 1, -kY3c * (4.0f * zz - xx - 3.0f * yy));
                add(11, 2, -8.0f * kY3c * y * z);
                break;
            case 12:
                add(12, 0, -6.0f * kY3d * x * z); add(12, 1, -6.0f * kY3d * y * z);
                add(12, 2, kY3d * (6.0f * zz - 3.0f * xx - 3.0f * yy));
                break;
            case 13:
                add(13, 0, -kY3c * (4.0f * zz - 3.0f * xx - yy)); add(13, 1, 2.0f * kY3c * x * y);
                add(13, 2, -8.0f * kY3c * x * z);
                break;
            case 14:
                add(14, 0, 2.0f * kY3e * x * z); add(14, 1, -2.0f * kY3e * y * z); add(14, 2, kY3e * (xx - yy));
                break;
            case 15: add(15, 0, -3.0f * kY3a * (xx - yy)); add(15, 1, 6.0f * kY3a * x * y); break;
            default: break;
        }
    }
}

// Gaussian i of a scene with P.n Gaussians; outputs go to slot `o` of O
// (with kJac also the colour's direction derivative, planes O.jac[9][n]).
// Returns (tiles touched, rectangle height in tiles), both 0 when culled.
template <bool kJac = false>
__device__ __forceinline__ uint2 preprocess_one(const ProjParams& P, const SceneParams& S, int64_t i,
                                               const SplatBuffers& O, int64_t o) {
    const int64_t n = P.n;

    // The scene's parameters are read once per render: non-temporal loads, so
    // that they do not displace this render's intermediate arrays from the
    // last-level cache.
    const double m0 = __builtin_nontemporal_load(&S.means[i]), m1 = __builtin_nontemporal_load(&S.means[n + i]),
                 m2 = __builtin_nontemporal_load(&S.means[2 * n + i]);
    // the other per-Gaussian inputs load with the means (one memory latency);
    // a line holds culled and visible Gaussians alike
    const float ls0 = __builtin_nontemporal_load(&S.log_scales[i]), ls1 = __builtin_nontemporal_load(&S.log_scales[n + i]),
                ls2 = __builtin_nontemporal_load(&S.log_scales[2 * n + i]);
    const float q0 = __builtin_nontemporal_load(&S.quats[i]), q1 = __builtin_nontemporal_load(&S.quats[n + i]),
                q2 = __builtin_nontemporal_load(&S.quats[2 * n + i]), q3 = __builtin_nontemporal_load(&S.quats[3 * n + i]);
    const float olog = __builtin_nontemporal_load(&S.opacity_logits[i]);
    const double tx = P.R[0] * m0 + P.R[1] * m1 + P.R[2] * m2 + P.t[0];
    const double ty = P.R[3] * m0 + P.R[4] * m1 + P.R[5] * m2 + P.t[1];
    const double tz = P.R[6] * m0 + P.R[7] * m1 + P.R[8] * m2 + P.t[2];

    bool visible = tz > P.near_plane;
    double A = 0, B = 0, C = 0, mx = 0, my = 0;
    int radius = 0;
    uint32_t tx0 = 0, ty0 = 0, tx1 = 0, ty1 = 0;
    uint8_t flags = 0;
    float mxf = 0.f, myf = 0.f;

    if (visible) {
        // 3D covariance Sigma = Rq diag(s^2) Rq^T, s = exp(log_scale)
        const double s0 = exp(2.0 * (double)ls0);
        const double s1 = exp(2.0 * (double)ls1);
        const double s2 = exp(2.0 * (double)ls2);
        double qw = q0, qx = q1, qy = q2, qz = q3;
        const double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
        qw /= qn; qx /= qn; qy /= qn; qz /= qn;
        const double r00 = 1.0 - 2.0 * (qy * qy + qz * qz), r01 = 2.0 * (qx * qy - qw * qz),
                     r02 = 2.0 * (qx * qz + qw * qy);
        const double r10 = 2.0 * (qx * qy + qw * qz), r11 = 1.0 - 2.0 * (qx * qx + qz * qz),
                     r12 = 2.0 * (qy * qz - qw * qx);
        const double r20 = 2.0 * (qx * qz - qw * qy), r21 = 2.0 * (qy * qz + qw * qx),
                     r22 = 1.0 - 2.0 * (qx * qx + qy * qy);
        const double S00 = r00 * r00 * s0 + r01 * r01 * s1 + r02 * r02 * s2;
        const double S01 = r00 * r10 * s0 + r01 * r11 * s1 + r02 * r12 * s2;
        const double S02 = r00 * r20 * s0 + r01 * r21 * s1 + r02 * r22 * s2;
        const double S11 = r10 * r10 * s0 + r11 * r11 * s1 + r12 * r12 * s2;
        const double S12 = r10 * r20 * s0 + r11 * r21 * s1 + r12 * r22 * s2;
        const double S22 = r20 * r20 * s0 + r21 * r21 * s1 + r22 * r22 * s2;

        // EWA Jacobian of the perspective projection, ratios limited to the guard band
        double ux = tx / tz, uy = ty / tz;
        if (ux > P.limx) { ux = P.limx; flags |= 8; }
        if (ux < -P.limx) { ux = -P.limx; flags |= 8; }
        if (uy > P.limy) { uy = P.limy; flags |= 16; }
        if (uy < -P.limy) { uy = -P.limy; flags |= 16; }
        const double j00 = P.fx / tz, j02 = -P.fx * ux / tz;
        const double j11 = P.fy / tz, j12 = -P.fy * uy / tz;
        // M = J * Rcam (2 x 3)
        const double a0 = j00 * P.R[0] + j02 * P.R[6], a1 = j00 * P.R[1] + j02 * P.R[7],
                     a2 = j00 * P.R[2] + j02 * P.R[8];
        const double b0 = j11 * P.R[3] + j12 * P.R[6], b1 = j11 * P.R[4] + j12 * P.R[7],
                     b2 = j11 * P.R[5] + j12 * P.R[8];
        // v = Sigma M0^T, w = Sigma M1^T
        const double v0 = S00 * a0 + S01 * a1 + S02 * a2;
        const double v1 = S01 * a0 + S11 * a1 + S12 * a2;
        const double v2 = S02 * a0 + S12 * a1 + S22 * a2;
        const double w0 = S00 * b0 + S01 * b1 + S02 * b2;
        const double w1 = S01 * b0 + S11 * b1 + S12 * b2;
        const double w2 = S02 * b0 + S12 * b1 + S22 * b2;
        const double ca = a0 * v0 + a1 * v1 + a2 * v2 + 0.3;
        const double cb = b0 * v0 + b1 * v1 + b2 * v2;
        const double cc = b0 * w0 + b1 * w1 + b2 * w2 + 0.3;
        const double det = ca * cc - cb * cb;
        if (!(det > 0.0)) {
            visible = false;
        } else {
            A = cc / det;
            B = -cb / det;
            C = ca / det;
            const double mid = 0.5 * (ca + cc);
            const double disc = mid * mid - det;
            const double lam = mid + sqrt(disc > 0.1 ? disc : 0.1);
            const double rr = ceil(3.0 * sqrt(lam));
            mx = P.fx * tx / tz + P.cx;
            my = P.fy * ty / tz + P.cy;
            mxf = (float)mx;
            myf = (float)my;
            // covered pixels |p - mean| <= r per axis (mean as stored, float32)
            double lox = ceil((double)mxf - rr), hix = floor((double)mxf + rr);
            double loy = ceil((double)myf - rr), hiy = floor((double)myf + rr);
            lox = lox < 0.0 ? 0.0 : lox;
            loy = loy < 0.0 ? 0.0 : loy;
            hix = hix > P.width - 1 ? (double)(P.width - 1) : hix;
            hiy = hiy > P.height - 1 ? (double)(P.height - 1) : hiy;
            if (lox > hix || loy > hiy) {
                visible = false;
            } else {
                radius = rr > 2147483647.0 ? 2147483647 : (int)rr;
                tx0 = (uint32_t)lox / kTile; tx1 = (uint32_t)hix / kTile;
                ty0 = (uint32_t)loy / kTile; ty1 = (uint32_t)hiy / kTile;
            }
        }
    }

    if (!visible) {
        O.mean2d[o] = make_float2(0.f, 0.f);
        O.conic_opacity[o] = make_float4(0.f, 0.f, 0.f, 0.f);
        O.rgb[o] = make_float4(0.f, 0.f, 0.f, 0.f);
        O.depth_bits[o] = 0u;
        O.radius[o] = 0;
        O.rect[o] = make_uint2(0u, 0u);
        O.touched[o] = 0u;
        O.clamp_flags[o] = 0;
        return make_uint2(0u, 0u);
    }

    const float opacity = (float)(1.0 / (1.0 + exp(-(double)olog)));

    // colour: view direction from the camera centre, SH up to degree 3
    double dx = m0 - P.campos[0], dy = m1 - P.campos[1], dz = m2 - P.campos[2];
    const double dl = sqrt(dx * dx + dy * dy + dz * dz);
    float basis[16];
    const float ux = (float)(dx / dl), uy = (float)(dy / dl), uz = (float)(dz / dl);
    sh_basis_f32(ux, uy, uz, P.sh_degree, basis);
    float col[3] = {0.f, 0.f, 0.f};
    float J[9];
    switch (P.sh_degree) {  // uniform
        case 0: sh_colour<1, false>(S.sh, n, i, basis, col, ux, uy, uz, J); break;
        case 1: sh_colour<4, kJac>(S.sh, n, i, basis, col, ux, uy, uz, J); break;
        case 2: sh_colour<9, kJac>(S.sh, n, i, basis, col, ux, uy, uz, J); break;
        default: sh_colour<16, kJac>(S.sh, n, i, basis, col, ux, uy, uz, J); break;
    }
    if constexpr (kJac) {
        if (P.sh_degree > 0)  // uniform
#pragma unroll
            // read once, by the backward pass: non-temporal, like the other
            // write-once streams, so it leaves no dirty lines in the
            // last-level cache for the rest of the frame to write back
            for (int e = 0; e < 9; ++e) __builtin_nontemporal_store(J[e], &O.jac[(int64_t)e * n + o]);
    }
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        col[ch] += 0.5f;
        if (col[ch] < 0.0f) {
            col[ch] = 0.0f;
            flags |= (uint8_t)(1u << ch);
        }
    }

    const float dzf = (float)tz;
    O.mean2d[o] = make_float2(mxf, myf);
    O.conic_opacity[o] = make_float4((float)A, (float)B, (float)C, opacity);
    O.rgb[o] = make_float4(col[0], col[1], col[2], 0.f);
    O.depth_bits[o] = __float_as_uint(dzf);
    O.radius[o] = radius;
    O.rect[o] = make_uint2(tx0 | (ty0 << 16), tx1 | (ty1 << 16));
    const uint32_t touched = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
    O.touched[o] = touched;
    O.clamp_flags[o] = flags;
    return make_uint2(touched, ty1 - ty0 + 1);
}

template <bool kJac>
__global__ __launch_bounds__(256) void k_preprocess(ProjParams P, SceneParams S, SplatBuffers O) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    preprocess_one<kJac>(P, S, i, O, i);
}

// The same, and per workgroup of 256 Gaussians the number of visible splats,
// the sum of their tiles touched and of their rectangle heights (the inputs
// of the visible compaction's scan), and the clearing of C's word ranges.
template <bool kJac>
__global__ __launch_bounds__(256) void k_preprocess_counted(ProjParams P, SceneParams S, SplatBuffers O,
                                                            PreCounts C) {
    __shared__ uint32_t s_part[3][256 / kWave];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
    for (int j = 0; j < 1 + kZeroSpans; ++j)
        for (int64_t k = i; k < C.clear[j].n; k += (int64_t)gridDim.x * blockDim.x) C.clear[j].p[k] = 0u;
    uint2 r = make_uint2(0u, 0u);
    if (i < P.n) r = preprocess_one<kJac>(P, S, i, O, i);
    // a block's sums fit 32 bits (at most 256 splats of at most 2^24 tiles each)
    uint32_t v = r.x ? 1u : 0u, k = r.x, h = r.y;
    v = wave_sum_u32(v);
    k = wave_sum_u32(k);
    h = wave_sum_u32(h);
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) {
        s_part[0][w] = v;
        s_part[1][w] = k;
        s_part[2][w] = h;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        uint64_t t = 0;
#pragma unroll
        for (int q = 0; q < 256 / kWave; ++q) t += s_part[threadIdx.x][q];
        uint64_t* dst = threadIdx.x == 0 ? C.vis : threadIdx.x == 1 ? C.keys : C.h;
        if (dst) dst[(int64_t)(blockIdx.x % C.group) * C.stride + blockIdx.x / C.group] = t;
    }
}

// Several scenes at once: global index g over the concatenated scenes of a
// batch; each lane finds its scene by binary search over the item bases.
__global__ __launch_bounds__(256) void k_preprocess_batch(const BatchItem* __restrict__ items, int nitems,
                                                          int64_t total, SplatBuffers O) {
    const int64_t g0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t g = g0 + threadIdx.x;
    const int64_t glast = (g0 + blockDim.x < total ? g0 + blockDim.x : total) - 1;
    // a block almost always lies inside one item: then the item is looked up
    // once and, uniform, its parameters load as scalars
    const int r0 = find_item_by_gaussian(items, nitems, g0);
    if (r0 == find_item_by_gaussian(items, nitems, glast)) {  // uniform
        const int r = __builtin_amdgcn_readfirstlane(r0);
        if (g < total) preprocess_one(items[r].P, items[r].S, g - items[r].gauss_base, O, g);
    } else if (g < total) {
        const int r = find_item_by_gaussian(items, nitems, g);
        preprocess_one(items[r].P, items[r].S, g - items[r].gauss_base, O, g);
    }
}

}  // namespace

hipError_t launch_preprocess_batch(const BatchItem* items, int nitems, int64_t total, const SplatBuffers& out,
                                   hipStream_t stream) {
    if (total == 0) return hipSuccess;
    const int64_t nb = (total + 255) / 256;
    hipLaunchKernelGGL(k_preprocess_batch, dim3((unsigned)nb), dim3(256), 0, stream, items, nitems, total, out);
    return hipGetLastError();
}

hipError_t launch_preprocess_counted(const ProjParams& p, const SceneParams& s, const SplatBuffers& out,
                                     const PreCounts& c, hipStream_t stream) {
    const int64_t nb = preprocess_blocks(p.n);
    if (nb == 0) {  // nothing to count: only the clearing
        for (int j = 0; j < 1 + kZeroSpans; ++j) {
            const hipError_t e = launch_fill_u32(c.clear[j].p, c.clear[j].n, 0u, stream);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    if (out.jac && p.sh_degree > 0)
        hipLaunchKernelGGL(k_preprocess_counted<true>, dim3((unsigned)nb), dim3(256), 0, stream, p, s, out, c);
    else
        hipLaunchKernelGGL(k_preprocess_counted<false>, dim3((unsigned)nb), dim3(256), 0, stream, p, s, out, c);
    return hipGetLastError();
}

hipError_t launch_preprocess(const ProjParams& p, const SceneParams& s, const SplatBuffers& out,
                             hipStream_t stream) {
    if (p.n == 0) return hipSuccess;
    const int nt = 256;
    const int64_t nb = (p.n + nt - 1) / nt;
    if (out.jac && p.sh_degree > 0)
        hipLaunchKernelGGL(k_preprocess<true>, dim3((unsigned)nb), dim3(nt), 0, stream, p, s, out);
    else
        hipLaunchKernelGGL(k_preprocess<false>, dim3((unsigned)nb), dim3(nt), 0, stream, p, s, out);
    return hipGetLastError();
}

}  // namespace cds
