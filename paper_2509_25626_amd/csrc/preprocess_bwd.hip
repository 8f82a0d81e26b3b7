// Backward of the per-Gaussian preprocessing: from the gradients of the 2D
// splat quantities (mean, conic, opacity, colour) to the raw parameters
// (means, log-scales, quaternions, opacity logits, SH coefficients).  The
// projection is recomputed in float64 exactly as the forward computed it and
// every decision (culls, Jacobian guard band, colour clamp) is held fixed.
// One Gaussian per lane; structure-of-arrays loads and stores.
#include "device_utils.h"
#include "internal.h"

namespace cds {
namespace {

// Real SH basis (degree <= 3, orthonormal, Condon-Shortley phase), float64.
__device__ __forceinline__ void sh_basis64(double x, double y, double z, double Y[16]) {
    const double k0 = 0.28209479177387814, k1 = 0.48860251190291992, k2a = 1.0925484305920792,
                 k2b = 0.31539156525252005, k2c = 0.54627421529603959, k3a = 0.59004358992664352,
                 k3b = 2.8906114426405538, k3c = 0.45704579946446572, k3d = 0.3731763325901154,
                 k3e = 1.4453057213202769;
    const double xx = x * x, yy = y * y, zz = z * z;
    Y[0] = k0;
    Y[1] = -k1 * y; Y[2] = k1 * z; Y[3] = -k1 * x;
    Y[4] = k2a * x * y; Y[5] = -k2a * y * z; Y[6] = k2b * (2 * zz - xx - yy);
    Y[7] = -k2a * x * z; Y[8] = k2c * (xx - yy);
    Y[9] = -k3a * y * (3 * xx - yy); Y[10] = k3b * x * y * z; Y[11] = -k3c * y * (4 * zz - xx - yy);
    Y[12] = k3d * z * (2 * zz - 3 * xx - 3 * yy); Y[13] = -k3c * x * (4 * zz - xx - yy);
    Y[14] = k3e * z * (xx - yy); Y[15] = -k3a * x * (xx - 3 * yy);
}

// sum_k w_k grad Y_k (gradient with respect to the direction components), w_k = 0 beyond the degree.
__device__ __forceinline__ void sh_weighted_grad64(double x, double y, double z, const double w[16],
                                                   double g[3]) {
    const double k1 = 0.48860251190291992, k2a = 1.0925484305920792, k2b = 0.31539156525252005,
                 k2c = 0.54627421529603959, k3a = 0.59004358992664352, k3b = 2.8906114426405538,
                 k3c = 0.45704579946446572, k3d = 0.3731763325901154, k3e = 1.4453057213202769;
    const double xx = x * x, yy = y * y, zz = z * z;
    g[0] = -k1 * w[3] + k2a * y * w[4] - 2 * k2b * x * w[6] - k2a * z * w[7] + 2 * k2c * x * w[8]
           - 6 * k3a * x * y * w[9] + k3b * y * z * w[10] + 2 * k3c * x * y * w[11]
           - 6 * k3d * x * z * w[12] - k3c * (4 * zz - 3 * xx - yy) * w[13] + 2 * k3e * x * z * w[14]
           - 3 * k3a * (xx - yy) * w[15];
    g[1] = -k1 * w[1] + k2a * x * w[4] - k2a * z * w[5] - 2 * k2b * y * w[6] - 2 * k2c * y * w[8]
           - 3 * k3a * (xx - yy) * w[9] + k3b * x * z * w[10] - k3c * (4 * zz - xx - 3 * yy) * w[11]
           - 6 * k3d * y * z * w[12] + 2 * k3c * x * y * w[13] - 2 * k3e * y * z * w[14]
           + 6 * k3a * x * y * w[15];
    g[2] = k1 * w[2] - k2a * y * w[5] + 4 * k2b * z * w[6] - k2a * x * w[7] + k3b * x * y * w[10]
           - 8 * k3c * y * z * w[11] + k3d * (6 * zz - 3 * xx - 3 * yy) * w[12] - 8 * k3c * x * z * w[13]
           + k3e * (xx - yy) * w[14];
}

template <bool kJac>
__global__ __launch_bounds__(256) void k_preprocess_bwd(ProjParams P, SceneParams S, PreBwdArgs A) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    const int64_t n = P.n;
    const int nb = (P.sh_degree + 1) * (P.sh_degree + 1);

    // Culled splats get zero gradients.  In a wave with live splats they run
    // the same code and their results are replaced by zero at the store, so
    // every output plane is written by one full-wave store (a culled lane's
    // early store and a live lane's late store to the same line would each
    // write back a partial line).
    const bool live = A.radius[i] != 0;
    if (!__any(live)) {  // the whole wave is culled: zeros, still one full-wave store per plane
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            __builtin_nontemporal_store(0.f, &A.g_means[k * n + i]);
            __builtin_nontemporal_store(0.f, &A.g_log_scales[k * n + i]);
        }
        for (int k = 0; k < 4; ++k) __builtin_nontemporal_store(0.f, &A.g_quats[k * n + i]);
        __builtin_nontemporal_store(0.f, &A.g_opacity_logits[i]);
        for (int k = 0; k < nb * 3; ++k) __builtin_nontemporal_store(0.f, &A.g_sh[(int64_t)k * n + i]);
        return;
    }
    // The gradients are written once and not read again by this library; they
    // go out non-temporal so that they do not fill the last-level cache with
    // dirty lines that the next forward pass would have to write back.
    auto put = [live](float* dst, double v) { __builtin_nontemporal_store(live ? (float)v : 0.0f, dst); };
    const uint8_t flags = A.clamp_flags[i];
    const float* G2 = A.grad2d + (size_t)i * kGrad2d;

    // ---- recompute the forward projection (float64)
    const double m0 = S.means[i], m1 = S.means[n + i], m2 = S.means[2 * n + i];
    const double* R = P.R;
    const double tx = R[0] * m0 + R[1] * m1 + R[2] * m2 + P.t[0];
    const double ty = R[3] * m0 + R[4] * m1 + R[5] * m2 + P.t[1];
    const double tz = R[6] * m0 + R[7] * m1 + R[8] * m2 + P.t[2];
    double s2[3];
    for (int k = 0; k < 3; ++k) s2[k] = exp(2.0 * (double)S.log_scales[k * n + i]);
    double q[4];
    for (int k = 0; k < 4; ++k) q[k] = S.quats[k * n + i];
    const double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const double iqn = 1.0 / qn;
    for (int k = 0; k < 4; ++k) q[k] *= iqn;
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    const double Rq[9] = {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y),
                          2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x),
                          2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)};
    double Sig[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            Sig[3 * r + c] = Rq[3 * r] * Rq[3 * c] * s2[0] + Rq[3 * r + 1] * Rq[3 * c + 1] * s2[1] +
                             Rq[3 * r + 2] * Rq[3 * c + 2] * s2[2];
    const bool clx = flags & 8, cly = flags & 16;
    const double itz = 1.0 / tz;  // one division; the gradients below multiply by it
    double ux = tx * itz, uy = ty * itz;
    if (clx) ux = ux > 0 ? P.limx : -P.limx;
    if (cly) uy = uy > 0 ? P.limy : -P.limy;
    const double J[6] = {P.fx * itz, 0.0, -P.fx * ux * itz, 0.0, P.fy * itz, -P.fy * uy * itz};
    double M[6];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c)
            M[3 * r + c] = J[3 * r] * R[c] + J[3 * r + 1] * R[3 + c] + J[3 * r + 2] * R[6 + c];
    double MS[6];  // M Sigma
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c)
            MS[3 * r + c] = M[3 * r] * Sig[c] + M[3 * r + 1] * Sig[3 + c] + M[3 * r + 2] * Sig[6 + c];
    const double a = MS[0] * M[0] + MS[1] * M[1] + MS[2] * M[2] + 0.3;
    const double b = MS[0] * M[3] + MS[1] * M[4] + MS[2] * M[5];
    const double c = MS[3] * M[3] + MS[4] * M[4] + MS[5] * M[5] + 0.3;
    const double det = a * c - b * b;
    const double idet = 1.0 / det;
    const double id2 = idet * idet;
    // sums over the splat's pixels of dL/dpower times dx, dy, dx^2, dx dy, dy^2
    // (dx, dy = 2D mean - pixel)
    const double s_x = G2[0], s_y = G2[1], s_xx = G2[2], s_xy = G2[3], s_yy = G2[4];
    // power = -(a' dx^2 + 2 b' dx dy + c' dy^2) / 2 with the conic (a', b', c') = (c, -b, a) / det:
    // dpower/dmean = -(a' dx + b' dy, b' dx + c' dy), dpower/d(a', b', c') = -(dx^2 / 2, dx dy, dy^2 / 2)
    const double gmx = -(c * s_x - b * s_y) * idet;
    const double gmy = -(a * s_y - b * s_x) * idet;
    const double gA = -0.5 * s_xx, gB = -s_xy, gC = -0.5 * s_yy;
    // 2D mean = (fx tx / tz, fy ty / tz) + principal point
    const double itz2 = itz * itz, itz3 = itz2 * itz;
    double gt0 = gmx * P.fx * itz;
    double gt1 = gmy * P.fy * itz;
    double gt2 = -gmx * P.fx * tx * itz2 - gmy * P.fy * ty * itz2;
    gt2 += -(double)G2[9] * itz2;  // dL / d(1 / depth), depth = t_cam z

    // ---- conic (c, -b, a)/det -> (a, b, c)
    const double ga = (gA * (-c * c) + gB * (b * c) + gC * (-b * b)) * id2;
    const double gb = (gA * (2.0 * b * c) + gB * (-(a * c + b * b)) + gC * (2.0 * a * b)) * id2;
    const double gc = (gA * (-b * b) + gB * (a * b) + gC * (-a * a)) * id2;
    const double Gs[4] = {ga, 0.5 * gb, 0.5 * gb, gc};
    // dL/dM = 2 G M Sigma ; dL/dSigma = M^T G M
    double gM[6];
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < 3; ++k) gM[3 * r + k] = 2.0 * (Gs[2 * r] * MS[k] + Gs[2 * r + 1] * MS[3 + k]);
    double GM[6];  // G M
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < 3; ++k) GM[3 * r + k] = Gs[2 * r] * M[k] + Gs[2 * r + 1] * M[3 + k];
    double gSig[9];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) gSig[3 * r + k] = M[r] * GM[k] + M[3 + r] * GM[3 + k];
    // M = J Rcam -> dL/dJ = dL/dM Rcam^T
    double gJ[6];
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < 3; ++k)
            gJ[3 * r + k] = gM[3 * r] * R[3 * k] + gM[3 * r + 1] * R[3 * k + 1] + gM[3 * r + 2] * R[3 * k + 2];
    gt2 += gJ[0] * (-P.fx * itz2) + gJ[4] * (-P.fy * itz2);
    if (!clx) { gt0 += gJ[2] * (-P.fx * itz2); gt2 += gJ[2] * (2.0 * P.fx * tx * itz3); }
    else      { gt2 += gJ[2] * (P.fx * ux * itz2); }
    if (!cly) { gt1 += gJ[5] * (-P.fy * itz2); gt2 += gJ[5] * (2.0 * P.fy * ty * itz3); }
    else      { gt2 += gJ[5] * (P.fy * uy * itz2); }

    // ---- Sigma = Rq diag(s2) Rq^T
    double GR[9];  // gSig Rq
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k)
            GR[3 * r + k] = gSig[3 * r] * Rq[k] + gSig[3 * r + 1] * Rq[3 + k] + gSig[3 * r + 2] * Rq[6 + k];
    double gR[9];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) gR[3 * r + k] = 2.0 * GR[3 * r + k] * s2[k];
    for (int k = 0; k < 3; ++k) {
        // (Rq^T gSig Rq)_kk
        const double d = Rq[k] * GR[k] + Rq[3 + k] * GR[3 + k] + Rq[6 + k] * GR[6 + k];
        put(&A.g_log_scales[k * n + i], 2.0 * s2[k] * d);
    }
    double gq[4];
    gq[0] = 2.0 * (-z * gR[1] + y * gR[2] + z * gR[3] - x * gR[5] - y * gR[6] + x * gR[7]);
    gq[1] = 2.0 * (y * gR[1] + z * gR[2] + y * gR[3] - 2.0 * x * gR[4] - w * gR[5] + z * gR[6] +
                   w * gR[7] - 2.0 * x * gR[8]);
    gq[2] = 2.0 * (-2.0 * y * gR[0] + x * gR[1] + w * gR[2] + x * gR[3] + z * gR[5] - w * gR[6] +
                   z * gR[7] - 2.0 * y * gR[8]);
    gq[3] = 2.0 * (-2.0 * z * gR[0] - w * gR[1] + x * gR[2] + w * gR[3] - 2.0 * z * gR[4] + y * gR[5] +
                   x * gR[6] + y * gR[7]);
    const double dot = q[0] * gq[0] + q[1] * gq[1] + q[2] * gq[2] + q[3] * gq[3];
    for (int k = 0; k < 4; ++k) put(&A.g_quats[k * n + i], (gq[k] - q[k] * dot) * iqn);

    // ---- opacity
    const double go = G2[5];
    const double o = 1.0 / (1.0 + exp(-(double)S.opacity_logits[i]));
    put(&A.g_opacity_logits[i], go * o * (1.0 - o));

    // ---- colour
    double gm[3] = {0.0, 0.0, 0.0};
    {
        double grgb[3] = {G2[6], G2[7], G2[8]};
        for (int ch = 0; ch < 3; ++ch)
            if (flags & (1u << ch)) grgb[ch] = 0.0;
        double v[3] = {m0 - P.campos[0], m1 - P.campos[1], m2 - P.campos[2]};
        const double vl = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        const double ivl = 1.0 / vl;
        const double dx = v[0] * ivl, dy = v[1] * ivl, dz = v[2] * ivl;
        double Y[16], wsum[16];
        sh_basis64(dx, dy, dz, Y);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            wsum[k] = 0.0;
            if (k < nb) {
                const float* cf = S.sh + (int64_t)k * 3 * n + i;
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    put(&A.g_sh[((int64_t)k * 3 + ch) * n + i], Y[k] * grgb[ch]);
                    if constexpr (!kJac) wsum[k] += (double)cf[(int64_t)ch * n] * grgb[ch];
                }
            }
        }
        // dL/ddir = sum_ch dL/drgb_ch drgb_ch/ddir: from the forward's
        // derivative (kJac) or from the coefficients
        double gdir[3];
        if constexpr (kJac) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
                gdir[c] = grgb[0] * (double)A.jac[(int64_t)c * n + i] +
                          grgb[1] * (double)A.jac[(int64_t)(3 + c) * n + i] +
                          grgb[2] * (double)A.jac[(int64_t)(6 + c) * n + i];
        } else {
            sh_weighted_grad64(dx, dy, dz, wsum, gdir);
        }
        const double dd = dx * gdir[0] + dy * gdir[1] + dz * gdir[2];
        gm[0] = (gdir[0] - dx * dd) * ivl;
        gm[1] = (gdir[1] - dy * dd) * ivl;
        gm[2] = (gdir[2] - dz * dd) * ivl;
    }
    // t_cam = Rcam m + t
    for (int k = 0; k < 3; ++k) gm[k] += R[k] * gt0 + R[3 + k] * gt1 + R[6 + k] * gt2;
    for (int k = 0; k < 3; ++k) put(&A.g_means[k * n + i], gm[k]);
}

}  // namespace

hipError_t launch_preprocess_backward(const ProjParams& p, const SceneParams& s, const PreBwdArgs& a,
                                      hipStream_t stream) {
    if (p.n == 0) return hipSuccess;
    const int64_t nb = (p.n + 255) / 256;
    if (a.jac && p.sh_degree > 0)
        hipLaunchKernelGGL(k_preprocess_bwd<true>, dim3((unsigned)nb), dim3(256), 0, stream, p, s, a);
    else
        hipLaunchKernelGGL(k_preprocess_bwd<false>, dim3((unsigned)nb), dim3(256), 0, stream, p, s, a);
    return hipGetLastError();
}

}  // namespace cds
