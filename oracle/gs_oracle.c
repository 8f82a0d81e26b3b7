/*
 * gs_oracle.c -- plain, slow, double-precision CPU reference for the 3D
 * Gaussian-splatting rasterisation pipeline.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU library; the only thing both sides
 * consume is the seeded input generator (which holds no rendering arithmetic).
 *
 * What is computed (paper: Section II-B "Structure of Gaussian Splatting
 * Rendering Pipeline", Eq. (1) and Algorithm 1; the projection and colour
 * stages are those of 3DGS, the pipeline the paper cites as its baseline):
 *
 *   project   per Gaussian: activations, view transform, near cull, 3D
 *             covariance, EWA 2D covariance (+0.3 dilation), conic, 3-sigma
 *             radius, 2D mean, covered tile rectangle, depth   (Sec. II-B(1))
 *   colour    real spherical harmonics up to degree 3, +0.5, clamp at 0
 *   keys      (tile id << 32 | float32 depth bits), one per covered tile,
 *             stably sorted (ties by Gaussian index)            (Sec. II-B(1))
 *   ranges    [start, end) of each tile in the sorted list      (Alg. 1, step 2)
 *   blend     per pixel, front to back: alpha = min(0.99, o*exp(power)),
 *             skip alpha < 1/255, stop when T*(1-alpha) < 1e-4,
 *             C += c*alpha*T; out = C + T*bg              (Sec. II-B(2), Alg. 1)
 *   backward  exact derivative of all of the above with every discrete
 *             decision held fixed.
 *
 * Every arithmetic operation is double precision.  The three blending
 * thresholds are the single-precision literals the paper's kernels use
 * (0.99f, 1.0f/255.0f, 0.0001f), converted exactly to double.  Where the
 * paper's pipeline stores an intermediate as float (2D mean, conic, opacity,
 * colour, depth; Appendix B kernel arguments) the caller may ask for those
 * intermediates rounded to float (round_f32 = 1); with round_f32 = 0 the whole
 * chain stays double, which is what the finite-difference checks use.
 *
 * Decision margins: wherever a double-precision value decides an integer
 * (cull, depth bits, radius, rectangle, alpha thresholds) the oracle reports
 * how close the value came to the boundary, so a test can tell a genuine
 * disagreement from one that any two correct roundings may produce.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TILE 16

typedef struct {
    int32_t width, height;
    double fx, fy, cx, cy;
    double view[12]; /* row-major [R | t], world -> camera */
    double near_plane;
    double bg[3];
} ora_camera;

/* The paper's single-precision blending constants, held as doubles. */
static double alpha_max(void) { volatile float f = 0.99f; return (double)f; }
static double alpha_min(void) { volatile float one = 1.0f, d = 255.0f; float q = one / d; return (double)q; }
static double t_min(void) { volatile float f = 0.0001f; return (double)f; }

/* near_flags bits (per Gaussian) */
#define NF_NEAR_PLANE 1u   /* t_z within rounding of the near plane          */
#define NF_DEPTH_ROUND 2u  /* t_z within rounding of a float32 midpoint      */
#define NF_RADIUS 4u       /* 3*sqrt(lambda) within rounding of an integer   */
#define NF_MEAN_ROUND 8u   /* 2D mean within rounding of a float32 midpoint  */
#define NF_DET 16u         /* determinant within rounding of zero            */
#define NF_JCLAMP 32u      /* x/z or y/z within rounding of the clamp limit  */
#define NF_RGB 64u         /* colour within rounding of the clamp at zero    */

/* clamp_flags bits (per Gaussian) */
#define CF_R 1u
#define CF_G 2u
#define CF_B 4u
#define CF_JX 8u
#define CF_JY 16u

/* True when v lies within a millionth of an ulp of a float32 rounding
 * midpoint without sitting exactly on it.  A value exactly on a midpoint
 * rounds to even in every IEEE implementation, so it is only ambiguous when a
 * different evaluation order could land on either side; the callers use this
 * for values the pipeline computes in one fixed order of double operations,
 * where an exact tie is reproduced exactly and is not a disagreement. */
static int near_f32_midpoint(double v) {
    float f = (float)v;
    double df = (double)f;
    double up = (double)nextafterf(f, INFINITY);
    double dn = (double)nextafterf(f, -INFINITY);
    double ulp = up - df;
    double mid_hi = 0.5 * (df + up), mid_lo = 0.5 * (df + dn);
    return (v != mid_hi && fabs(v - mid_hi) < 1e-6 * ulp) || (v != mid_lo && fabs(v - mid_lo) < 1e-6 * (df - dn));
}

static double round_to_f32(double v) { return (double)(float)v; }

/* ---------------------------------------------------------------------- */
/* Real spherical harmonics, degree <= 3, orthonormal on the unit sphere,   */
/* Condon-Shortley phase, order m = -l..l.  Constants from closed forms.    */
/* ---------------------------------------------------------------------- */
static void sh_basis(const double d[3], int degree, double Y[16], double dY[16][3]) {
    const double pi = 3.14159265358979323846;
    const double x = d[0], y = d[1], z = d[2];
    const double k0 = 0.5 / sqrt(pi);
    const double k1 = sqrt(3.0 / (4.0 * pi));
    const double k2a = sqrt(15.0 / (4.0 * pi));
    const double k2b = sqrt(5.0 / (16.0 * pi));
    const double k2c = sqrt(15.0 / (16.0 * pi));
    const double k3a = sqrt(35.0 / (32.0 * pi));
    const double k3b = sqrt(105.0 / (4.0 * pi));
    const double k3c = sqrt(21.0 / (32.0 * pi));
    const double k3d = sqrt(7.0 / (16.0 * pi));
    const double k3e = sqrt(105.0 / (16.0 * pi));
    int i, j;
    for (i = 0; i < 16; ++i) {
        Y[i] = 0.0;
        if (dY) for (j = 0; j < 3; ++j) dY[i][j] = 0.0;
    }
    Y[0] = k0;
    if (degree >= 1) {
        Y[1] = -k1 * y; Y[2] = k1 * z; Y[3] = -k1 * x;
        if (dY) { dY[1][1] = -k1; dY[2][2] = k1; dY[3][0] = -k1; }
    }
    if (degree >= 2) {
        Y[4] = k2a * x * y;
        Y[5] = -k2a * y * z;
        Y[6] = k2b * (2.0 * z * z - x * x - y * y);
        Y[7] = -k2a * x * z;
        Y[8] = k2c * (x * x - y * y);
        if (dY) {
            dY[4][0] = k2a * y; dY[4][1] = k2a * x;
            dY[5][1] = -k2a * z; dY[5][2] = -k2a * y;
            dY[6][0] = -2.0 * k2b * x; dY[6][1] = -2.0 * k2b * y; dY[6][2] = 4.0 * k2b * z;
            dY[7][0] = -k2a * z; dY[7][2] = -k2a * x;
            dY[8][0] = 2.0 * k2c * x; dY[8][1] = -2.0 * k2c * y;
        }
    }
    if (degree >= 3) {
        Y[9] = -k3a * y * (3.0 * x * x - y * y);
        Y[10] = k3b * x * y * z;
        Y[11] = -k3c * y * (4.0 * z * z - x * x - y * y);
        Y[12] = k3d * z * (2.0 * z * z - 3.0 * x * x - 3.0 * y * y);
        Y[13] = -k3c * x * (4.0 * z * z - x * x - y * y);
        Y[14] = k3e * z * (x * x - y * y);
        Y[15] = -k3a * x * (x * x - 3.0 * y * y);
        if (dY) {
            dY[9][0] = -k3a * 6.0 * x * y;
            dY[9][1] = -k3a * (3.0 * x * x - 3.0 * y * y);
            dY[10][0] = k3b * y * z; dY[10][1] = k3b * x * z; dY[10][2] = k3b * x * y;
            dY[11][0] = -k3c * y * (-2.0 * x);
            dY[11][1] = -k3c * (4.0 * z * z - x * x - 3.0 * y * y);
            dY[11][2] = -k3c * y * 8.0 * z;
            dY[12][0] = k3d * z * (-6.0 * x);
            dY[12][1] = k3d * z * (-6.0 * y);
            dY[12][2] = k3d * (6.0 * z * z - 3.0 * x * x - 3.0 * y * y);
            dY[13][0] = -k3c * (4.0 * z * z - 3.0 * x * x - y * y);
            dY[13][1] = -k3c * x * (-2.0 * y);
            dY[13][2] = -k3c * x * 8.0 * z;
            dY[14][0] = k3e * z * 2.0 * x; dY[14][1] = -k3e * z * 2.0 * y;
            dY[14][2] = k3e * (x * x - y * y);
            dY[15][0] = -k3a * (3.0 * x * x - 3.0 * y * y);
            dY[15][1] = -k3a * x * (-6.0 * y);
        }
    }
}

/* Exported for the basis tests (orthonormality, library cross-check). */
void ora_sh_basis(const double* dirs, int64_t count, int degree, double* out /*[count][16]*/) {
    int64_t i;
    for (i = 0; i < count; ++i) sh_basis(dirs + 3 * i, degree, out + 16 * i, NULL);
}

/* ---------------------------------------------------------------------- */
/* Small dense matrix helpers (row-major).                                 */
/* ---------------------------------------------------------------------- */
static void quat_to_rot(const double q[4], double R[9]) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z); R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z); R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y); R[7] = 2.0 * (y * z + w * x); R[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* C[r x c] = A[r x k] * B[k x c] */
static void matmul(const double* A, const double* B, double* C, int r, int k, int c) {
    int i, j, l;
    for (i = 0; i < r; ++i)
        for (j = 0; j < c; ++j) {
            double s = 0.0;
            for (l = 0; l < k; ++l) s += A[i * k + l] * B[l * c + j];
            C[i * c + j] = s;
        }
}

static void transpose(const double* A, double* At, int r, int c) {
    int i, j;
    for (i = 0; i < r; ++i)
        for (j = 0; j < c; ++j) At[j * r + i] = A[i * c + j];
}

/* Per-Gaussian projected state, double precision, before any rounding. */
typedef struct {
    int visible;
    double tcam[3];
    double qn[4], qnorm;
    double Rq[9], s2[3], Sigma[9];
    double ux, uy, uxc, uyc; /* x/z, y/z and their clamped values */
    int clampx, clampy;
    double J[6], M[6];       /* M = J * R_cam, 2 x 3 */
    double a, b, c, det;     /* dilated 2D covariance [[a,b],[b,c]] */
    double mean2d[2];
    double conic[3];
    double opacity;
    double dir[3], dirlen;
    double rgb_raw[3];
    double rgb[3];
    int radius;
    int rect[4];             /* tile span tx0, ty0, tx1, ty1 (inclusive) */
    uint8_t clamp, nearf;
} gstate;

static void project_one(int64_t n, int64_t i, int degree,
                        const float* means, const float* log_scales, const float* quats,
                        const float* opac_logits, const float* sh,
                        const ora_camera* cam, gstate* g) {
    const double* V = cam->view;
    const double Rc[9] = {V[0], V[1], V[2], V[4], V[5], V[6], V[8], V[9], V[10]};
    const double tc[3] = {V[3], V[7], V[11]};
    double m[3], Cov2[4], Mt[6], tmp[6], ls[3];
    int k, ch, W = cam->width, H = cam->height;
    memset(g, 0, sizeof(*g));
    for (k = 0; k < 3; ++k) m[k] = means[k * n + i];
    for (k = 0; k < 3; ++k)
        g->tcam[k] = Rc[3 * k] * m[0] + Rc[3 * k + 1] * m[1] + Rc[3 * k + 2] * m[2] + tc[k];
    {
        double tz = g->tcam[2];
        if (fabs(tz - cam->near_plane) < 1e-12 * fmax(1.0, fabs(tz))) g->nearf |= NF_NEAR_PLANE;
        if (near_f32_midpoint(tz)) g->nearf |= NF_DEPTH_ROUND;
        if (!(tz > cam->near_plane)) return; /* near cull */
    }
    /* activations */
    for (k = 0; k < 3; ++k) { ls[k] = log_scales[k * n + i]; g->s2[k] = exp(2.0 * ls[k]); }
    {
        double q[4], nq = 0.0;
        for (k = 0; k < 4; ++k) { q[k] = quats[k * n + i]; nq += q[k] * q[k]; }
        g->qnorm = sqrt(nq);
        for (k = 0; k < 4; ++k) g->qn[k] = q[k] / g->qnorm;
    }
    quat_to_rot(g->qn, g->Rq);
    /* Sigma = Rq diag(s^2) Rq^T */
    {
        double RS[9], RqT[9];
        int r, c;
        for (r = 0; r < 3; ++r)
            for (c = 0; c < 3; ++c) RS[3 * r + c] = g->Rq[3 * r + c] * g->s2[c];
        transpose(g->Rq, RqT, 3, 3);
        matmul(RS, RqT, g->Sigma, 3, 3, 3);
    }
    /* EWA: J (with the 1.3x field-of-view guard band on x/z and y/z) */
    {
        double tz = g->tcam[2];
        double limx = 1.3 * (0.5 * W / cam->fx), limy = 1.3 * (0.5 * H / cam->fy);
        g->ux = g->tcam[0] / tz;
        g->uy = g->tcam[1] / tz;
        g->uxc = g->ux; g->uyc = g->uy;
        if (fabs(fabs(g->ux) - limx) < 1e-12 * limx) g->nearf |= NF_JCLAMP;
        if (fabs(fabs(g->uy) - limy) < 1e-12 * limy) g->nearf |= NF_JCLAMP;
        if (g->ux > limx) { g->uxc = limx; g->clampx = 1; }
        if (g->ux < -limx) { g->uxc = -limx; g->clampx = 1; }
        if (g->uy > limy) { g->uyc = limy; g->clampy = 1; }
        if (g->uy < -limy) { g->uyc = -limy; g->clampy = 1; }
        g->J[0] = cam->fx / tz; g->J[1] = 0.0; g->J[2] = -cam->fx * g->uxc / tz;
        g->J[3] = 0.0; g->J[4] = cam->fy / tz; g->J[5] = -cam->fy * g->uyc / tz;
        if (g->clampx) g->clamp |= CF_JX;
        if (g->clampy) g->clamp |= CF_JY;
    }
    matmul(g->J, Rc, g->M, 2, 3, 3);
    transpose(g->M, Mt, 2, 3);
    matmul(g->M, g->Sigma, tmp, 2, 3, 3);
    matmul(tmp, Mt, Cov2, 2, 3, 2);
    g->a = Cov2[0] + 0.3;
    g->b = Cov2[1];
    g->c = Cov2[3] + 0.3;
    g->det = g->a * g->c - g->b * g->b;
    if (fabs(g->det) < 1e-12 * fabs(g->a * g->c)) g->nearf |= NF_DET;
    if (!(g->det > 0.0)) return;
    g->conic[0] = g->c / g->det;
    g->conic[1] = -g->b / g->det;
    g->conic[2] = g->a / g->det;
    {
        double mid = 0.5 * (g->a + g->c);
        double disc = mid * mid - g->det;
        double lam = mid + sqrt(disc > 0.1 ? disc : 0.1);
        double rr = ceil(3.0 * sqrt(lam));
        double x3 = 3.0 * sqrt(lam);
        if (fabs(x3 - nearbyint(x3)) < 1e-10 * fmax(1.0, x3)) g->nearf |= NF_RADIUS;
        g->radius = rr > 2147483647.0 ? 2147483647 : (int)rr;
    }
    g->mean2d[0] = cam->fx * g->tcam[0] / g->tcam[2] + cam->cx;
    g->mean2d[1] = cam->fy * g->tcam[1] / g->tcam[2] + cam->cy;
    if (near_f32_midpoint(g->mean2d[0]) || near_f32_midpoint(g->mean2d[1])) g->nearf |= NF_MEAN_ROUND;
    /* covered pixels: |p - mean| <= r per axis, mean as stored (float32) */
    {
        double mx = round_to_f32(g->mean2d[0]), my = round_to_f32(g->mean2d[1]);
        double r = (double)g->radius;
        double lox = ceil(mx - r), hix = floor(mx + r), loy = ceil(my - r), hiy = floor(my + r);
        if (lox < 0) lox = 0;
        if (loy < 0) loy = 0;
        if (hix > W - 1) hix = W - 1;
        if (hiy > H - 1) hiy = H - 1;
        if (lox > hix || loy > hiy) { g->radius = 0; return; }
        g->rect[0] = (int)lox / TILE; g->rect[1] = (int)loy / TILE;
        g->rect[2] = (int)hix / TILE; g->rect[3] = (int)hiy / TILE;
    }
    g->opacity = 1.0 / (1.0 + exp(-(double)opac_logits[i]));
    /* colour */
    {
        double Rt[9], cw[3], Y[16];
        int nb = (degree + 1) * (degree + 1);
        transpose(Rc, Rt, 3, 3);
        for (k = 0; k < 3; ++k) cw[k] = -(Rt[3 * k] * tc[0] + Rt[3 * k + 1] * tc[1] + Rt[3 * k + 2] * tc[2]);
        for (k = 0; k < 3; ++k) g->dir[k] = m[k] - cw[k];
        g->dirlen = sqrt(g->dir[0] * g->dir[0] + g->dir[1] * g->dir[1] + g->dir[2] * g->dir[2]);
        for (k = 0; k < 3; ++k) g->dir[k] /= g->dirlen;
        sh_basis(g->dir, degree, Y, NULL);
        for (ch = 0; ch < 3; ++ch) {
            double s = 0.0;
            for (k = 0; k < nb; ++k) s += Y[k] * (double)sh[((int64_t)k * 3 + ch) * n + i];
            s += 0.5;
            g->rgb_raw[ch] = s;
            if (fabs(s) < 1e-12) g->nearf |= NF_RGB;
            if (s < 0.0) { g->rgb[ch] = 0.0; g->clamp |= (uint8_t)(CF_R << ch); }
            else g->rgb[ch] = s;
        }
    }
    g->visible = 1;
}

/*
 * Project every Gaussian.  Outputs are structure-of-arrays; culled Gaussians
 * have radius 0, tiles_touched 0 and zero values elsewhere.
 */
int ora_project(int64_t n, int degree,
                const float* means, const float* log_scales, const float* quats,
                const float* opac_logits, const float* sh, const ora_camera* cam, int round_f32,
                double* mean2d /*[2][n]*/, double* conic /*[3][n]*/, double* opacity /*[n]*/,
                double* rgb /*[3][n]*/, double* depth /*[n]*/, uint32_t* depth_bits /*[n]*/,
                int32_t* radius /*[n]*/, int32_t* rect /*[4][n]*/, uint32_t* tiles_touched /*[n]*/,
                uint8_t* clamp_flags /*[n]*/, uint8_t* near_flags /*[n]*/) {
    int64_t i;
    if (n < 0 || degree < 0 || degree > 3 || !cam) return 1;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; ++i) {
        gstate g;
        int k;
        project_one(n, i, degree, means, log_scales, quats, opac_logits, sh, cam, &g);
        near_flags[i] = g.nearf;
        clamp_flags[i] = g.clamp;
        {
            float dz = (float)g.tcam[2];
            uint32_t bits;
            memcpy(&bits, &dz, 4);
            depth[i] = g.tcam[2];
            depth_bits[i] = g.visible ? bits : 0u;
        }
        if (!g.visible) {
            radius[i] = 0;
            tiles_touched[i] = 0;
            for (k = 0; k < 2; ++k) mean2d[k * n + i] = 0.0;
            for (k = 0; k < 3; ++k) { conic[k * n + i] = 0.0; rgb[k * n + i] = 0.0; }
            for (k = 0; k < 4; ++k) rect[k * n + i] = 0;
            opacity[i] = 0.0;
            continue;
        }
        radius[i] = g.radius;
        for (k = 0; k < 4; ++k) rect[k * n + i] = g.rect[k];
        tiles_touched[i] = (uint32_t)((g.rect[2] - g.rect[0] + 1) * (g.rect[3] - g.rect[1] + 1));
        for (k = 0; k < 2; ++k) mean2d[k * n + i] = round_f32 ? round_to_f32(g.mean2d[k]) : g.mean2d[k];
        for (k = 0; k < 3; ++k) {
            conic[k * n + i] = round_f32 ? round_to_f32(g.conic[k]) : g.conic[k];
            rgb[k * n + i] = round_f32 ? round_to_f32(g.rgb[k]) : g.rgb[k];
        }
        opacity[i] = round_f32 ? round_to_f32(g.opacity) : g.opacity;
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Keys, stable sort, ranges                                               */
/* ---------------------------------------------------------------------- */
int64_t ora_count_keys(int64_t n, const uint32_t* tiles_touched) {
    int64_t i, k = 0;
    for (i = 0; i < n; ++i) k += tiles_touched[i];
    return k;
}

/* Keys in generation order: ascending Gaussian index, tiles of its
 * rectangle in row-major order. */
int ora_build_keys(int64_t n, const int32_t* rect, const uint32_t* tiles_touched,
                   const uint32_t* depth_bits, int tiles_x, uint64_t* keys, uint32_t* vals) {
    int64_t i, o = 0;
    for (i = 0; i < n; ++i) {
        int tx, ty;
        if (!tiles_touched[i]) continue;
        for (ty = rect[1 * n + i]; ty <= rect[3 * n + i]; ++ty)
            for (tx = rect[0 * n + i]; tx <= rect[2 * n + i]; ++tx) {
                uint64_t tile = (uint64_t)ty * (uint64_t)tiles_x + (uint64_t)tx;
                keys[o] = (tile << 32) | (uint64_t)depth_bits[i];
                vals[o] = (uint32_t)i;
                ++o;
            }
    }
    return 0;
}

typedef struct { uint64_t k; uint32_t v; } kv;

static int kv_cmp(const void* a, const void* b) {
    const kv* x = (const kv*)a;
    const kv* y = (const kv*)b;
    if (x->k != y->k) return x->k < y->k ? -1 : 1;
    if (x->v != y->v) return x->v < y->v ? -1 : 1;
    return 0;
}

/* A stable sort by key of keys generated in ascending-index order equals a
 * sort by (key, index): each Gaussian emits a key at most once per tile. */
int ora_sort_keys(int64_t count, uint64_t* keys, uint32_t* vals) {
    int64_t i;
    kv* buf = (kv*)malloc(sizeof(kv) * (size_t)(count > 0 ? count : 1));
    if (!buf) return 2;
    for (i = 0; i < count; ++i) { buf[i].k = keys[i]; buf[i].v = vals[i]; }
    qsort(buf, (size_t)count, sizeof(kv), kv_cmp);
    for (i = 0; i < count; ++i) { keys[i] = buf[i].k; vals[i] = buf[i].v; }
    free(buf);
    return 0;
}

int ora_ranges(int64_t count, const uint64_t* sorted_keys, int ntiles, uint32_t* ranges /*[ntiles][2]*/) {
    int64_t i;
    memset(ranges, 0, sizeof(uint32_t) * 2 * (size_t)ntiles);
    for (i = 0; i < count; ++i) {
        uint32_t t = (uint32_t)(sorted_keys[i] >> 32);
        if ((int)t >= ntiles) return 1;
        if (i == 0 || (uint32_t)(sorted_keys[i - 1] >> 32) != t) ranges[2 * t] = (uint32_t)i;
        if (i == count - 1 || (uint32_t)(sorted_keys[i + 1] >> 32) != t) ranges[2 * t + 1] = (uint32_t)(i + 1);
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Blending                                                                */
/* ---------------------------------------------------------------------- */
typedef struct {
    double Tfinal;
    double C[3];
    double D;                     /* expected inverse depth: sum of a T / depth */
    uint32_t ncontrib;
    uint32_t nused;               /* Gaussians actually blended */
    uint32_t neval;               /* list entries examined: up to and including the
                                     one that stops the pixel, else the whole list */
    double m_power, m_alpha, m_T; /* smallest relative decision margins */
} pixres;

/* Blend one pixel over an ordered list of Gaussian indices.  `invd` (1 /
 * depth per Gaussian, or NULL) is composited like a colour channel without
 * a background term: the expected inverse depth of the optional output of
 * the Appendix B kernels. */
static void blend_pixel(int px, int py, const uint32_t* list, int64_t len, int64_t n,
                        const double* mean2d, const double* conic, const double* opacity,
                        const double* rgb, const double* invd, pixres* out,
                        /* optional per-contribution record for the backward pass */
                        int64_t* c_pos, double* c_T, double* c_alpha, double* c_G, int* c_clamped,
                        int64_t* c_count) {
    const double amax = alpha_max(), amin = alpha_min(), tmin = t_min();
    double T = 1.0, C[3] = {0.0, 0.0, 0.0}, D = 0.0;
    double m_power = INFINITY, m_alpha = INFINITY, m_T = INFINITY;
    uint32_t last = 0;
    int64_t j, nc = 0;
    for (j = 0; j < len; ++j) {
        const uint32_t g = list[j];
        const double dx = mean2d[g] - px, dy = mean2d[n + g] - py;
        const double A = conic[g], B = conic[n + g], Cc = conic[2 * n + g];
        const double power = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy;
        const double scale = 0.5 * (fabs(A) * dx * dx + fabs(Cc) * dy * dy) + fabs(B * dx * dy);
        double G, a, Tn;
        int clamped;
        if (scale > 0.0) {
            double mp = fabs(power) / scale;
            if (mp < m_power) m_power = mp;
        }
        if (power > 0.0) continue;
        G = exp(power);
        a = opacity[g] * G;
        clamped = a > amax;
        if (clamped) a = amax;
        {
            double ma = fabs(a / amin - 1.0);
            if (ma < m_alpha) m_alpha = ma;
        }
        if (a < amin) continue;
        Tn = T * (1.0 - a);
        {
            double mt = fabs(Tn / tmin - 1.0);
            if (mt < m_T) m_T = mt;
        }
        if (Tn < tmin) { ++j; break; }
        if (c_count) {
            c_pos[nc] = j; c_T[nc] = T; c_alpha[nc] = a; c_G[nc] = G; c_clamped[nc] = clamped;
        }
        ++nc;
        C[0] += rgb[g] * a * T;
        C[1] += rgb[n + g] * a * T;
        C[2] += rgb[2 * n + g] * a * T;
        if (invd) D += invd[g] * a * T;
        T = Tn;
        last = (uint32_t)(j + 1);
    }
    if (c_count) *c_count = nc;
    out->Tfinal = T;
    out->C[0] = C[0]; out->C[1] = C[1]; out->C[2] = C[2];
    out->D = D;
    out->ncontrib = last;
    out->nused = (uint32_t)nc;
    out->neval = (uint32_t)j;
    out->m_power = m_power; out->m_alpha = m_alpha; out->m_T = m_T;
}

static void store_pixel(const pixres* r, int64_t pix, int64_t npix, const double* bg,
                        double* out_rgb, double* out_T, uint32_t* n_contrib, double* margins,
                        uint32_t* n_used, double* out_invdepth, uint32_t* n_eval) {
    int ch;
    if (n_used) n_used[pix] = r->nused;
    if (n_eval) n_eval[pix] = r->neval;
    if (out_invdepth) out_invdepth[pix] = r->D;
    for (ch = 0; ch < 3; ++ch) out_rgb[ch * npix + pix] = r->C[ch] + r->Tfinal * bg[ch];
    out_T[pix] = r->Tfinal;
    n_contrib[pix] = r->ncontrib;
    if (margins) {
        margins[pix] = r->m_power;
        margins[npix + pix] = r->m_alpha;
        margins[2 * npix + pix] = r->m_T;
    }
}

/* Tile path: each pixel walks its tile's [start, end) slice of the sorted
 * Gaussian list (Algorithm 1). */
int ora_blend_tiles(int W, int H, int64_t n, const uint32_t* ranges, const uint32_t* point_list,
                    const double* mean2d, const double* conic, const double* opacity,
                    const double* rgb, const double* bg,
                    double* out_rgb /*[3][H][W]*/, double* out_T /*[H][W]*/,
                    uint32_t* n_contrib /*[H][W]*/, double* margins /*[3][H][W] or NULL*/,
                    uint32_t* n_used /*[H][W] or NULL*/, const double* invd /*[n] or NULL*/,
                    double* out_invdepth /*[H][W] or NULL*/, uint32_t* n_eval /*[H][W] or NULL*/) {
    const int tiles_x = (W + TILE - 1) / TILE;
    const int64_t npix = (int64_t)W * H;
    int64_t p;
#pragma omp parallel for schedule(dynamic, 64)
    for (p = 0; p < npix; ++p) {
        const int x = (int)(p % W), y = (int)(p / W);
        const int t = (y / TILE) * tiles_x + x / TILE;
        const uint32_t s = ranges[2 * t], e = ranges[2 * t + 1];
        pixres r;
        blend_pixel(x, y, point_list + s, (int64_t)e - s, n, mean2d, conic, opacity, rgb, invd, &r,
                    NULL, NULL, NULL, NULL, NULL, NULL);
        store_pixel(&r, p, npix, bg, out_rgb, out_T, n_contrib, margins, n_used, out_invdepth, n_eval);
    }
    return 0;
}

typedef struct { uint32_t d; uint32_t i; } di;

static int di_cmp(const void* a, const void* b) {
    const di* x = (const di*)a;
    const di* y = (const di*)b;
    if (x->d != y->d) return x->d < y->d ? -1 : 1;
    return x->i < y->i ? -1 : (x->i > y->i);
}

/*
 * Brute force: for every pixel, every visible Gaussian in (depth, index)
 * order.  With tile_filter = 1 a Gaussian is considered only when its tile
 * rectangle contains the pixel's tile (what the tile lists encode); with
 * tile_filter = 0 every visible Gaussian is considered.
 */
int ora_blend_brute(int W, int H, int64_t n, const int32_t* radius, const int32_t* rect,
                    const uint32_t* depth_bits, int tile_filter,
                    const double* mean2d, const double* conic, const double* opacity,
                    const double* rgb, const double* bg,
                    double* out_rgb, double* out_T, uint32_t* n_contrib, double* margins,
                    uint32_t* n_used, const double* invd, double* out_invdepth) {
    const int64_t npix = (int64_t)W * H;
    int64_t i, nv = 0, p;
    di* order = (di*)malloc(sizeof(di) * (size_t)(n > 0 ? n : 1));
    uint32_t* sorted;
    if (!order) return 2;
    for (i = 0; i < n; ++i)
        if (radius[i] > 0) { order[nv].d = depth_bits[i]; order[nv].i = (uint32_t)i; ++nv; }
    qsort(order, (size_t)nv, sizeof(di), di_cmp);
    sorted = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(nv > 0 ? nv : 1));
    if (!sorted) { free(order); return 2; }
    for (i = 0; i < nv; ++i) sorted[i] = order[i].i;
    free(order);
#pragma omp parallel for schedule(dynamic, 16)
    for (p = 0; p < npix; ++p) {
        const int x = (int)(p % W), y = (int)(p / W);
        const int tx = x / TILE, ty = y / TILE;
        uint32_t* list = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(nv > 0 ? nv : 1));
        int64_t len = 0, j;
        pixres r;
        for (j = 0; j < nv; ++j) {
            const uint32_t g = sorted[j];
            if (tile_filter && (tx < rect[g] || tx > rect[2 * n + g] || ty < rect[n + g] || ty > rect[3 * n + g]))
                continue;
            list[len++] = g;
        }
        blend_pixel(x, y, list, len, n, mean2d, conic, opacity, rgb, invd, &r, NULL, NULL, NULL, NULL, NULL,
                    NULL);
        store_pixel(&r, p, npix, bg, out_rgb, out_T, n_contrib, margins, n_used, out_invdepth, NULL);
        free(list);
    }
    free(sorted);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Backward                                                                */
/* ---------------------------------------------------------------------- */

/*
 * Gradients of L with respect to the per-Gaussian 2D quantities, given
 * dL/d(out_rgb).  The forward transmittance of every contribution is stored
 * (not reconstructed by division).
 *
 * For the contributions i = 1..N of a pixel (T_i the transmittance before i,
 * T_final after N):  out = sum_i rgb_i a_i T_i + T_final bg, and
 *   d out / d rgb_i  = a_i T_i
 *   d out / d a_i    = T_i (rgb_i - S_i),  S_N = bg,  S_{i-1} = a_i rgb_i + (1 - a_i) S_i
 *   d a / d o        = G (0 if clamped),  d a / d power = a (0 if clamped)
 * The expected inverse depth D = sum_i (1 / depth_i) a_i T_i is one more
 * channel with background 0: given dL/dD (or NULL), d D / d a_i = T_i
 * (1 / depth_i - S^D_i) and d D / d (1 / depth_i) = a_i T_i, into g_invd.
 */
int ora_backward_2d(int W, int H, int64_t n, const uint32_t* ranges, const uint32_t* point_list,
                    const double* mean2d, const double* conic, const double* opacity,
                    const double* rgb, const double* bg, const double* dL_dout /*[3][H][W]*/,
                    double* g_mean2d /*[2][n]*/, double* g_conic /*[3][n]*/,
                    double* g_opacity /*[n]*/, double* g_rgb /*[3][n]*/,
                    const double* invd /*[n] or NULL*/, const double* dL_dinvdepth /*[H][W] or NULL*/,
                    double* g_invd /*[n] or NULL*/) {
    const int depth_on = invd && dL_dinvdepth && g_invd;
    const int tiles_x = (W + TILE - 1) / TILE, tiles_y = (H + TILE - 1) / TILE;
    const int64_t npix = (int64_t)W * H;
    /* per-thread accumulator: mean2d[2][n] conic[3][n] opacity[n] rgb[3][n] invd[n] */
    const int64_t nacc = 10 * n;
    int64_t maxlen = 0, t, ntiles = (int64_t)tiles_x * tiles_y;
    int nthreads = 1, failed = 0;
    double* acc;
    for (t = 0; t < ntiles; ++t) {
        int64_t len = (int64_t)ranges[2 * t + 1] - ranges[2 * t];
        if (len > maxlen) maxlen = len;
    }
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    acc = (double*)calloc((size_t)(nacc > 0 ? nacc : 1) * (size_t)nthreads, sizeof(double));
    if (!acc) return 2;
    /* Tiles are dealt to threads round-robin (a fixed assignment for a fixed
     * thread count); each thread sums into its own accumulator, and the
     * accumulators are added in thread order at the end. */
#pragma omp parallel num_threads(nthreads) reduction(| : failed)
    {
        int tid = 0;
        double *a_mean, *a_conic, *a_op, *a_rgb, *a_invd;
        int64_t* c_pos = (int64_t*)malloc(sizeof(int64_t) * (size_t)(maxlen + 1));
        double* c_T = (double*)malloc(sizeof(double) * (size_t)(maxlen + 1));
        double* c_alpha = (double*)malloc(sizeof(double) * (size_t)(maxlen + 1));
        double* c_G = (double*)malloc(sizeof(double) * (size_t)(maxlen + 1));
        int* c_clamped = (int*)malloc(sizeof(int) * (size_t)(maxlen + 1));
        int64_t tt;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        a_mean = acc + (size_t)tid * (size_t)nacc;
        a_conic = a_mean + 2 * n;
        a_op = a_conic + 3 * n;
        a_rgb = a_op + n;
        a_invd = a_rgb + 3 * n;
        if (!c_pos || !c_T || !c_alpha || !c_G || !c_clamped) failed = 1;
#pragma omp for schedule(static, 1)
        for (tt = 0; tt < ntiles; ++tt) {
            const int tx = (int)(tt % tiles_x), ty = (int)(tt / tiles_x);
            const uint32_t s = ranges[2 * tt], e = ranges[2 * tt + 1];
            const uint32_t* list = point_list + s;
            int x, y;
            if (failed) continue;
            for (y = ty * TILE; y < H && y < (ty + 1) * TILE; ++y)
                for (x = tx * TILE; x < W && x < (tx + 1) * TILE; ++x) {
                    const int64_t p = (int64_t)y * W + x;
                    double go[3], S[3], gd = 0.0, Sd = 0.0;
                    int64_t nc = 0, k;
                    int ch;
                    pixres r;
                    blend_pixel(x, y, list, (int64_t)e - s, n, mean2d, conic, opacity, rgb, NULL, &r,
                                c_pos, c_T, c_alpha, c_G, c_clamped, &nc);
                    for (ch = 0; ch < 3; ++ch) { go[ch] = dL_dout[ch * npix + p]; S[ch] = bg[ch]; }
                    if (depth_on) gd = dL_dinvdepth[p];
                    for (k = nc - 1; k >= 0; --k) {
                        const uint32_t g = list[c_pos[k]];
                        const double a = c_alpha[k], T = c_T[k], G = c_G[k];
                        const double dx = mean2d[g] - x, dy = mean2d[n + g] - y;
                        const double A = conic[g], B = conic[n + g], Cc = conic[2 * n + g];
                        double dLda = 0.0;
                        for (ch = 0; ch < 3; ++ch) {
                            const double c = rgb[ch * n + g];
                            a_rgb[ch * n + g] += a * T * go[ch];
                            dLda += T * (c - S[ch]) * go[ch];
                            S[ch] = a * c + (1.0 - a) * S[ch];
                        }
                        if (depth_on) {
                            a_invd[g] += a * T * gd;
                            dLda += T * (invd[g] - Sd) * gd;
                            Sd = a * invd[g] + (1.0 - a) * Sd;
                        }
                        if (!c_clamped[k]) {
                            const double dLdp = dLda * a;
                            a_op[g] += dLda * G;
                            /* power = -0.5 (A dx^2 + C dy^2) - B dx dy, dx = mean_x - px */
                            a_mean[g] += dLdp * (-(A * dx + B * dy));
                            a_mean[n + g] += dLdp * (-(Cc * dy + B * dx));
                            a_conic[g] += dLdp * (-0.5 * dx * dx);
                            a_conic[n + g] += dLdp * (-dx * dy);
                            a_conic[2 * n + g] += dLdp * (-0.5 * dy * dy);
                        }
                    }
                }
        }
        free(c_pos); free(c_T); free(c_alpha); free(c_G); free(c_clamped);
    }
    if (failed) { free(acc); return 2; }
    /* sum the accumulators in thread order */
#pragma omp parallel for schedule(static)
    for (t = 0; t < n; ++t) {
        double s[10] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int th, k;
        for (th = 0; th < nthreads; ++th) {
            const double* b = acc + (size_t)th * (size_t)nacc;
            for (k = 0; k < 10; ++k) s[k] += b[k * n + t];
        }
        g_mean2d[t] = s[0]; g_mean2d[n + t] = s[1];
        g_conic[t] = s[2]; g_conic[n + t] = s[3]; g_conic[2 * n + t] = s[4];
        g_opacity[t] = s[5];
        g_rgb[t] = s[6]; g_rgb[n + t] = s[7]; g_rgb[2 * n + t] = s[8];
        if (g_invd) g_invd[t] = s[9];
    }
    free(acc);
    return 0;
}

/*
 * Chain rule from the per-Gaussian 2D gradients to the raw parameters,
 * recomputing the projection in double precision.  Culled Gaussians get 0.
 * Gradient arrays have the parameter layouts (structure-of-arrays).
 */
int ora_backward_params(int64_t n, int degree,
                        const float* means, const float* log_scales, const float* quats,
                        const float* opac_logits, const float* sh, const ora_camera* cam,
                        const double* g_mean2d, const double* g_conic, const double* g_opacity,
                        const double* g_rgb,
                        double* g_means /*[3][n]*/, double* g_log_scales /*[3][n]*/,
                        double* g_quats /*[4][n]*/, double* g_opac_logits /*[n]*/,
                        double* g_sh /*[(deg+1)^2][3][n]*/,
                        const double* g_invd /*[n] or NULL: dL / d(1 / depth)*/) {
    const int nb = (degree + 1) * (degree + 1);
    const double* V = cam->view;
    const double Rc[9] = {V[0], V[1], V[2], V[4], V[5], V[6], V[8], V[9], V[10]};
    int64_t i;
    if (degree < 0 || degree > 3) return 1;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; ++i) {
        gstate g;
        int k, ch, r, c;
        double gt[3] = {0.0, 0.0, 0.0}; /* dL / d t_cam */
        double gm[3] = {0.0, 0.0, 0.0};
        project_one(n, i, degree, means, log_scales, quats, opac_logits, sh, cam, &g);
        for (k = 0; k < 3; ++k) { g_means[k * n + i] = 0.0; g_log_scales[k * n + i] = 0.0; }
        for (k = 0; k < 4; ++k) g_quats[k * n + i] = 0.0;
        g_opac_logits[i] = 0.0;
        for (k = 0; k < nb * 3; ++k) g_sh[(int64_t)k * n + i] = 0.0;
        if (!g.visible) continue;

        /* opacity = sigmoid(logit) */
        g_opac_logits[i] = g_opacity[i] * g.opacity * (1.0 - g.opacity);

        /* colour: rgb = max(0, sum_k Y_k(dir) sh_k + 0.5), dir = (m - c)/|m - c| */
        {
            double Y[16], dY[16][3], gdir[3] = {0.0, 0.0, 0.0}, grgb[3];
            sh_basis(g.dir, degree, Y, dY);
            for (ch = 0; ch < 3; ++ch) grgb[ch] = (g.clamp & (CF_R << ch)) ? 0.0 : g_rgb[ch * n + i];
            for (k = 0; k < nb; ++k) {
                double acc = 0.0;
                for (ch = 0; ch < 3; ++ch) {
                    g_sh[((int64_t)k * 3 + ch) * n + i] = Y[k] * grgb[ch];
                    acc += (double)sh[((int64_t)k * 3 + ch) * n + i] * grgb[ch];
                }
                for (c = 0; c < 3; ++c) gdir[c] += dY[k][c] * acc;
            }
            /* d dir / d v = (I - dir dir^T) / |v| */
            {
                double dd = g.dir[0] * gdir[0] + g.dir[1] * gdir[1] + g.dir[2] * gdir[2];
                for (c = 0; c < 3; ++c) gm[c] += (gdir[c] - g.dir[c] * dd) / g.dirlen;
            }
        }

        /* conic = (c, -b, a) / det  ->  d L / d (a, b, c) */
        {
            const double a = g.a, b = g.b, cc = g.c, det = g.det, d2 = det * det;
            const double gA = g_conic[i], gB = g_conic[n + i], gC = g_conic[2 * n + i];
            const double ga = gA * (-cc * cc / d2) + gB * (b * cc / d2) + gC * (-b * b / d2);
            const double gb = gA * (2.0 * b * cc / d2) + gB * (-(a * cc + b * b) / d2) + gC * (2.0 * a * b / d2);
            const double gc = gA * (-b * b / d2) + gB * (a * b / d2) + gC * (-a * a / d2);
            /* Cov2 = M Sigma M^T; as a symmetric matrix G = [[ga, gb/2], [gb/2, gc]] */
            const double Gs[4] = {ga, 0.5 * gb, 0.5 * gb, gc};
            double GM[6], gM[6], Mt[6], tmp[6], gSigma[9], gJ[6], Rt[9];
            matmul(Gs, g.M, GM, 2, 2, 3);
            matmul(GM, g.Sigma, gM, 2, 3, 3);
            for (k = 0; k < 6; ++k) gM[k] *= 2.0;              /* dL/dM = 2 G M Sigma */
            transpose(g.M, Mt, 2, 3);
            matmul(Mt, Gs, tmp, 3, 2, 2);
            matmul(tmp, g.M, gSigma, 3, 2, 3);                  /* dL/dSigma = M^T G M */
            /* M = J Rc -> dL/dJ = dL/dM Rc^T */
            transpose(Rc, Rt, 3, 3);
            matmul(gM, Rt, gJ, 2, 3, 3);
            /* J entries as functions of t_cam */
            {
                const double tz = g.tcam[2], fx = cam->fx, fy = cam->fy;
                gt[2] += gJ[0] * (-fx / (tz * tz)) + gJ[4] * (-fy / (tz * tz));
                if (!g.clampx) {
                    gt[0] += gJ[2] * (-fx / (tz * tz));
                    gt[2] += gJ[2] * (2.0 * fx * g.tcam[0] / (tz * tz * tz));
                } else {
                    gt[2] += gJ[2] * (fx * g.uxc / (tz * tz));
                }
                if (!g.clampy) {
                    gt[1] += gJ[5] * (-fy / (tz * tz));
                    gt[2] += gJ[5] * (2.0 * fy * g.tcam[1] / (tz * tz * tz));
                } else {
                    gt[2] += gJ[5] * (fy * g.uyc / (tz * tz));
                }
            }
            /* Sigma = Rq diag(s2) Rq^T: dL/dRq = 2 gSigma Rq diag(s2), dL/ds2_k = (Rq^T gSigma Rq)_kk */
            {
                double gR[9], RtG[9], RtGR[9], RqT[9], GR[9];
                matmul(gSigma, g.Rq, GR, 3, 3, 3);
                for (r = 0; r < 3; ++r)
                    for (c = 0; c < 3; ++c) gR[3 * r + c] = 2.0 * GR[3 * r + c] * g.s2[c];
                transpose(g.Rq, RqT, 3, 3);
                matmul(RqT, gSigma, RtG, 3, 3, 3);
                matmul(RtG, g.Rq, RtGR, 3, 3, 3);
                /* s2_k = exp(2 l_k) */
                for (k = 0; k < 3; ++k) g_log_scales[k * n + i] = RtGR[4 * k] * 2.0 * g.s2[k];
                /* rotation entries as functions of the unit quaternion (w, x, y, z) */
                {
                    const double w = g.qn[0], x = g.qn[1], y = g.qn[2], z = g.qn[3];
                    double gq[4], dot = 0.0;
                    gq[0] = 2.0 * (-z * gR[1] + y * gR[2] + z * gR[3] - x * gR[5] - y * gR[6] + x * gR[7]);
                    gq[1] = 2.0 * (y * gR[1] + z * gR[2] + y * gR[3] - 2.0 * x * gR[4] - w * gR[5]
                                   + z * gR[6] + w * gR[7] - 2.0 * x * gR[8]);
                    gq[2] = 2.0 * (-2.0 * y * gR[0] + x * gR[1] + w * gR[2] + x * gR[3] + z * gR[5]
                                   - w * gR[6] + z * gR[7] - 2.0 * y * gR[8]);
                    gq[3] = 2.0 * (-2.0 * z * gR[0] - w * gR[1] + x * gR[2] + w * gR[3] - 2.0 * z * gR[4]
                                   + y * gR[5] + x * gR[6] + y * gR[7]);
                    /* qn = q / |q| */
                    for (k = 0; k < 4; ++k) dot += g.qn[k] * gq[k];
                    for (k = 0; k < 4; ++k) g_quats[k * n + i] = (gq[k] - g.qn[k] * dot) / g.qnorm;
                }
            }
        }
        /* 2D mean = (fx tx / tz + cx, fy ty / tz + cy) */
        {
            const double tz = g.tcam[2];
            const double gmx = g_mean2d[i], gmy = g_mean2d[n + i];
            gt[0] += gmx * cam->fx / tz;
            gt[1] += gmy * cam->fy / tz;
            gt[2] += -gmx * cam->fx * g.tcam[0] / (tz * tz) - gmy * cam->fy * g.tcam[1] / (tz * tz);
        }
        /* 1 / depth with depth = t_cam z */
        if (g_invd) gt[2] += -g_invd[i] / (g.tcam[2] * g.tcam[2]);
        /* t_cam = Rc m + t  ->  dL/dm += Rc^T dL/dt */
        for (c = 0; c < 3; ++c) gm[c] += Rc[c] * gt[0] + Rc[3 + c] * gt[1] + Rc[6 + c] * gt[2];
        for (c = 0; c < 3; ++c) g_means[c * n + i] = gm[c];
    }
    return 0;
}

/* Threads the OpenMP loops use from now on (the CPU baseline's one-thread run). */
void ora_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int ora_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

const char* ora_version(void) { return "gs_oracle 1"; }
