/*
 * slag_oracle.c -- plain FP64 CPU oracle for the loss-free embedding lift.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code with the GPU library.
 *
 * What it computes (paper, Method section, "Semantic Embedding"):
 *   - each Gaussian is projected to a screen mean and a 2D covariance
 *     (the rasterizer call with K_i, R_i, t_i), here by EWA splatting;
 *   - at every pixel p the Gaussians are visited front to back and each gets
 *     the blend weight w_kp = alpha_kp * T_kp (the rasterizer's contribution
 *     weight, our reading of the weight the modified rasterizer captures);
 *   - the weight is masked by the segment that owns the pixel (parameter
 *     masking, w'_kp = w_kp * M_j(p)) and summed per (Gaussian, segment)
 *     (the aggregation equation's numerator and denominator sums over p).
 * The view sums are returned as sparse (Gaussian, segment, W) triples; the
 * contraction with the feature table and the normalisation are done by the
 * Python half of the oracle.
 *
 * Conventions the paper leaves open (taken from 3D Gaussian splatting; the
 * defaults below, settable with orc_set_constants like the library's
 * options):
 *   alpha = min(0.99, o * exp(-q/2)), q = d^T Sigma2^{-1} d, d = p - mu2,
 *   p = pixel centre (u+0.5, v+0.5); contributions with alpha < 1/255 are
 *   skipped; the walk stops *before* a Gaussian whose blend would take the
 *   transmittance below 1e-4; Sigma2 gets +0.3 px^2 on its diagonal; the
 *   Jacobian is evaluated at x/z, y/z clamped to 1.3 x the half-FOV tangent;
 *   Gaussians with camera z <= 0.01 are culled.  q is clamped at 0 (a
 *   positive-definite conic never gives q < 0; only rounding could).
 *
 * Depth order and culling are integer decisions taken from floating point,
 * so they are taken in the kernel's precision: this file carries its own
 * FP32 evaluation of camera depth and of the conservative pixel box, written
 * op by op from the normative sequence documented with the library (fmaf
 * where a fused multiply-add is specified, correctly rounded / and sqrt, no
 * other contraction; build with -ffp-contract=off).  Everything that weighs a
 * contribution is FP64.
 *
 * Error model and decision margins.  The weights are exact (FP64) here; an
 * FP32 evaluation of the same walk deviates from them in two ways, and this
 * file bounds both, per (Gaussian, segment) triple, from the FP64 values:
 *   - rounding mass r: to first order, the relative error of an FP32 weight
 *     w = alpha T is at most eps_alpha + rho_T + 2^-24, where eps_alpha
 *     bounds the relative error of alpha (alpha_eps below: the exponent is
 *     a quadratic in the pixel offset, evaluated in FP32 from FP32-rounded
 *     coefficients as an expansion about a point within 3.5 px of the pixel
 *     in each axis; every rounding is counted with the magnitude of the
 *     value it rounds; exp2 adds 2 ulp) and rho_T bounds the relative error
 *     of the transmittance, which grows by eps_alpha alpha / (1 - alpha) +
 *     2^-24 per blend (alpha clamped at 0.99 on both sides carries no error);
 *   - decision mass U: a threshold decision (alpha against 1/255, T' against
 *     1e-4) whose FP64 operand lies within that error bound of the threshold
 *     may go the other way in FP32; U bounds how much W could move because
 *     of it (see composite_pixel).  With U = 0 a triple must match exactly
 *     in membership.
 * Both bounds are derived from the operation sequence, not fitted to any
 * observed error; a test re-walks the same per-pixel lists in FP32
 * (orc_lift_view_f32) and checks that it stays inside them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    float fx, fy, cx, cy;
    float R[9];
    float t[3];
    int32_t width, height;
} orc_camera;

typedef struct {
    int64_t n_contrib;          /* accepted blends, all pixels (background included) */
    int64_t n_tests;            /* box candidates evaluated before termination */
    int64_t n_visible;          /* Gaussians with z > near, det > 0, non-empty box */
    int64_t n_uncertain;        /* near-threshold decisions met */
} orc_counts;

/* ---- Rasterizer constants (3D Gaussian splatting's by default; settable,
 * orc_set_constants, to mirror the library's options).  FP32 decision values
 * (exact bit patterns) and the FP64 weighting values. ---- */
static float F_NEAR = 0.01f;
static float F_DIL = 0.3f;
static float F_CLAMP = 1.3f;
static float F_RHO2 = 0x1.62a41p+3f;       /* float nearest to 2 ln 255: q bound of alpha >= 1/255 */
static float F_AMIN = 1.0f / 255.0f, F_AMAX = 0.99f, F_TMIN = 1e-4f;
static double D_AMIN = 1.0 / 255.0;
static double D_AMAX = 0.99;
static double D_TMIN = 1e-4;
static double D_DIL = 0.3;
static double D_CLAMP = 1.3;
/* Weight of a blended Gaussian: 0 = alpha T (the front-to-back blend weight,
 * the default reading), 1 = the Gaussian kernel exp(-q/2) itself (the
 * paper's weight equation) for each Gaussian the walk blends. */
static int g_kernel_w = 0;

/* Non-default constants, each given as the float the library receives:
 * c = (alpha_max, alpha_min, t_min, dilation, near_z, guard, weight mode),
 * 0 = default (weight mode 1: kernel weights).
 * The FP64 values are those floats widened; rho^2 = 2 ln(1 / alpha_min) is
 * rounded once to float (the default keeps the float nearest to 2 ln 255). */
void orc_set_constants(const float* c)
{
    F_AMAX = c[0] > 0.0f ? c[0] : 0.99f;
    D_AMAX = c[0] > 0.0f ? (double)c[0] : 0.99;
    F_AMIN = c[1] > 0.0f ? c[1] : 1.0f / 255.0f;
    D_AMIN = c[1] > 0.0f ? (double)c[1] : 1.0 / 255.0;
    F_RHO2 = c[1] > 0.0f ? (float)(2.0 * log(1.0 / (double)c[1])) : 0x1.62a41p+3f;
    F_TMIN = c[2] > 0.0f ? c[2] : 1e-4f;
    D_TMIN = c[2] > 0.0f ? (double)c[2] : 1e-4;
    F_DIL = c[3] > 0.0f ? c[3] : 0.3f;
    D_DIL = c[3] > 0.0f ? (double)c[3] : 0.3;
    F_NEAR = c[4] > 0.0f ? c[4] : 0.01f;
    F_CLAMP = c[5] > 0.0f ? c[5] : 1.3f;
    D_CLAMP = c[5] > 0.0f ? (double)c[5] : 1.3;
    g_kernel_w = c[6] > 0.0f;
}

#define D_L2E 1.4426950408889634074      /* log2(e) */
#define D_LN2 0.69314718055994530942
#define U32 0x1p-24                          /* unit roundoff of FP32 */
#define ORC_MAX_LABELS 8                     /* masks a pixel may lie in (overlapping masks) */
/* FP32 thresholds differ from the FP64 ones by at most this relative amount
 * ((float)(1/255) and 1e-4f are rounded) */
#define CONST_REL 0x1p-23

/* ========================================================================
 * FP32 mirror: camera depth, culling and the conservative pixel box.
 * ====================================================================== */
typedef struct {
    int vis_depth;      /* z32 > near and det32 > 0 */
    int vis;            /* vis_depth and the box is non-empty */
    float z32;
    int32_t x0, x1, y0, y1;
    float u, v, c00, c01, c11;
} mirror_out;

static void mirror_project(const float* m, const float* s, const float* q,
                           const orc_camera* c, mirror_out* o)
{
    const float* R = c->R;
    memset(o, 0, sizeof(*o));
    float X = fmaf(R[0], m[0], fmaf(R[1], m[1], fmaf(R[2], m[2], c->t[0])));
    float Y = fmaf(R[3], m[0], fmaf(R[4], m[1], fmaf(R[5], m[2], c->t[1])));
    float Z = fmaf(R[6], m[0], fmaf(R[7], m[1], fmaf(R[8], m[2], c->t[2])));
    o->z32 = Z;
    if (!(Z > F_NEAR)) return;

    float nq = fmaf(q[0], q[0], fmaf(q[1], q[1], fmaf(q[2], q[2], q[3] * q[3])));
    float rn = 1.0f / sqrtf(nq);
    float w = q[0] * rn, x = q[1] * rn, y = q[2] * rn, z = q[3] * rn;
    float r[9];
    r[0] = 1.0f - 2.0f * fmaf(y, y, z * z);
    r[1] = 2.0f * fmaf(x, y, -(w * z));
    r[2] = 2.0f * fmaf(x, z, (w * y));
    r[3] = 2.0f * fmaf(x, y, (w * z));
    r[4] = 1.0f - 2.0f * fmaf(x, x, z * z);
    r[5] = 2.0f * fmaf(y, z, -(w * x));
    r[6] = 2.0f * fmaf(x, z, -(w * y));
    r[7] = 2.0f * fmaf(y, z, (w * x));
    r[8] = 1.0f - 2.0f * fmaf(x, x, y * y);
    float M[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) M[3 * i + j] = r[3 * i + j] * s[j];
    float S[9];
    for (int i = 0; i < 3; i++)
        for (int j = i; j < 3; j++) {
            float v = fmaf(M[3 * i + 0], M[3 * j + 0],
                           fmaf(M[3 * i + 1], M[3 * j + 1], M[3 * i + 2] * M[3 * j + 2]));
            S[3 * i + j] = v;
            S[3 * j + i] = v;
        }

    float iz = 1.0f / Z;
    float txr = X * iz, tyr = Y * iz;
    float limx = F_CLAMP * ((0.5f * (float)c->width) / c->fx);
    float limy = F_CLAMP * ((0.5f * (float)c->height) / c->fy);
    float tx = fminf(limx, fmaxf(-limx, txr));
    float ty = fminf(limy, fmaxf(-limy, tyr));
    float j00 = c->fx * iz, j02 = -(j00 * tx);
    float j11 = c->fy * iz, j12 = -(j11 * ty);
    float A[6];
    for (int k = 0; k < 3; k++) {
        A[k] = fmaf(j00, R[k], j02 * R[6 + k]);
        A[3 + k] = fmaf(j11, R[3 + k], j12 * R[6 + k]);
    }
    float B[6];
    for (int i = 0; i < 2; i++)
        for (int k = 0; k < 3; k++)
            B[3 * i + k] = fmaf(A[3 * i + 0], S[0 + k],
                                fmaf(A[3 * i + 1], S[3 + k], A[3 * i + 2] * S[6 + k]));
    float c00 = fmaf(B[0], A[0], fmaf(B[1], A[1], B[2] * A[2])) + F_DIL;
    float c01 = fmaf(B[0], A[3], fmaf(B[1], A[4], B[2] * A[5]));
    float c11 = fmaf(B[3], A[3], fmaf(B[4], A[4], B[5] * A[5])) + F_DIL;
    float det = fmaf(c00, c11, -(c01 * c01));
    if (!(det > 0.0f)) return;
    o->vis_depth = 1;

    float u = fmaf(c->fx, txr, c->cx);
    float v = fmaf(c->fy, tyr, c->cy);
    float ex = sqrtf(F_RHO2 * c00);
    float ey = sqrtf(F_RHO2 * c11);
    float x0 = ceilf(u - (ex + 1.5f)), x1 = floorf(u + (ex + 0.5f));
    float y0 = ceilf(v - (ey + 1.5f)), y1 = floorf(v + (ey + 0.5f));
    float wm1 = (float)(c->width - 1), hm1 = (float)(c->height - 1);
    o->u = u; o->v = v; o->c00 = c00; o->c01 = c01; o->c11 = c11;
    if (!(x0 <= wm1 && x1 >= 0.0f && y0 <= hm1 && y1 >= 0.0f)) return;
    x0 = fmaxf(x0, 0.0f); x1 = fminf(x1, wm1);
    y0 = fmaxf(y0, 0.0f); y1 = fminf(y1, hm1);
    o->x0 = (int32_t)x0; o->x1 = (int32_t)x1;
    o->y0 = (int32_t)y0; o->y1 = (int32_t)y1;
    o->vis = 1;
}

/* ========================================================================
 * FP64 EWA projection (the rasterizer's projection step).
 * ====================================================================== */
typedef struct {
    double mu[2];
    double cov[3];      /* Sigma2 (with dilation): xx, xy, yy */
    double conic[3];    /* Sigma2^{-1}: xx, xy, yy */
    double zc;          /* camera-space depth */
    double o;
    double lo2;         /* log2(o) */
} proj64;

static void project64(const float* mf, const float* sf, const float* qf, float opac,
                      const orc_camera* c, proj64* p)
{
    double R[9], t[3], m[3];
    for (int i = 0; i < 9; i++) R[i] = c->R[i];
    for (int i = 0; i < 3; i++) { t[i] = c->t[i]; m[i] = mf[i]; }
    /* camera-space mean: m_c = R mu + t */
    double X = R[0] * m[0] + R[1] * m[1] + R[2] * m[2] + t[0];
    double Y = R[3] * m[0] + R[4] * m[1] + R[5] * m[2] + t[1];
    double Z = R[6] * m[0] + R[7] * m[1] + R[8] * m[2] + t[2];
    /* rotation of the Gaussian from its unit quaternion (w, x, y, z) */
    double qn = sqrt((double)qf[0] * qf[0] + (double)qf[1] * qf[1] +
                     (double)qf[2] * qf[2] + (double)qf[3] * qf[3]);
    double w = qf[0] / qn, x = qf[1] / qn, y = qf[2] / qn, z = qf[3] / qn;
    double Rq[9] = {
        1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
        2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
        2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
    /* world covariance Sigma3 = Rq diag(s^2) Rq^T */
    double S[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double acc = 0;
            for (int k = 0; k < 3; k++)
                acc += Rq[3 * i + k] * ((double)sf[k] * sf[k]) * Rq[3 * j + k];
            S[3 * i + j] = acc;
        }
    /* camera covariance C = R Sigma3 R^T */
    double RS[9], C[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double acc = 0;
            for (int k = 0; k < 3; k++) acc += R[3 * i + k] * S[3 * k + j];
            RS[3 * i + j] = acc;
        }
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double acc = 0;
            for (int k = 0; k < 3; k++) acc += RS[3 * i + k] * R[3 * j + k];
            C[3 * i + j] = acc;
        }
    /* Jacobian of (fx X/Z + cx, fy Y/Z + cy) at the guard-clamped point */
    double limx = D_CLAMP * (0.5 * c->width / (double)c->fx);
    double limy = D_CLAMP * (0.5 * c->height / (double)c->fy);
    double txz = X / Z, tyz = Y / Z;
    double cx_ = fmin(limx, fmax(-limx, txz)), cy_ = fmin(limy, fmax(-limy, tyz));
    double J[6] = {c->fx / Z, 0.0, -c->fx * cx_ / Z, 0.0, c->fy / Z, -c->fy * cy_ / Z};
    /* Sigma2 = J C J^T + 0.3 I */
    double JC[6];
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 3; j++) {
            double acc = 0;
            for (int k = 0; k < 3; k++) acc += J[3 * i + k] * C[3 * k + j];
            JC[3 * i + j] = acc;
        }
    double s2[4];
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) {
            double acc = 0;
            for (int k = 0; k < 3; k++) acc += JC[3 * i + k] * J[3 * j + k];
            s2[2 * i + j] = acc;
        }
    double a = s2[0] + D_DIL, b = 0.5 * (s2[1] + s2[2]), d = s2[3] + D_DIL;
    double det = a * d - b * b;
    p->cov[0] = a; p->cov[1] = b; p->cov[2] = d;
    p->conic[0] = d / det; p->conic[1] = -b / det; p->conic[2] = a / det;
    p->mu[0] = c->fx * txz + c->cx;
    p->mu[1] = c->fy * tyz + c->cy;
    p->zc = Z;
    p->o = opac;
    p->lo2 = log2((double)opac);
}

/* ========================================================================
 * growable arrays and a (g,s) -> (W,U) hash map
 * ====================================================================== */
typedef struct { int32_t g, s; double w, u, r; } contrib;
typedef struct { contrib* a; int64_t n, cap; } cbuf;

static int cbuf_push(cbuf* b, int32_t g, int32_t s, double w, double u, double r)
{
    if (b->n == b->cap) {
        int64_t nc = b->cap ? 2 * b->cap : 256;
        contrib* na = (contrib*)realloc(b->a, (size_t)nc * sizeof(contrib));
        if (!na) return -1;
        b->a = na; b->cap = nc;
    }
    b->a[b->n].g = g; b->a[b->n].s = s; b->a[b->n].w = w; b->a[b->n].u = u;
    b->a[b->n].r = r;
    b->n++;
    return 0;
}

typedef struct { uint64_t* key; double* w; double* u; double* r; int64_t cap, n; } hmap;
#define HEMPTY 0xFFFFFFFFFFFFFFFFull

/* One contribution to every mask that contains the pixel (overlapping masks:
 * the weight goes to each of the pixel's labels). */
static int push_labels(cbuf* b, int32_t g, const int32_t* segs, int nl, double w, double u,
                       double r)
{
    for (int i = 0; i < nl; i++)
        if (cbuf_push(b, g, segs[i], w, u, r)) return 1;
    return 0;
}

static int hmap_init(hmap* h, int64_t cap)
{
    int64_t c = 1024;
    while (c < 2 * cap) c <<= 1;
    h->key = (uint64_t*)malloc((size_t)c * 8);
    h->w = (double*)calloc((size_t)c, 8);
    h->u = (double*)calloc((size_t)c, 8);
    h->r = (double*)calloc((size_t)c, 8);
    if (!h->key || !h->w || !h->u || !h->r) return -1;
    memset(h->key, 0xFF, (size_t)c * 8);
    h->cap = c; h->n = 0;
    return 0;
}

static void hmap_free(hmap* h) { free(h->key); free(h->w); free(h->u); free(h->r); }

static int64_t hslot(const hmap* h, uint64_t k)
{
    uint64_t x = k * 0x9E3779B97F4A7C15ull;
    int64_t i = (int64_t)(x >> 17) & (h->cap - 1);
    while (h->key[i] != HEMPTY && h->key[i] != k) i = (i + 1) & (h->cap - 1);
    return i;
}

static int hmap_add(hmap* h, uint64_t k, double w, double u, double r)
{
    if (2 * (h->n + 1) > h->cap) {
        hmap nh;
        if (hmap_init(&nh, h->cap)) return -1;
        for (int64_t i = 0; i < h->cap; i++)
            if (h->key[i] != HEMPTY) {
                int64_t j = hslot(&nh, h->key[i]);
                nh.key[j] = h->key[i]; nh.w[j] = h->w[i]; nh.u[j] = h->u[i];
                nh.r[j] = h->r[i]; nh.n++;
            }
        hmap_free(h);
        *h = nh;
    }
    int64_t i = hslot(h, k);
    if (h->key[i] == HEMPTY) { h->key[i] = k; h->n++; }
    h->w[i] += w;
    h->u[i] += u;
    h->r[i] += r;
    return 0;
}

/* ========================================================================
 * per-pixel front-to-back walk
 * ====================================================================== */
typedef struct {
    const proj64* P;
    const mirror_out* Mi;
} view_ctx;

/* alpha = min(0.99, o exp(-q/2)) with q = d^T Sigma2^{-1} d; also returns
 * the unclamped value */
static inline double alpha_at(const proj64* p, double px, double py, double* unclamped)
{
    double dx = px - p->mu[0], dy = py - p->mu[1];
    double q = p->conic[0] * dx * dx + 2.0 * p->conic[1] * dx * dy + p->conic[2] * dy * dy;
    if (q < 0.0) q = 0.0;
    double a = p->o * exp(-0.5 * q);
    if (unclamped) *unclamped = a;
    return a < D_AMAX ? a : D_AMAX;
}

/*
 * Bound on the relative error of an FP32 alpha at pixel centre (px, py).
 * The FP32 exponent is e = log2(o) + A dx^2 + B dx dy + C dy^2 with
 * A = -log2(e) conic_xx / 2, B = -log2(e) conic_xy, C = -log2(e) conic_yy / 2
 * and (dx, dy) the offset of the pixel from the mean, evaluated from FP32
 * roundings of A, B, C, log2(o) and of the mean's offset from the box corner
 * (x0, y0), as a quadratic expanded about a point within L = 3.5 px of the
 * pixel in each axis:  c0 + lx (cx + A lx + B ly) + ly (cy + C ly), with c0,
 * cx, cy the value and gradient at the expansion point (three FMA chains).
 * Magnitudes (a, b, c = |A|, |B|, |C|; U, V bound the expansion point's
 * offset from the mean; X, Y its gradient; M0 its value):
 *   coefficient rounding         u (a dx^2 + b |dx dy| + c dy^2 + |log2 o|)
 *   mean-offset rounding         u (2a|dx| + b|dy|)(|u - x0| + U) + (same in y)
 *   value and gradient at the
 *   expansion point (5 + 2 ops)  <= 7 u M0
 *   per-pixel chains             <= 6 u L (X + Y) + 4 u L^2 (a + b + c)
 * (each rounding bounded by u = 2^-24 times the magnitude it rounds,
 * propagated through the multiplications by lx, ly, |lx|, |ly| <= L).
 * alpha = 2^e then has relative error ln 2 |de| + 2^-22 (exp2: 2 ulp).
 */
static double alpha_eps(const proj64* p, const mirror_out* mo, double px, double py)
{
    const double a = 0.5 * D_L2E * fabs(p->conic[0]);
    const double b = D_L2E * fabs(p->conic[1]);
    const double c = 0.5 * D_L2E * fabs(p->conic[2]);
    const double lo2 = fabs(p->lo2);
    const double dx = fabs(px - p->mu[0]), dy = fabs(py - p->mu[1]);
    const double L = 3.5, U = dx + L, V = dy + L;
    const double Mpix = a * dx * dx + b * dx * dy + c * dy * dy + lo2;
    const double M0 = a * U * U + b * U * V + c * V * V + lo2;
    const double X = 2.0 * a * U + b * V, Y = b * U + 2.0 * c * V;
    const double ur = fabs(p->mu[0] - (double)mo->x0), vr = fabs(p->mu[1] - (double)mo->y0);
    const double G = (2.0 * a * dx + b * dy) * (ur + U) + (b * dx + 2.0 * c * dy) * (vr + V);
    const double de = U32 * (Mpix + 7.0 * M0 + 6.0 * L * (X + Y) + 4.0 * L * L * (a + b + c) + G);
    return D_LN2 * de * (1.0 + 1e-6) + 0x1p-22;
}

/*
 * Walk the depth-ordered candidates of one pixel.  Emits (g, s, w, u, r) for
 * accepted blends when the pixel has a segment (s >= 0).
 *
 * rho is the bound on the FP32 transmittance's relative error (given the
 * same decisions so far); eps that of alpha (alpha_eps, plus the rounding of
 * the FP32 threshold constants).  r = w (eps + rho + 2^-24) bounds the
 * rounding of the weight.  u bounds how far a flipped decision could move a
 * contribution:
 *  - alpha with alpha (1 - eps) < 1/255 <= alpha may be skipped (u = w), and
 *    one with alpha < 1/255 <= alpha (1 + eps) may be taken (a zero-weight
 *    entry with u = its possible weight); either flip scales the
 *    transmittance seen by everything behind it by (1 - alpha), so later
 *    blends get u += w delta with delta += alpha / (1 - alpha);
 *  - a stop decision with |T' - 1e-4| within (rho' + delta) of T' may go the
 *    other way: if the walk continues here, this and every later blend may
 *    vanish (u = w, delta = 1); if it stops here, this Gaussian and the next
 *    acceptable one may still be blended (entries with u = their weights).
 * Returns the final T, the sum of weights, the final rho, and whether any
 * decision of the pixel lay inside its band.
 */
static int composite_pixel(const view_ctx* vc, const int32_t* cand, int64_t nc,
                           int ix, int iy, const int32_t* segs, int nl, cbuf* out,
                           double* T_out, double* wsum_out, double* rho_out, int* near_out,
                           int64_t* n_c, int64_t* n_q, int64_t* n_unc, int count_box_only)
{
    const double px = ix + 0.5, py = iy + 0.5;
    double T = 1.0, rho = 0.0, delta = 0.0, sumw = 0.0;
    int any_near = 0;
    for (int64_t k = 0; k < nc; k++) {
        const int32_t g = cand[k];
        const proj64* p = &vc->P[g];
        const mirror_out* mo = &vc->Mi[g];
        if (!count_box_only || (mo->vis && ix >= mo->x0 && ix <= mo->x1 && iy >= mo->y0 && iy <= mo->y1))
            (*n_q)++;
        double au;
        const double alpha = alpha_at(p, px, py, &au);
        const double eps = alpha_eps(p, mo, px, py) + CONST_REL;
        /* both sides clamp at 0.99 when even the lower FP32 value exceeds it */
        const double ea = (au * (1.0 - eps) >= D_AMAX) ? 0.0 : eps;
        const double dl = delta < 1.0 ? delta : 1.0;
        const double grow = 1.0 + dl;
        /* the weight this Gaussian would get: alpha T, or its kernel value
         * (unclamped alpha / o); with kernel weights T carries no error */
        const double kv = au / p->o;
        const double wt = g_kernel_w ? kv : alpha * T;
        const double rt = g_kernel_w ? 0.0 : rho;
        if (alpha < D_AMIN) {
            if (alpha * (1.0 + eps) >= D_AMIN) {
                (*n_unc)++;
                any_near = 1;
                if (push_labels(out, g, segs, nl, 0.0, wt * grow * (1.0 + eps + rt), 0.0))
                    return -1;
                delta += alpha / (1.0 - alpha);
            }
            continue;
        }
        const int near_a = alpha * (1.0 - eps) < D_AMIN;
        const double Tn = T * (1.0 - alpha);
        const double rho_n = rho + ea * alpha / (1.0 - alpha) + U32;
        const double band = (rho_n + CONST_REL + dl) * (Tn > D_TMIN ? Tn : D_TMIN);
        const int near_t = fabs(Tn - D_TMIN) <= band;
        if (near_a || near_t) { (*n_unc)++; any_near = 1; }
        if (Tn < D_TMIN) {
            if (near_t && nl > 0) {
                if (push_labels(out, g, segs, nl, 0.0, wt * grow * (1.0 + ea + rt), 0.0))
                    return -1;
                for (int64_t h = k + 1; h < nc; h++) {
                    const proj64* ph = &vc->P[cand[h]];
                    double ahu;
                    const double ah = alpha_at(ph, px, py, &ahu);
                    const double eh = alpha_eps(ph, &vc->Mi[cand[h]], px, py) + CONST_REL;
                    if (ah * (1.0 + eh) >= D_AMIN) {
                        const double wh = g_kernel_w ? ahu / ph->o : ah * Tn;
                        if (push_labels(out, cand[h], segs, nl, 0.0,
                                        wh * grow * (1.0 + eh + (g_kernel_w ? 0.0 : rho_n)), 0.0))
                            return -1;
                        break;
                    }
                }
            }
            break;
        }
        /* kernel weights: exp2 of the exponent less log2(o), one more
         * subtraction and the exp2 of the FP32 path */
        const double w = wt;
        const double r = g_kernel_w ? w * (eps + U32 * (5.0 + D_LN2 * (fabs(p->lo2) - log2(kv))))
                                    : w * (ea + rho + U32);
        double u = w * dl;
        if (near_a) u = w * grow;
        if (near_t) { u = w * grow; delta = 1.0; }
        (*n_c)++;
        sumw += w;
        if (push_labels(out, g, segs, nl, w, u, r)) return -1;
        if (near_a) delta += alpha / (1.0 - alpha);
        T = Tn;
        rho = rho_n;
    }
    *T_out = T;
    *wsum_out = sumw;
    *rho_out = rho;
    *near_out = any_near;
    return 0;
}

/*
 * The same per-pixel walk in FP32, evaluated the way a tile rasterizer with
 * 8x8-pixel wave blocks does it: the exponent is expanded about the centre of
 * the pixel's aligned 8x8 block (lx, ly in -3.5 .. 3.5), from coefficients
 * rounded to FP32 once per Gaussian (the mean as an offset from the box
 * corner).  Test infrastructure for the error model above: its weights must
 * stay within r + U of the FP64 walk's.  Decisions are taken in FP32.
 */
static int composite_pixel_f32(const view_ctx* vc, const int32_t* cand, int64_t nc,
                               int ix, int iy, const int32_t* segs, int nl, cbuf* out, double* T_out,
                               double* wsum_out)
{
    const float AMIN_F = F_AMIN, AMAX_F = F_AMAX, TMIN_F = F_TMIN;
    const int bx0 = ix & ~7, by0 = iy & ~7;
    const float lx = (float)(ix & 7) - 3.5f, ly = (float)(iy & 7) - 3.5f;
    float T = 1.0f;
    double sumw = 0.0;
    for (int64_t k = 0; k < nc; k++) {
        const int32_t g = cand[k];
        const proj64* p = &vc->P[g];
        const mirror_out* mo = &vc->Mi[g];
        const float A = (float)(-0.5 * D_L2E * p->conic[0]);
        const float B = (float)(-D_L2E * p->conic[1]);
        const float C = (float)(-0.5 * D_L2E * p->conic[2]);
        const float lo2 = (float)p->lo2;
        const float urel = (float)(p->mu[0] - (double)mo->x0);
        const float vrel = (float)(p->mu[1] - (double)mo->y0);
        const float du = urel + (float)(mo->x0 - bx0 - 4);   /* mean minus block centre */
        const float dv = vrel + (float)(mo->y0 - by0 - 4);
        const float cx = -fmaf(2.0f * A, du, B * dv);
        const float cy = -fmaf(B, du, 2.0f * C * dv);
        const float c0 = fmaf(A * du, du, fmaf(B * du, dv, C * dv * dv)) + lo2;
        const float tx = fmaf(B, ly, fmaf(A, lx, cx));
        const float ty = fmaf(C, ly, cy);
        const float e = fmaf(ty, ly, fmaf(tx, lx, c0));
        const float alpha = fminf(AMAX_F, exp2f(e));
        if (!(alpha >= AMIN_F)) continue;
        const float Tn = fmaf(-alpha, T, T);
        if (Tn < TMIN_F) break;
        const float w = g_kernel_w ? exp2f(e - lo2) : alpha * T;
        sumw += (double)w;
        if (push_labels(out, g, segs, nl, (double)w, 0.0, 0.0)) return -1;
        T = Tn;
    }
    *T_out = (double)T;
    *wsum_out = sumw;
    return 0;
}

/* depth order: ascending FP32 camera z, ties to the lower Gaussian index */
static const float* g_sort_z;
static int cmp_depth(const void* a, const void* b)
{
    int32_t ga = *(const int32_t*)a, gb = *(const int32_t*)b;
    float za = g_sort_z[ga], zb = g_sort_z[gb];
    if (za < zb) return -1;
    if (za > zb) return 1;
    return (ga > gb) - (ga < gb);
}

typedef struct { const float* z; int32_t* a; } sort_job;

/* insertion/merge sort on a small array with the same order as cmp_depth;
 * thread-safe (no global state) */
static void sort_depth(int32_t* a, int64_t n, const float* z, int32_t* tmp)
{
    if (n < 24) {
        for (int64_t i = 1; i < n; i++) {
            int32_t v = a[i];
            int64_t j = i - 1;
            while (j >= 0 && (z[a[j]] > z[v] || (z[a[j]] == z[v] && a[j] > v))) {
                a[j + 1] = a[j];
                j--;
            }
            a[j + 1] = v;
        }
        return;
    }
    int64_t h = n / 2;
    sort_depth(a, h, z, tmp);
    sort_depth(a + h, n - h, z, tmp);
    int64_t i = 0, j = h, k = 0;
    while (i < h && j < n) {
        int32_t x = a[i], y = a[j];
        int take_y = (z[y] < z[x]) || (z[y] == z[x] && y < x);
        tmp[k++] = take_y ? a[j++] : a[i++];
    }
    while (i < h) tmp[k++] = a[i++];
    while (j < n) tmp[k++] = a[j++];
    memcpy(a, tmp, (size_t)n * sizeof(int32_t));
}

typedef struct {
    int64_t n_triples;
    int32_t* g;
    int32_t* s;
    double* w;
    double* u;
    double* r;
} view_result;

static int cmp_u64(const void* a, const void* b)
{
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return (x > y) - (x < y);
}

/*
 * Per-pixel candidate lists of the box mode: start[npix + 1] (zeroed by the
 * caller) receives the offsets, the returned array the Gaussians whose
 * conservative pixel box contains each pixel, in index order (NULL when out
 * of memory).
 */
static int32_t* box_candidates(int64_t n, const mirror_out* Mi, int W, int H, int64_t* start)
{
    const int64_t npix = (int64_t)W * H;
    for (int64_t g = 0; g < n; g++) {
        const mirror_out* m = &Mi[g];
        if (!m->vis) continue;
        for (int y = m->y0; y <= m->y1; y++)
            for (int x = m->x0; x <= m->x1; x++) start[(int64_t)y * W + x + 1]++;
    }
    for (int64_t i = 0; i < npix; i++) start[i + 1] += start[i];
    int32_t* cand = (int32_t*)malloc((size_t)(start[npix] ? start[npix] : 1) * sizeof(int32_t));
    int64_t* fill = (int64_t*)malloc((size_t)(npix ? npix : 1) * sizeof(int64_t));
    if (!cand || !fill) { free(cand); free(fill); return NULL; }
    memcpy(fill, start, (size_t)npix * sizeof(int64_t));
    for (int64_t g = 0; g < n; g++) {
        const mirror_out* m = &Mi[g];
        if (!m->vis) continue;
        for (int y = m->y0; y <= m->y1; y++)
            for (int x = m->x0; x <= m->x1; x++) cand[fill[(int64_t)y * W + x]++] = (int32_t)g;
    }
    free(fill);
    return cand;
}

/*
 * Lift one view.  mode bit 0: 0 = brute (every Gaussian in front of the
 * camera is a candidate of every pixel), 1 = box (only Gaussians whose
 * conservative pixel box contains the pixel).  Both walk candidates in the
 * same depth order, so the two must agree bit for bit.  Mode bit 1 selects the
 * FP32 walk (composite_pixel_f32; box candidates only, no margins or counts).
 * pix_rho (optional) receives the final T's relative error bound, or -1 at
 * pixels where some decision lay inside its band.
 */
void* orc_lift_view(int64_t n, const float* means, const float* scales, const float* quats,
                    const float* opacity, const orc_camera* cam, const int32_t* ids, int32_t L,
                    int32_t mode, int32_t nthreads, double* pix_T, double* pix_wsum,
                    double* pix_rho, orc_counts* counts, int64_t* n_triples)
{
    const int f32 = (mode & 2) != 0;
    mode &= 1;
    if (L < 1 || L > ORC_MAX_LABELS) return NULL;
    const int W = cam->width, H = cam->height;
    proj64* P = (proj64*)malloc((size_t)(n ? n : 1) * sizeof(proj64));
    mirror_out* Mi = (mirror_out*)malloc((size_t)(n ? n : 1) * sizeof(mirror_out));
    float* z = (float*)malloc((size_t)(n ? n : 1) * sizeof(float));
    if (!P || !Mi || !z) return NULL;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int64_t nvis = 0;
#pragma omp parallel for schedule(static) reduction(+ : nvis)
    for (int64_t g = 0; g < n; g++) {
        mirror_project(means + 3 * g, scales + 3 * g, quats + 4 * g, cam, &Mi[g]);
        z[g] = Mi[g].z32;
        if (Mi[g].vis_depth) project64(means + 3 * g, scales + 3 * g, quats + 4 * g, opacity[g], cam, &P[g]);
        nvis += Mi[g].vis;
    }

    /* candidate lists */
    const int64_t npix = (int64_t)W * H;
    int64_t* start = (int64_t*)calloc((size_t)npix + 1, sizeof(int64_t));
    int32_t* cand = NULL;
    int32_t* all = NULL;
    int64_t nall = 0;
    if (!start) return NULL;
    if (mode == 0) {
        all = (int32_t*)malloc((size_t)(n ? n : 1) * sizeof(int32_t));
        if (!all) return NULL;
        for (int64_t g = 0; g < n; g++)
            if (Mi[g].vis_depth) all[nall++] = (int32_t)g;
        g_sort_z = z;
        qsort(all, (size_t)nall, sizeof(int32_t), cmp_depth);
    } else {
        cand = box_candidates(n, Mi, W, H, start);
        if (!cand) return NULL;
    }

    /* walk every pixel; rows in parallel, contributions kept per row */
    view_ctx vc = {P, Mi};
    cbuf* rows = (cbuf*)calloc((size_t)(H ? H : 1), sizeof(cbuf));
    int64_t nc_tot = 0, nq_tot = 0, nu_tot = 0;
    int failed = 0;
    int64_t maxc = 0;
    if (mode == 1)
        for (int64_t i = 0; i < npix; i++)
            if (start[i + 1] - start[i] > maxc) maxc = start[i + 1] - start[i];
#pragma omp parallel reduction(+ : nc_tot, nq_tot, nu_tot)
    {
        int32_t* tmp = (int32_t*)malloc((size_t)(maxc + 1) * sizeof(int32_t));
#pragma omp for schedule(dynamic, 1)
        for (int y = 0; y < H; y++) {
            for (int x = 0; x < W; x++) {
                const int64_t pi = (int64_t)y * W + x;
                /* the pixel's labels (masks containing it), -1 entries skipped */
                int32_t segs[ORC_MAX_LABELS];
                int nl = 0;
                for (int l = 0; l < L; l++) {
                    const int32_t sl = ids[pi * L + l];
                    if (sl >= 0) segs[nl++] = sl;
                }
                const int32_t* c;
                int64_t ncand;
                if (mode == 0) {
                    c = all;
                    ncand = nall;
                } else {
                    ncand = start[pi + 1] - start[pi];
                    sort_depth(cand + start[pi], ncand, z, tmp);
                    c = cand + start[pi];
                }
                double Tf = 1.0, ws = 0.0, rf = 0.0;
                int nr = 0;
                const int bad = f32 ? composite_pixel_f32(&vc, c, ncand, x, y, segs, nl, &rows[y], &Tf, &ws)
                                    : composite_pixel(&vc, c, ncand, x, y, segs, nl, &rows[y], &Tf, &ws,
                                                      &rf, &nr, &nc_tot, &nq_tot, &nu_tot, mode == 0);
                if (bad) failed = 1;
                if (pix_T) pix_T[pi] = Tf;
                if (pix_rho) pix_rho[pi] = nr ? -1.0 : rf;
                if (pix_wsum) pix_wsum[pi] = ws;
            }
        }
        free(tmp);
    }

    /* accumulate in pixel order (row-major, then depth order) */
    int64_t tot = 0;
    for (int y = 0; y < H; y++) tot += rows[y].n;
    hmap hm;
    if (failed || hmap_init(&hm, tot / 4 + 16)) return NULL;
    for (int y = 0; y < H; y++) {
        for (int64_t i = 0; i < rows[y].n; i++) {
            const contrib* e = &rows[y].a[i];
            if (hmap_add(&hm, ((uint64_t)(uint32_t)e->g << 32) | (uint32_t)e->s, e->w, e->u, e->r))
                return NULL;
        }
        free(rows[y].a);
    }
    free(rows);

    view_result* vr = (view_result*)calloc(1, sizeof(view_result));
    uint64_t* keys = (uint64_t*)malloc((size_t)(hm.n ? hm.n : 1) * 8);
    int64_t k = 0;
    for (int64_t i = 0; i < hm.cap; i++)
        if (hm.key[i] != HEMPTY) keys[k++] = hm.key[i];
    qsort(keys, (size_t)k, 8, cmp_u64);
    vr->n_triples = k;
    vr->g = (int32_t*)malloc((size_t)(k ? k : 1) * 4);
    vr->s = (int32_t*)malloc((size_t)(k ? k : 1) * 4);
    vr->w = (double*)malloc((size_t)(k ? k : 1) * 8);
    vr->u = (double*)malloc((size_t)(k ? k : 1) * 8);
    vr->r = (double*)malloc((size_t)(k ? k : 1) * 8);
    for (int64_t i = 0; i < k; i++) {
        int64_t sl = hslot(&hm, keys[i]);
        vr->g[i] = (int32_t)(keys[i] >> 32);
        vr->s[i] = (int32_t)(keys[i] & 0xFFFFFFFFu);
        vr->w[i] = hm.w[sl];
        vr->u[i] = hm.u[sl];
        vr->r[i] = hm.r[sl];
    }
    free(keys);
    hmap_free(&hm);
    free(start); free(cand); free(all); free(P); free(Mi); free(z);
    if (counts) {
        counts->n_contrib = nc_tot;
        counts->n_tests = nq_tot;
        counts->n_visible = nvis;
        counts->n_uncertain = nu_tot;
    }
    if (n_triples) *n_triples = k;
    return vr;
}

/*
 * Render per-Gaussian attributes attr [n][C] into one view with the weights
 * of the lift (Method, the rendering equation with w = alpha T, or the
 * kernel weights): every pixel walks its depth-ordered candidates exactly as
 * the lift does (composite_pixel, one pseudo-label, no masking) and gets
 *   out[p][c] = sum_k w_k attr[g_k][c] / sum_k w_k   (0 where the sum is 0),
 * with wsum[p] = sum_k w_k, bw[p] = sum_k (u_k + r_k) (the bound on the
 * FP32 weights' total deviation, decision flips included) and nb[p] = the
 * number of contributions (blended or possibly blended).  Returns 0, or -1
 * when out of memory.
 */
int32_t orc_render_view(int64_t n, const float* means, const float* scales, const float* quats,
                        const float* opacity, const orc_camera* cam, const float* attr, int32_t C,
                        int32_t nthreads, double* out, double* wsum, double* bw, int32_t* nb)
{
    const int W = cam->width, H = cam->height;
    const int64_t npix = (int64_t)W * H;
    proj64* P = (proj64*)malloc((size_t)(n ? n : 1) * sizeof(proj64));
    mirror_out* Mi = (mirror_out*)malloc((size_t)(n ? n : 1) * sizeof(mirror_out));
    float* z = (float*)malloc((size_t)(n ? n : 1) * sizeof(float));
    int64_t* start = (int64_t*)calloc((size_t)npix + 1, sizeof(int64_t));
    if (!P || !Mi || !z || !start) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < n; g++) {
        mirror_project(means + 3 * g, scales + 3 * g, quats + 4 * g, cam, &Mi[g]);
        z[g] = Mi[g].z32;
        if (Mi[g].vis_depth) project64(means + 3 * g, scales + 3 * g, quats + 4 * g, opacity[g], cam, &P[g]);
    }
    int32_t* cand = box_candidates(n, Mi, W, H, start);
    if (!cand) return -1;
    int64_t maxc = 0;
    for (int64_t i = 0; i < npix; i++)
        if (start[i + 1] - start[i] > maxc) maxc = start[i + 1] - start[i];
    view_ctx vc = {P, Mi};
    int failed = 0;
#pragma omp parallel
    {
        int32_t* tmp = (int32_t*)malloc((size_t)(maxc + 1) * sizeof(int32_t));
        cbuf cb = {NULL, 0, 0};
        const int32_t seg0 = 0;
#pragma omp for schedule(dynamic, 1)
        for (int y = 0; y < H; y++) {
            for (int x = 0; x < W; x++) {
                const int64_t pi = (int64_t)y * W + x;
                const int64_t nc = start[pi + 1] - start[pi];
                if (!tmp) { failed = 1; continue; }
                sort_depth(cand + start[pi], nc, z, tmp);
                double Tf, ws, rf;
                int nr;
                int64_t c0 = 0, c1 = 0, c2 = 0;
                cb.n = 0;
                if (composite_pixel(&vc, cand + start[pi], nc, x, y, &seg0, 1, &cb, &Tf, &ws,
                                            &rf, &nr, &c0, &c1, &c2, 0)) {
                    failed = 1;
                    continue;
                }
                double* o = out + pi * C;
                for (int c = 0; c < C; c++) o[c] = 0.0;
                double sw = 0.0, sb = 0.0;
                for (int64_t i = 0; i < cb.n; i++) {
                    const contrib* e = &cb.a[i];
                    const float* a = attr + (int64_t)e->g * C;
                    for (int c = 0; c < C; c++) o[c] += e->w * (double)a[c];
                    sw += e->w;
                    sb += e->u + e->r;
                }
                if (sw > 0.0)
                    for (int c = 0; c < C; c++) o[c] /= sw;
                wsum[pi] = sw;
                bw[pi] = sb;
                nb[pi] = (int32_t)cb.n;
            }
        }
        free(cb.a);
        free(tmp);
    }
    free(start); free(cand); free(P); free(Mi); free(z);
    return failed ? -1 : 0;
}

void orc_view_fetch(void* h, int32_t* g, int32_t* s, double* w, double* u, double* r)
{
    view_result* vr = (view_result*)h;
    size_t k = (size_t)vr->n_triples;
    if (g) memcpy(g, vr->g, k * 4);
    if (s) memcpy(s, vr->s, k * 4);
    if (w) memcpy(w, vr->w, k * 8);
    if (u) memcpy(u, vr->u, k * 8);
    if (r) memcpy(r, vr->r, k * 8);
}

void orc_view_free(void* h)
{
    view_result* vr = (view_result*)h;
    if (!vr) return;
    free(vr->g); free(vr->s); free(vr->w); free(vr->u); free(vr->r);
    free(vr);
}

/* FP32 mirror for every Gaussian of one view: visibility, depth and box. */
void orc_mirror_view(int64_t n, const float* means, const float* scales, const float* quats,
                     const orc_camera* cam, uint8_t* vis, float* z32, int32_t* box,
                     float* mu, float* cov)
{
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < n; g++) {
        mirror_out m;
        mirror_project(means + 3 * g, scales + 3 * g, quats + 4 * g, cam, &m);
        if (vis) vis[g] = (uint8_t)(m.vis ? 1 : (m.vis_depth ? 2 : 0));
        if (z32) z32[g] = m.z32;
        if (box) { box[4 * g] = m.x0; box[4 * g + 1] = m.x1; box[4 * g + 2] = m.y0; box[4 * g + 3] = m.y1; }
        if (mu) { mu[2 * g] = m.u; mu[2 * g + 1] = m.v; }
        if (cov) { cov[3 * g] = m.c00; cov[3 * g + 1] = m.c01; cov[3 * g + 2] = m.c11; }
    }
}

/* FP64 projection of every Gaussian for one view (for closed-form checks). */
void orc_project64_view(int64_t n, const float* means, const float* scales, const float* quats,
                        const float* opacity, const orc_camera* cam, double* mu, double* cov,
                        double* conic, double* zc)
{
    for (int64_t g = 0; g < n; g++) {
        proj64 p;
        project64(means + 3 * g, scales + 3 * g, quats + 4 * g, opacity[g], cam, &p);
        if (mu) { mu[2 * g] = p.mu[0]; mu[2 * g + 1] = p.mu[1]; }
        if (cov) for (int i = 0; i < 3; i++) cov[3 * g + i] = p.cov[i];
        if (conic) for (int i = 0; i < 3; i++) conic[3 * g + i] = p.conic[i];
        if (zc) zc[g] = p.zc;
    }
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
