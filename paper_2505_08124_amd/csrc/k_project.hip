// EWA projection of (view, Gaussian) pairs, culling, compaction of visible
// pairs and their records (paper, Method: the rasterizer's projection of each
// Gaussian to a screen mean mu'_k and covariance Sigma_k with K_i, R_i, t_i).
//
// Every value that feeds an integer decision (camera depth for culling and
// ordering, the conservative pixel box for tile membership) follows one fixed
// FP32 operation sequence: fmaf exactly where written, correctly rounded / and
// sqrt, no other contraction (this file is built with -ffp-contract=off).
// The same sequence written independently on the CPU reproduces the depth
// keys and tile lists bit for bit.
#include <algorithm>

#include "slag_internal.h"

namespace slag {

namespace {

// The near plane, the screen-space dilation and the pixel box's q bound
// (rho^2 = 2 ln(1 / alpha_min)) come with each view (the context's options).
constexpr int PER_THREAD = 8;
constexpr int CPB = 256 * PER_THREAD;    // Gaussians per block and view
static_assert(CPB == GBLOCK, "projection blocks are the Gaussian blocks of the view lists");

struct Proj {
    float u, v, ca, cb, cc, z;
    int x0, x1, y0, y1;
};

// World covariance Sigma3 = M M^T, M = Rq diag(s), from the normalised quaternion.
__device__ __forceinline__ void world_cov(const float* s, const float* q, float* S)
{
    float nq = fmaf(q[0], q[0], fmaf(q[1], q[1], fmaf(q[2], q[2], q[3] * q[3])));
    float rn = 1.0f / sqrtf(nq);
    float w = q[0] * rn, x = q[1] * rn, y = q[2] * rn, z = q[3] * rn;
    float r00 = 1.0f - 2.0f * fmaf(y, y, z * z);
    float r01 = 2.0f * fmaf(x, y, -(w * z));
    float r02 = 2.0f * fmaf(x, z, (w * y));
    float r10 = 2.0f * fmaf(x, y, (w * z));
    float r11 = 1.0f - 2.0f * fmaf(x, x, z * z);
    float r12 = 2.0f * fmaf(y, z, -(w * x));
    float r20 = 2.0f * fmaf(x, z, -(w * y));
    float r21 = 2.0f * fmaf(y, z, (w * x));
    float r22 = 1.0f - 2.0f * fmaf(x, x, y * y);
    float m00 = r00 * s[0], m01 = r01 * s[1], m02 = r02 * s[2];
    float m10 = r10 * s[0], m11 = r11 * s[1], m12 = r12 * s[2];
    float m20 = r20 * s[0], m21 = r21 * s[1], m22 = r22 * s[2];
    S[0] = fmaf(m00, m00, fmaf(m01, m01, m02 * m02));   // xx
    S[1] = fmaf(m00, m10, fmaf(m01, m11, m02 * m12));   // xy
    S[2] = fmaf(m00, m20, fmaf(m01, m21, m02 * m22));   // xz
    S[3] = fmaf(m10, m10, fmaf(m11, m11, m12 * m12));   // yy
    S[4] = fmaf(m10, m20, fmaf(m11, m21, m12 * m22));   // yz
    S[5] = fmaf(m20, m20, fmaf(m21, m21, m22 * m22));   // zz
}

// Projection of one Gaussian into one view.  Returns false when culled (depth
// at or in front of the near plane, degenerate covariance, empty pixel box).
__device__ __forceinline__ bool project(const ViewDev& V, float mx, float my, float mz,
                                        const float* S, Proj& P)
{
    const float* R = V.R;
    float X = fmaf(R[0], mx, fmaf(R[1], my, fmaf(R[2], mz, V.t[0])));
    float Y = fmaf(R[3], mx, fmaf(R[4], my, fmaf(R[5], mz, V.t[1])));
    float Z = fmaf(R[6], mx, fmaf(R[7], my, fmaf(R[8], mz, V.t[2])));
    P.z = Z;
    if (!(Z > V.near_z)) return false;
    float iz = 1.0f / Z;
    float txr = X * iz, tyr = Y * iz;
    float tx = fminf(V.limx, fmaxf(-V.limx, txr));
    float ty = fminf(V.limy, fmaxf(-V.limy, tyr));
    float j00 = V.fx * iz, j02 = -(j00 * tx);
    float j11 = V.fy * iz, j12 = -(j11 * ty);
    // A = J R (2x3), Sigma2 = A Sigma3 A^T
    float a0 = fmaf(j00, R[0], j02 * R[6]), a1 = fmaf(j00, R[1], j02 * R[7]),
          a2 = fmaf(j00, R[2], j02 * R[8]);
    float a3 = fmaf(j11, R[3], j12 * R[6]), a4 = fmaf(j11, R[4], j12 * R[7]),
          a5 = fmaf(j11, R[5], j12 * R[8]);
    const float sxx = S[0], sxy = S[1], sxz = S[2], syy = S[3], syz = S[4], szz = S[5];
    float b0 = fmaf(a0, sxx, fmaf(a1, sxy, a2 * sxz));
    float b1 = fmaf(a0, sxy, fmaf(a1, syy, a2 * syz));
    float b2 = fmaf(a0, sxz, fmaf(a1, syz, a2 * szz));
    float b3 = fmaf(a3, sxx, fmaf(a4, sxy, a5 * sxz));
    float b4 = fmaf(a3, sxy, fmaf(a4, syy, a5 * syz));
    float b5 = fmaf(a3, sxz, fmaf(a4, syz, a5 * szz));
    float c00 = fmaf(b0, a0, fmaf(b1, a1, b2 * a2)) + V.dil;
    float c01 = fmaf(b0, a3, fmaf(b1, a4, b2 * a5));
    float c11 = fmaf(b3, a3, fmaf(b4, a4, b5 * a5)) + V.dil;
    float det = fmaf(c00, c11, -(c01 * c01));
    if (!(det > 0.0f)) return false;
    float idet = 1.0f / det;
    P.ca = c11 * idet;
    P.cb = -(c01 * idet);
    P.cc = c00 * idet;
    float u = fmaf(V.fx, txr, V.cx);
    float v = fmaf(V.fy, tyr, V.cy);
    P.u = u;
    P.v = v;
    float ex = sqrtf(V.rho2 * c00);
    float ey = sqrtf(V.rho2 * c11);
    float x0 = ceilf(u - (ex + 1.5f)), x1 = floorf(u + (ex + 0.5f));
    float y0 = ceilf(v - (ey + 1.5f)), y1 = floorf(v + (ey + 0.5f));
    float wm1 = (float)(V.W - 1), hm1 = (float)(V.H - 1);
    if (!(x0 <= wm1 && x1 >= 0.0f && y0 <= hm1 && y1 >= 0.0f)) return false;
    P.x0 = (int)fmaxf(x0, 0.0f);
    P.x1 = (int)fminf(x1, wm1);
    P.y0 = (int)fmaxf(y0, 0.0f);
    P.y1 = (int)fminf(y1, hm1);
    return true;
}

// Compositing form of a visible pair, in FP64 from the FP64 world covariance
// (same operations as the FP32 path, so the conic is the exact inverse of the
// projected covariance up to FP64 rounding): the prescaled conic
// (A, B, C) = -log2(e) (conic_xx / 2, conic_xy, conic_yy / 2) and the screen
// mean as an offset from the pixel box's corner (x0, y0), each rounded to FP32
// once.  alpha = 2^(lo2 + A dx^2 + B dx dy + C dy^2).
__device__ __forceinline__ void project_fine(const ViewDev& V, float mx, float my, float mz,
                                             const double* S, int x0, int y0, float4& r0,
                                             float& rc)
{
    const float* R = V.R;
    const double X = (double)R[0] * mx + (double)R[1] * my + (double)R[2] * mz + (double)V.t[0];
    const double Y = (double)R[3] * mx + (double)R[4] * my + (double)R[5] * mz + (double)V.t[1];
    const double Z = (double)R[6] * mx + (double)R[7] * my + (double)R[8] * mz + (double)V.t[2];
    const double limx = V.guard_d * (0.5 * (double)V.W / (double)V.fx);
    const double limy = V.guard_d * (0.5 * (double)V.H / (double)V.fy);
    const double txz = X / Z, tyz = Y / Z;
    const double tx = fmin(limx, fmax(-limx, txz)), ty = fmin(limy, fmax(-limy, tyz));
    const double j00 = (double)V.fx / Z, j02 = -j00 * tx;
    const double j11 = (double)V.fy / Z, j12 = -j11 * ty;
    double a[6];
#pragma unroll
    for (int k = 0; k < 3; k++) {
        a[k] = j00 * R[k] + j02 * R[6 + k];
        a[3 + k] = j11 * R[3 + k] + j12 * R[6 + k];
    }
    const double sxx = S[0], sxy = S[1], sxz = S[2], syy = S[3], syz = S[4], szz = S[5];
    const double b0 = a[0] * sxx + a[1] * sxy + a[2] * sxz;
    const double b1 = a[0] * sxy + a[1] * syy + a[2] * syz;
    const double b2 = a[0] * sxz + a[1] * syz + a[2] * szz;
    const double b3 = a[3] * sxx + a[4] * sxy + a[5] * sxz;
    const double b4 = a[3] * sxy + a[4] * syy + a[5] * syz;
    const double b5 = a[3] * sxz + a[4] * syz + a[5] * szz;
    const double c00 = b0 * a[0] + b1 * a[1] + b2 * a[2] + V.dil_d;
    const double c01 = b0 * a[3] + b1 * a[4] + b2 * a[5];
    const double c11 = b3 * a[3] + b4 * a[4] + b5 * a[5] + V.dil_d;
    const double idet = 1.0 / (c00 * c11 - c01 * c01);
    const double L2E = 1.4426950408889634074;
    const double u = (double)V.fx * txz + (double)V.cx;
    const double v = (double)V.fy * tyz + (double)V.cy;
    r0 = make_float4((float)(u - (double)x0), (float)(v - (double)y0),
                     (float)(-0.5 * L2E * c11 * idet), (float)(L2E * c01 * idet));
    rc = (float)(-0.5 * L2E * c00 * idet);
}

// Tiles of the pixel box (tsh = log2 of the tile edge; the box is clamped to
// the image, so its corners are not negative).
__device__ __forceinline__ uint32_t tiles_of(const Proj& P, int tsh)
{
    return (uint32_t)(((P.x1 >> tsh) - (P.x0 >> tsh) + 1) * ((P.y1 >> tsh) - (P.y0 >> tsh) + 1));
}

__device__ __forceinline__ void load_cov(const float* cov3, int64_t n, int64_t g, float* S)
{
#pragma unroll
    for (int k = 0; k < 6; k++) S[k] = cov3[k * n + g];
}

// Exclusive scan of one value per thread over a 256-thread block.
__device__ __forceinline__ uint32_t block_exscan(uint32_t v, uint32_t* lds, uint32_t& total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) lds[w] = x;
    __syncthreads();
    uint32_t off = 0;
    for (int i = 0; i < w; i++) off += lds[i];
    total = lds[0] + lds[1] + lds[2] + lds[3];
    __syncthreads();
    return off + x - v;
}

// Per block of CPB consecutive (Morton-ordered) Gaussians: the bounding box
// of the means and the largest trace of the world covariance (a bound of
// the variance along any axis): geo[8 blk + (0..2: min xyz, 3..5: max xyz,
// 6: max trace)].
__global__ __launch_bounds__(256) void k_block_geo(int64_t n, const float* __restrict__ means,
                                                   const float* __restrict__ cov3,
                                                   float* __restrict__ geo)
{
    __shared__ float red[4][7];
    const int64_t b0 = (int64_t)blockIdx.x * CPB;
    float v[7] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, 0.0f};
    for (int64_t g = b0 + threadIdx.x; g < n && g < b0 + CPB; g += 256) {
        for (int k = 0; k < 3; k++) {
            const float m = means[3 * g + k];
            v[k] = fminf(v[k], m);
            v[3 + k] = fmaxf(v[3 + k], m);
        }
        v[6] = fmaxf(v[6], cov3[g] + cov3[3 * n + g] + cov3[5 * n + g]);
    }
    for (int o = 32; o >= 1; o >>= 1)
        for (int k = 0; k < 7; k++) {
            const float w = __shfl_xor(v[k], o, 64);
            v[k] = (k < 3) ? fminf(v[k], w) : fmaxf(v[k], w);
        }
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 7; k++) red[threadIdx.x >> 6][k] = v[k];
    __syncthreads();
    if (threadIdx.x < 7) {
        const int k = threadIdx.x;
        float r = red[0][k];
        for (int w = 1; w < 4; w++) r = (k < 3) ? fminf(r, red[w][k]) : fmaxf(r, red[w][k]);
        geo[8 * blockIdx.x + k] = r;
    }
}

// Can no Gaussian of a block have a non-empty pixel box in view V?  A
// conservative bound, with margins far beyond any FP32 rounding: the camera
// depth and the screen coordinates x/z, y/z of the means are extreme at the
// corners of the block's box (affine and linear-fractional maps of a box in
// front of the camera), and a pixel box's half-extent is at most
// sqrt(rho^2 ((f / z_min)^2 (1 + lim^2) trace + dilation)) (the Jacobian row
// has squared norm (f / z)^2 (1 + t^2), t the clamped x/z).  Blocks that the
// bound cannot rule out are projected Gaussian by Gaussian as before, so
// every visibility decision is unchanged.
__device__ __forceinline__ bool block_outside(const ViewDev& V, const float* __restrict__ g8)
{
    const float* R = V.R;
    float zmin = INFINITY, zmax = -INFINITY, xmn = INFINITY, xmx = -INFINITY, ymn = INFINITY,
          ymx = -INFINITY, mag = fabsf(V.t[0]) + fabsf(V.t[1]) + fabsf(V.t[2]);
    float X[8], Y[8], Z[8];
#pragma unroll
    for (int c = 0; c < 8; c++) {
        const float mx = g8[(c & 1) ? 3 : 0], my = g8[(c & 2) ? 4 : 1], mz = g8[(c & 4) ? 5 : 2];
        X[c] = fmaf(R[0], mx, fmaf(R[1], my, fmaf(R[2], mz, V.t[0])));
        Y[c] = fmaf(R[3], mx, fmaf(R[4], my, fmaf(R[5], mz, V.t[1])));
        Z[c] = fmaf(R[6], mx, fmaf(R[7], my, fmaf(R[8], mz, V.t[2])));
        zmin = fminf(zmin, Z[c]);
        zmax = fmaxf(zmax, Z[c]);
        mag = fmaxf(mag, fabsf(mx) + fabsf(my) + fabsf(mz));
    }
    const float tol = 1e-4f * (1.0f + 2.0f * mag);
    if (zmax < V.near_z - tol) return true;       // every mean behind the near plane
    if (!(zmin > V.near_z + tol) || !(g8[6] >= 0.0f) || !isfinite(g8[6])) return false;
#pragma unroll
    for (int c = 0; c < 8; c++) {
        xmn = fminf(xmn, X[c] / Z[c]);
        xmx = fmaxf(xmx, X[c] / Z[c]);
        ymn = fminf(ymn, Y[c] / Z[c]);
        ymx = fmaxf(ymx, Y[c] / Z[c]);
    }
    const float iz = 1.0f / (zmin - tol);
    const float ex = sqrtf(V.rho2 * (V.fx * V.fx * iz * iz * (1.0f + V.limx * V.limx) * g8[6] * 1.01f + V.dil)) + 2.0f;
    const float ey = sqrtf(V.rho2 * (V.fy * V.fy * iz * iz * (1.0f + V.limy * V.limy) * g8[6] * 1.01f + V.dil)) + 2.0f;
    const float umn = fmaf(V.fx, xmn, V.cx), umx = fmaf(V.fx, xmx, V.cx);
    const float vmn = fmaf(V.fy, ymn, V.cy), vmx = fmaf(V.fy, ymx, V.cy);
    const float su = 2.0f + 1e-3f * (fabsf(umn) + fabsf(umx));
    const float sv = 2.0f + 1e-3f * (fabsf(vmn) + fabsf(vmx));
    return (umn - ex - 1.5f > (float)(V.W - 1) + su) || (umx + ex + 0.5f < -su) ||
           (vmn - ey - 1.5f > (float)(V.H - 1) + sv) || (vmx + ey + 0.5f < -sv);
}

// Upload: validation, the FP32 world covariance of the decision path, and
// the FP64 world covariance and log2 of the opacity that the records of the
// compositing are formed from (so that alpha carries only the rounding of the
// stored coefficients, not that of an FP32 projection).
__global__ __launch_bounds__(256) void k_prep_gauss(int64_t n, const float* __restrict__ means,
                                                    const float* __restrict__ scales,
                                                    const float* __restrict__ quats,
                                                    const float* __restrict__ opac,
                                                    float* __restrict__ cov3,
                                                    double* __restrict__ covd,
                                                    float* __restrict__ lo2, uint32_t* err)
{
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    float s[3] = {scales[3 * g], scales[3 * g + 1], scales[3 * g + 2]};
    float q[4] = {quats[4 * g], quats[4 * g + 1], quats[4 * g + 2], quats[4 * g + 3]};
    float o = opac[g];
    bool ok = isfinite(means[3 * g]) && isfinite(means[3 * g + 1]) && isfinite(means[3 * g + 2]);
    ok = ok && s[0] > 0.0f && s[1] > 0.0f && s[2] > 0.0f && isfinite(s[0]) && isfinite(s[1]) &&
         isfinite(s[2]);
    float nq = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    ok = ok && nq > 0.0f && isfinite(nq) && o > 0.0f && o <= 1.0f;
    if (!ok) {
        atomicOr(err, 1u);
        for (int k = 0; k < 6; k++) {
            cov3[k * n + g] = 0.0f;
            covd[k * n + g] = 0.0;
        }
        lo2[g] = 0.0f;
        return;
    }
    float S[6];
    world_cov(s, q, S);
#pragma unroll
    for (int k = 0; k < 6; k++) cov3[k * n + g] = S[k];
    // FP64: Sigma3 = Rq diag(s^2) Rq^T from the normalised quaternion
    const double qn = sqrt((double)q[0] * q[0] + (double)q[1] * q[1] + (double)q[2] * q[2] +
                           (double)q[3] * q[3]);
    const double w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
    const double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                         2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                         2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
    const double s2[3] = {(double)s[0] * s[0], (double)s[1] * s[1], (double)s[2] * s[2]};
    const int ij[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
#pragma unroll
    for (int k = 0; k < 6; k++) {
        const int i = ij[k][0], j = ij[k][1];
        covd[k * n + g] = R[3 * i] * s2[0] * R[3 * j] + R[3 * i + 1] * s2[1] * R[3 * j + 1] +
                          R[3 * i + 2] * s2[2] * R[3 * j + 2];
    }
    lo2[g] = (float)log2((double)o);
}

__global__ __launch_bounds__(256) void k_validate_ids(int64_t npix, const int32_t* __restrict__ ids,
                                                      int lpp, int32_t nseg, uint32_t* err)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    for (; i < npix; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t lab[MAX_LABELS];
        for (int l = 0; l < lpp; l++) {
            const int32_t s = ids[i * lpp + l];
            lab[l] = s;
            bad |= (s < -1) || (s >= nseg);
            for (int m = 0; m < l; m++) bad |= s >= 0 && lab[m] == s;   // one mask listed twice
        }
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(err, 2u);
}

__global__ __launch_bounds__(256) void k_expand_labels(int64_t npix, const int32_t* __restrict__ src,
                                                       int lin, int32_t* __restrict__ dst, int lout)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npix * lout;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = i / lout;
        const int l = (int)(i - p * lout);
        dst[i] = l < lin ? src[p * lin + l] : -1;
    }
}

// Pass 1: tile count of every (view, Gaussian) pair (0 = not visible), the
// number of visible pairs per block, and the range of visible depth keys.
// Thread t of a block handles Gaussians base + i * 256 + t, i < PER_THREAD
// (coalesced loads and stores).
__global__ __launch_bounds__(256) void k_count(int64_t n, const ViewDev* __restrict__ views,
                                               const float* __restrict__ means,
                                               const float* __restrict__ cov3,
                                               const float* __restrict__ geo,
                                               uint32_t* __restrict__ tcnt,
                                               uint32_t* __restrict__ blk_vis,
                                               uint32_t* __restrict__ zrange)
{
    __shared__ uint32_t lds[4];
    // grid (view, Gaussian block): consecutive workgroups are the views of one
    // Gaussian block, whose data they then share through the caches
    const int vl = blockIdx.x;
    const int blk = blockIdx.y, nblk = gridDim.y;
    const ViewDev V = views[vl];
    if (block_outside(V, geo + 8 * blk)) {
        // no Gaussian of the block is visible: no pair (the emission skips
        // the block without reading its tile counts)
        if (threadIdx.x == 0) {
            const int64_t bi = (int64_t)vl * nblk + blk;
            blk_vis[bi] = 0;
            zrange[2 * bi] = 0xFFFFFFFFu;
            zrange[2 * bi + 1] = 0;
        }
        return;
    }
    const int64_t g0 = (int64_t)blk * CPB + threadIdx.x;
    uint32_t* out = tcnt + (int64_t)vl * n;
    uint32_t nvis = 0, zmin = 0xFFFFFFFFu, zmax = 0;
    // the next Gaussian's inputs are loaded (clamped, unconditionally) while
    // the current one is projected
    float nc[6], nm[3];
    auto load_in = [&](int i) {
        const int64_t g = g0 + (int64_t)i * 256;
        const int64_t gc = g < n ? g : n - 1;
        load_cov(cov3, n, gc, nc);
        nm[0] = means[3 * gc];
        nm[1] = means[3 * gc + 1];
        nm[2] = means[3 * gc + 2];
    };
    load_in(0);
#pragma unroll 1
    for (int i = 0; i < PER_THREAD; i++) {
        const int64_t g = g0 + (int64_t)i * 256;
        if (g >= n) break;
        float S[6];
#pragma unroll
        for (int k = 0; k < 6; k++) S[k] = nc[k];
        const float mx = nm[0], my = nm[1], mz = nm[2];
        if (i + 1 < PER_THREAD) load_in(i + 1);
        Proj P;
        uint32_t tc = 0;
        if (project(V, mx, my, mz, S, P)) {
            tc = tiles_of(P, V.tsh);
            nvis++;
            const uint32_t zb = __float_as_uint(P.z);
            zmin = min(zmin, zb);
            zmax = max(zmax, zb);
        }
        out[g] = tc;
    }
    uint32_t total;
    block_exscan(nvis, lds, total);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        zmin = min(zmin, (uint32_t)__shfl_xor((int)zmin, d, 64));
        zmax = max(zmax, (uint32_t)__shfl_xor((int)zmax, d, 64));
    }
    __shared__ uint32_t zl[8];
    if ((threadIdx.x & 63) == 0) {
        zl[threadIdx.x >> 6] = zmin;
        zl[4 + (threadIdx.x >> 6)] = zmax;
    }
    __syncthreads();
    const int64_t bi = (int64_t)vl * nblk + blk;
    if (threadIdx.x == 0) {
        blk_vis[bi] = total;
        zrange[2 * bi] = min(min(zl[0], zl[1]), min(zl[2], zl[3]));
        zrange[2 * bi + 1] = max(max(zl[4], zl[5]), max(zl[6], zl[7]));
    }
}

// Pass 2: compact visible pairs in (view, Gaussian) order (Gaussians are
// stored in Morton order) and write their records, depth-sort keys, part-list
// capacities, the caller's index of each pair's Gaussian (pgauss: the depth
// order breaks ties by it) and the (view, Morton rank) -> pair map (NONE
// where not visible); pz (depth bits per pair) only when given, for the
// debug exports.  Same striped layout as pass 1.
__global__ __launch_bounds__(256) void k_emit_pairs(
    int64_t n, const ViewDev* __restrict__ views, const float* __restrict__ means,
    const float* __restrict__ cov3, const double* __restrict__ covd,
    const float* __restrict__ lo2, uint32_t* __restrict__ tcnt,
    const uint32_t* __restrict__ blk_off, float4* __restrict__ rec, uint32_t* __restrict__ pgauss,
    uint16_t* __restrict__ pview, uint64_t* __restrict__ dkey, uint32_t* __restrict__ dval,
    uint32_t* __restrict__ psz, uint32_t* __restrict__ pz, const uint32_t* __restrict__ sat,
    uint32_t zmin, int zbits, int pbits, int plocal, uint32_t* __restrict__ blk_tot,
    const uint32_t* __restrict__ perm, uint32_t* __restrict__ pair_of_m, uint2* __restrict__ prect,
    int lbits)
{
    __shared__ uint32_t cnt[PER_THREAD][4];
    __shared__ uint64_t msk[4][PER_THREAD];
    const int vl = blockIdx.x;                       // grid (view, Gaussian block)
    const int blk = blockIdx.y, nblk = gridDim.y;
    const int64_t bi0 = (int64_t)vl * nblk + blk;
    if (blk_off[bi0 + 1] == blk_off[bi0]) {
        // no visible pair in this (view, block): nothing to emit, and the pair
        // map is not written (its readers skip such (view, block)s by the
        // scanned counts)
        if (threadIdx.x == 0) {
            blk_tot[2 * bi0] = 0;
            blk_tot[2 * bi0 + 1] = 0;
        }
        return;
    }
    const ViewDev V = views[vl];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t g0 = (int64_t)blk * CPB + threadIdx.x;
    const uint32_t* io = tcnt + (int64_t)vl * n;
    uint32_t tc[PER_THREAD];   // all loads in flight before the first is used
#pragma unroll
    for (int i = 0; i < PER_THREAD; i++) {
        const int64_t g = g0 + (int64_t)i * 256;
        const uint32_t v = io[g < n ? g : n - 1];   // unconditional: no branch between loads
        tc[i] = g < n ? v : 0u;
    }
#pragma unroll
    for (int i = 0; i < PER_THREAD; i++) {
        const uint64_t m = __ballot(tc[i] != 0);
        if (lane == 0) {
            cnt[i][wv] = (uint32_t)__popcll(m);
            msk[wv][i] = m;
        }
    }
    __syncthreads();
    uint32_t run = blk_off[(int64_t)vl * nblk + blk];
    const uint32_t vbase = blk_off[(int64_t)vl * nblk];   // the view's first pair
    const int sw = V.ntx + 1;
    const uint32_t* S = sat + V.sat_off;
    unsigned long long n_isect = 0, n_part = 0;
    // the next Gaussian's inputs are loaded (clamped, unconditionally) while
    // the current one is projected and written
    struct GIn {
        float C[6], x, y, z, lo2;
        uint32_t pg;
    };
    auto load_in = [&](int i, GIn& a) {
        const int64_t g = g0 + (int64_t)i * 256;
        const int64_t gc = g < n ? g : n - 1;
        load_cov(cov3, n, gc, a.C);
        a.x = means[3 * gc];
        a.y = means[3 * gc + 1];
        a.z = means[3 * gc + 2];
        a.lo2 = lo2[gc];
        a.pg = perm[gc];
    };
    GIn nx;
    load_in(0, nx);
#pragma unroll 1
    for (int i = 0; i < PER_THREAD; i++) {
        const GIn cur = nx;
        if (i + 1 < PER_THREAD) load_in(i + 1, nx);
        const int64_t g = g0 + (int64_t)i * 256;
        const uint64_t m = msk[wv][i];
        uint32_t before = 0;
        for (int w = 0; w < wv; w++) before += cnt[i][w];
        const uint32_t pidx = run + before + (uint32_t)__popcll(m & lt);
        run += cnt[i][0] + cnt[i][1] + cnt[i][2] + cnt[i][3];
        if (g >= n) continue;
        if (!((m >> lane) & 1ull)) {
            pair_of_m[(int64_t)vl * n + g] = NONE;
            continue;
        }
        Proj P;
        project(V, cur.x, cur.y, cur.z, cur.C, P);
        // compositing form (FP64 projection): mean offset from the box corner,
        // prescaled conic, log2 of the opacity, pixel box
        double Sd[6];
#pragma unroll
        for (int k = 0; k < 6; k++) Sd[k] = covd[k * n + g];
        float4 r0;
        float rc;
        project_fine(V, cur.x, cur.y, cur.z, Sd, P.x0, P.y0, r0, rc);
        rec[2 * (size_t)pidx] = r0;
        rec[2 * (size_t)pidx + 1] =
            make_float4(rc, cur.lo2, __uint_as_float((uint32_t)P.x0 | ((uint32_t)P.y0 << 16)),
                        __uint_as_float((uint32_t)P.x1 | ((uint32_t)P.y1 << 16)));
        pgauss[pidx] = cur.pg;                       // the caller's index of the Gaussian
        pview[pidx] = (uint16_t)vl;
        const uint64_t dk = ((uint64_t)vl << zbits) | (uint64_t)(__float_as_uint(P.z) - zmin);
        if (pbits) {
            // the pair index (or, plocal, its index within the view) rides in
            // the low bits
            dkey[pidx] = (dk << pbits) | (plocal ? pidx - vbase : pidx);
        } else {
            dkey[pidx] = dk;
            dval[pidx] = pidx;
        }
        if (pz) pz[pidx] = __float_as_uint(P.z);      // debug exports only
        // part slots of this pair: sum of the tile segment counts over its tile rect
        const int tx0 = P.x0 >> V.tsh, tx1 = P.x1 >> V.tsh, ty0 = P.y0 >> V.tsh, ty1 = P.y1 >> V.tsh;
        const uint32_t ps = S[(ty1 + 1) * sw + tx1 + 1] - S[ty0 * sw + tx1 + 1] -
                            S[(ty1 + 1) * sw + tx0] + S[ty0 * sw + tx0];
        psz[pidx] = ps;
        const uint32_t rw = (uint32_t)(tx1 - tx0 + 1), rh = (uint32_t)(ty1 - ty0 + 1);
        const uint32_t tc = rw * rh;
        // tile rectangle: (entry key of its top-left tile, width | height << 16)
        prect[pidx] = make_uint2(((uint32_t)vl << lbits) + (uint32_t)(ty0 * V.ntx + tx0),
                                 rw | (rh << 16));
        n_isect += tc;
        n_part += ps;
        pair_of_m[(int64_t)vl * n + g] = pidx;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        n_isect += __shfl_xor(n_isect, d, 64);
        n_part += __shfl_xor(n_part, d, 64);
    }
    __shared__ unsigned long long tl[8];
    if (lane == 0) {
        tl[wv] = n_isect;
        tl[4 + wv] = n_part;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // per-block totals (saturated: a block never exceeds 2^32 - 1 in practice,
        // and the host rejects totals that do)
        const unsigned long long a = tl[0] + tl[1] + tl[2] + tl[3];
        const unsigned long long b = tl[4] + tl[5] + tl[6] + tl[7];
        const int64_t bi = (int64_t)vl * nblk + blk;
        blk_tot[2 * bi] = a > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)a;
        blk_tot[2 * bi + 1] = b > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)b;
    }
}

// Reduction of per-block results: out[0] = min over even entries (u32 min),
// out[1] = max over odd entries; or (sum mode) 64-bit sums of even and odd
// entries.  Grid-stride blocks, one integer atomic per block into out
// (initialised by k_reduce_init): integer min, max and sums do not depend on
// the order, so the results are deterministic.
__global__ __launch_bounds__(256) void k_reduce_init(int sum_mode, unsigned long long* __restrict__ out)
{
    if (threadIdx.x == 0) {
        out[0] = sum_mode ? 0ull : 0xFFFFFFFFull;
        out[1] = 0ull;
    }
}

__global__ __launch_bounds__(256) void k_reduce_pairs(const uint32_t* __restrict__ in, uint64_t npairs,
                                                      int sum_mode, unsigned long long* __restrict__ out)
{
    __shared__ unsigned long long a_l[4], b_l[4];
    unsigned long long a = sum_mode ? 0ull : 0xFFFFFFFFull, b = 0ull;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < npairs;
         i += (uint64_t)gridDim.x * 256) {
        const uint2 xy = reinterpret_cast<const uint2*>(in)[i];
        if (sum_mode) { a += xy.x; b += xy.y; }
        else { a = min(a, (unsigned long long)xy.x); b = max(b, (unsigned long long)xy.y); }
    }
    for (int o = 32; o >= 1; o >>= 1) {
        const unsigned long long ao = __shfl_xor(a, o, 64), bo = __shfl_xor(b, o, 64);
        if (sum_mode) { a += ao; b += bo; }
        else { a = min(a, ao); b = max(b, bo); }
    }
    if ((threadIdx.x & 63) == 0) {
        a_l[threadIdx.x >> 6] = a;
        b_l[threadIdx.x >> 6] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; w++) {
            if (sum_mode) { a += a_l[w]; b += b_l[w]; }
            else { a = min(a, a_l[w]); b = max(b, b_l[w]); }
        }
        if (sum_mode) {
            atomicAdd(&out[0], a);
            atomicAdd(&out[1], b);
        } else {
            atomicMin(&out[0], a);
            atomicMax(&out[1], b);
        }
    }
}

// ---- Morton order of the Gaussians (block structure of the contraction) ----

// Order-preserving integer image of a float (for min/max with integer atomics).
__device__ __forceinline__ uint32_t ord_of(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__global__ __launch_bounds__(256) void k_bbox(int64_t n, const float* __restrict__ means,
                                              uint32_t* __restrict__ box6)
{
    uint32_t lo[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, hi[3] = {0u, 0u, 0u};
    for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < n; g += (int64_t)gridDim.x * 256)
        for (int k = 0; k < 3; k++) {
            const uint32_t o = ord_of(means[3 * g + k]);
            lo[k] = min(lo[k], o);
            hi[k] = max(hi[k], o);
        }
    __shared__ uint32_t bl[4][6];
    for (int k = 0; k < 3; k++) {
        for (int d = 32; d >= 1; d >>= 1) {
            lo[k] = min(lo[k], (uint32_t)__shfl_xor((int)lo[k], d, 64));
            hi[k] = max(hi[k], (uint32_t)__shfl_xor((int)hi[k], d, 64));
        }
        if ((threadIdx.x & 63) == 0) {
            bl[threadIdx.x >> 6][k] = lo[k];
            bl[threadIdx.x >> 6][3 + k] = hi[k];
        }
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int k = threadIdx.x;
        atomicMin(&box6[k], min(min(bl[0][k], bl[1][k]), min(bl[2][k], bl[3][k])));
        atomicMax(&box6[3 + k], max(max(bl[0][3 + k], bl[1][3 + k]), max(bl[2][3 + k], bl[3][3 + k])));
    }
}

__device__ __forceinline__ uint64_t spread3(uint64_t x)   // 21 bits -> every third bit
{
    x &= 0x1FFFFFull;
    x = (x | (x << 32)) & 0x1F00000000FFFFull;
    x = (x | (x << 16)) & 0x1F0000FF0000FFull;
    x = (x | (x << 8)) & 0x100F00F00F00F00Full;
    x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__global__ __launch_bounds__(256) void k_morton(int64_t n, const float* __restrict__ means,
                                                const float* __restrict__ lo_scale,
                                                uint64_t* __restrict__ keys,
                                                uint32_t* __restrict__ vals)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= n) return;
    uint64_t c[3];
    for (int k = 0; k < 3; k++) {
        float f = (means[3 * g + k] - lo_scale[k]) * lo_scale[3 + k];
        f = fminf(fmaxf(f, 0.0f), 2097151.0f);
        c[k] = (uint64_t)f;
    }
    keys[g] = spread3(c[0]) | (spread3(c[1]) << 1) | (spread3(c[2]) << 2);
    vals[g] = (uint32_t)g;
}

__global__ __launch_bounds__(256) void k_invert(int64_t n, const uint32_t* __restrict__ perm,
                                                uint32_t* __restrict__ rank)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q < n) rank[perm[q]] = (uint32_t)q;
}

// Gaussian q of the Morton order from input Gaussian perm[q]: means [n][3],
// covariances [6][n], opacities [n].
__global__ __launch_bounds__(256) void k_gather_gauss(int64_t n, const uint32_t* __restrict__ perm,
                                                      const float* __restrict__ means,
                                                      const float* __restrict__ cov3,
                                                      const double* __restrict__ covd,
                                                      const float* __restrict__ lo2,
                                                      float* __restrict__ means_o,
                                                      float* __restrict__ cov3_o,
                                                      double* __restrict__ covd_o,
                                                      float* __restrict__ lo2_o)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    const int64_t g = perm[q];
#pragma unroll
    for (int k = 0; k < 3; k++) means_o[3 * q + k] = means[3 * g + k];
#pragma unroll
    for (int k = 0; k < 6; k++) {
        cov3_o[k * n + q] = cov3[k * n + g];
        covd_o[k * n + q] = covd[k * n + g];
    }
    lo2_o[q] = lo2[g];
}

}  // namespace

int count_blocks_per_view(int64_t n) { return (int)((n + CPB - 1) / CPB); }

void launch_prep_gauss(int64_t n, const float* means, const float* scales, const float* quats,
                       const float* opac, float* cov3, double* covd, float* lo2, uint32_t* err,
                       hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_prep_gauss, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, means,
                       scales, quats, opac, cov3, covd, lo2, err);
}

void launch_expand_labels(int64_t npix, const int32_t* src, int lin, int32_t* dst, int lout,
                          hipStream_t st)
{
    if (npix <= 0) return;
    const int64_t blocks = std::min<int64_t>((npix * lout + 255) / 256, 65536);
    hipLaunchKernelGGL(k_expand_labels, dim3((unsigned)blocks), dim3(256), 0, st, npix, src, lin, dst,
                       lout);
}

void launch_validate_ids(int64_t npix, const int32_t* ids, int lpp, int32_t nseg, uint32_t* err,
                         hipStream_t st)
{
    if (npix <= 0) return;
    int64_t blocks = (npix + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_validate_ids, dim3((unsigned)blocks), dim3(256), 0, st, npix, ids,
                       lpp < 1 ? 1 : lpp, nseg, err);
}

void launch_block_geo(int64_t n, const float* means, const float* cov3, float* geo, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_block_geo, dim3((unsigned)count_blocks_per_view(n)), dim3(256), 0, st, n,
                       means, cov3, geo);
}

void launch_count(int nb, int64_t n, const ViewDev* views, const float* means, const float* cov3,
                  const float* geo, uint32_t* tcnt, uint32_t* blk_vis, uint32_t* zrange,
                  hipStream_t st)
{
    if (n <= 0 || nb <= 0) return;
    hipLaunchKernelGGL(k_count, dim3((unsigned)nb, (unsigned)count_blocks_per_view(n)), dim3(256),
                       0, st, n, views, means, cov3, geo, tcnt, blk_vis, zrange);
}

void launch_emit_pairs(int nb, int64_t n, const ViewDev* views, const float* means,
                       const float* cov3, const double* covd, const float* lo2,
                       uint32_t* tcnt_pairof,
                       const uint32_t* blk_off, float4* rec, uint32_t* pgauss, uint16_t* pview,
                       uint64_t* dkey, uint32_t* dval, uint32_t* psz, uint32_t* pz,
                       const uint32_t* sat, uint32_t zmin, int zbits, int pbits, int plocal,
                       uint32_t* blk_tot, const uint32_t* perm, uint32_t* pair_of_m, uint2* prect,
                       int lbits, hipStream_t st)
{
    if (n <= 0 || nb <= 0) return;
    hipLaunchKernelGGL(k_emit_pairs, dim3((unsigned)nb, (unsigned)count_blocks_per_view(n)),
                       dim3(256), 0, st, n, views, means, cov3, covd, lo2, tcnt_pairof, blk_off, rec,
                       pgauss, pview, dkey, dval, psz, pz, sat, zmin, zbits, pbits, plocal, blk_tot,
                       perm, pair_of_m, prect, lbits);
}

void launch_reduce_pairs(const uint32_t* in, uint64_t npairs, bool sum_mode,
                         unsigned long long* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce_init, dim3(1), dim3(64), 0, st, sum_mode ? 1 : 0, out);
    if (!npairs) return;
    const uint64_t blocks = std::min<uint64_t>((npairs + 255) / 256, 1024);
    hipLaunchKernelGGL(k_reduce_pairs, dim3((unsigned)blocks), dim3(256), 0, st, in, npairs,
                       sum_mode ? 1 : 0, out);
}

void launch_bbox(int64_t n, const float* means, uint32_t* box6, hipStream_t st)
{
    if (n <= 0) return;
    int64_t g = (n + 255) / 256;
    if (g > 2048) g = 2048;
    hipLaunchKernelGGL(k_bbox, dim3((unsigned)g), dim3(256), 0, st, n, means, box6);
}

void launch_morton(int64_t n, const float* means, const float* lo_scale, uint64_t* keys,
                   uint32_t* vals, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_morton, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, means,
                       lo_scale, keys, vals);
}

void launch_invert(int64_t n, const uint32_t* perm, uint32_t* rank, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_invert, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, perm,
                       rank);
}

void launch_gather_gauss(int64_t n, const uint32_t* perm, const float* means, const float* cov3,
                         const double* covd, const float* lo2, float* means_o, float* cov3_o,
                         double* covd_o, float* lo2_o, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gather_gauss, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, perm,
                       means, cov3, covd, lo2, means_o, cov3_o, covd_o, lo2_o);
}

}  // namespace slag
