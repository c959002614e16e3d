// Per-tile front-to-back compositing with segment masking, and the per-pair
// merge of the partial weight sums (paper, Method: the rasterizer's weights
// w_kp of the contributing set K_p, the parameter masking w'_kp = w_kp M_j(p),
// and the per-view part of the aggregation sums over p in M_j).
//
// A 16x16 tile is one 256-thread workgroup: four wave64s, each owning an 8x8
// pixel block.  The tile's depth-ordered list is staged through LDS BATCH
// entries at a time.  For every entry each lane blends its pixel
// (alpha = min(0.99, o exp(-q/2)), skip below 1/255, stop before T < 1e-4,
// w = alpha T) and the wave reduces w over the lanes of each segment with DPP
// row reductions -- no global atomics, no float atomics, so the sums are
// deterministic.  The four waves' sums are added in fixed order and written to
// the entry's part slots: one float per (pair, tile, tile segment), laid out
// pair-major so the merge reads each pair's slots contiguously.
#include "slag_internal.h"

namespace slag {

namespace {

constexpr float AMIN = 1.0f / 255.0f;
constexpr float AMAX = 0.99f;
constexpr float TMIN = 1e-4f;
constexpr float NHALF_LOG2E = -0.72134752044448170368f;   // -log2(e) / 2
constexpr float NLOG2E = -1.44269504088896340736f;        // -log2(e)

__device__ __forceinline__ void box_of(const float4& r1, int& x0, int& x1, int& y0, int& y1)
{
    const uint32_t a = __float_as_uint(r1.z), b = __float_as_uint(r1.w);
    x0 = (int)(a & 0xFFFFu); y0 = (int)(a >> 16);
    x1 = (int)(b & 0xFFFFu); y1 = (int)(b >> 16);
}

__device__ __forceinline__ float dpp_f(float v, int ctrl);

template <int CTRL>
__device__ __forceinline__ float dpp_add(float v)
{
    return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ float readlane_f(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Sum over the 64 lanes; the result is valid in lane 0.  Call with all lanes
// active.  Fixed association order: deterministic.
__device__ __forceinline__ float wave_sum(float v)
{
    v = dpp_add<0xB1>(v);    // quad_perm [1,0,3,2]
    v = dpp_add<0x4E>(v);    // quad_perm [2,3,0,1]
    v = dpp_add<0x124>(v);   // row_ror:4
    v = dpp_add<0x128>(v);   // row_ror:8  -> every lane holds its row total
    return ((v + readlane_f(v, 16)) + readlane_f(v, 32)) + readlane_f(v, 48);
}

// Rectangle sum over a view's summed-area table (inclusive tile bounds).
__device__ __forceinline__ uint32_t sat_rect(const uint32_t* S, int sw, int xa, int xb, int ya,
                                             int yb)
{
    if (xa > xb || ya > yb) return 0;
    return S[(yb + 1) * sw + xb + 1] - S[ya * sw + xb + 1] - S[(yb + 1) * sw + xa] + S[ya * sw + xa];
}

// Distinct segment ids of each tile, ascending (sort + unique in LDS).
__global__ __launch_bounds__(256) void k_tile_segs(const uint32_t* __restrict__ bucket_view,
                                                   const ViewDev* __restrict__ views,
                                                   const int32_t* __restrict__ ids,
                                                   uint32_t* __restrict__ ns_tile,
                                                   uint16_t* __restrict__ segl)
{
    __shared__ uint32_t s[TILE_PIX];
    __shared__ uint32_t wsum[4];
    const uint32_t b = blockIdx.x;
    const ViewDev& V = views[bucket_view[b]];
    const uint32_t tile = b - V.tile_base;
    const int tx = (int)(tile % (uint32_t)V.ntx), ty = (int)(tile / (uint32_t)V.ntx);
    const int t = threadIdx.x;
    const int px = tx * TILE + (t & (TILE - 1)), py = ty * TILE + t / TILE;
    int32_t id = -1;
    if (px < V.W && py < V.H) id = ids[V.pix_off + (uint64_t)py * V.W + px];
    s[t] = id >= 0 ? (uint32_t)id : 0xFFFFFFFFu;
    __syncthreads();
    for (int k = 2; k <= TILE_PIX; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            const int o = t ^ j;
            if (o > t) {
                const uint32_t a = s[t], c = s[o];
                const bool up = (t & k) == 0;
                if ((a > c) == up) { s[t] = c; s[o] = a; }
            }
            __syncthreads();
        }
    }
    const uint32_t k = s[t];
    const uint32_t flag = (k != 0xFFFFFFFFu) && (t == 0 || s[t - 1] != k);
    // block exclusive scan of flags
    const int lane = t & 63, w = t >> 6;
    const uint64_t m = __ballot(flag);
    const uint32_t below = (uint32_t)__popcll(m & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
    if (lane == 0) wsum[w] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t off = 0;
    for (int i = 0; i < w; i++) off += wsum[i];
    if (flag) segl[(uint64_t)b * TILE_PIX + off + below] = (uint16_t)k;
    if (t == 0) ns_tile[b] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// Per-view summed-area table of the tile segment counts: (nty+1) x (ntx+1).
__global__ __launch_bounds__(256) void k_sat(const ViewDev* __restrict__ views,
                                             const uint32_t* __restrict__ ns_tile,
                                             uint32_t* __restrict__ sat)
{
    const ViewDev& V = views[blockIdx.x];
    const int sw = V.ntx + 1;
    uint32_t* S = sat + V.sat_off;
    for (int x = threadIdx.x; x < sw; x += 256) S[x] = 0;
    for (int y = threadIdx.x + 1; y <= V.nty; y += 256) {
        uint32_t run = 0;
        S[y * sw] = 0;
        for (int x = 1; x <= V.ntx; x++) {
            run += ns_tile[V.tile_base + (uint32_t)((y - 1) * V.ntx + (x - 1))];
            S[y * sw + x] = run;
        }
    }
    __syncthreads();
    for (int x = threadIdx.x + 1; x <= V.ntx; x += 256)
        for (int y = 1; y <= V.nty; y++) S[y * sw + x] += S[(y - 1) * sw + x];
}

template <bool COUNT>
__global__ __launch_bounds__(256) void k_composite(
    const uint32_t* __restrict__ bucket_view, const ViewDev* __restrict__ views,
    const uint32_t* __restrict__ bstart, const uint32_t* __restrict__ bend,
    const uint32_t* __restrict__ ival, const float4* __restrict__ rec,
    const uint32_t* __restrict__ part_base, const uint32_t* __restrict__ sat,
    const uint32_t* __restrict__ ns_tile, const uint16_t* __restrict__ segl,
    const int32_t* __restrict__ ids, float* __restrict__ part,
    unsigned long long* __restrict__ counters)
{
    __shared__ float4 s_p0[BATCH];            // u, v, A, B   (exponent e = A dx^2 + B dx dy + C dy^2)
    __shared__ float2 s_p1[BATCH];            // C, opacity
    __shared__ uint32_t s_off[BATCH];         // part slot of (pair, this tile, first tile segment)
    __shared__ uint2 s_box[COUNT ? BATCH : 1];
    __shared__ float s_acc[4][BATCH][NS_CAP];
    __shared__ uint16_t s_seg[TILE_PIX];

    const uint32_t b = blockIdx.x;
    const uint32_t start = bstart[b], end = bend[b];
    if (start >= end) return;
    const uint32_t ns = ns_tile[b];
    if (!COUNT && ns == 0) return;
    const ViewDev& V = views[bucket_view[b]];
    const uint32_t tile = b - V.tile_base;
    const int tx = (int)(tile % (uint32_t)V.ntx), ty = (int)(tile / (uint32_t)V.ntx);
    const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
    const int px = tx * TILE + (wv & 1) * 8 + (lane & 7);
    const int py = ty * TILE + (wv >> 1) * 8 + (lane >> 3);
    const bool valid = px < V.W && py < V.H;
    const int32_t seg = valid ? ids[V.pix_off + (uint64_t)py * V.W + px] : -1;
    for (uint32_t i = t; i < ns; i += 256) s_seg[i] = segl[(uint64_t)b * TILE_PIX + i];
    __syncthreads();
    int ls = -1;   // index of this pixel's segment among the tile's segments
    if (seg >= 0) {
        int lo = 0, hi = (int)ns - 1;
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if ((int)s_seg[mid] < seg) lo = mid + 1; else hi = mid;
        }
        ls = lo;
    }
    const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
    const uint32_t* S = sat + V.sat_off;
    const int sw = V.ntx + 1;
    unsigned long long n_acc = 0, n_box = 0, n_tile = 0;

    const int npass = ns == 0 ? 1 : (int)((ns + NS_CAP - 1) / NS_CAP);
    for (int pass = 0; pass < npass; pass++) {
        const int g0 = pass * NS_CAP;
        const int nsc = min(NS_CAP, (int)ns - g0);
        const bool counting = COUNT && pass == 0;
        const int slot = (ls >= g0 && ls < g0 + NS_CAP) ? ls - g0 : -1;
        // wave-uniform slot when every accumulating lane shares one segment
        int uslot = -1;
        {
            const uint64_t has = __ballot(slot >= 0);
            if (has) {
                const int first = __builtin_amdgcn_readlane(slot, __ffsll((long long)has) - 1);
                uslot = __ballot(slot >= 0 && slot != first) ? -2 : first;
            }
        }
        bool done = counting ? !valid : (slot < 0);
        float T = 1.0f;
        for (int i = t; i < 4 * BATCH * NS_CAP; i += 256) (&s_acc[0][0][0])[i] = 0.0f;
        __syncthreads();
        for (uint32_t base = start; base < end; base += BATCH) {
            const int nb = (int)min((uint32_t)BATCH, end - base);
            if (t < nb) {
                const uint32_t p = ival[base + t];
                const float4 r0 = rec[2 * (size_t)p];
                const float4 r1 = rec[2 * (size_t)p + 1];
                s_p0[t] = make_float4(r0.x, r0.y, r0.z * NHALF_LOG2E, r0.w * NLOG2E);
                s_p1[t] = make_float2(r1.x * NHALF_LOG2E, r1.y);
                int x0, x1, y0, y1;
                box_of(r1, x0, x1, y0, y1);
                const int tx0 = x0 / TILE, tx1 = x1 / TILE, ty0 = y0 / TILE;
                s_off[t] = part_base[p] + sat_rect(S, sw, tx0, tx1, ty0, ty - 1) +
                           sat_rect(S, sw, tx0, tx - 1, ty, ty) + (uint32_t)g0;
                if (COUNT) s_box[t] = make_uint2((uint32_t)x0 | ((uint32_t)x1 << 16),
                                                 (uint32_t)y0 | ((uint32_t)y1 << 16));
            }
            __syncthreads();
            if (!__all(done)) {
                for (int j = 0; j < nb; j++) {
                    const float4 p0 = s_p0[j];
                    const float2 p1 = s_p1[j];
                    float w = 0.0f;
                    if (!done) {
                        const float dx = fpx - p0.x, dy = fpy - p0.y;
                        float e = fmaf(dx, fmaf(p0.z, dx, p0.w * dy), p1.x * dy * dy);
                        e = fminf(e, 0.0f);
                        const float alpha = fminf(AMAX, p1.y * __builtin_amdgcn_exp2f(e));
                        if (counting) {
                            n_tile++;
                            const uint2 bx = s_box[j];
                            n_box += (px >= (int)(bx.x & 0xFFFFu) && px <= (int)(bx.x >> 16) &&
                                      py >= (int)(bx.y & 0xFFFFu) && py <= (int)(bx.y >> 16));
                        }
                        if (alpha >= AMIN) {
                            const float Tn = fmaf(-alpha, T, T);
                            if (Tn < TMIN) {
                                done = true;
                            } else {
                                w = alpha * T;
                                T = Tn;
                                if (counting) n_acc++;
                            }
                        }
                    }
                    if (uslot >= 0) {
                        const float wm = slot >= 0 ? w : 0.0f;
                        if (__any(wm > 0.0f)) {
                            const float s = wave_sum(wm);
                            if (lane == 0) s_acc[wv][j][uslot] = s;
                        }
                    } else if (uslot == -2) {
                        const float wm = slot >= 0 ? w : 0.0f;
                        uint64_t m = __ballot(wm > 0.0f);
                        while (m) {
                            const int sl = __builtin_amdgcn_readlane(slot, __ffsll((long long)m) - 1);
                            const bool mine = slot == sl;
                            const float s = wave_sum(mine ? wm : 0.0f);
                            if (lane == 0) s_acc[wv][j][sl] = s;
                            m &= ~__ballot(mine);
                        }
                    }
                }
            }
            __syncthreads();
            for (int i = t; i < nb * nsc; i += 256) {
                const int j = i / nsc, k = i - j * nsc;
                const float s = ((s_acc[0][j][k] + s_acc[1][j][k]) + s_acc[2][j][k]) + s_acc[3][j][k];
                if (s != 0.0f) part[s_off[j] + k] = s;
                s_acc[0][j][k] = 0.0f; s_acc[1][j][k] = 0.0f;
                s_acc[2][j][k] = 0.0f; s_acc[3][j][k] = 0.0f;
            }
            if (__syncthreads_count(!done) == 0) break;
        }
        __syncthreads();
    }
    if (COUNT) {
        // wave totals, one atomic per wave
        for (int d = 32; d >= 1; d >>= 1) {
            n_acc += __shfl_xor(n_acc, d, 64);
            n_box += __shfl_xor(n_box, d, 64);
            n_tile += __shfl_xor(n_tile, d, 64);
        }
        if (lane == 0) {
            atomicAdd(&counters[0], n_acc);
            atomicAdd(&counters[1], n_box);
            atomicAdd(&counters[2], n_tile);
        }
    }
}

// One thread per pair: walk its tiles in row-major order and keep the
// non-zero partial sums as (global segment row, weight).
__global__ __launch_bounds__(256) void k_merge(uint64_t npairs, const float4* __restrict__ rec,
                                               const uint16_t* __restrict__ pview,
                                               const ViewDev* __restrict__ views,
                                               const uint32_t* __restrict__ part_base,
                                               const float* __restrict__ part,
                                               const uint32_t* __restrict__ ns_tile,
                                               const uint16_t* __restrict__ segl,
                                               uint2* __restrict__ wrow,
                                               uint32_t* __restrict__ wlen,
                                               unsigned long long* __restrict__ nnz)
{
    const uint64_t p = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    uint32_t n = 0;
    if (p < npairs) {
        int x0, x1, y0, y1;
        box_of(rec[2 * p + 1], x0, x1, y0, y1);
        const ViewDev& V = views[pview[p]];
        const uint32_t base = part_base[p];
        uint32_t k = 0;
        for (int ty = y0 / TILE; ty <= y1 / TILE; ty++)
            for (int tx = x0 / TILE; tx <= x1 / TILE; tx++) {
                const uint32_t bk = V.tile_base + (uint32_t)(ty * V.ntx + tx);
                const uint32_t ns = ns_tile[bk];
                for (uint32_t i = 0; i < ns; i++) {
                    const float w = part[base + k++];
                    if (w > 0.0f) {
                        wrow[base + n] = make_uint2(V.seg_off + segl[(uint64_t)bk * TILE_PIX + i],
                                                    __float_as_uint(w));
                        n++;
                    }
                }
            }
        wlen[p] = n;
    }
    unsigned long long c = n;
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(nnz, c);
}

}  // namespace

void launch_tile_segs(uint32_t nbuckets, const uint32_t* bucket_view, const ViewDev* views,
                      const int32_t* ids, uint32_t* ns_tile, uint16_t* segl, hipStream_t st)
{
    if (!nbuckets) return;
    hipLaunchKernelGGL(k_tile_segs, dim3(nbuckets), dim3(256), 0, st, bucket_view, views, ids,
                       ns_tile, segl);
}

void launch_sat(int nb, const ViewDev* views, const uint32_t* ns_tile, uint32_t* sat,
                hipStream_t st)
{
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_sat, dim3(nb), dim3(256), 0, st, views, ns_tile, sat);
}

void launch_composite(bool count, uint32_t nbuckets, const uint32_t* bucket_view,
                      const ViewDev* views, const uint32_t* bstart, const uint32_t* bend,
                      const uint32_t* ival, const float4* rec, const uint32_t* part_base,
                      const uint32_t* sat, const uint32_t* ns_tile, const uint16_t* segl,
                      const int32_t* ids, float* part, unsigned long long* counters,
                      hipStream_t st)
{
    if (!nbuckets) return;
    if (count)
        hipLaunchKernelGGL(k_composite<true>, dim3(nbuckets), dim3(256), 0, st, bucket_view, views,
                           bstart, bend, ival, rec, part_base, sat, ns_tile, segl, ids, part,
                           counters);
    else
        hipLaunchKernelGGL(k_composite<false>, dim3(nbuckets), dim3(256), 0, st, bucket_view,
                           views, bstart, bend, ival, rec, part_base, sat, ns_tile, segl, ids,
                           part, counters);
}

void launch_merge(uint64_t npairs, const float4* rec, const uint16_t* pview, const ViewDev* views,
                  const uint32_t* part_base, const float* part, const uint32_t* ns_tile,
                  const uint16_t* segl, uint2* wrow, uint32_t* wlen, unsigned long long* nnz,
                  hipStream_t st)
{
    if (!npairs) return;
    hipLaunchKernelGGL(k_merge, dim3((unsigned)((npairs + 255) / 256)), dim3(256), 0, st, npairs,
                       rec, pview, views, part_base, part, ns_tile, segl, wrow, wlen, nnz);
}

}  // namespace slag
