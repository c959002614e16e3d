// Per-tile front-to-back compositing with segment masking, and the per-pair
// merge of the partial weight sums (paper, Method: the rasterizer's weights
// w_kp of the contributing set K_p, the parameter masking w'_kp = w_kp M_j(p),
// and the per-view part of the aggregation sums over p in M_j).
//
// A 16x16 tile is one 256-thread workgroup: four wave64s, each owning an 8x8
// pixel block (an 8x8 tile, the other tile size, is one wave).  The tile's depth-ordered list is staged through LDS BATCH
// entries at a time.  For every entry each lane blends its pixel
// (alpha = min(0.99, o exp(-q/2)), skip below 1/255, stop before T < 1e-4,
// w = alpha T) and each 16-lane row reduces w over the lanes of each segment
// with DPP -- no global atomics, no float atomics, so the sums are
// deterministic.  The sixteen row sums are added in fixed order and written to
// the entry's part slots: one (tile-local segment id, weight) slot per (pair,
// tile, tile segment), laid out pair-major so each pair's slots are
// contiguous for the contraction.
#include <algorithm>

#include "slag_internal.h"

namespace slag {

namespace {

// alpha_min, alpha_max, the transmittance stop t_min and log2(alpha_min)
// come with each view (the context's options; 3D Gaussian splatting's
// 1/255, 0.99 and 1e-4 by default).

__device__ __forceinline__ void box_of(const float4& r1, int& x0, int& x1, int& y0, int& y1)
{
    const uint32_t a = __float_as_uint(r1.z), b = __float_as_uint(r1.w);
    x0 = (int)(a & 0xFFFFu); y0 = (int)(a >> 16);
    x1 = (int)(b & 0xFFFFu); y1 = (int)(b >> 16);
}

template <int CTRL>
__device__ __forceinline__ float dpp_add(float v)
{
    return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Sum over each 16-lane row of the wave; every lane receives its row's total.
// Call with all lanes active.  Fixed association order: deterministic.
__device__ __forceinline__ float row_sum(float v)
{
    v = dpp_add<0xB1>(v);    // quad_perm [1,0,3,2]
    v = dpp_add<0x4E>(v);    // quad_perm [2,3,0,1]
    v = dpp_add<0x124>(v);   // row_ror:4
    v = dpp_add<0x128>(v);   // row_ror:8
    return v;
}

// Rectangle sum over a view's summed-area table (inclusive tile bounds).
__device__ __forceinline__ uint32_t sat_rect(const uint32_t* S, int sw, int xa, int xb, int ya,
                                             int yb)
{
    if (xa > xb || ya > yb) return 0;
    return S[(yb + 1) * sw + xb + 1] - S[ya * sw + xb + 1] - S[(yb + 1) * sw + xa] + S[ya * sw + xa];
}

// Distinct segment ids of each tile, ascending, over every label layer of
// its pixels (a pixel lies in up to lpp masks; -1 = none).  One wave per
// tile, four tiles per workgroup: each lane holds TS^2 / 64 pixels of the
// TS x TS tile (column lane % TS, rows lane / TS + (64 / TS) r) with their
// NL = 1 or MAX_LABELS layers.  A ballot loop finds one distinct id per iteration (the
// first remaining value of the first lane that has one), clears it in every
// lane and appends it to the wave's list in LDS; each id of the list then
// goes to the position given by the number of smaller ids.  Tiles hold few
// segments, so both loops are short.  More than TS^2 distinct ids in one
// tile (only possible with several layers) set bit 4 of *err and keep the
// TS^2 smallest.
template <int NL, int TS>
__global__ __launch_bounds__(256) void k_tile_segs(uint32_t nbuckets,
                                                   const uint32_t* __restrict__ bucket_view,
                                                   const ViewDev* __restrict__ views,
                                                   const int32_t* __restrict__ ids, int lpp,
                                                   uint32_t* __restrict__ ns_tile,
                                                   uint16_t* __restrict__ segl,
                                                   unsigned long long* __restrict__ err)
{
    constexpr int TPX = TS * TS, NR = TPX / 64, RPP = 64 / TS;
    constexpr int NV = NR * NL;   // values per lane
    __shared__ uint32_t cand[4][64 * NV];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t b = blockIdx.x * 4u + (uint32_t)w;
    if (b >= nbuckets) return;   // whole waves; nothing below waits for other waves
    const ViewDev& V = views[bucket_view[b]];
    const uint32_t tile = b - V.tile_base;
    const int tx = (int)(tile % (uint32_t)V.ntx), ty = (int)(tile / (uint32_t)V.ntx);
    const int px = tx * TS + lane % TS;
    int32_t idv[NV];
    uint32_t left = 0;   // bit k: value k is an id not yet taken
#pragma unroll
    for (int r = 0; r < NR; r++) {
        const int py = ty * TS + lane / TS + RPP * r;
        const bool inside = px < V.W && py < V.H;
        const uint64_t pb = (V.pix_off + (uint64_t)py * V.W + px) * (uint64_t)lpp;
#pragma unroll
        for (int l = 0; l < NL; l++) {
            const int32_t id = (inside && l < lpp) ? ids[pb + l] : -1;
            idv[r * NL + l] = id;
            if (id >= 0) left |= 1u << (r * NL + l);
        }
    }
    uint32_t nc = 0;   // wave-uniform
    for (;;) {
        const uint64_t act = __ballot(left != 0);
        if (!act) break;
        int mine = 0;
#pragma unroll
        for (int k = NV - 1; k >= 0; k--)
            if ((left >> k) & 1u) mine = idv[k];
        const int v = __builtin_amdgcn_readlane(mine, __ffsll((long long)act) - 1);
#pragma unroll
        for (int k = 0; k < NV; k++)
            if (idv[k] == v) left &= ~(1u << k);
        if (lane == 0) cand[w][nc] = (uint32_t)v;
        nc++;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (uint32_t i = (uint32_t)lane; i < nc; i += 64) {
        const uint32_t c = cand[w][i];
        uint32_t pos = 0;
        for (uint32_t j = 0; j < nc; j++) pos += cand[w][j] < c;
        if (pos < (uint32_t)TPX) segl[(uint64_t)b * TPX + pos] = (uint16_t)c;
    }
    if (lane == 0) {
        ns_tile[b] = nc < (uint32_t)TPX ? nc : (uint32_t)TPX;
        if (nc > (uint32_t)TPX) atomicOr(err, 4ull);
    }
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

// Sum over the 64 lanes of v; valid in every lane.  Fixed order.
__device__ __forceinline__ float wave_total(float v)
{
    v = row_sum(v);
    const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    return ((r0 + r1) + r2) + r3;
}

enum { MODE_NONE = 0, MODE_UNIFORM = 1, MODE_MIXED = 2 };

// max over t in [t0, t1] of P a^2 + Q a t + R t^2 (R < 0): the vertex
// -Q a / (2 R), clamped to the interval (the reciprocal's rounding moves the
// point, and so the value, by far less than the caller's margin)
__device__ __forceinline__ float qmax_edge(float a, float t0, float t1, float P, float Q, float R)
{
    const float t = fminf(fmaxf(-0.5f * (Q * a) * __builtin_amdgcn_rcpf(R), t0), t1);
    return fmaf(fmaf(R, t, Q * a), t, P * a * a);
}

// Can an entry reach alpha >= 1/255 at any pixel of the active rectangle
// (offsets dx in [x0, x1], dy in [y0, y1] from its mean)?  The exponent
// log2(o) + A dx^2 + B dx dy + C dy^2 is concave, so its maximum over the
// rectangle is 0 + log2(o) when the mean lies inside, else the largest of the
// four edge maxima.  An entry is dropped only when that maximum stays below
// log2(1/255) by a margin (0.01, plus 1e-6 of the magnitude of the terms the
// blend sums) beyond any rounding of the blend's own evaluation: then every
// pixel gets alpha < 1/255 and is left unchanged, so dropping it is exact.
__device__ __forceinline__ bool reaches_amin(float A, float B, float C, float lo2, float x0,
                                             float x1, float y0, float y1, float l2amin)
{
    float m = 0.0f;
    if (!(x0 <= 0.0f && x1 >= 0.0f && y0 <= 0.0f && y1 >= 0.0f))
        m = fmaxf(fmaxf(qmax_edge(x0, y0, y1, A, B, C), qmax_edge(x1, y0, y1, A, B, C)),
                  fmaxf(qmax_edge(y0, x0, x1, C, B, A), qmax_edge(y1, x0, x1, C, B, A)));
    const float d = fmaxf(fmaxf(fabsf(x0), fabsf(x1)), fmaxf(fabsf(y0), fabsf(y1))) + 8.0f;
    const float mag = 3.0f * (fabsf(A) + fabsf(B) + fabsf(C)) * d * d + fabsf(lo2);
    return lo2 + m >= l2amin - 0.01f - 1e-6f * mag;
}

// Wave sums of four per-lane values: on return every lane of row r (lanes
// 16 r .. 16 r + 15) holds the sum of value r over all 64 lanes.  Two lane
// swaps across the wave halves, one across rows, then a DPP row sum: about
// ten instructions for four sums.
__device__ __forceinline__ float wave_sum4(float v0, float v1, float v2, float v3)
{
    const auto a = __builtin_amdgcn_permlane32_swap(__float_as_uint(v0), __float_as_uint(v2),
                                                    false, false);
    const auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(v1), __float_as_uint(v3),
                                                    false, false);
    const float x0 = __uint_as_float(a[0]) + __uint_as_float(a[1]);   // lanes 0-31: v0, 32-63: v2
    const float x1 = __uint_as_float(b[0]) + __uint_as_float(b[1]);   // lanes 0-31: v1, 32-63: v3
    const auto c = __builtin_amdgcn_permlane16_swap(__float_as_uint(x0), __float_as_uint(x1),
                                                    false, false);
    return row_sum(__uint_as_float(c[0]) + __uint_as_float(c[1]));    // row r: value r
}

// Blend this wave's compacted entries of one batch into its 64 pixels, four
// entries at a time; the four entries' per-segment weight sums over the
// wave's pixels go to acc[batch entry][segment slot].
// A lane's pixel inside its wave's 8x8 block, relative to the block centre (lx, ly in
// -3.5 .. 3.5).
struct LaneXY {
    float lx, ly;
};

template <int MODE, bool COUNTING, bool PAD, bool KW>
__device__ __forceinline__ void blend_batch(const float4* __restrict__ w0, const float4* __restrict__ w1,
                                            const float* __restrict__ wlo,
                                            const int* __restrict__ wj, int cnt, const LaneXY& Q,
                                            int px, int py, uint32_t sbits, int uslot,
                                            uint32_t slot_mask,
                                            float& T, bool& done, float (*acc)[NS_CAP], int lane,
                                            unsigned long long& n_acc, unsigned long long& n_box,
                                            unsigned long long& n_tile, float& wsum, float amin,
                                            float amax, float tmin)
{
    const bool slot_ok = sbits != 0;   // the pixel lies in a segment of this pass
    const int r = lane >> 4;
    const bool writer = (lane & 15) == 0;
    for (int g = 0; g < cnt; g += 4) {
        float w[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            // PAD: entries past cnt (up to the next multiple of four) are null:
            // opacity 0, so alpha = 0 and nothing changes; else skip them
            const int jj = g + u;
            if (!PAD) {
                w[u] = 0.0f;
                if (jj >= cnt) continue;                 // wave-uniform
            }
            // alpha = min(0.99, o exp(-q/2)) = min(0.99, 2^e) with
            // e = log2(o) - q log2(e) / 2 a quadratic in the lane's block
            // coordinates (coefficients from the compaction step)
            const float4 p0 = w0[jj];
            const float4 p1 = w1[jj];
            const float tx = fmaf(p1.x, Q.ly, fmaf(p0.w, Q.lx, p0.y));   // cx + cxx lx + cxy ly
            const float ty = fmaf(p1.y, Q.ly, p0.z);                       // cy + cyy ly
            const float e = fmaf(ty, Q.ly, fmaf(tx, Q.lx, p0.x));
            const float alpha = fminf(amax, __builtin_amdgcn_exp2f(e));
            const float Tn = fmaf(-alpha, T, T);
            // the weight: alpha T, or (KW) the Gaussian kernel exp(-q/2) =
            // 2^(e - log2 o) of each blended Gaussian (the paper's weight
            // equation)
            const float wv = KW ? __builtin_amdgcn_exp2f(e - wlo[jj]) : alpha * T;
            if (COUNTING) {
                const bool ok = !done && alpha >= amin;
                const bool stop = ok && Tn < tmin;
                const bool take = ok && !stop;
                w[u] = (take && slot_ok) ? wv : 0.0f;
                if (!done && jj < cnt) {
                    n_tile++;
                    const uint32_t a = __float_as_uint(p1.z), b = __float_as_uint(p1.w);
                    n_box += (px >= (int)(a & 0xFFFFu) && px <= (int)(b & 0xFFFFu) &&
                              py >= (int)(a >> 16) && py <= (int)(b >> 16));
                }
                n_acc += take;
                wsum += take ? wv : 0.0f;
                T = take ? Tn : T;
                done = done || stop;
            } else {
                // T = 0 marks a finished pixel (stopped, or nothing to add in
                // this pass): then Tn = 0 < tmin and w = 0 from here on
                const bool ok = alpha >= amin;
                const bool keep = Tn >= tmin;
                w[u] = (ok && keep) ? wv : 0.0f;
                T = ok ? (keep ? Tn : 0.0f) : T;
            }
        }
        if (!COUNTING) done = T == 0.0f;
        const int jr = g + r;
        if (MODE == MODE_UNIFORM) {
            const float s = wave_sum4(w[0], w[1], w[2], w[3]);
            if (writer && jr < cnt) acc[wj[jr]][uslot] = s;
        } else if (MODE == MODE_MIXED) {
            uint32_t sm = slot_mask;
            while (sm) {
                const int sl = __builtin_ctz(sm);
                sm &= sm - 1u;
                const bool mine = (sbits >> sl) & 1u;
                const float s = wave_sum4(mine ? w[0] : 0.0f, mine ? w[1] : 0.0f,
                                          mine ? w[2] : 0.0f, mine ? w[3] : 0.0f);
                if (writer && jr < cnt) acc[wj[jr]][sl] = s;
            }
        }
        if (__all(done)) break;
    }
}

// One tile (bucket b: a (view, tile) with a non-empty list) composited by the
// workgroup: TS x TS pixels, one wave per 8x8 block (four waves, or one).  Variants (same arithmetic, bitwise-equal results): MINW (of the
// kernel) = waves per SIMD the register budget must allow; PAD = four-entry
// groups padded with null entries (loads of a group can be issued together)
// or cut at the end.
template <bool COUNT, bool PAD, int LMAX, bool KW, int BT, int TS>
__device__ __forceinline__ void composite_tile(
    const uint32_t b, const int t,
    const uint32_t* __restrict__ bucket_view, const ViewDev* __restrict__ views,
    const uint32_t* __restrict__ bstart, const uint32_t* __restrict__ bend,
    const uint32_t* __restrict__ ival, uint2* __restrict__ pinfo,
    const float4* __restrict__ rec, const uint32_t* __restrict__ ns_tile,
    const uint16_t* __restrict__ segl, const int32_t* __restrict__ ids, int lpp,
    uint2* __restrict__ part, unsigned long long* __restrict__ counters,
    float* __restrict__ pix_t, float* __restrict__ pix_w, uint32_t* __restrict__ pix_n)
{
    static_assert(BT % 4 == 0 && BT <= 64, "one batch entry per lane, groups of four");
    static_assert(TS == 16 || TS == 8, "tiles of 16 x 16 or 8 x 8 pixels");
    constexpr int NW = TS * TS / 64, NTH = 64 * NW, TPX = TS * TS;
    __shared__ float4 s_w0[NW][BT];           // per wave: entries touching its block, exponent
    __shared__ float4 s_w1[NW][BT];           //   coefficients (c0, cx, cy, cxx), (cxy, cyy, box, box)
    __shared__ int s_wj[NW][BT];              //   their index in the batch
    __shared__ float s_lo[NW][BT];            //   log2(opacity) (kernel weights)
    __shared__ float s_acc[NW][BT][NS_CAP];   // per wave weight sums [entry][segment]
    __shared__ uint32_t s_pair[BT];           // pair of each batch entry
    __shared__ uint32_t s_tir[BT];            // index of this tile in the pair's tile rectangle
    __shared__ uint16_t s_seg[TPX];

    const uint32_t start = bstart[b], end = bend[b];
    if (start >= end) return;
    const uint32_t ns = ns_tile[b];
    if (!COUNT && ns == 0) return;
    const ViewDev& V = views[bucket_view[b]];
    const uint32_t tile = b - V.tile_base;
    const int tx = (int)(tile % (uint32_t)V.ntx), ty = (int)(tile / (uint32_t)V.ntx);
    const int wv = t >> 6, lane = t & 63;
    const float amin = V.amin, amax = V.amax, tmin = V.tmin, l2amin = V.l2amin;
    const int bx0 = tx * TS + (wv & 1) * 8;    // this wave's 8x8 pixel block
    const int by0 = ty * TS + (wv >> 1) * 8;
    const int px = bx0 + (lane & 7);
    const int py = by0 + (lane >> 3);
    const bool valid = px < V.W && py < V.H;
    // the pixel's segments (masks containing it; LMAX = 1: one id per pixel)
    int32_t seg[LMAX];
#pragma unroll
    for (int l = 0; l < LMAX; l++)
        seg[l] = (valid && l < lpp) ? ids[(V.pix_off + (uint64_t)py * V.W + px) * (uint64_t)lpp + l] : -1;
    for (uint32_t i = t; i < ns; i += NTH) s_seg[i] = segl[(uint64_t)b * TPX + i];
    __syncthreads();
    int ls[LMAX];   // index of each of the pixel's segments among the tile's segments
#pragma unroll
    for (int l = 0; l < LMAX; l++) {
        ls[l] = -1;
        if (seg[l] >= 0) {
            int lo = 0, hi = (int)ns - 1;
            while (lo < hi) {
                int mid = (lo + hi) >> 1;
                if ((int)s_seg[mid] < seg[l]) lo = mid + 1; else hi = mid;
            }
            ls[l] = (int)s_seg[lo] == seg[l] ? lo : -1;   // not kept: a tile over capacity
        }
    }
    // lane offsets from the block centre (bx0 + 4, by0 + 4): the exponent is
    // expanded there, so no lane is more than 3.5 px from the expansion point
    LaneXY Q;
    Q.lx = (float)(lane & 7) - 3.5f;
    Q.ly = (float)(lane >> 3) - 3.5f;
    unsigned long long n_acc = 0, n_box = 0, n_tile = 0;
    float wsum = 0.0f;   // counting pass: the pixel's accepted weight
    const uint32_t last = end - 1;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    const int npass = ns == 0 ? 1 : (int)((ns + NS_CAP - 1) / NS_CAP);
    for (int pass = 0; pass < npass; pass++) {
        const int g0 = pass * NS_CAP;
        const int nsc = min(NS_CAP, (int)ns - g0);
        const bool counting = COUNT && pass == 0;
        // this pass's slots of the pixel's segments, as bits
        uint32_t sbits = 0;
#pragma unroll
        for (int l = 0; l < LMAX; l++)
            if (ls[l] >= g0 && ls[l] < g0 + NS_CAP) sbits |= 1u << (ls[l] - g0);
        // wave-uniform slot when every accumulating lane has the same single
        // segment; else the set of slots present in the wave
        int mode = MODE_NONE, uslot = -1;
        uint32_t slot_mask = 0;
        {
            const uint64_t has = __ballot(sbits != 0);
            if (has) {
                const uint32_t first =
                    (uint32_t)__builtin_amdgcn_readlane((int)sbits, __ffsll((long long)has) - 1);
                const bool mixed = (first & (first - 1u)) != 0 ||
                                   __ballot(sbits != 0 && sbits != first) != 0;
                mode = mixed ? MODE_MIXED : MODE_UNIFORM;
                uslot = __builtin_ctz(first);
                for (int k = 0; k < nsc; k++)
                    if (__ballot((sbits >> k) & 1u)) slot_mask |= 1u << k;
            }
        }
        bool done = counting ? !valid : (sbits == 0);
        float T = (counting || sbits != 0) ? 1.0f : 0.0f;
        for (int i = lane; i < BT * NS_CAP; i += 64) (&s_acc[wv][0][0])[i] = 0.0f;
        // lane l holds entry l of the batch (lanes past BT repeat the last
        // one).  Two-deep prefetch: records of the next batch and list
        // entries of the one after are in flight while a batch blends
        // (unconditional clamped loads: every address is inside the list;
        // nothing waits on them until they are used).
        const uint32_t le = (uint32_t)min(lane, BT - 1);
        uint32_t e = min(start + le, last);
        uint32_t pcur = ival[e];
        float4 q0 = rec[2 * (size_t)pcur], q1 = rec[2 * (size_t)pcur + 1];
        e = min(start + BT + le, last);
        uint32_t pn = ival[e];
        for (uint32_t base = start; base < end; base += BT) {
            const int nb = (int)min((uint32_t)BT, end - base);
            // the bounding box of this wave's pixels that can still take
            // weight (lane = 8 y + x), from the active-lane mask
            const uint64_t am = __ballot(!done);
            int ax0 = 0, ax1 = -1, ay0 = 0, ay1 = -1;
            if (am) {
                uint64_t c = am | (am >> 32);
                c |= c >> 16;
                c |= c >> 8;
                const uint32_t cols = (uint32_t)(c & 0xFFu);
                ax0 = __builtin_ctz(cols);
                ax1 = 31 - __builtin_clz(cols);
                ay0 = __builtin_ctzll(am) >> 3;
                ay1 = (63 - __builtin_clzll(am)) >> 3;
            }
            // compact the entries whose pixel box meets those pixels' box (and,
            // outside the counting pass, that can reach alpha >= 1/255 there)
            const uint32_t ba = __float_as_uint(q1.z), bb = __float_as_uint(q1.w);
            bool hit = lane < nb && (int)(bb & 0xFFFFu) >= bx0 + ax0 &&
                       (int)(ba & 0xFFFFu) <= bx0 + ax1 && (int)(bb >> 16) >= by0 + ay0 &&
                       (int)(ba >> 16) <= by0 + ay1;
            // exponent log2(o) + A dx^2 + B dx dy + C dy^2 with dx = lx - du,
            // dy = ly - dv (pixel centre relative to the entry's mean; du, dv:
            // the mean relative to the block centre, from its offset to the box
            // corner)
            const float A = q0.z, B = q0.w, C = q1.x;   // prescaled in the record
            const float du = q0.x + (float)((int)(ba & 0xFFFFu) - bx0 - 4);
            const float dv = q0.y + (float)((int)(ba >> 16) - by0 - 4);
            const float lo2 = q1.y;                        // log2(o)
            if (!COUNT && hit)
                hit = reaches_amin(A, B, C, lo2, (float)ax0 - 3.5f - du, (float)ax1 - 3.5f - du,
                                   (float)ay0 - 3.5f - dv, (float)ay1 - 3.5f - dv, l2amin);
            const uint64_t hm = __ballot(hit);
            const int cnt = __popcll(hm);
            if (hit) {
                // the exponent expanded in the block coordinates lx, ly: six
                // coefficients
                const int k = __popcll(hm & lt);
                const float cx = -fmaf(2.0f * A, du, B * dv);
                const float cy = -fmaf(B, du, 2.0f * C * dv);
                const float c0 = fmaf(A * du, du, fmaf(B * du, dv, C * dv * dv)) + lo2;
                s_w0[wv][k] = make_float4(c0, cx, cy, A);
                s_w1[wv][k] = make_float4(B, C, q1.z, q1.w);
                s_wj[wv][k] = lane;
                if (KW) s_lo[wv][k] = lo2;
            }
            if (PAD && lane >= cnt && lane < ((cnt + 3) & ~3)) {   // null entries up to a multiple of 4
                s_w0[wv][lane] = make_float4(-1e30f, 0.0f, 0.0f, 0.0f);   // 2^e = 0
                s_w1[wv][lane] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if (KW) s_lo[wv][lane] = 0.0f;
            }
            if (wv == 0 && lane < nb) {
                const int rtx0 = (int)(ba & 0xFFFFu) / TS, rty0 = (int)(ba >> 16) / TS;
                const int rw = (int)(bb & 0xFFFFu) / TS - rtx0 + 1;
                s_pair[lane] = pcur;
                s_tir[lane] = (uint32_t)((ty - rty0) * rw + (tx - rtx0));
            }
            q0 = rec[2 * (size_t)pn];
            q1 = rec[2 * (size_t)pn + 1];
            pcur = pn;
            e = min(base + 2 * BT + le, last);
            pn = ival[e];
            __builtin_amdgcn_wave_barrier();
            if (cnt && !__all(done)) {
                if (counting) {
                    if (mode == MODE_UNIFORM)
                        blend_batch<MODE_UNIFORM, true, PAD, KW>(s_w0[wv], s_w1[wv], s_lo[wv], s_wj[wv], cnt, Q, px, py, sbits, uslot, slot_mask, T, done, s_acc[wv], lane, n_acc, n_box, n_tile, wsum, amin, amax, tmin);
                    else if (mode == MODE_MIXED)
                        blend_batch<MODE_MIXED, true, PAD, KW>(s_w0[wv], s_w1[wv], s_lo[wv], s_wj[wv], cnt, Q, px, py, sbits, uslot, slot_mask, T, done, s_acc[wv], lane, n_acc, n_box, n_tile, wsum, amin, amax, tmin);
                    else
                        blend_batch<MODE_NONE, true, PAD, KW>(s_w0[wv], s_w1[wv], s_lo[wv], s_wj[wv], cnt, Q, px, py, sbits, uslot, slot_mask, T, done, s_acc[wv], lane, n_acc, n_box, n_tile, wsum, amin, amax, tmin);
                } else {
                    if (mode == MODE_UNIFORM)
                        blend_batch<MODE_UNIFORM, false, PAD, KW>(s_w0[wv], s_w1[wv], s_lo[wv], s_wj[wv], cnt, Q, px, py, sbits, uslot, slot_mask, T, done, s_acc[wv], lane, n_acc, n_box, n_tile, wsum, amin, amax, tmin);
                    else
                        blend_batch<MODE_MIXED, false, PAD, KW>(s_w0[wv], s_w1[wv], s_lo[wv], s_wj[wv], cnt, Q, px, py, sbits, uslot, slot_mask, T, done, s_acc[wv], lane, n_acc, n_box, n_tile, wsum, amin, amax, tmin);
                }
            }
            __syncthreads();
            // one thread per batch entry: the waves' sums per segment, in a
            // fixed order; the non-zero ones are appended to the pair's part
            // list (one atomic per (pair, tile) with output; the lists'
            // order is arbitrary, so readers visit entries by key)
            if (t < nb) {
                float sv[NS_CAP];
                int nz = 0;
#pragma unroll
                for (int k = 0; k < NS_CAP; k++) {
                    sv[k] = 0.0f;
                    if (k < nsc) {
                        if constexpr (NW == 4) {
                            sv[k] = ((s_acc[0][t][k] + s_acc[1][t][k]) + s_acc[2][t][k]) + s_acc[3][t][k];
                            s_acc[0][t][k] = 0.0f; s_acc[1][t][k] = 0.0f;
                            s_acc[2][t][k] = 0.0f; s_acc[3][t][k] = 0.0f;
                        } else {
                            sv[k] = s_acc[0][t][k];
                            s_acc[0][t][k] = 0.0f;
                        }
                        nz += sv[k] != 0.0f;
                    }
                }
                if (nz) {
                    const uint32_t p = s_pair[t];
                    // pinfo[p] = (list base, fill count); the capacity is the
                    // next list's base (neighbouring record, same line mostly)
                    const uint32_t b0 = pinfo[p].x, b1 = pinfo[p + 1].x;
                    const uint32_t o = atomicAdd(&pinfo[p].y, (uint32_t)nz);
                    if (o + (uint32_t)nz <= b1 - b0) {   // always, by construction of the capacity
                        uint2* dst = part + b0 + o;
                        const uint32_t tk = (s_tir[t] & 0xFFFFu) << 16;
#pragma unroll
                        for (int k = 0; k < NS_CAP; k++)
                            if (sv[k] != 0.0f)
                                *dst++ = make_uint2(tk | (uint32_t)s_seg[g0 + k], __float_as_uint(sv[k]));
                    } else {
                        // a capacity error would lose weight: count it, the
                        // fetch of the result reports it
                        atomicAdd(&counters[3], (unsigned long long)nz);
                    }
                }
            }
            if (__syncthreads_count(!done) == 0) break;
        }
        if (counting && pix_t && valid) {
            // per-pixel debug outputs of the counting pass (every pixel walked)
            const uint64_t pi = V.pix_off + (uint64_t)py * V.W + px;
            pix_t[pi] = T;
            pix_w[pi] = wsum;
            pix_n[pi] = (uint32_t)n_acc;
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

// The compositing kernel.  Buckets are taken in the given order (longest
// lists first, over all views of the launch): either one workgroup per
// bucket (the hardware hands out workgroups in index order), or PERSIST: a
// grid of resident workgroups that each take the next bucket from a queue
// counter (*queue = 0 at launch) until all nbk are taken.
template <bool COUNT, int MINW, bool PAD, int LMAX, bool KW, bool PERSIST, int BT, int TS>
__global__ __launch_bounds__(TS * TS, TS == 16 ? MINW : 4 * MINW) void k_composite(
    const uint32_t* __restrict__ order, uint32_t obase, uint32_t nbk,
    uint32_t* __restrict__ queue,
    const uint32_t* __restrict__ bucket_view, const ViewDev* __restrict__ views,
    const uint32_t* __restrict__ bstart, const uint32_t* __restrict__ bend,
    const uint32_t* __restrict__ ival, uint2* __restrict__ pinfo,
    const float4* __restrict__ rec, const uint32_t* __restrict__ ns_tile,
    const uint16_t* __restrict__ segl, const int32_t* __restrict__ ids, int lpp,
    uint2* __restrict__ part, unsigned long long* __restrict__ counters,
    float* __restrict__ pix_t, float* __restrict__ pix_w, uint32_t* __restrict__ pix_n)
{
    if (!PERSIST) {
        composite_tile<COUNT, PAD, LMAX, KW, BT, TS>(order[obase + blockIdx.x], (int)threadIdx.x,
                                             bucket_view, views,
                                             bstart, bend, ival, pinfo, rec, ns_tile, segl, ids,
                                             lpp, part, counters, pix_t, pix_w, pix_n);
        return;
    }
    __shared__ uint32_t s_q;
    for (;;) {
        // the two barriers: every thread has left the previous tile before
        // the next index is published, and has read it before it changes
        if (threadIdx.x == 0) s_q = atomicAdd(queue, 1u);
        __syncthreads();
        const uint32_t i = s_q;
        __syncthreads();
        if (i >= nbk) break;   // the counter only grows: every workgroup gets here
        // the thread index passed as a value the compiler cannot carry across
        // tiles: what the tile derives from it is formed per tile, not held
        // in registers over the loop
        int t = (int)threadIdx.x;
        asm volatile("" : "+v"(t));
        composite_tile<COUNT, PAD, LMAX, KW, BT, TS>(order[obase + i], t, bucket_view, views, bstart, bend,
                                             ival, pinfo, rec, ns_tile, segl, ids, lpp, part,
                                             counters, pix_t, pix_w, pix_n);
    }
}

// Render-back of per-Gaussian attributes into one view (the paper's
// rendering equation with the lift's weights: C_p = sum_k w_kp a_k /
// sum_k w_kp over the Gaussians the front-to-back walk blends at p, every
// pixel, no masking).  One workgroup per TS x TS tile of the view, one wave
// per 8x8 pixels; the tile's list is staged BATCH entries at a time with the
// entries' attribute channels [c0, c0 + 16); every lane evaluates every
// entry with the compositing's own exponent expansion (about its wave's
// block centre), so its weights and decisions are the lift's, bit for bit.
template <bool KW, int TS>
__global__ __launch_bounds__(TS * TS) void k_render(const ViewDev* __restrict__ views, int vi,
                                                const uint32_t* __restrict__ bstart,
                                                const uint32_t* __restrict__ bend,
                                                const uint32_t* __restrict__ ival,
                                                const float4* __restrict__ rec,
                                                const uint32_t* __restrict__ pgauss,
                                                const float* __restrict__ attr, int C, int c0,
                                                float* __restrict__ out,
                                                float* __restrict__ wsum_out)
{
    __shared__ float4 s_r0[BATCH], s_r1[BATCH];
    __shared__ float s_a[BATCH][16];
    const ViewDev& V = views[vi];
    const uint32_t tile = blockIdx.x;
    const uint32_t b = V.tile_base + tile;
    const int tx = (int)(tile % (uint32_t)V.ntx), ty = (int)(tile / (uint32_t)V.ntx);
    const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
    const int bx0 = tx * TS + (wv & 1) * 8, by0 = ty * TS + (wv >> 1) * 8;
    const int px = bx0 + (lane & 7), py = by0 + (lane >> 3);
    const bool valid = px < V.W && py < V.H;
    const float lx = (float)(lane & 7) - 3.5f, ly = (float)(lane >> 3) - 3.5f;
    const float amin = V.amin, amax = V.amax, tmin = V.tmin;
    const int cn = min(16, C - c0);
    float T = 1.0f, ws = 0.0f, acc[16];
#pragma unroll
    for (int c = 0; c < 16; c++) acc[c] = 0.0f;
    bool done = !valid;
    const uint32_t start = bstart[b], end = bend[b];
    for (uint32_t base = start; base < end; base += BATCH) {
        const int nb = (int)min((uint32_t)BATCH, end - base);
        if (t < nb) {
            const uint32_t p = ival[base + t];
            s_r0[t] = rec[2 * (size_t)p];
            s_r1[t] = rec[2 * (size_t)p + 1];
            const float* ar = attr + (size_t)pgauss[p] * C + c0;
            for (int c = 0; c < cn; c++) s_a[t][c] = ar[c];
        }
        __syncthreads();
        for (int j = 0; j < nb && !__all(done); j++) {
            const float4 q0 = s_r0[j], q1 = s_r1[j];
            const uint32_t ba = __float_as_uint(q1.z);
            const float A = q0.z, B = q0.w, Cq = q1.x, lo2 = q1.y;
            const float du = q0.x + (float)((int)(ba & 0xFFFFu) - bx0 - 4);
            const float dv = q0.y + (float)((int)(ba >> 16) - by0 - 4);
            const float cx = -fmaf(2.0f * A, du, B * dv);
            const float cy = -fmaf(B, du, 2.0f * Cq * dv);
            const float e0 = fmaf(A * du, du, fmaf(B * du, dv, Cq * dv * dv)) + lo2;
            const float tq = fmaf(B, ly, fmaf(A, lx, cx));
            const float tw = fmaf(Cq, ly, cy);
            const float e = fmaf(tw, ly, fmaf(tq, lx, e0));
            const float alpha = fminf(amax, __builtin_amdgcn_exp2f(e));
            const float Tn = fmaf(-alpha, T, T);
            const bool ok = !done && alpha >= amin;
            const bool stop = ok && Tn < tmin;
            const bool take = ok && !stop;
            const float w = take ? (KW ? __builtin_amdgcn_exp2f(e - lo2) : alpha * T) : 0.0f;
            ws += w;
#pragma unroll
            for (int c = 0; c < 16; c++)
                if (c < cn) acc[c] = fmaf(w, s_a[j][c], acc[c]);
            T = take ? Tn : T;
            done = done || stop;
        }
        if (__syncthreads_count(!done) == 0) break;
    }
    if (valid) {
        const size_t pi = (size_t)py * V.W + px;
        const float inv = ws > 0.0f ? 1.0f / ws : 0.0f;
        for (int c = 0; c < cn; c++) out[pi * C + c0 + c] = acc[c] * inv;
        if (wsum_out && c0 == 0) wsum_out[pi] = ws;
    }
}

// Part-list records: pinfo[p] = (base, 0) from the scanned capacities, and
// the sentinel pinfo[npairs] = (total, 0), so a list's capacity is the next
// record's base minus its own.
__global__ __launch_bounds__(256) void k_init_pinfo(uint64_t npairs, const uint32_t* __restrict__ base,
                                                    uint32_t total, uint2* __restrict__ pinfo)
{
    const uint64_t p = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (p < npairs) pinfo[p] = make_uint2(base[p], 0u);
    else if (p == npairs) pinfo[p] = make_uint2(total, 0u);
}

// Debug export and training rows: one thread per pair copies its part list
// (pinfo[p] = (base, filled length)) as (global segment row, weight), to
// wrow at the list's base.
__global__ __launch_bounds__(256) void k_merge(uint64_t npairs, const uint16_t* __restrict__ pview,
                                               const ViewDev* __restrict__ views,
                                               const uint2* __restrict__ pinfo,
                                               const uint2* __restrict__ part,
                                               uint2* __restrict__ wrow,
                                               uint32_t* __restrict__ wlen,
                                               unsigned long long* __restrict__ nnz)
{
    const uint64_t p = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    uint32_t n = 0;
    if (p < npairs) {
        const ViewDev& V = views[pview[p]];
        const uint32_t base = pinfo[p].x, cnt = pinfo[p].y;
        for (uint32_t k = 0; k < cnt; k++) {
            const uint2 e = part[base + k];
            if (__uint_as_float(e.y) > 0.0f)
                wrow[base + n++] = make_uint2(V.seg_off + (e.x & 0xFFFFu), e.y);
        }
        wlen[p] = n;
    }
    unsigned long long c = n;
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(nnz, c);
}

}  // namespace

void launch_render(bool kernel_w, int ts, int ntiles, const ViewDev* views, int vi,
                   const uint32_t* bstart, const uint32_t* bend, const uint32_t* ival,
                   const float4* rec, const uint32_t* pgauss, const float* attr, int C, float* out,
                   float* wsum, hipStream_t st)
{
    if (ntiles <= 0) return;
#define SLAG_RENDER(K, T)                                                                         \
    hipLaunchKernelGGL((k_render<K, T>), dim3((unsigned)ntiles), dim3(T * T), 0, st, views, vi,   \
                       bstart, bend, ival, rec, pgauss, attr, C, c0, out, wsum)
    for (int c0 = 0; c0 < C; c0 += 16) {
        if (ts == 8) {
            if (kernel_w) SLAG_RENDER(true, 8); else SLAG_RENDER(false, 8);
        } else {
            if (kernel_w) SLAG_RENDER(true, 16); else SLAG_RENDER(false, 16);
        }
    }
#undef SLAG_RENDER
}

void launch_tile_segs(int ts, uint32_t nbuckets, const uint32_t* bucket_view, const ViewDev* views,
                      const int32_t* ids, int lpp, uint32_t* ns_tile, uint16_t* segl,
                      unsigned long long* err, hipStream_t st)
{
    if (!nbuckets) return;
    const dim3 grid((nbuckets + 3) / 4);
#define SLAG_SEGS(L, T)                                                                           \
    hipLaunchKernelGGL((k_tile_segs<L, T>), grid, dim3(256), 0, st, nbuckets, bucket_view, views, \
                       ids, lpp, ns_tile, segl, err)
    if (ts == 8) {
        if (lpp <= 1) SLAG_SEGS(1, 8); else SLAG_SEGS(MAX_LABELS, 8);
    } else {
        if (lpp <= 1) SLAG_SEGS(1, 16); else SLAG_SEGS(MAX_LABELS, 16);
    }
#undef SLAG_SEGS
}

void launch_sat(int nb, const ViewDev* views, const uint32_t* ns_tile, uint32_t* sat,
                hipStream_t st)
{
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_sat, dim3(nb), dim3(256), 0, st, views, ns_tile, sat);
}

int composite_variants() { return 7; }

const char* composite_variant_name(int v)
{
    static const char* names[7] = {"occupancy 8, padded groups", "occupancy 6, padded groups",
                                   "occupancy 5, padded groups", "occupancy 8, cut groups",
                                   "occupancy 8, cut groups, persistent queue",
                                   "occupancy 8, padded groups, persistent queue",
                                   "occupancy 8, cut groups, batches of 32"};
    return (v >= 0 && v < 7) ? names[v] : "";
}

template <int TS>
static void composite_ts(bool count, int variant, uint32_t grid, uint32_t nbuckets,
                         const uint32_t* order, uint32_t obase, const uint32_t* bucket_view,
                         const ViewDev* views, const uint32_t* bstart, const uint32_t* bend,
                         const uint32_t* ival, uint2* pinfo, const float4* rec,
                         const uint32_t* ns_tile, const uint16_t* segl, const int32_t* ids, int lpp,
                         bool kernel_w, uint2* part, unsigned long long* counters, float* pix_t,
                         float* pix_w, uint32_t* pix_n, uint32_t* queue, hipStream_t st)
{
#define SLAG_COMP(C, W, P, LM, K, Q, BT)                                                           \
    hipLaunchKernelGGL((k_composite<C, W, P, LM, K, Q, BT, TS>), dim3(grid), dim3(TS * TS), 0, st, \
                       order, obase, nbuckets, queue, bucket_view, views, bstart, bend, ival,      \
                       pinfo, rec, ns_tile, segl, ids, lpp, part, counters, pix_t, pix_w, pix_n)
#define SLAG_COMP_V(LM)                                                                            \
    do {                                                                                           \
        if (count) {                                                                               \
            SLAG_COMP(true, 8, false, LM, false, false, 64);                                       \
            break;                                                                                 \
        }                                                                                          \
        switch (variant) {                                                                         \
        case 1: SLAG_COMP(false, 6, true, LM, false, false, 64); break;                            \
        case 2: SLAG_COMP(false, 5, true, LM, false, false, 64); break;                            \
        case 3: SLAG_COMP(false, 8, false, LM, false, false, 64); break;                           \
        case 4: SLAG_COMP(false, 8, false, LM, false, true, 64); break;                            \
        case 5: SLAG_COMP(false, 8, true, LM, false, true, 64); break;                             \
        case 6: SLAG_COMP(false, 8, false, LM, false, false, 32); break;                           \
        default: SLAG_COMP(false, 8, true, LM, false, false, 64); break;                           \
        }                                                                                          \
    } while (0)
    if (kernel_w) {
        // kernel weights: the occupancy-8, cut-groups shape only (no tuning)
        if (count) {
            if (lpp <= 1) SLAG_COMP(true, 8, false, 1, true, false, 64);
            else SLAG_COMP(true, 8, false, MAX_LABELS, true, false, 64);
        } else {
            if (lpp <= 1) SLAG_COMP(false, 8, false, 1, true, false, 64);
            else SLAG_COMP(false, 8, false, MAX_LABELS, true, false, 64);
        }
    } else if (lpp <= 1) {
        SLAG_COMP_V(1);
    } else {
        SLAG_COMP_V(MAX_LABELS);
    }
#undef SLAG_COMP_V
#undef SLAG_COMP
}

void launch_composite(bool count, int variant, int ts, uint32_t nbuckets, const uint32_t* order,
                      uint32_t obase, const uint32_t* bucket_view, const ViewDev* views,
                      const uint32_t* bstart, const uint32_t* bend, const uint32_t* ival,
                      uint2* pinfo, const float4* rec, const uint32_t* ns_tile,
                      const uint16_t* segl, const int32_t* ids, int lpp, bool kernel_w,
                      uint2* part, unsigned long long* counters, float* pix_t, float* pix_w,
                      uint32_t* pix_n, uint32_t* queue, uint32_t pgrid, hipStream_t st)
{
    if (!nbuckets) return;
    const bool persist = !count && !kernel_w && (variant == 4 || variant == 5);
    uint32_t grid = nbuckets;
    if (persist) {
        // pgrid: eight 4-wave workgroups per CU; 8 x 8 tiles are 1-wave workgroups
        launch_fill_u32(queue, 1, 0u, st);
        grid = std::min(nbuckets, std::max(pgrid * (ts == 8 ? 4u : 1u), 1u));
    }
    if (ts == 8)
        composite_ts<8>(count, variant, grid, nbuckets, order, obase, bucket_view, views, bstart,
                        bend, ival, pinfo, rec, ns_tile, segl, ids, lpp, kernel_w, part, counters,
                        pix_t, pix_w, pix_n, queue, st);
    else
        composite_ts<16>(count, variant, grid, nbuckets, order, obase, bucket_view, views, bstart,
                         bend, ival, pinfo, rec, ns_tile, segl, ids, lpp, kernel_w, part, counters,
                         pix_t, pix_w, pix_n, queue, st);
}

void launch_init_pinfo(uint64_t npairs, const uint32_t* base, uint32_t total, uint2* pinfo,
                       hipStream_t st)
{
    if (!npairs) return;
    hipLaunchKernelGGL(k_init_pinfo, dim3((unsigned)((npairs + 256) / 256)), dim3(256), 0, st,
                       npairs, base, total, pinfo);
}

void launch_merge(uint64_t npairs, const uint16_t* pview, const ViewDev* views, const uint2* pinfo,
                  const uint2* part, uint2* wrow, uint32_t* wlen, unsigned long long* nnz,
                  hipStream_t st)
{
    if (!npairs) return;
    hipLaunchKernelGGL(k_merge, dim3((unsigned)((npairs + 255) / 256)), dim3(256), 0, st, npairs,
                       pview, views, pinfo, part, wrow, wlen, nnz);
}

}  // namespace slag
