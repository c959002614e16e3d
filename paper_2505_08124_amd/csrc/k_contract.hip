// Aggregation (paper, Method: E_k = sum_i sum_j sum_{p in M_j} w_kp E_j /
// sum_i sum_j sum_{p in M_j} w_kp) on the matrix cores.
//
// num = W F is a sparse-times-dense product: each Gaussian touches about one
// segment per view, out of ~10^2 per view.  Gaussians are taken in blocks of
// G = 16 RT consecutive along a Morton curve of their means, so the rows of a
// block tend to see the same segments.  A workgroup (4 waves) owns one block;
// the block walks its pairs VPT 256 / G views per step, VPT (row, view) pairs
// per thread, reading each pair's part list of (segment, weight) entries
// (appended by the compositing in arbitrary order; the sums below are exact
// fixed-point sums, so the order does not matter); the segments the
// rows touch are deduplicated per view with LDS bitmaps over view-local ids,
// numbered in (view, id) order by a block scan, and the weights are summed
// into a shared fixed-point A[G x K].  K-chunks of 32 columns then go to the matrix
// cores: each wave loads the feature rows B[32 x 16] of its column tiles
// once and multiplies them with all RT row tiles of A (RT-fold reuse of every
// feature load, the scarce resource: the same segment rows are fetched again
// by every block that touches them):
//   BF16 features: v_mfma_f32_16x16x32_bf16, with A split exactly enough into
//                  hi + lo BF16 parts (two MFMAs, error ~2^-16 relative);
//   FP32 features: v_mfma_f32_16x16x4_f32, eight per chunk.
// Accumulation is FP32.  The weight sums (denominators) are FP32 sums in view
// order; every chunk is filled in a fixed order, so results are
// deterministic.
#include <algorithm>

#include "slag_internal.h"

namespace slag {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int KC = 32;          // K columns per chunk

constexpr int KMAX = 128;       // K columns staged per round of a step

// Weights are summed in 64-bit fixed point with 40 fraction bits: integer
// addition is exact, so the sums do not depend on the order in which the
// compositing appended a pair's entries (a (view, segment) sum is at most the
// segment's pixel count, < 2^23, well inside the range).
constexpr float kFx = 1099511627776.0f;          // 2^40
constexpr float kFxInv = 1.0f / 1099511627776.0f;
__device__ __forceinline__ int64_t to_fx(float w) { return (int64_t)(w * kFx); }
__device__ __forceinline__ float from_fx(int64_t x) { return (float)x * kFxInv; }
// Blocks per XCD chunk of the contraction's launch order (0: plain order):
// the fused kernel and the walk, and the chunk multiply.
constexpr int kXcdChunk = 16;
constexpr int kXcdChunkMul = 16;
constexpr int kContractRT = 1;  // row tiles per block (G = 16 Gaussians; 2 and 4 measured slower)

// G = 16 RT rows per block; thread t walks row t % G and views
// v0 + t / G + (256 / G) j, j < VPT: GV = VPT 256 / G views per step.
constexpr int VPT = 2;   // (a thread numbers the bitmap words 2 t, 2 t + 1: view slot t / 4)
static_assert(VPT == 2, "the walk reads one view offset per thread per step");
// Part-list entries of one step staged in LDS (a step with more reads them
// from global memory in both passes); SU loads per thread in flight.
constexpr int STAGE = 2048;
constexpr int SU = 4;
template <int RT>
struct BlockLds {
    static constexpr int G = 16 * RT, GT = 256 / G, GV = VPT * GT;
    uint32_t bits[GV * 8];      // word i: view i >> 3 of the step, ids w0 + 32 (i & 7) + [0, 32)
    uint32_t wbase[GV * 8];     // first step column of each word
    uint32_t ks[KMAX];          // feature row of each column of the round
    int64_t A[G][KMAX + 1];     // weights of the round's columns, fixed point
    float dpart[GV][G];         // per-view row weight sums of the step
    uint64_t dfx[GV][G];        //   the same, fixed point
    uint32_t scan[8];
    uint32_t chead, clast, cbase;   // chunk list of the block (walk-only launch)
    // the step's part-list entries, staged once (both passes read them);
    // the high half of .x (the entry's tile in its pair's rectangle, unused
    // here) is replaced by the entry's owner, view slot G + row
    uint2 stage[STAGE];
    uint32_t soff[256];         // first staged entry of each thread
    uint32_t spb[256][VPT];     // list base and length of each thread's pairs
    uint32_t scnt[256][VPT];
};

// Output column of lane m (of 16) in column tile i of a wave whose first
// column is c0.  BF16 features, NT = 12 or 16 (D = 768, 1024): lane m holds the
// four consecutive columns c0 + 64 (i / 4) + 4 m + (0 .. 3) of tiles
// 4 (i / 4) .. + 3, so that one 8-byte load of a feature row feeds four
// tiles; else tile i is columns c0 + 16 i + (0 .. 15).
template <int NT, bool BF16>
__device__ __forceinline__ int tile_col(int c0, int i, int m)
{
    if constexpr (BF16 && NT >= 12 && NT % 4 == 0) return c0 + 64 * (i >> 2) + 4 * m + (i & 3);
    else return c0 + 16 * i + m;
}

// One 32-column chunk on the matrix cores for D >= 768 BF16 features (one
// row tile): this lane's K rows k = 8 kq + j at byte offsets roff[j] (bit j
// of live: a real column; others are read as zero), weights split hi + lo.
// The feature loads go in batches of GF groups of four columns (8 rows x 8
// bytes per group, the last batch possibly short), each batch in flight at
// once; GF keeps a batch within the registers the occupancy leaves.
template <int NT, int GF>
__device__ __forceinline__ void wide_mfma(const char* __restrict__ Fb, const uint32_t (&roff)[8],
                                          uint32_t live, bf16x8 ahi, bf16x8 alo, floatx4* acc)
{
    constexpr int NG = NT / 4;
#pragma unroll
    for (int g0 = 0; g0 < NG; g0 += GF) {
        uint2 raw[8][GF];
#pragma unroll
        for (int j = 0; j < 8; j++)
#pragma unroll
            for (int gg = 0; gg < GF; gg++)
                raw[j][gg] = ((live >> j) & 1u) && g0 + gg < NG
                                 ? *reinterpret_cast<const uint2*>(Fb + (roff[j] + 128u * (uint32_t)(g0 + gg)))
                                 : make_uint2(0u, 0u);
#pragma unroll
        for (int gg = 0; gg < GF; gg++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                if (g0 + gg >= NG) continue;
                u32x4 w;
#pragma unroll
                for (int jj = 0; jj < 4; jj++) {
                    const uint32_t x0 = (e < 2) ? raw[2 * jj][gg].x : raw[2 * jj][gg].y;
                    const uint32_t x1 = (e < 2) ? raw[2 * jj + 1][gg].x : raw[2 * jj + 1][gg].y;
                    w[jj] = (e & 1) ? ((x0 >> 16) | (x1 & 0xFFFF0000u)) : ((x0 & 0xFFFFu) | (x1 << 16));
                }
                const bf16x8 b = __builtin_bit_cast(bf16x8, w);
                const int ti = 4 * (g0 + gg) + e;
                acc[ti] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, b, acc[ti], 0, 0, 0);
                acc[ti] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, b, acc[ti], 0, 0, 0);
            }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Multiply columns [k0, k0 + kn) of the staged round into the accumulators
// acc[r][t] (row tile r, column tile t).
template <int NT, bool BF16, int RT>
__device__ __forceinline__ void mfma_chunk(const BlockLds<RT>& L, int k0, int kn, const void* feats,
                                           int d, int c0, floatx4 (*acc)[NT], int lane)
{
    const int m = lane & 15, kq = lane >> 4;
    if constexpr (BF16 && NT >= 12 && NT % 4 == 0) {
        static_assert(RT == 1, "the wide-load path multiplies one row tile");
        bf16x8 ahi, alo;
        uint32_t roff[8];   // byte offset of this lane's four columns in each K row
        uint32_t live = 0;
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const int k = 8 * kq + j;
            live |= (k < kn ? 1u : 0u) << j;
            roff[j] = ((k < kn ? L.ks[k0 + k] : 0u) * (uint32_t)d + (uint32_t)(c0 + 4 * m)) * 2u;
            const float a = k < kn ? from_fx(L.A[m][k0 + k]) : 0.0f;
            const __bf16 h = (__bf16)a;
            ahi[j] = h;
            alo[j] = (__bf16)(a - (float)h);
        }
        wide_mfma<NT, NT == 12 ? 3 : 1>(reinterpret_cast<const char*>(feats), roff, live, ahi, alo, acc[0]);
    } else if constexpr (BF16) {
        bf16x8 ahi[RT], alo[RT];
        uint32_t roff[8];          // byte offset of this lane's column in each K row (row 0
        uint32_t live = 0;         // stands in for unused K slots; their values become zero)
        const char* Fb = reinterpret_cast<const char*>(feats);
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const int k = 8 * kq + j;
#pragma unroll
            for (int r = 0; r < RT; r++) {
                const float a = k < kn ? from_fx(L.A[16 * r + m][k0 + k]) : 0.0f;
                const __bf16 h = (__bf16)a;
                ahi[r][j] = h;
                alo[r][j] = (__bf16)(a - (float)h);
            }
            const uint32_t kr = k < kn ? L.ks[k0 + k] : 0u;
            live |= (k < kn ? 1u : 0u) << j;
            roff[j] = (kr * (uint32_t)d + (uint32_t)(c0 + m)) * 2u;
        }
#pragma unroll
        for (int t = 0; t < NT; t++) {
            bf16x8 b;
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const uint16_t v = *reinterpret_cast<const uint16_t*>(Fb + (roff[j] + 32u * (uint32_t)t));
                b[j] = __builtin_bit_cast(__bf16, ((live >> j) & 1u) ? v : (uint16_t)0);
            }
#pragma unroll
            for (int r = 0; r < RT; r++) {
                acc[r][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[r], b, acc[r][t], 0, 0, 0);
                acc[r][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[r], b, acc[r][t], 0, 0, 0);
            }
            // keep at most two tiles of feature loads in flight (register pressure)
            if (t & 1) __builtin_amdgcn_sched_barrier(0);
        }
    } else {
        const float* F = reinterpret_cast<const float*>(feats);
#pragma unroll
        for (int kk = 0; kk < KC / 4; kk++) {
            const int k = 4 * kk + kq;
            float a[RT];
#pragma unroll
            for (int r = 0; r < RT; r++) a[r] = k < kn ? from_fx(L.A[16 * r + m][k0 + k]) : 0.0f;
            const uint32_t krow = k < kn ? L.ks[k0 + k] : NONE;
#pragma unroll
            for (int t = 0; t < NT; t++) {
                const int col = c0 + 16 * t + m;
                const float b = krow != NONE ? F[(size_t)krow * d + col] : 0.0f;
#pragma unroll
                for (int r = 0; r < RT; r++)
                    acc[r][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r], b, acc[r][t], 0, 0, 0);
            }
        }
    }
}

// Exclusive scan of one value per thread over the 256-thread block.  The
// caller must pass a block barrier before scratch is written again (every
// caller does, right after the scan).
__device__ __forceinline__ uint32_t block_exscan(uint32_t x, uint32_t* scratch, uint32_t& total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t v = x;
#pragma unroll
    for (int dd = 1; dd < 64; dd <<= 1) {
        const uint32_t y = __shfl_up(v, dd, 64);
        if (lane >= dd) v += y;
    }
    if (lane == 63) scratch[w] = v;
    __syncthreads();
    uint32_t off = 0;
    for (int i = 0; i < w; i++) off += scratch[i];
    total = scratch[0] + scratch[1] + scratch[2] + scratch[3];
    return off + v - x;
}

// Three workgroups per CU while the accumulators fit beside the walk's
// registers (NT <= 8 column tiles per wave, D <= 512); wider rows take two,
// so that the 12 or 16 accumulator tiles of D = 768 or 1024 do not spill.
template <int NT>
constexpr int contract_min_blocks() { return NT <= 8 ? 3 : 2; }

// SPLIT: the walk alone (no accumulators, so three workgroups per CU at any
// D): each round's columns and weights go to a chunk list of the block and
// the rows' weight sums to co.rowden; k_contract_chunks multiplies them.
template <int NT, bool BF16, int RT, bool SPLIT>
__global__ __launch_bounds__(256, contract_min_blocks<SPLIT ? 1 : NT>()) void k_contract_mfma(
    int64_t n, int nb, int d, const uint32_t* __restrict__ perm,
    const uint32_t* __restrict__ pair_of_m, const ViewDev* __restrict__ views,
    const uint16_t* __restrict__ vlist, const uint32_t* __restrict__ vcnt,
    const uint2* __restrict__ pinfo,
    const uint2* __restrict__ part, const void* __restrict__ feats, float* __restrict__ num,
    float* __restrict__ den, int first, int last, int64_t q_begin, int64_t q_end, int local,
    const uint32_t* __restrict__ gorder, ChunkOut co)
{
    constexpr int G = BlockLds<RT>::G, GT = BlockLds<RT>::GT, GV = BlockLds<RT>::GV;
    __shared__ BlockLds<RT> L;
    const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
    // Morton ranks [q_begin, q_end) (q_begin a multiple of G); output row of
    // rank q: its caller index perm[q], or q - q_begin (local rows of a chunk)
    // Dispatch order: the Gaussian blocks (GBLOCK ranks) of the range,
    // heaviest first (gorder: by descending visible pair count), so the
    // blocks with the most views do not form the kernel's tail; inside one,
    // its GBLOCK / G workgroups in Morton order.  XCD-aware: workgroups are
    // dealt to the 8 XCDs round-robin; each group of 8 C workgroups gives
    // XCD x the C consecutive blocks x C .. x C + C - 1 of the group, so
    // neighbouring blocks (which touch the same segments) share one L2
    // (the grid is whole groups).
    constexpr int BPG = GBLOCK / G;
    int64_t lb = blockIdx.x;
    if (kXcdChunk > 0) {
        const int64_t gs = 8 * kXcdChunk, w = lb % gs;
        lb = lb - w + (w % 8) * kXcdChunk + w / 8;
    }
    const int64_t ng = (q_end + GBLOCK - 1) / GBLOCK - q_begin / GBLOCK;
    if (lb >= ng * BPG) return;
    const int64_t q0 = (int64_t)gorder[lb / BPG] * GBLOCK + (lb % BPG) * G;  // first Morton rank
    if (q0 < q_begin || q0 >= q_end) return;
    auto orow = [&](int64_t q) -> int64_t { return local ? q - q_begin : (int64_t)perm[q]; };
    const int c0 = wv * 16 * NT;                          // this wave's first feature column
    const bool wact = c0 < d;                             // (d < 64: waves past d only walk)
    const int m = lane & 15, kq = lane >> 4;
    const int row = t % G, vt = t / G;                    // walking role
    const bool row_ok = q0 + row < q_end;
    const int64_t qr = row_ok ? q0 + row : q0;

    floatx4 acc[RT][NT];
    float dsum = 0.0f;   // running weight sum of row t (threads t < G)
    if (SPLIT) {
        // the rows' sums so far: the earlier view launches' walks left them
        // in co.rowden_in (a walk run again reads the same)
        if (t == 0) { L.chead = NONE; L.clast = NONE; }
        if (!first && t < G) dsum = co.rowden_in[((q0 - q_begin) / G) * G + t];
    } else if (first) {
#pragma unroll
        for (int r = 0; r < RT; r++)
#pragma unroll
            for (int i = 0; i < NT; i++) acc[r][i] = floatx4{0.f, 0.f, 0.f, 0.f};
    } else {
        // clamped (always valid) loads, all in flight before the first is used
        int64_t gq[RT][4];
#pragma unroll
        for (int r = 0; r < RT; r++)
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int64_t q = q0 + 16 * r + 4 * kq + j;
                gq[r][j] = orow(q < q_end ? q : q_end - 1);
            }
#pragma unroll
        for (int r = 0; r < RT; r++)
#pragma unroll
            for (int i = 0; i < NT; i++)
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    const int64_t q = q0 + 16 * r + 4 * kq + j;
                    const float x = num[(size_t)gq[r][j] * d + (wact ? tile_col<NT, BF16>(c0, i, m) : 0)];
                    acc[r][i][j] = (wact && q < q_end) ? x : 0.0f;
                }
        if (t < G && q0 + t < q_end) dsum = den[orow(q0 + t)];
    }

    // only the views in which this block's Gaussian block has visible pairs
    // (ascending): slot i of the walk is view vl[i]
    const int64_t cb = q0 / GBLOCK;
    const uint16_t* vl = vlist + (size_t)cb * (size_t)nb;
    const int nvb = (int)vcnt[cb];
    auto pair_at = [&](int i) -> uint32_t {
        const int v = i < nvb ? (int)vl[i] : 0;            // clamped: always a valid address
        const uint32_t p = pair_of_m[(int64_t)v * n + qr];
        return (row_ok && i < nvb) ? p : NONE;
    };
    // Everything a step needs from global memory before its entries is
    // loaded one step ahead (the pairs two steps ahead): the pairs' (base,
    // fill) records, the views' segment counts and the segment offset of
    // the view whose bitmap words this thread numbers (slot t / 4)
    auto view_at = [&](int i) -> const ViewDev* { return &views[i < nvb ? (int)vl[i] : (int)vl[0]]; };
    uint32_t pc[VPT], pn[VPT], nsc[VPT], soc;
    uint2 pin[VPT];
#pragma unroll
    for (int j = 0; j < VPT; j++) pc[j] = pair_at(vt + GT * j);
#pragma unroll
    for (int j = 0; j < VPT; j++) {
        pin[j] = pc[j] != NONE ? pinfo[pc[j]] : make_uint2(0u, 0u);
        nsc[j] = vt + GT * j < nvb ? view_at(vt + GT * j)->nseg : 0u;
        pn[j] = pair_at(GV + vt + GT * j);
    }
    soc = (t >> 2) < nvb ? view_at(t >> 2)->seg_off : 0u;

    for (int i = t; i < GV * 8; i += 256) L.bits[i] = 0;
    for (int v0 = 0; v0 < nvb; v0 += GV) {
        // this step's pairs (slot v0 + vt + GT j)
        uint32_t pb[VPT], cnt[VPT], nsv = 0;
        bool any = false;
        const uint32_t so_step = soc;
#pragma unroll
        for (int j = 0; j < VPT; j++) {
            const uint32_t p = pc[j];
            const uint2 pi = pin[j];
            any = any || p != NONE;
            pb[j] = p != NONE ? pi.x : 0u;
            cnt[j] = p != NONE ? pi.y : 0u;
            nsv = max(nsv, nsc[j]);
            // the next step's
            const int in = v0 + GV + vt + GT * j;
            pc[j] = pn[j];
            pin[j] = pn[j] != NONE ? pinfo[pn[j]] : make_uint2(0u, 0u);
            nsc[j] = in < nvb ? view_at(in)->nseg : 0u;
            pn[j] = pair_at(v0 + 2 * GV + vt + GT * j);
        }
        {
            const int in = v0 + GV + (t >> 2);
            soc = in < nvb ? view_at(in)->seg_off : 0u;
        }
        if (!__syncthreads_or(any)) continue;
        // stage the step's entries: thread t's lists go to [soff[t], ...) in
        // pair order; all threads load, SU clamped (always valid) loads each
        // in flight, the owner of entry i found by binary search over soff
        bool staged;
        uint32_t tot_st = 0;   // entries staged (block-uniform)
        {
            uint32_t ct = 0;
#pragma unroll
            for (int j = 0; j < VPT; j++) {
                ct += cnt[j];
                L.spb[t][j] = pb[j];
                L.scnt[t][j] = cnt[j];
            }
            uint32_t tot;
            const uint32_t off = block_exscan(ct, L.scan, tot);
            L.soff[t] = off;
            staged = tot <= (uint32_t)STAGE;
            tot_st = staged ? tot : 0u;
            __syncthreads();
            if (staged && tot) {
                for (uint32_t i0 = 0; i0 < tot; i0 += 256 * SU) {
                    uint2 xv[SU];
                    uint16_t ow[SU];
#pragma unroll
                    for (int u = 0; u < SU; u++) {
                        const uint32_t i = min(i0 + (uint32_t)(u * 256 + t), tot - 1u);
                        int lo = 0, hi = 255;
                        while (lo < hi) {
                            const int mid = (lo + hi + 1) >> 1;
                            if (L.soff[mid] <= i) lo = mid; else hi = mid - 1;
                        }
                        uint32_t k = i - L.soff[lo];
                        int jj = 0;
#pragma unroll
                        for (int j = 0; j + 1 < VPT; j++)
                            if (jj == j && k >= L.scnt[lo][j]) { k -= L.scnt[lo][j]; jj = j + 1; }
                        xv[u] = part[L.spb[lo][jj] + k];
                        ow[u] = (uint16_t)((lo / G + GT * jj) * G + lo % G);
                    }
#pragma unroll
                    for (int u = 0; u < SU; u++) {
                        const uint32_t i = i0 + (uint32_t)(u * 256 + t);
                        if (i < tot) {
                            L.stage[i] = make_uint2((xv[u].x & 0xFFFFu) | ((uint32_t)ow[u] << 16), xv[u].y);
                        }
                    }
                }
                __syncthreads();
            }
        }
        // bitmap words: word i covers view v0 + (i >> 3), ids w0 + 32 (i & 7) + [0, 32).
        // Staged steps are walked entry by entry (every thread the same
        // count; same-slot sums by integer LDS atomics, exact in any order),
        // others list by list.
        for (int i = t; i < GV * G; i += 256) (&L.dfx[0][0])[i] = 0ull;
        for (uint32_t w0 = 0; __syncthreads_or(w0 < nsv); w0 += 256) {
            // (the bitmaps are zero here: cleared before the walk and after
            // each window's last reader)
            // 1. mark the segments the rows touch, and add the weights into
            //    the per-view row sums
            if (staged) {
                for (uint32_t i = t; i < tot_st; i += 256) {
                    const uint2 x = L.stage[i];
                    const uint32_t s = (x.x & 0xFFFFu) - w0;
                    const float w = __uint_as_float(x.y);
                    if (s < 256u && w > 0.0f) {
                        const uint32_t ow = x.x >> 16, sl = ow / G;
                        atomicOr(&L.bits[sl * 8 + (s >> 5)], 1u << (s & 31));
                        atomicAdd(&L.dfx[sl][ow % G], (unsigned long long)to_fx(w));
                    }
                }
            } else {
#pragma unroll
                for (int j = 0; j < VPT; j++) {
                    const int vw = (vt + GT * j) * 8;
                    for (uint32_t k = 0; k < cnt[j]; k++) {
                        const uint2 x = part[pb[j] + k];
                        const uint32_t s = (x.x & 0xFFFFu) - w0;
                        const float w = __uint_as_float(x.y);
                        if (s < 256u && w > 0.0f) {
                            atomicOr(&L.bits[vw + (s >> 5)], 1u << (s & 31));
                            atomicAdd(&L.dfx[vt + GT * j][row], (unsigned long long)to_fx(w));
                        }
                    }
                }
            }
            __syncthreads();
            // 2. columns: marked segments in (view, id) order; thread t owns
            //    words VPT t .. VPT t + VPT - 1
            uint32_t wb[VPT], npop = 0;
#pragma unroll
            for (int j = 0; j < VPT; j++) {
                const int i = VPT * t + j;
                wb[j] = i < GV * 8 ? L.bits[i] : 0u;
                npop += (uint32_t)__popc(wb[j]);
            }
            uint32_t ktot;
            uint32_t base = block_exscan(npop, L.scan, ktot);
#pragma unroll
            for (int j = 0; j < VPT; j++) {
                const int i = VPT * t + j;
                if (i < GV * 8) L.wbase[i] = base;
                base += (uint32_t)__popc(wb[j]);
            }
            __syncthreads();
            for (uint32_t kr = 0; kr < ktot; kr += KMAX) {
                // feature rows of this round's columns
#pragma unroll
                for (int j = 0; j < VPT; j++) {
                    const int i = VPT * t + j;
                    uint32_t bb = wb[j];
                    if (!bb) continue;
                    const uint32_t so = so_step;   // view slot i >> 3 = t >> 2
                    uint32_t c = L.wbase[i];
                    while (bb) {
                        const uint32_t bit = (uint32_t)(__ffs((int)bb) - 1);
                        if (c >= kr && c < kr + KMAX)
                            L.ks[c - kr] = so + w0 + 32u * (uint32_t)(i & 7) + bit;
                        bb &= bb - 1u;
                        c++;
                    }
                }
                for (int i = t; i < G * (KMAX + 1); i += 256) (&L.A[0][0])[i] = 0;
                __syncthreads();
                // 3. weights into A (entry by entry with integer atomics, or
                //    each thread its own pairs' lists, which no other
                //    thread's entries share a (row, column) with)
                if (staged) {
                    for (uint32_t i = t; i < tot_st; i += 256) {
                        const uint2 x = L.stage[i];
                        const uint32_t s = (x.x & 0xFFFFu) - w0;
                        const float w = __uint_as_float(x.y);
                        if (s >= 256u || !(w > 0.0f)) continue;
                        const uint32_t ow = x.x >> 16;
                        const int wi = (int)(ow / G) * 8 + (int)(s >> 5);
                        const uint32_t bit = 1u << (s & 31);
                        const uint32_t col = L.wbase[wi] + (uint32_t)__popc(L.bits[wi] & (bit - 1u));
                        if (col >= kr && col < kr + KMAX)
                            atomicAdd(reinterpret_cast<unsigned long long*>(&L.A[ow % G][col - kr]),
                                      (unsigned long long)to_fx(w));
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < VPT; j++) {
                        const int vw = (vt + GT * j) * 8;
                        for (uint32_t k = 0; k < cnt[j]; k++) {
                            const uint2 x = part[pb[j] + k];
                            const uint32_t s = (x.x & 0xFFFFu) - w0;
                            const float w = __uint_as_float(x.y);
                            if (s >= 256u || !(w > 0.0f)) continue;
                            const int wi = vw + (int)(s >> 5);
                            const uint32_t bit = 1u << (s & 31);
                            const uint32_t col = L.wbase[wi] + (uint32_t)__popc(L.bits[wi] & (bit - 1u));
                            if (col >= kr && col < kr + KMAX) L.A[row][col - kr] += to_fx(w);
                        }
                    }
                }
                __syncthreads();
                const int kc = (int)min((uint32_t)KMAX, ktot - kr);
                if constexpr (SPLIT) {
                    // 4. the round's columns, 32 to a chunk (feature row, or
                    //    NONE past kc; the 16 rows' weights), appended to the
                    //    block's chunk list; nothing is written past co.cap
                    //    (the counter still counts: the host then re-runs)
                    const int nchk = (kc + KC - 1) / KC;
                    if (t == 0) L.cbase = atomicAdd(co.counter, (uint32_t)nchk);
                    __syncthreads();
                    const uint32_t cb0 = L.cbase;
                    if ((uint64_t)cb0 + (uint64_t)nchk <= (uint64_t)co.cap) {
                        for (int i = t; i < nchk * KC; i += 256)
                            co.cks[(size_t)cb0 * KC + i] = i < kc ? L.ks[i] : NONE;
                        for (int i = t; i < nchk * KC * G; i += 256) {
                            const int c = i / (KC * G), r = (i / KC) % G, k = i % KC, col = c * KC + k;
                            co.cA[((size_t)cb0 + c) * (KC * G) + r * KC + k] =
                                col < kc ? from_fx(L.A[r][col]) : 0.0f;
                        }
                        if (t == 0) {
                            for (int c = 0; c < nchk; c++)
                                co.cnext[cb0 + c] = c + 1 < nchk ? cb0 + c + 1 : NONE;
                            if (L.clast != NONE) co.cnext[L.clast] = cb0;
                            else L.chead = cb0;
                            L.clast = cb0 + (uint32_t)nchk - 1u;
                        }
                    }
                } else {
                    // 4. matrix cores, 32 columns at a time
                    if (wact)
                        for (int k0 = 0; k0 < kc; k0 += KC)
                            mfma_chunk<NT, BF16, RT>(L, k0, min(KC, kc - k0), feats, d, c0, acc, lane);
                }
                __syncthreads();
            }
            // the bitmaps' last reader is behind a barrier: clear them for the
            // next window or step
            for (int i = t; i < GV * 8; i += 256) L.bits[i] = 0;
        }
        // row weight sums, views in order
        for (int i = t; i < GV * G; i += 256)
            (&L.dpart[0][0])[i] = from_fx((int64_t)(&L.dfx[0][0])[i]);
        __syncthreads();
        if (t < G) {
            const int nv = min(GV, nvb - v0);
            for (int i = 0; i < nv; i++) dsum += L.dpart[i][t];
        }
    }
    if constexpr (SPLIT) {
        const int64_t bl = (q0 - q_begin) / G;   // the block's index in the range
        if (t < G) co.rowden[bl * G + t] = dsum;
        if (t == 0) co.head[bl] = L.chead;
        return;
    }
    __syncthreads();
    float* drow = &L.dpart[0][0];
    if (t < G) drow[t] = dsum;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RT; r++)
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int rr = 16 * r + 4 * kq + j;
            const int64_t q = q0 + rr;
            if (q >= q_end || !wact) continue;
            const int64_t g = orow(q);
            const float dn = drow[rr];
#pragma unroll
            for (int i = 0; i < NT; i++) {
                const float a = acc[r][i][j];
                num[(size_t)g * d + tile_col<NT, BF16>(c0, i, m)] = last ? (dn > 0.0f ? a / dn : 0.0f) : a;
            }
        }
    if (t < G && q0 + t < q_end) den[orow(q0 + t)] = dsum;
}

template <int NT, int RT>
void launch_nt(int64_t n, int nb, int d, bool bf16, const uint32_t* perm, const uint32_t* pair_of_m,
               const ViewDev* views, const uint16_t* vlist, const uint32_t* vcnt, const uint2* pinfo,
               const uint2* part, const void* feats, float* num, float* den, bool first, bool last,
               int64_t q_begin, int64_t q_end, bool local, const uint32_t* gorder, hipStream_t st)
{
    constexpr int G = 16 * RT;
    static_assert(GBLOCK % G == 0, "contraction blocks lie inside one Gaussian block");
    const int64_t gs = kXcdChunk > 0 ? 8 * kXcdChunk : 1;
    const int64_t ng = (q_end + GBLOCK - 1) / GBLOCK - q_begin / GBLOCK;   // Gaussian blocks met
    const dim3 grid((unsigned)((ng * (GBLOCK / G) + gs - 1) / gs * gs));
    const ChunkOut none{};
    if (bf16)
        hipLaunchKernelGGL((k_contract_mfma<NT, true, RT, false>), grid, dim3(256), 0, st, n, nb, d,
                           perm, pair_of_m, views, vlist, vcnt, pinfo, part, feats, num, den,
                           (int)first, (int)last, q_begin, q_end, (int)local, gorder, none);
    else
        hipLaunchKernelGGL((k_contract_mfma<NT, false, RT, false>), grid, dim3(256), 0, st, n, nb, d,
                           perm, pair_of_m, views, vlist, vcnt, pinfo, part, feats, num, den,
                           (int)first, (int)last, q_begin, q_end, (int)local, gorder, none);
}

// Grid of a contraction launch over [q_begin, q_end): the Gaussian blocks met,
// GBLOCK / 16 workgroups each, in whole XCD groups.
dim3 contract_grid(int64_t q_begin, int64_t q_end, int chunk = kXcdChunk)
{
    const int64_t gs = chunk > 0 ? 8 * chunk : 1;
    const int64_t ng = (q_end + GBLOCK - 1) / GBLOCK - q_begin / GBLOCK;
    return dim3((unsigned)((ng * (GBLOCK / 16) + gs - 1) / gs * gs));
}

// The chunk multiply, once per lift: one workgroup per block of 16
// Gaussians (the walk's dispatch order), four independent waves of NT column
// tiles; each follows the block's chunk lists of every view launch in order
// (nlists lists of nblocks heads) and multiplies every chunk with the same
// operations as the fused kernel (FP32 accumulation in the same order, so
// the results equal a fused contraction per launch carried over in num),
// then writes E and den.
template <int NT>
__global__ __launch_bounds__(256, 3) void k_contract_chunks(
    int64_t n, int d, const uint32_t* __restrict__ perm, const uint32_t* __restrict__ head,
    int nlists, const uint32_t* __restrict__ cnext, const uint32_t* __restrict__ cks,
    const float* __restrict__ cA, const float* __restrict__ rowden, const void* __restrict__ feats,
    float* __restrict__ num, float* __restrict__ den, int64_t q_begin, int64_t q_end, int local,
    const uint32_t* __restrict__ gorder)
{
    constexpr int G = 16, BPG = GBLOCK / G;
    int64_t lb = blockIdx.x;
    if (kXcdChunkMul > 0) {
        const int64_t gs = 8 * kXcdChunkMul, w = lb % gs;
        lb = lb - w + (w % 8) * kXcdChunkMul + w / 8;
    }
    const int64_t ng = (q_end + GBLOCK - 1) / GBLOCK - q_begin / GBLOCK;
    if (lb >= ng * BPG) return;
    const int64_t q0 = (int64_t)gorder[lb / BPG] * GBLOCK + (lb % BPG) * G;
    if (q0 < q_begin || q0 >= q_end) return;
    const int64_t bl = (q0 - q_begin) / G;
    auto orow = [&](int64_t q) -> int64_t { return local ? q - q_begin : (int64_t)perm[q]; };
    const int t = threadIdx.x, wv = t >> 6, lane = t & 63, m = lane & 15, kq = lane >> 4;
    const int c0 = wv * 16 * NT;   // d = 64 NT: every wave has columns
    const int64_t nblocks = (q_end - q_begin + G - 1) / G;
    floatx4 acc[NT];
#pragma unroll
    for (int i = 0; i < NT; i++) acc[i] = floatx4{0.f, 0.f, 0.f, 0.f};
    const char* Fb = reinterpret_cast<const char*>(feats);
    for (int li = 0; li < nlists; li++)
    for (uint32_t ch = head[(int64_t)li * nblocks + bl]; ch != NONE;) {
        const uint32_t nx = cnext[ch];
        const float* ap = cA + (size_t)ch * (KC * G) + m * KC + 8 * kq;
        const uint32_t* kp = cks + (size_t)ch * KC + 8 * kq;
        bf16x8 ahi, alo;
        uint32_t roff[8], live = 0;
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const uint32_t kr = kp[j];
            live |= (kr != NONE ? 1u : 0u) << j;
            roff[j] = ((kr != NONE ? kr : 0u) * (uint32_t)d + (uint32_t)(c0 + 4 * m)) * 2u;
            const float a = ap[j];
            const __bf16 h = (__bf16)a;
            ahi[j] = h;
            alo[j] = (__bf16)(a - (float)h);
        }
        wide_mfma<NT, NT == 12 ? 2 : 1>(Fb, roff, live, ahi, alo, acc);
        ch = nx;
    }
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int rr = 4 * kq + j;
        const int64_t q = q0 + rr;
        if (q >= q_end) continue;
        const int64_t g = orow(q);
        const float dn = rowden[bl * G + rr];
#pragma unroll
        for (int i = 0; i < NT; i++) {
            const float a = acc[i][j];
            num[(size_t)g * d + tile_col<NT, true>(c0, i, m)] = dn > 0.0f ? a / dn : 0.0f;
        }
    }
    if (t < G && q0 + t < q_end) den[orow(q0 + t)] = rowden[bl * G + t];
}

// Views in which each Gaussian block has visible pairs, ascending:
// vlist[blk nb + i], i < vcnt[blk]; blk_off = exclusive scan of the visible
// pair counts per (view, block), nb nblk + 1 entries.  Also the dispatch key
// of the block for the contraction over Gaussian blocks [gb0, gb1): blocks
// in range by descending pair count (the block's work), the rest after them
// (wkey = 2^27 - 1 - pairs, or 2^27), with gidx = the block.
__global__ __launch_bounds__(256) void k_view_lists(int nb, int nblk, const uint32_t* __restrict__ blk_off,
                                                    uint16_t* __restrict__ vlist,
                                                    uint32_t* __restrict__ vcnt, int64_t gb0,
                                                    int64_t gb1, uint32_t* __restrict__ wkey,
                                                    uint32_t* __restrict__ gidx)
{
    __shared__ uint32_t wc[4], wp[4];
    const int blk = blockIdx.x, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t base = 0, pairs = 0;
    for (int v0 = 0; v0 < nb; v0 += 256) {
        const int v = v0 + (int)threadIdx.x;
        uint32_t np = 0;
        if (v < nb) {
            const int64_t bi = (int64_t)v * nblk + blk;
            np = blk_off[bi + 1] - blk_off[bi];
        }
        const bool vis = np != 0;
        const uint64_t m = __ballot(vis);
        uint32_t ps = np;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) ps += __shfl_xor(ps, o, 64);
        if (lane == 0) { wc[wv] = (uint32_t)__popcll(m); wp[wv] = ps; }
        __syncthreads();
        uint32_t off = 0;
        for (int w = 0; w < wv; w++) off += wc[w];
        const uint32_t tot = wc[0] + wc[1] + wc[2] + wc[3];
        pairs += wp[0] + wp[1] + wp[2] + wp[3];
        if (vis) vlist[(size_t)blk * nb + base + off + (uint32_t)__popcll(m & lt)] = (uint16_t)v;
        base += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        vcnt[blk] = base;
        if (wkey) {
            const bool in = blk >= gb0 && blk < gb1;
            wkey[blk] = in ? (1u << 27) - 1u - min(pairs, (1u << 27) - 1u) : (1u << 27);
            gidx[blk] = (uint32_t)blk;
        }
    }
}

__global__ __launch_bounds__(256) void k_f32_to_bf16(uint64_t n, const float* __restrict__ in,
                                                     uint16_t* __restrict__ out)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * 256) {
        const uint32_t b = __float_as_uint(in[i]);
        out[i] = (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
    }
}

}  // namespace

void launch_f32_to_bf16(uint64_t n, const float* in, uint16_t* out, hipStream_t st)
{
    if (!n) return;
    const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_f32_to_bf16, dim3((unsigned)blocks), dim3(256), 0, st, n, in, out);
}

bool contract_supported(int d)
{
    return d == 64 || d == 128 || d == 256 || d == 512 || d == 768 || d == 1024;
}

bool contract_supported_codes(int d) { return d == 16 || d == 32 || d == 48 || contract_supported(d); }

void launch_view_lists(int nb, int nblk, const uint32_t* blk_off, uint16_t* vlist, uint32_t* vcnt,
                       int64_t gb0, int64_t gb1, uint32_t* wkey, uint32_t* gidx, hipStream_t st)
{
    if (nb <= 0 || nblk <= 0) return;
    hipLaunchKernelGGL(k_view_lists, dim3((unsigned)nblk), dim3(256), 0, st, nb, nblk, blk_off, vlist,
                       vcnt, gb0, gb1, wkey, gidx);
}

void launch_contract(int64_t n, int nb, int d, bool bf16, const uint32_t* perm,
                     const uint32_t* pair_of_m, const ViewDev* views, const uint16_t* vlist,
                     const uint32_t* vcnt, const uint2* pinfo, const uint2* part, const void* feats,
                     float* num, float* den, bool first, bool last, int64_t q_begin, int64_t q_end,
                     bool local, const uint32_t* gorder, hipStream_t st)
{
    if (n <= 0 || q_end <= q_begin) return;
#define SLAG_NT(NTV) launch_nt<NTV, kContractRT>(n, nb, d, bf16, perm, pair_of_m, views, vlist, vcnt, \
                                    pinfo, part, feats, num, den, first, last, q_begin, q_end,     \
                                    local, gorder, st)
    switch (d) {
    case 16:
    case 32:
    case 48:
    case 64: SLAG_NT(1); break;
    case 128: SLAG_NT(2); break;
    case 256: SLAG_NT(4); break;
    case 512: SLAG_NT(8); break;
    case 768: SLAG_NT(12); break;
    case 1024: SLAG_NT(16); break;
    default: break;
    }
#undef SLAG_NT
}

bool contract_split(int d, bool bf16) { return bf16 && (d == 768 || d == 1024); }

void launch_contract_walk(int64_t n, int nb, int d, const uint32_t* perm, const uint32_t* pair_of_m,
                          const ViewDev* views, const uint16_t* vlist, const uint32_t* vcnt,
                          const uint2* pinfo, const uint2* part, const float* den, bool first,
                          int64_t q_begin, int64_t q_end, bool local, const uint32_t* gorder,
                          const ChunkOut& co, hipStream_t st)
{
    if (n <= 0 || q_end <= q_begin || !contract_split(d, true)) return;
    static_assert(kContractRT == 1, "the chunk multiply takes blocks of 16 Gaussians");
    const dim3 grid = contract_grid(q_begin, q_end);
    float* dn = const_cast<float*>(den);   // read only (when not first)
    if (d == 768)
        hipLaunchKernelGGL((k_contract_mfma<12, true, 1, true>), grid, dim3(256), 0, st, n, nb, d,
                           perm, pair_of_m, views, vlist, vcnt, pinfo, part, nullptr, nullptr, dn,
                           (int)first, 0, q_begin, q_end, (int)local, gorder, co);
    else
        hipLaunchKernelGGL((k_contract_mfma<16, true, 1, true>), grid, dim3(256), 0, st, n, nb, d,
                           perm, pair_of_m, views, vlist, vcnt, pinfo, part, nullptr, nullptr, dn,
                           (int)first, 0, q_begin, q_end, (int)local, gorder, co);
}

void launch_contract_chunks(int64_t n, int d, const uint32_t* perm, const ChunkOut& co, int nlists,
                            const void* feats, float* num, float* den, int64_t q_begin,
                            int64_t q_end, bool local, const uint32_t* gorder, hipStream_t st)
{
    if (n <= 0 || q_end <= q_begin || !contract_split(d, true)) return;
    const dim3 grid = contract_grid(q_begin, q_end, kXcdChunkMul);
    if (d == 768)
        hipLaunchKernelGGL(k_contract_chunks<12>, grid, dim3(256), 0, st, n, d, perm, co.head, nlists,
                           co.cnext, co.cks, co.cA, co.rowden, feats, num, den, q_begin, q_end,
                           (int)local, gorder);
    else
        hipLaunchKernelGGL(k_contract_chunks<16>, grid, dim3(256), 0, st, n, d, perm, co.head, nlists,
                           co.cnext, co.cks, co.cA, co.rowden, feats, num, den, q_begin, q_end,
                           (int)local, gorder);
}

}  // namespace slag
