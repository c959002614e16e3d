// Aggregation (paper, Method: E_k = sum_i sum_j sum_{p in M_j} w_kp E_j /
// sum_i sum_j sum_{p in M_j} w_kp) on the matrix cores.
//
// num = W F is a sparse-times-dense product: each Gaussian touches about one
// segment per view, out of ~10^2 per view.  Gaussians are taken in blocks of
// 16 consecutive along a Morton curve of their means, so the 16 rows of a
// block tend to see the same segments.  A workgroup (4 waves) owns one block;
// the block walks its pairs sixteen views per step, one (row, view) pair per
// thread reading the pair's packed (segment, weight) slots; the segments the
// rows touch are deduplicated per view with LDS bitmaps over view-local ids,
// numbered in (view, id) order by a block scan, and the weights are summed
// into a shared A[16 x K].  K-chunks of 32 columns then go to the matrix
// cores: A[16 x 32] holds the weights, B[32 x 16] the feature rows of those
// segments, and each wave multiplies for its quarter of the feature columns:
//   BF16 features: v_mfma_f32_16x16x32_bf16, with A split exactly enough into
//                  hi + lo BF16 parts (two MFMAs, error ~2^-16 relative);
//   FP32 features: v_mfma_f32_16x16x4_f32, eight per chunk.
// Accumulation is FP32.  The weight sums (denominators) are FP32 sums in a
// fixed order; every chunk is filled in a fixed order, so results are
// deterministic.
#include "slag_internal.h"

namespace slag {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int KC = 32;          // K columns per chunk

constexpr int GV = 16;          // views per step: thread t walks (row t & 15, view v0 + (t >> 4))
constexpr int KMAX = 128;       // K columns staged per round of a step

struct BlockLds {
    uint32_t bits[GV * 8];      // word i: view i >> 3 of the step, ids w0 + 32 (i & 7) + [0, 32)
    uint32_t wbase[GV * 8];     // first step column of each word
    uint32_t ks[KMAX];          // feature row of each column of the round
    float A[16][KMAX + 1];      // weights of the round's columns
    float dpart[GV][16];        // per-view row weight sums of the step
    uint32_t scan[8];
};

// Multiply columns [k0, k0 + kn) of the staged round into the accumulators.
template <int NT, bool BF16>
__device__ __forceinline__ void mfma_chunk(const BlockLds& L, int k0, int kn, const void* feats,
                                           int d, int c0, floatx4* acc, int lane)
{
    const int m = lane & 15, kq = lane >> 4;
    if constexpr (BF16) {
        bf16x8 ahi, alo;
        const uint16_t* rowp[8];   // this lane's column in each K row (row 0 stands in for
        uint32_t live = 0;         // unused K slots; their values are replaced by zero)
        const uint16_t* F = reinterpret_cast<const uint16_t*>(feats) + c0 + m;
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const int k = 8 * kq + j;
            const float a = k < kn ? L.A[m][k0 + k] : 0.0f;
            const __bf16 h = (__bf16)a;
            ahi[j] = h;
            alo[j] = (__bf16)(a - (float)h);
            const uint32_t kr = k < kn ? L.ks[k0 + k] : 0u;
            live |= (k < kn ? 1u : 0u) << j;
            rowp[j] = F + (size_t)kr * d;
        }
#pragma unroll
        for (int t = 0; t < NT; t++) {
            bf16x8 b;
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const uint16_t v = rowp[j][16 * t];
                b[j] = __builtin_bit_cast(__bf16, ((live >> j) & 1u) ? v : (uint16_t)0);
            }
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, b, acc[t], 0, 0, 0);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, b, acc[t], 0, 0, 0);
            // keep at most two tiles of feature loads in flight (register pressure)
            if (t & 1) __builtin_amdgcn_sched_barrier(0);
        }
    } else {
        const float* F = reinterpret_cast<const float*>(feats);
#pragma unroll
        for (int kk = 0; kk < KC / 4; kk++) {
            const int k = 4 * kk + kq;
            const float a = k < kn ? L.A[m][k0 + k] : 0.0f;
            const uint32_t krow = k < kn ? L.ks[k0 + k] : NONE;
#pragma unroll
            for (int t = 0; t < NT; t++) {
                const int col = c0 + 16 * t + m;
                const float b = krow != NONE ? F[(size_t)krow * d + col] : 0.0f;
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[t], 0, 0, 0);
            }
        }
    }
}

// Exclusive scan of one value per thread over the 256-thread block.
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
    __syncthreads();
    return off + v - x;
}

template <int NT, bool BF16>
__global__ __launch_bounds__(256) void k_contract_mfma(
    int64_t n, int nb, int d, const uint32_t* __restrict__ perm,
    const uint32_t* __restrict__ pair_of_m, const ViewDev* __restrict__ views,
    const uint32_t* __restrict__ part_base, const uint32_t* __restrict__ pcnt,
    const uint2* __restrict__ part, const void* __restrict__ feats, float* __restrict__ num,
    float* __restrict__ den, int first, int last)
{
    __shared__ BlockLds L;
    const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
    const int64_t q0 = (int64_t)blockIdx.x * 16;          // first Morton rank of the block
    const int c0 = wv * 16 * NT;                          // this wave's first feature column
    const bool wact = c0 < d;                             // (d < 64: waves past d only walk)
    const int m = lane & 15, kq = lane >> 4;
    const int row = t & 15, vi = t >> 4;                  // walking role
    const bool row_ok = q0 + row < n;
    const int64_t qr = row_ok ? q0 + row : q0;

    floatx4 acc[NT];
    float dsum = 0.0f;   // running weight sum of row t (threads t < 16)
    if (first) {
#pragma unroll
        for (int i = 0; i < NT; i++) acc[i] = floatx4{0.f, 0.f, 0.f, 0.f};
    } else {
#pragma unroll
        for (int i = 0; i < NT; i++)
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int64_t q = q0 + 4 * kq + j;
                acc[i][j] = (wact && q < n) ? num[(size_t)perm[q] * d + c0 + 16 * i + m] : 0.0f;
            }
        if (t < 16 && q0 + t < n) dsum = den[perm[q0 + t]];
    }

    auto pair_at = [&](int v) -> uint32_t {
        const int vc = v < nb ? v : nb - 1;                 // clamped: always a valid address
        const uint32_t p = pair_of_m[(int64_t)vc * n + qr];
        return (row_ok && v < nb) ? p : NONE;
    };
    uint32_t pn = pair_at(vi);

    for (int v0 = 0; v0 < nb; v0 += GV) {
        const uint32_t p = pn;
        pn = pair_at(v0 + GV + vi);                         // next step, in flight meanwhile
        if (!__syncthreads_or(p != NONE)) continue;
        const int v = v0 + vi;
        const uint32_t pb = p != NONE ? part_base[p] : 0u, cnt = p != NONE ? pcnt[p] : 0u;
        const uint32_t nsv = v < nb ? views[v].nseg : 0u;
        const int vw = v0 + (t >> 3);                       // view of bitmap word t (t < 128)
        const uint32_t so_w = (t < GV * 8 && vw < nb) ? views[vw].seg_off : 0u;
        float dv = 0.0f;
        for (uint32_t w0 = 0; __syncthreads_or(w0 < nsv); w0 += 256) {
            if (t < GV * 8) L.bits[t] = 0;
            __syncthreads();
            // 1. mark the segments the rows touch (slot order: dv does not
            //    depend on how columns are cut)
            auto mark = [&](const uint2 x) {
                const uint32_t s = x.x - w0;
                const float w = __uint_as_float(x.y);
                if (s < 256u && w > 0.0f) {
                    atomicOr(&L.bits[vi * 8 + (s >> 5)], 1u << (s & 31));
                    dv += w;
                }
            };
#pragma unroll 4
            for (uint32_t k = 0; k < cnt; k++) mark(part[pb + k]);
            __syncthreads();
            // 2. columns: marked segments in (view, id) order
            const uint32_t wb = t < GV * 8 ? L.bits[t] : 0u;
            uint32_t ktot;
            const uint32_t base = block_exscan((uint32_t)__popc(wb), L.scan, ktot);
            if (t < GV * 8) L.wbase[t] = base;
            for (uint32_t kr = 0; kr < ktot; kr += KMAX) {
                // feature rows of this round's columns
                if (wb) {
                    uint32_t c = base, bb = wb;
                    while (bb) {
                        const uint32_t bit = (uint32_t)(__ffs((int)bb) - 1);
                        if (c >= kr && c < kr + KMAX)
                            L.ks[c - kr] = so_w + w0 + 32u * (uint32_t)(t & 7) + bit;
                        bb &= bb - 1u;
                        c++;
                    }
                }
                for (int i = t; i < 16 * (KMAX + 1); i += 256) (&L.A[0][0])[i] = 0.0f;
                __syncthreads();
                // 3. weights: each thread adds its pair's slots into its row
                auto add = [&](const uint2 x) {
                    const uint32_t s = x.x - w0;
                    const float w = __uint_as_float(x.y);
                    if (s >= 256u || !(w > 0.0f)) return;
                    const int wi = vi * 8 + (int)(s >> 5);
                    const uint32_t bit = 1u << (s & 31);
                    const uint32_t col = L.wbase[wi] + (uint32_t)__popc(L.bits[wi] & (bit - 1u));
                    if (col >= kr && col < kr + KMAX) L.A[row][col - kr] += w;
                };
#pragma unroll 4
                for (uint32_t k = 0; k < cnt; k++) add(part[pb + k]);
                __syncthreads();
                // 4. matrix cores, 32 columns at a time
                const int kc = (int)min((uint32_t)KMAX, ktot - kr);
                if (wact)
                    for (int k0 = 0; k0 < kc; k0 += KC)
                        mfma_chunk<NT, BF16>(L, k0, min(KC, kc - k0), feats, d, c0, acc, lane);
                __syncthreads();
            }
        }
        // row weight sums, views in order
        L.dpart[vi][row] = dv;
        __syncthreads();
        if (t < 16) {
#pragma unroll
            for (int i = 0; i < GV; i++) dsum += L.dpart[i][t];
        }
    }
    __syncthreads();
    if (t < 16) L.dpart[0][t] = dsum;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int rr = 4 * kq + j;
        const int64_t q = q0 + rr;
        if (q >= n || !wact) continue;
        const uint32_t g = perm[q];
        const float dn = L.dpart[0][rr];
#pragma unroll
        for (int i = 0; i < NT; i++) {
            const float a = acc[i][j];
            num[(size_t)g * d + c0 + 16 * i + m] = last ? (dn > 0.0f ? a / dn : 0.0f) : a;
        }
    }
    if (t < 16 && q0 + t < n) den[perm[q0 + t]] = dsum;
}

template <int NT>
void launch_nt(int64_t n, int nb, int d, bool bf16, const uint32_t* perm, const uint32_t* pair_of_m,
               const ViewDev* views, const uint32_t* part_base, const uint32_t* pcnt,
               const uint2* part, const void* feats, float* num, float* den, bool first, bool last,
               hipStream_t st)
{
    const dim3 grid((unsigned)((n + 15) / 16));
    if (bf16)
        hipLaunchKernelGGL((k_contract_mfma<NT, true>), grid, dim3(256), 0, st, n, nb, d, perm,
                           pair_of_m, views, part_base, pcnt, part, feats, num, den, (int)first,
                           (int)last);
    else
        hipLaunchKernelGGL((k_contract_mfma<NT, false>), grid, dim3(256), 0, st, n, nb, d, perm,
                           pair_of_m, views, part_base, pcnt, part, feats, num, den, (int)first,
                           (int)last);
}

}  // namespace

bool contract_supported(int d)
{
    return d == 64 || d == 128 || d == 256 || d == 512 || d == 768 || d == 1024;
}

bool contract_supported_codes(int d) { return d == 16 || d == 32 || d == 48 || contract_supported(d); }

void launch_contract(int64_t n, int nb, int d, bool bf16, const uint32_t* perm,
                     const uint32_t* pair_of_m, const ViewDev* views, const uint32_t* part_base,
                     const uint32_t* pcnt, const uint2* part, const void* feats, float* num,
                     float* den, bool first, bool last, hipStream_t st)
{
    if (n <= 0) return;
#define SLAG_NT(NTV) launch_nt<NTV>(n, nb, d, bf16, perm, pair_of_m, views, part_base, pcnt, part, \
                                    feats, num, den, first, last, st)
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

}  // namespace slag
