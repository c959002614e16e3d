// Aggregation (paper, Method: E_k = sum_i sum_j sum_{p in M_j} w_kp E_j /
// sum_i sum_j sum_{p in M_j} w_kp) on the matrix cores.
//
// num = W F is a sparse-times-dense product: each Gaussian touches about one
// segment per view, out of ~10^2 per view.  Gaussians are taken in blocks of
// 16 consecutive along a Morton curve of their means, so the 16 rows of a
// block tend to see the same segments.  A workgroup (4 waves) owns one block;
// every wave walks the block's pairs eight views per step (each lane walks two
// (row, view) pairs, reading their packed (segment, weight) slots),
// deduplicates the segments the rows touch (an LDS bitmap per view over
// view-local segment ids), and packs them into K-chunks of 32 columns: A[16 x 32] holds the weights, B[32 x 16] the
// feature rows of those segments.  Each wave multiplies for its quarter of
// the feature columns:
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

constexpr int VG = 8;           // views per step: lane l walks (row l & 15) in views
                                // v0 + (l >> 4) and v0 + 4 + (l >> 4)
constexpr int SL = 4;           // slots of one pair held in registers at a time

struct WaveLds {
    uint32_t bits[64];          // word i: view i >> 3 of the step, ids w0 + 32 (i & 7) + [0, 32)
    uint32_t piece[64];         // bits placed in the open chunk by the current piece
    uint32_t pbase[64];         // first chunk column of each piece word
    uint32_t ks[KC];            // feature row of each K column of the open chunk
    float A[16][KC + 1];        // weights of the open chunk
    float dpart[VG][16];        // per-view weight sums of the step
    float den[16];
};

// Multiply the open chunk (kn columns) into the accumulators and clear it.
template <int NT, bool BF16>
__device__ __forceinline__ void flush(WaveLds& L, int kn, const void* feats, int d, int c0,
                                      floatx4* acc, int lane)
{
    const int m = lane & 15, kq = lane >> 4;
    if constexpr (BF16) {
        bf16x8 ahi, alo;
        uint32_t krow[8];
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const int k = 8 * kq + j;
            const float a = L.A[m][k];
            const __bf16 h = (__bf16)a;
            ahi[j] = h;
            alo[j] = (__bf16)(a - (float)h);
            krow[j] = k < kn ? L.ks[k] : NONE;
        }
        const uint16_t* F = reinterpret_cast<const uint16_t*>(feats);
#pragma unroll
        for (int t = 0; t < NT; t++) {
            const int col = c0 + 16 * t + m;
            bf16x8 b;
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const uint16_t v = krow[j] != NONE ? F[(size_t)krow[j] * d + col] : (uint16_t)0;
                b[j] = __builtin_bit_cast(__bf16, v);
            }
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, b, acc[t], 0, 0, 0);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, b, acc[t], 0, 0, 0);
        }
    } else {
        const float* F = reinterpret_cast<const float*>(feats);
#pragma unroll
        for (int kk = 0; kk < KC / 4; kk++) {
            const int k = 4 * kk + kq;
            const float a = L.A[m][k];
            const uint32_t krow = k < kn ? L.ks[k] : NONE;
#pragma unroll
            for (int t = 0; t < NT; t++) {
                const int col = c0 + 16 * t + m;
                const float b = krow != NONE ? F[(size_t)krow * d + col] : 0.0f;
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[t], 0, 0, 0);
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
    for (int i = lane; i < 16 * (KC + 1); i += 64) (&L.A[0][0])[i] = 0.0f;
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint32_t wave_exscan(uint32_t x, int lane, uint32_t& total)
{
    uint32_t v = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(v, d, 64);
        if (lane >= d) v += y;
    }
    total = (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
    return v - x;
}

// The lowest k set bits of b.
__device__ __forceinline__ uint32_t lowest_bits(uint32_t b, uint32_t k)
{
    if (k >= (uint32_t)__popc(b)) return b;
    uint32_t keep = 0;
    for (uint32_t i = 0; i < k; i++) {
        const uint32_t low = b & (~b + 1u);
        keep |= low;
        b ^= low;
    }
    return keep;
}

template <int NT, bool BF16>
__global__ __launch_bounds__(256) void k_contract_mfma(
    int64_t n, int nb, int d, const uint32_t* __restrict__ perm,
    const uint32_t* __restrict__ pair_of_m, const ViewDev* __restrict__ views,
    const uint32_t* __restrict__ part_base, const uint32_t* __restrict__ pcnt,
    const uint2* __restrict__ part, const void* __restrict__ feats, float* __restrict__ num,
    float* __restrict__ den, int first, int last)
{
    __shared__ WaveLds lds[4];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    WaveLds& L = lds[wv];
    const int64_t q0 = (int64_t)blockIdx.x * 16;          // first Morton rank of the block
    const int c0 = wv * 16 * NT;                          // this wave's first feature column
    const int m = lane & 15, kq = lane >> 4;
    const int r = lane & 15, vq = lane >> 4;              // walking role
    const bool row_ok = q0 + r < n;
    const int64_t qr = row_ok ? q0 + r : q0;

    for (int i = lane; i < 16 * (KC + 1); i += 64) (&L.A[0][0])[i] = 0.0f;
    L.bits[lane] = 0;
    floatx4 acc[NT];
    float dsum = 0.0f;   // running weight sum of row r (held by lanes vq == 0)
    if (first) {
#pragma unroll
        for (int t = 0; t < NT; t++) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
    } else {
#pragma unroll
        for (int t = 0; t < NT; t++)
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int64_t q = q0 + 4 * kq + j;
                acc[t][j] = q < n ? num[(size_t)perm[q] * d + c0 + 16 * t + m] : 0.0f;
            }
        if (vq == 0 && row_ok) dsum = den[perm[q0 + r]];
    }
    __builtin_amdgcn_wave_barrier();
    int kn = 0;   // open chunk fill

    auto pair_at = [&](int v) -> uint32_t {
        const int vc = v < nb ? v : nb - 1;                 // clamped: always a valid address
        const uint32_t p = pair_of_m[(int64_t)vc * n + qr];
        return (row_ok && v < nb) ? p : NONE;
    };
    uint32_t nA = pair_at(vq), nB = pair_at(4 + vq);

    for (int v0 = 0; v0 < nb; v0 += VG) {
        const uint32_t pA = nA, pB = nB;
        nA = pair_at(v0 + VG + vq);                         // next step, in flight meanwhile
        nB = pair_at(v0 + VG + 4 + vq);
        if (!__ballot(pA != NONE || pB != NONE)) continue;
        const int vA = v0 + vq, vB = v0 + 4 + vq;
        const uint32_t pbA = pA != NONE ? part_base[pA] : 0u, cA = pA != NONE ? pcnt[pA] : 0u;
        const uint32_t pbB = pB != NONE ? part_base[pB] : 0u, cB = pB != NONE ? pcnt[pB] : 0u;
        const uint32_t nsA = vA < nb ? views[vA].nseg : 0u, nsB = vB < nb ? views[vB].nseg : 0u;
        const int vw = v0 + (lane >> 3);                    // view of bitmap word `lane`
        const uint32_t so_w = vw < nb ? views[vw].seg_off : 0u;
        const uint32_t cmax = max(cA, cB);
        float dA = 0.0f, dB = 0.0f;
        for (uint32_t w0 = 0; __ballot(w0 < nsA || w0 < nsB); w0 += 256) {
            // 1. mark the segments the rows touch
            for (uint32_t kb = 0; __ballot(kb < cmax); kb += SL) {
                uint2 ea[SL], eb[SL];
#pragma unroll
                for (int k = 0; k < SL; k++) {
                    ea[k] = kb + k < cA ? part[pbA + kb + k] : make_uint2(0u, 0u);
                    eb[k] = kb + k < cB ? part[pbB + kb + k] : make_uint2(0u, 0u);
                }
#pragma unroll
                for (int k = 0; k < SL; k++) {
                    const uint32_t sa = ea[k].x - w0, sb = eb[k].x - w0;
                    const float wa = __uint_as_float(ea[k].y), wb = __uint_as_float(eb[k].y);
                    if (sa < 256u && wa > 0.0f) {
                        atomicOr(&L.bits[vq * 8 + (sa >> 5)], 1u << (sa & 31));
                        dA += wa;
                    }
                    if (sb < 256u && wb > 0.0f) {
                        atomicOr(&L.bits[(vq + 4) * 8 + (sb >> 5)], 1u << (sb & 31));
                        dB += wb;
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            uint32_t b = L.bits[lane];                      // lane owns word `lane`
            __builtin_amdgcn_wave_barrier();
            L.bits[lane] = 0;
            // 2. place the marked segments into chunks (views in order, ids ascending)
            for (;;) {
                uint32_t total;
                const uint32_t c = (uint32_t)__popc(b);
                const uint32_t pre = wave_exscan(c, lane, total);
                if (!total) break;
                const uint32_t room = (uint32_t)(KC - kn);
                const uint32_t want = pre < room ? room - pre : 0u;
                const uint32_t piece = lowest_bits(b, want);
                b ^= piece;
                const uint32_t taken = total < room ? total : room;
                const uint32_t pbase = (uint32_t)kn + (pre < room ? pre : room);
                L.piece[lane] = piece;
                L.pbase[lane] = pbase;
                {
                    uint32_t cc = pbase, bb = piece;
                    while (bb) {
                        const uint32_t bit = (uint32_t)(__ffs((int)bb) - 1);
                        L.ks[cc++] = so_w + w0 + 32u * (uint32_t)(lane & 7) + bit;
                        bb &= bb - 1u;
                    }
                }
                __builtin_amdgcn_wave_barrier();
                // weights of the placed segments, each lane into its row
                for (uint32_t kb = 0; __ballot(kb < cmax); kb += SL) {
                    uint2 ea[SL], eb[SL];
#pragma unroll
                    for (int k = 0; k < SL; k++) {
                        ea[k] = kb + k < cA ? part[pbA + kb + k] : make_uint2(0u, 0u);
                        eb[k] = kb + k < cB ? part[pbB + kb + k] : make_uint2(0u, 0u);
                    }
#pragma unroll
                    for (int k = 0; k < SL; k++) {
#pragma unroll
                        for (int h = 0; h < 2; h++) {
                            const uint2 e = h ? eb[k] : ea[k];
                            const uint32_t s = e.x - w0;
                            const float w = __uint_as_float(e.y);
                            if (s >= 256u || !(w > 0.0f)) continue;
                            const int wi = (vq + 4 * h) * 8 + (int)(s >> 5);
                            const uint32_t pw = L.piece[wi];
                            const uint32_t bit = 1u << (s & 31);
                            if (!(pw & bit)) continue;
                            const int col = (int)L.pbase[wi] + __popc(pw & (bit - 1u));
                            L.A[r][col] += w;
                        }
                    }
                }
                __builtin_amdgcn_wave_barrier();
                kn += (int)taken;
                if (kn == KC) {
                    flush<NT, BF16>(L, kn, feats, d, c0, acc, lane);
                    kn = 0;
                }
            }
        }
        // row weight sums, views in order
        L.dpart[vq][r] = dA;
        L.dpart[vq + 4][r] = dB;
        __builtin_amdgcn_wave_barrier();
        if (vq == 0) {
#pragma unroll
            for (int i = 0; i < VG; i++) dsum += L.dpart[i][r];
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (kn) flush<NT, BF16>(L, kn, feats, d, c0, acc, lane);
    if (vq == 0) L.den[r] = dsum;
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int rr = 4 * kq + j;
        const int64_t q = q0 + rr;
        if (q >= n) continue;
        const uint32_t g = perm[q];
        const float dn = L.den[rr];
#pragma unroll
        for (int t = 0; t < NT; t++) {
            const float a = acc[t][j];
            num[(size_t)g * d + c0 + 16 * t + m] = last ? (dn > 0.0f ? a / dn : 0.0f) : a;
        }
    }
    if (vq == 0 && row_ok && wv == 0) den[perm[q0 + r]] = dsum;
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

void launch_contract(int64_t n, int nb, int d, bool bf16, const uint32_t* perm,
                     const uint32_t* pair_of_m, const ViewDev* views, const uint32_t* part_base,
                     const uint32_t* pcnt, const uint2* part, const void* feats, float* num,
                     float* den, bool first, bool last, hipStream_t st)
{
    if (n <= 0) return;
#define SLAG_NT(NTV) launch_nt<NTV>(n, nb, d, bf16, perm, pair_of_m, views, part_base, pcnt, part, \
                                    feats, num, den, first, last, st)
    switch (d) {
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
