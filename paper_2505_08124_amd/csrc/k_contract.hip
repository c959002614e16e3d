// Aggregation (paper, Method: E_k = sum_i sum_j sum_{p in M_j} w_kp E_j /
// sum_i sum_j sum_{p in M_j} w_kp): the per-view masked weight sums W_i[k, j]
// are contracted with the segment feature table and normalised.
//
// One wave64 owns one Gaussian: it walks the Gaussian's pairs in view order
// and their (segment row, weight) entries in row order, so every output is
// summed in a fixed order (deterministic).  Lane l owns feature columns
// [l*KPL, (l+1)*KPL); BF16 tables are widened exactly to FP32 and all sums are
// FP32.  Output rows are written in input Gaussian order.
#include "slag_internal.h"

namespace slag {

namespace {

template <int KPL, bool BF16>
__device__ __forceinline__ void load_row(const void* feats, uint32_t row, int d, int lane, float* f)
{
    if constexpr (BF16) {
        const uint16_t* p = reinterpret_cast<const uint16_t*>(feats) + (size_t)row * d + lane * KPL;
        if constexpr (KPL % 8 == 0) {
#pragma unroll
            for (int i = 0; i < KPL / 8; i++) {
                const uint4 q = reinterpret_cast<const uint4*>(p)[i];
                const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    f[8 * i + 2 * k] = __uint_as_float(w[k] << 16);
                    f[8 * i + 2 * k + 1] = __uint_as_float(w[k] & 0xFFFF0000u);
                }
            }
        } else if constexpr (KPL % 4 == 0) {
#pragma unroll
            for (int i = 0; i < KPL / 4; i++) {
                const uint2 q = reinterpret_cast<const uint2*>(p)[i];
                f[4 * i] = __uint_as_float(q.x << 16);
                f[4 * i + 1] = __uint_as_float(q.x & 0xFFFF0000u);
                f[4 * i + 2] = __uint_as_float(q.y << 16);
                f[4 * i + 3] = __uint_as_float(q.y & 0xFFFF0000u);
            }
        } else {
#pragma unroll
            for (int i = 0; i < KPL; i++) f[i] = __uint_as_float((uint32_t)p[i] << 16);
        }
    } else {
        const float* p = reinterpret_cast<const float*>(feats) + (size_t)row * d + lane * KPL;
        if constexpr (KPL % 4 == 0) {
#pragma unroll
            for (int i = 0; i < KPL / 4; i++) {
                const float4 q = reinterpret_cast<const float4*>(p)[i];
                f[4 * i] = q.x; f[4 * i + 1] = q.y; f[4 * i + 2] = q.z; f[4 * i + 3] = q.w;
            }
        } else {
#pragma unroll
            for (int i = 0; i < KPL; i++) f[i] = p[i];
        }
    }
}

template <int KPL, bool BF16>
__global__ __launch_bounds__(256) void k_contract(int64_t n, int nb, int d,
                                                  const uint32_t* __restrict__ pair_of,
                                                  const uint32_t* __restrict__ wlen,
                                                  const uint32_t* __restrict__ part_base,
                                                  const uint2* __restrict__ wrow,
                                                  const void* __restrict__ feats,
                                                  float* __restrict__ num, float* __restrict__ den,
                                                  int first, int last)
{
    const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (g >= n) return;
    const int lane = threadIdx.x & 63;
    float acc[KPL];
    float dsum = 0.0f;
    float* nrow = num + (size_t)g * d + lane * KPL;
    if (first) {
#pragma unroll
        for (int k = 0; k < KPL; k++) acc[k] = 0.0f;
    } else {
#pragma unroll
        for (int k = 0; k < KPL; k++) acc[k] = nrow[k];
        dsum = den[g];
    }
    for (int v0 = 0; v0 < nb; v0 += 64) {
        const int vl = v0 + lane;
        const uint32_t p = vl < nb ? pair_of[(int64_t)vl * n + g] : NONE;
        uint64_t m = __ballot(p != NONE);
        while (m) {
            const int l = __ffsll((long long)m) - 1;
            m &= m - 1;
            const uint32_t pp = (uint32_t)__builtin_amdgcn_readlane((int)p, l);
            const uint32_t cnt = wlen[pp];
            const uint32_t base = part_base[pp];
            for (uint32_t e0 = 0; e0 < cnt; e0 += 64) {
                const uint32_t ne = min(64u, cnt - e0);
                const uint2 ent = (uint32_t)lane < ne ? wrow[base + e0 + lane] : make_uint2(0u, 0u);
                for (uint32_t i = 0; i < ne; i++) {
                    const uint32_t s = (uint32_t)__builtin_amdgcn_readlane((int)ent.x, (int)i);
                    const float w = __int_as_float(__builtin_amdgcn_readlane((int)ent.y, (int)i));
                    dsum += w;
                    float f[KPL];
                    load_row<KPL, BF16>(feats, s, d, lane, f);
#pragma unroll
                    for (int k = 0; k < KPL; k++) acc[k] = fmaf(w, f[k], acc[k]);
                }
            }
        }
    }
    if (last) {
#pragma unroll
        for (int k = 0; k < KPL; k++) nrow[k] = dsum > 0.0f ? acc[k] / dsum : 0.0f;
    } else {
#pragma unroll
        for (int k = 0; k < KPL; k++) nrow[k] = acc[k];
    }
    if (lane == 0) den[g] = dsum;
}

template <int KPL>
void launch_kpl(int64_t n, int nb, int d, bool bf16, const uint32_t* pair_of, const uint32_t* wlen,
                const uint32_t* part_base, const uint2* wrow, const void* feats, float* num,
                float* den, bool first, bool last, hipStream_t st)
{
    const dim3 grid((unsigned)((n + 3) / 4));
    if (bf16)
        hipLaunchKernelGGL((k_contract<KPL, true>), grid, dim3(256), 0, st, n, nb, d, pair_of, wlen,
                           part_base, wrow, feats, num, den, (int)first, (int)last);
    else
        hipLaunchKernelGGL((k_contract<KPL, false>), grid, dim3(256), 0, st, n, nb, d, pair_of,
                           wlen, part_base, wrow, feats, num, den, (int)first, (int)last);
}

}  // namespace

bool contract_supported(int d)
{
    return d == 64 || d == 128 || d == 256 || d == 512 || d == 768 || d == 1024;
}

void launch_contract(int64_t n, int nb, int d, bool bf16, const uint32_t* pair_of,
                     const uint32_t* wlen, const uint32_t* part_base, const uint2* wrow,
                     const void* feats, float* num, float* den, bool first, bool last,
                     hipStream_t st)
{
    if (n <= 0) return;
    switch (d) {
    case 64: launch_kpl<1>(n, nb, d, bf16, pair_of, wlen, part_base, wrow, feats, num, den, first, last, st); break;
    case 128: launch_kpl<2>(n, nb, d, bf16, pair_of, wlen, part_base, wrow, feats, num, den, first, last, st); break;
    case 256: launch_kpl<4>(n, nb, d, bf16, pair_of, wlen, part_base, wrow, feats, num, den, first, last, st); break;
    case 512: launch_kpl<8>(n, nb, d, bf16, pair_of, wlen, part_base, wrow, feats, num, den, first, last, st); break;
    case 768: launch_kpl<12>(n, nb, d, bf16, pair_of, wlen, part_base, wrow, feats, num, den, first, last, st); break;
    case 1024: launch_kpl<16>(n, nb, d, bf16, pair_of, wlen, part_base, wrow, feats, num, den, first, last, st); break;
    default: break;
    }
}

}  // namespace slag
