// Cosine-similarity search over per-Gaussian embeddings (paper, Method,
// "Query processing for inference": query vectors are matched against the
// embedding tensor by cosine similarity; Experiments: a relevance threshold
// on the cosine, query responses of the best-matching Gaussians, and the
// per-Gaussian class of highest cosine similarity).
//
// Scores: S[q][g] = E_g . qhat_q / ||E_g||, qhat = q / ||q||, for every
// Gaussian with E_g != 0 (else -inf).  The product E QhatT is a dense
// [N x d] x [d x Qp] contraction on the matrix cores
// (v_mfma_f32_16x16x4_f32, FP32 operands and accumulation): a wave owns 16
// consecutive Gaussians, each lane loads 16 bytes of one embedding row per
// step (the four lanes of a row cover 64 consecutive bytes), and the same
// registers feed the four MFMAs of the step (k-slices permuted identically
// in A and B) and the row's sum of squares.  Reading E once is the bound
// (4 d bytes per Gaussian) while Qp stays below about 40.
#include <cmath>
#include <mutex>

#include "../../include/slag_query.h"
#include "slag_internal.h"

// Work area of slag_query_static (callers that cannot allocate): one static
// buffer per GPU, reserved with the code object and kept until the process
// ends.  Host code never uses this name as an address (on the host it is a
// stand-in, not device memory): it takes the per-device address returned by
// hipGetSymbolAddress in query_scratch_init.
static __device__ __align__(256) unsigned char scratch[SLAG_QUERY_SCRATCH_BYTES];

namespace slag {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};
}  // namespace

hipError_t query_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[device]) return hipSuccess;
    // the caller made `device` current
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess) g_scratch[device] = p;
    return e;
}

void* query_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch[device];
}

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Unit query vectors, transposed and zero-padded: qt[k][j], j < qp (a
// multiple of 16).  One workgroup per query; zero or non-finite norms set
// err[0] (the host rejects such queries).
__global__ __launch_bounds__(256) void k_qprep(int nq, int qp, int d, const float* __restrict__ q,
                                               float* __restrict__ qt, uint32_t* __restrict__ err)
{
    __shared__ float part[4];
    const int j = blockIdx.x, t = threadIdx.x;
    float s = 0.0f;
    if (j < nq)
        for (int k = t; k < d; k += 256) {
            const float x = q[(size_t)j * d + k];
            s = fmaf(x, x, s);
        }
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((t & 63) == 0) part[t >> 6] = s;
    __syncthreads();
    const float n2 = ((part[0] + part[1]) + part[2]) + part[3];
    const bool ok = j >= nq || (n2 > 0.0f && n2 < INFINITY);
    if (!ok && t == 0) atomicOr(err, 1u);
    const float inv = (j < nq && ok) ? 1.0f / sqrtf(n2) : 0.0f;
    for (int k = t; k < d; k += 256)
        qt[(size_t)k * qp + j] = j < nq ? q[(size_t)j * d + k] * inv : 0.0f;
}

// Monotone integer key of a float: larger floats give smaller keys, so an
// ascending stable sort lists the best scores first and ties in index order.
__device__ __forceinline__ uint32_t desc_key(float f)
{
    const uint32_t u = __float_as_uint(f);
    const uint32_t asc = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return ~asc;
}

__device__ __forceinline__ float from_desc_key(uint32_t k)
{
    const uint32_t asc = ~k;
    const uint32_t u = (asc & 0x80000000u) ? (asc & 0x7FFFFFFFu) : ~asc;
    return __uint_as_float(u);
}

// MODE 0: per-query counts of scores >= thr and, if keys != null, the sort
// keys (desc_key(score), index) of every (q, g) at [q n + g].
// MODE 1: per Gaussian, the class (query) of highest score, ties to the
// lower class, -1 for E_g = 0, and that score.
template <int NQT, int MODE>
__global__ __launch_bounds__(256) void k_scores(int64_t n, int d, int nq, const float* __restrict__ E,
                                                const float* __restrict__ qt, float thr,
                                                uint32_t* __restrict__ keys,
                                                uint32_t* __restrict__ vals,
                                                unsigned long long* __restrict__ counts,
                                                int32_t* __restrict__ label, float* __restrict__ best)
{
    constexpr int QP = 16 * NQT;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int64_t g0 = ((int64_t)blockIdx.x * 4 + wv) * 16;     // this wave's first Gaussian
    if (g0 >= n) return;                                       // wave-uniform
    const int m = lane & 15, kq = lane >> 4;
    const int64_t gm = g0 + m < n ? g0 + m : n - 1;            // clamped row (always valid)
    const float* row = E + (size_t)gm * d + 4 * kq;
    floatx4 acc[NQT];
#pragma unroll
    for (int i = 0; i < NQT; i++) acc[i] = floatx4{0.f, 0.f, 0.f, 0.f};
    float ss = 0.0f;
    // d is a multiple of 16: each step covers 16 columns, lane kq takes
    // columns k0 + 4 kq .. + 3 of its row; MFMA j multiplies column
    // k0 + 4 kk + j of A (lane kk's j-th value) with the same row of B
    for (int k0 = 0; k0 < d; k0 += 16) {
        const float4 a = *reinterpret_cast<const float4*>(row + k0);
        ss = fmaf(a.x, a.x, ss);
        ss = fmaf(a.y, a.y, ss);
        ss = fmaf(a.z, a.z, ss);
        ss = fmaf(a.w, a.w, ss);
        const float* qb = qt + (size_t)(k0 + 4 * kq) * QP + m;
        const float av[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
        for (int j = 0; j < 4; j++)
#pragma unroll
            for (int i = 0; i < NQT; i++)
                acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[j], qb[(size_t)j * QP + 16 * i],
                                                             acc[i], 0, 0, 0);
    }
    // row sums of squares: lanes m, m + 16, m + 32, m + 48 hold parts of row m
    ss += __shfl_xor(ss, 16, 64);
    ss += __shfl_xor(ss, 32, 64);
    // acc[i][j] is C[row 4 kq + j][column 16 i + m]; the norms of those rows
    float inv[4];
    bool live[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const float n2 = __shfl(ss, 4 * kq + j, 64);
        live[j] = n2 > 0.0f && g0 + 4 * kq + j < n;
        inv[j] = n2 > 0.0f ? 1.0f / sqrtf(n2) : 0.0f;
    }
    if (MODE == 0) {
        uint32_t cnt[NQT] = {};
#pragma unroll
        for (int i = 0; i < NQT; i++) {
            const int q = 16 * i + m;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int64_t g = g0 + 4 * kq + j;
                const float s = live[j] ? acc[i][j] * inv[j] : -INFINITY;
                if (q < nq && g < n) {
                    if (keys) {
                        keys[(size_t)q * n + g] = desc_key(s);
                        vals[(size_t)q * n + g] = (uint32_t)g;
                    }
                    cnt[i] += s >= thr;
                }
            }
        }
        // per-query counts: the four lanes kq of column m add up, one atomic each
#pragma unroll
        for (int i = 0; i < NQT; i++) {
            uint32_t c = cnt[i];
            c += __shfl_xor(c, 16, 64);
            c += __shfl_xor(c, 32, 64);
            if (kq == 0 && 16 * i + m < nq && c) atomicAdd(&counts[16 * i + m], (unsigned long long)c);
        }
    } else {
        // best class per row: over this lane's tiles, then across the 16
        // lanes of its DPP row (column m), ties to the lower class
#pragma unroll
        for (int j = 0; j < 4; j++) {
            float bv = -INFINITY;
            int bc = 0x7FFFFFFF;
#pragma unroll
            for (int i = 0; i < NQT; i++) {
                const int q = 16 * i + m;
                const float s = acc[i][j] * inv[j];
                if (q < nq && (s > bv || (s == bv && q < bc))) { bv = s; bc = q; }
            }
            for (int o = 1; o < 16; o <<= 1) {
                const float ov = __shfl_xor(bv, o, 64);
                const int oc = __shfl_xor(bc, o, 64);
                if (ov > bv || (ov == bv && oc < bc)) { bv = ov; bc = oc; }
            }
            const int64_t g = g0 + 4 * kq + j;
            if (m == 0 && g < n) {
                label[g] = live[j] ? bc : -1;
                if (best) best[g] = live[j] ? bv : -INFINITY;
            }
        }
    }
}

// First k entries of each query's sorted (key, index) list (query q's list
// at keys[q n], vals[q n]); past the scored Gaussians: index NONE, -inf.
__global__ __launch_bounds__(256) void k_topk_out(int nq, int k, int64_t n, const uint32_t* __restrict__ keys,
                                                  const uint32_t* __restrict__ vals, uint32_t* __restrict__ idx,
                                                  float* __restrict__ cosv)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int q = blockIdx.y;
    if (i >= k || q >= nq) return;
    uint32_t g = NONE;
    float s = -INFINITY;
    if (i < n) {
        const float v = from_desc_key(keys[(size_t)q * n + i]);
        if (v != -INFINITY) { g = vals[(size_t)q * n + i]; s = v; }
    }
    idx[(size_t)q * k + i] = g;
    cosv[(size_t)q * k + i] = s;
}

template <int MODE>
void launch_scores_t(int nqt, int64_t n, int d, int nq, const float* E, const float* qt, float thr,
                     uint32_t* keys, uint32_t* vals, unsigned long long* counts, int32_t* label,
                     float* best, hipStream_t st)
{
    const dim3 grid((unsigned)((n + 63) / 64));
#define SLAG_QS(NQ)                                                                              \
    hipLaunchKernelGGL((k_scores<NQ, MODE>), grid, dim3(256), 0, st, n, d, nq, E, qt, thr, keys, \
                       vals, counts, label, best)
    switch (nqt) {
    case 1: SLAG_QS(1); break;
    case 2: SLAG_QS(2); break;
    case 3: SLAG_QS(3); break;
    case 4: SLAG_QS(4); break;
    default: break;
    }
#undef SLAG_QS
}

}  // namespace

void launch_qprep(int nq, int qp, int d, const float* q, float* qt, uint32_t* err, hipStream_t st)
{
    hipLaunchKernelGGL(k_qprep, dim3((unsigned)qp), dim3(256), 0, st, nq, qp, d, q, qt, err);
}

void launch_scores(int nq, int64_t n, int d, const float* E, const float* qt, float thr,
                   uint32_t* keys, uint32_t* vals, unsigned long long* counts, hipStream_t st)
{
    if (n <= 0) return;
    launch_scores_t<0>((nq + 15) / 16, n, d, nq, E, qt, thr, keys, vals, counts, nullptr, nullptr,
                       st);
}

void launch_classify(int nc, int64_t n, int d, const float* E, const float* qt, int32_t* label,
                     float* best, hipStream_t st)
{
    if (n <= 0) return;
    launch_scores_t<1>((nc + 15) / 16, n, d, nc, E, qt, 0.0f, nullptr, nullptr, nullptr, label,
                       best, st);
}

void launch_topk_out(int nq, int k, int64_t n, const uint32_t* keys, const uint32_t* vals,
                     uint32_t* idx, float* cosv, hipStream_t st)
{
    if (k <= 0 || nq <= 0) return;
    hipLaunchKernelGGL(k_topk_out, dim3((unsigned)((k + 255) / 256), (unsigned)nq), dim3(256), 0, st,
                       nq, k, n, keys, vals, idx, cosv);
}

}  // namespace slag
