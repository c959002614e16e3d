// Learned segment-feature codec: encoder D -> H -> k and decoder k -> H -> D
// (tanh-form GELU), trained through the lift's mixing (each Gaussian's code
// is the weight-normalised sum of its segments' codes; the loss is the mean
// of 1 - cos(decoded code, plain-lift embedding)), and used by the codec lift.
// This is an extension of the paper's lift, which aggregates the full
// features; the aggregation of codes is the same weighted average.
//
// Products run on the matrix cores: v_mfma_f32_16x16x32_bf16 with operands
// rounded to bf16 (FP32 master weights, FP32 accumulation), or
// v_mfma_f32_16x16x4f32 in full FP32 (used to check gradients).
#include "slag_internal.h"

namespace slag {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int GT = 64;     // output tile edge per workgroup
constexpr int GK = 32;     // K per staged chunk

constexpr float kGeluC = 0.7978845608028654f;   // sqrt(2 / pi)
constexpr float kGeluA = 0.044715f;

__device__ __forceinline__ float gelu_f(float x)
{
    const float u = kGeluC * (x + kGeluA * x * x * x);
    return 0.5f * x * (1.0f + tanhf(u));
}

__device__ __forceinline__ float gelu_grad_f(float x)
{
    const float u = kGeluC * (x + kGeluA * x * x * x);
    const float th = tanhf(u);
    return 0.5f * (1.0f + th) + 0.5f * x * (1.0f - th * th) * kGeluC * (1.0f + 3.0f * kGeluA * x * x);
}

__device__ __forceinline__ float load_elem(const float* p, int64_t i) { return p[i]; }
__device__ __forceinline__ float load_elem(const uint16_t* p, int64_t i)
{
    return __uint_as_float((uint32_t)p[i] << 16);
}

__device__ __forceinline__ float epilogue(float v, int64_t row, int col, int64_t idx,
                                          const GemmEpi& e)
{
    if (e.bias) v += e.bias[col];
    if (e.zsave) e.zsave[idx] = v;
    if (e.act == GEMM_GELU) v = gelu_f(v);
    else if (e.act == GEMM_GELU_BWD) v *= gelu_grad_f(e.aux[idx]);
    if (e.rowmask && !(e.rowmask[row] > 0.0f)) v = 0.0f;
    return v;
}

// C[M][N] (row-major, leading dimension ldc) = op(A)[M][K] op(B)[K][N] with
// the epilogue; A(m, k) = A[m sam + k sak], B(k, n) = B[k sbk + n sbn].
// blockIdx.z selects a slice of K; with more than one slice the raw sums go
// to out + z M N (row-major, leading dimension N) and k_gemm_reduce finishes.
template <bool BF16, typename TA>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const TA* __restrict__ A,
                                              int64_t sam, int64_t sak,
                                              const float* __restrict__ B, int64_t sbk,
                                              int64_t sbn, int kper, float* __restrict__ out,
                                              int64_t ldc, GemmEpi epi)
{
    __shared__ float As[GT][GK + 1];
    __shared__ float Bs[GK][GT + 1];
    const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
    const int64_t m0 = (int64_t)blockIdx.y * GT;
    const int n0 = blockIdx.x * GT;
    const int kb = blockIdx.z * kper, ke = min(K, kb + kper);
    const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
    const int li = lane & 15, lq = lane >> 4;
    const bool a_kfast = sak == 1, b_nfast = sbn == 1;

    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    constexpr int TE = GT * GK / 256;   // tile elements per thread
    for (int k0 = kb; k0 < ke; k0 += GK) {
        // clamped (always valid) loads of both tiles, all in flight before
        // the first LDS store
        float av[TE], bv[TE];
#pragma unroll
        for (int i = 0; i < TE; i++) {
            const int e = t + 256 * i;
            const int mm = a_kfast ? (e >> 5) : (e & 63);
            const int kk = a_kfast ? (e & 31) : (e >> 6);
            const int64_t gm = m0 + mm;
            const int gk = k0 + kk;
            const bool oka = gm < M && gk < ke;
            const float xa = load_elem(A, oka ? gm * sam + (int64_t)gk * sak : 0);
            av[i] = oka ? xa : 0.0f;
            const int nn = b_nfast ? (e & 63) : (e >> 5);
            const int kb2 = b_nfast ? (e >> 6) : (e & 31);
            const int gn = n0 + nn, gk2 = k0 + kb2;
            const bool okb = gn < N && gk2 < ke;
            const float xb = B[okb ? (int64_t)gk2 * sbk + (int64_t)gn * sbn : 0];
            bv[i] = okb ? xb : 0.0f;
        }
#pragma unroll
        for (int i = 0; i < TE; i++) {
            const int e = t + 256 * i;
            As[a_kfast ? (e >> 5) : (e & 63)][a_kfast ? (e & 31) : (e >> 6)] = av[i];
            Bs[b_nfast ? (e >> 6) : (e & 31)][b_nfast ? (e & 63) : (e >> 5)] = bv[i];
        }
        __syncthreads();
        if constexpr (BF16) {
            bf16x8 a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; i++)
#pragma unroll
                for (int j = 0; j < 8; j++) {
                    a[i][j] = (__bf16)As[wm + 16 * i + li][8 * lq + j];
                    b[i][j] = (__bf16)Bs[8 * lq + j][wn + 16 * i + li];
                }
#pragma unroll
            for (int i = 0; i < 2; i++)
#pragma unroll
                for (int j = 0; j < 2; j++)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        } else {
#pragma unroll
            for (int kk = 0; kk < GK / 4; kk++) {
                float a[2], b[2];
#pragma unroll
                for (int i = 0; i < 2; i++) {
                    a[i] = As[wm + 16 * i + li][4 * kk + lq];
                    b[i] = Bs[4 * kk + lq][wn + 16 * i + li];
                }
#pragma unroll
                for (int i = 0; i < 2; i++)
#pragma unroll
                    for (int j = 0; j < 2; j++)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
            }
        }
        __syncthreads();
    }

    const bool split = gridDim.z > 1;
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int64_t row = m0 + wm + 16 * i + 4 * lq + r;
                const int col = n0 + wn + 16 * j + li;
                if (row >= M || col >= N) continue;
                if (split) {
                    out[((int64_t)blockIdx.z * M + row) * N + col] = acc[i][j][r];
                } else {
                    const int64_t idx = row * ldc + col;
                    out[idx] = epilogue(acc[i][j][r], row, col, idx, epi);
                }
            }
}

// Fused decoder for BF16 products, 64 code rows per workgroup: the hidden
// layer h = gelu(code W3^T + b3) is formed on the matrix cores and kept in
// LDS as bf16 (the rounding the two-product path applies when it stages h),
// then y = h W4^T + b4 is formed 128 output columns at a time (32 per wave)
// and written once, zero on rows whose rowmask <= 0.  The hidden layer never
// reaches HBM and each W4 row is read once per workgroup.  Codes are padded
// to KP columns with zeros; needs H % 64 == 0, H <= 384 and D % 128 == 0.
template <int KP>
__global__ __launch_bounds__(256) void k_decode_bf16(int M, int k, int H, int D,
                                                     const float* __restrict__ code,
                                                     const float* __restrict__ W3,
                                                     const float* __restrict__ b3,
                                                     const float* __restrict__ W4,
                                                     const float* __restrict__ b4,
                                                     const float* __restrict__ rowmask,
                                                     float* __restrict__ y)
{
    extern __shared__ __align__(16) unsigned char dsm[];
    const int HS = H + 8, KS = KP + 8;            // padded row strides (bf16)
    __bf16* hid = reinterpret_cast<__bf16*>(dsm);  // [64][HS]
    __bf16* cds = hid + 64 * HS;                   // [64][KS]
    const int t = threadIdx.x, wv = t >> 6, lane = t & 63, m = lane & 15, kq = lane >> 4;
    const int64_t r0 = (int64_t)blockIdx.x * 64;
    // clamped (always valid) loads, all in flight before the first LDS store
    constexpr int CE = 64 * KP / 256;
    float cv[CE];
#pragma unroll
    for (int u = 0; u < CE; u++) {
        const int e = t + 256 * u;
        const int rr = e / KP, kk = e - rr * KP;
        const int64_t gr = r0 + rr;
        const bool ok = gr < M && kk < k;
        const float x = code[(ok ? gr : 0) * k + (ok ? kk : 0)];
        cv[u] = ok ? x : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < CE; u++) {
        const int e = t + 256 * u;
        const int rr = e / KP, kk = e - rr * KP;
        cds[rr * KS + kk] = (__bf16)cv[u];
    }
    __syncthreads();
    // hidden layer: wave wv takes the 64-column groups c0 = 64 wv + 256 i
    for (int c0 = 64 * wv; c0 < H; c0 += 256) {
        floatx4 acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 4; j++) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < KP; kk += 32) {
            bf16x8 a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; i++)
                a[i] = *reinterpret_cast<const bf16x8*>(&cds[(16 * i + m) * KS + kk + 8 * kq]);
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const float* wr = W3 + (int64_t)(c0 + 16 * j + m) * k;
#pragma unroll
                for (int e = 0; e < 8; e++) {
                    const int kc = kk + 8 * kq + e;
                    const float x = wr[kc < k ? kc : k - 1];   // clamped: no branch between loads
                    b[j][e] = (__bf16)(kc < k ? x : 0.0f);
                }
            }
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int j = 0; j < 4; j++)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        float bias[4];
#pragma unroll
        for (int j = 0; j < 4; j++) bias[j] = b3[c0 + 16 * j + m];
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int col = c0 + 16 * j + m;
#pragma unroll
                for (int r = 0; r < 4; r++)
                    hid[(16 * i + 4 * kq + r) * HS + col] = (__bf16)gelu_f(acc[i][j][r] + bias[j]);
            }
    }
    // rows kept: inside the matrix and (with a mask) of positive mask value;
    // clamped mask loads, all in flight together
    float keep[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int64_t row = r0 + 16 * i + 4 * kq + r;
            keep[i][r] = row < M ? 1.0f : 0.0f;
        }
    if (rowmask) {
        float mk[4][4];
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int64_t row = r0 + 16 * i + 4 * kq + r;
                mk[i][r] = rowmask[row < M ? row : M - 1];
            }
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int r = 0; r < 4; r++)
                if (!(mk[i][r] > 0.0f)) keep[i][r] = 0.0f;
    }
    __syncthreads();
    // output: 128 columns per pass, wave wv takes columns n0 + 32 wv .. + 31
    for (int n0 = 0; n0 < D; n0 += 128) {
        const int cb = n0 + 32 * wv;
        floatx4 acc[4][2];
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 2; j++) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
        for (int kk = 0; kk < H; kk += 32) {
            bf16x8 a[4], b[2];
#pragma unroll
            for (int i = 0; i < 4; i++)
                a[i] = *reinterpret_cast<const bf16x8*>(&hid[(16 * i + m) * HS + kk + 8 * kq]);
#pragma unroll
            for (int j = 0; j < 2; j++) {
                const float4* wr = reinterpret_cast<const float4*>(
                    W4 + (int64_t)(cb + 16 * j + m) * H + kk + 8 * kq);
                const float4 u0 = wr[0], u1 = wr[1];
                b[j][0] = (__bf16)u0.x; b[j][1] = (__bf16)u0.y; b[j][2] = (__bf16)u0.z; b[j][3] = (__bf16)u0.w;
                b[j][4] = (__bf16)u1.x; b[j][5] = (__bf16)u1.y; b[j][6] = (__bf16)u1.z; b[j][7] = (__bf16)u1.w;
            }
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int j = 0; j < 2; j++)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        const float bias[2] = {b4[cb + m], b4[cb + 16 + m]};
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 2; j++) {
                const int col = cb + 16 * j + m;
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int64_t row = r0 + 16 * i + 4 * kq + r;
                    if (row < M) y[row * D + col] = keep[i][r] * (acc[i][j][r] + bias[j]);
                }
            }
    }
}

// Sum of the K slices in slice order, then the epilogue.
__global__ __launch_bounds__(256) void k_gemm_reduce(int M, int N, int splits,
                                                     const float* __restrict__ part,
                                                     float* __restrict__ out, int64_t ldc,
                                                     GemmEpi epi)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)M * N) return;
    const int64_t row = i / N;
    const int col = (int)(i - row * N);
    float s = 0.0f;
    for (int z = 0; z < splits; z++) s += part[(int64_t)z * M * N + i];
    const int64_t idx = row * ldc + col;
    out[idx] = epilogue(s, row, col, idx, epi);
}

// Column sums of X[R][N] over row slices (partials [slices][N]).
__global__ __launch_bounds__(256) void k_colsum_part(int R, int N, const float* __restrict__ X,
                                                     int rows_per, float* __restrict__ part)
{
    const int col = blockIdx.x * 256 + threadIdx.x;
    if (col >= N) return;
    const int r0 = blockIdx.y * rows_per, r1 = min(R, r0 + rows_per);
    float s = 0.0f;
    for (int r = r0; r < r1; r++) s += X[(int64_t)r * N + col];
    part[(int64_t)blockIdx.y * N + col] = s;
}

__global__ __launch_bounds__(256) void k_colsum_fin(int N, int slices, const float* __restrict__ part,
                                                    float* __restrict__ out)
{
    const int col = blockIdx.x * 256 + threadIdx.x;
    if (col >= N) return;
    float s = 0.0f;
    for (int z = 0; z < slices; z++) s += part[(int64_t)z * N + col];
    out[col] = s;
}

// code[r][c] = sum_j w[j] C[col[j]][c], j in [row_ptr[r], row_ptr[r + 1]).
__global__ __launch_bounds__(256) void k_mix(int R, int k, const uint32_t* __restrict__ row_ptr,
                                             const uint32_t* __restrict__ col,
                                             const float* __restrict__ w,
                                             const float* __restrict__ C, float* __restrict__ code)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)R * k) return;
    const int r = (int)(i / k), c = (int)(i - (int64_t)r * k);
    float s = 0.0f;
    for (uint32_t j = row_ptr[r]; j < row_ptr[r + 1]; j++) s += w[j] * C[(int64_t)col[j] * k + c];
    code[i] = s;
}

// Transpose of the mixing for the gradient: dC[s][c] = sum over the pool
// entries j of column s whose row lies in this batch of w[j] dcode[row][c].
// The pool's entries grouped by column (csc_j: entry indices, ascending
// within each column, so rows ascend too; column s owns [cbeg[s], cend[s]));
// the batch's entries (rows row0 .. row0 + R - 1, row pointers rp = the
// pool's from row0) are the index range [rp[0], rp[R]), found in each column by
// binary search; each (s, c) is summed by one thread in entry order, so the
// result is deterministic (no atomics).
__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t* a, uint32_t lo, uint32_t hi,
                                                    uint32_t x)
{
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_mix_bwd(int NS, int k, const uint32_t* __restrict__ rp, int R,
                                                 int64_t row0,
                                                 const uint32_t* __restrict__ cbeg,
                                                 const uint32_t* __restrict__ cend,
                                                 const uint32_t* __restrict__ csc_j,
                                                 const uint32_t* __restrict__ csc_row,
                                                 const float* __restrict__ w,
                                                 const float* __restrict__ dcode,
                                                 float* __restrict__ dC)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)NS * k) return;
    const int sidx = (int)(i / k), c = (int)(i - (int64_t)sidx * k);
    const uint32_t j0 = rp[0], j1 = rp[R];            // the batch's entry range
    const uint32_t b = cbeg[sidx], e = cend[sidx];
    const uint32_t lo = lower_bound_u32(csc_j, b, e, j0);
    const uint32_t hi = lower_bound_u32(csc_j, lo, e, j1);
    float acc = 0.0f;
    for (uint32_t q = lo; q < hi; q++) {
        const uint32_t j = csc_j[q];
        acc = fmaf(w[j], dcode[((int64_t)csc_row[q] - row0) * k + c], acc);
    }
    dC[i] = acc;
}

// Entries of the pool grouped by column: given the column-sorted entries
// (key = column, ascending; stable, so entry indices ascend within a
// column), the range [cbeg[s], cend[s]) of each column s (empty columns keep
// the zero-filled range) and the row of each sorted entry.
__global__ __launch_bounds__(256) void k_csc_ranges(uint32_t nnz, const uint32_t* __restrict__ key,
                                                    const uint32_t* __restrict__ csc_j,
                                                    const uint32_t* __restrict__ row_of,
                                                    uint32_t* __restrict__ cbeg,
                                                    uint32_t* __restrict__ cend,
                                                    uint32_t* __restrict__ csc_row)
{
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nnz) return;
    const uint32_t s = key[i];
    if (i == 0 || key[i - 1] != s) cbeg[s] = i;
    if (i + 1 == nnz || key[i + 1] != s) cend[s] = i + 1;
    csc_row[i] = row_of[csc_j[i]];
}

// Row of every pool entry from the row pointers (one thread per row).
__global__ __launch_bounds__(256) void k_row_of(uint32_t R, const uint32_t* __restrict__ row_ptr,
                                                uint32_t* __restrict__ row_of,
                                                uint32_t* __restrict__ key,
                                                uint32_t* __restrict__ ent,
                                                const uint32_t* __restrict__ col)
{
    const uint32_t r = blockIdx.x * 256 + threadIdx.x;
    if (r >= R) return;
    for (uint32_t j = row_ptr[r]; j < row_ptr[r + 1]; j++) {
        row_of[j] = r;
        key[j] = col[j];
        ent[j] = j;
    }
}

// Per row (one wave each): loss_r = 1 - cos(y_r, t_r) and
// dy_r = -(t_r / (|y||t|) - cos y_r / |y|^2) / R.  Per-block loss sums.
__global__ __launch_bounds__(256) void k_cos_loss(int R, int d, const float* __restrict__ y,
                                                  const float* __restrict__ tg, float inv_r,
                                                  float* __restrict__ dy,
                                                  float* __restrict__ loss_part)
{
    __shared__ float s_l[4];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + wv;
    float l = 0.0f;
    if (r < R) {
        const float* yr = y + r * d;
        const float* tr = tg + r * d;
        float yy = 0.f, tt = 0.f, yt = 0.f;
        for (int c = lane; c < d; c += 64) {
            const float a = yr[c], b = tr[c];
            yy += a * a;
            tt += b * b;
            yt += a * b;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            yy += __shfl_xor(yy, o, 64);
            tt += __shfl_xor(tt, o, 64);
            yt += __shfl_xor(yt, o, 64);
        }
        const float ny = sqrtf(yy), nt = sqrtf(tt);
        const bool ok = ny > 0.0f && nt > 0.0f;
        const float cs = ok ? yt / (ny * nt) : 0.0f;
        const float at = ok ? inv_r / (ny * nt) : 0.0f, ay = ok ? inv_r * cs / yy : 0.0f;
        for (int c = lane; c < d; c += 64) dy[r * d + c] = -(at * tr[c] - ay * yr[c]);
        l = 1.0f - cs;
    }
    if (lane == 0) s_l[wv] = l;
    __syncthreads();
    if (threadIdx.x == 0) loss_part[blockIdx.x] = s_l[0] + s_l[1] + s_l[2] + s_l[3];
}

// Mean of the per-block loss sums (one block; fixed order).
__global__ __launch_bounds__(256) void k_loss_fin(int nb, const float* __restrict__ part,
                                                  float inv_r, float* __restrict__ out)
{
    __shared__ float s[256];
    float a = 0.0f;
    for (int i = threadIdx.x; i < nb; i += 256) a += part[i];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0] * inv_r;
}

// Adam with bias correction; step is 1-based.
__global__ __launch_bounds__(256) void k_adam(int64_t n, float* __restrict__ p,
                                              const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, float lr, float b1, float b2,
                                              float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// BF16 (bits) or FP32 rows to FP32.
__global__ __launch_bounds__(256) void k_to_f32(int64_t n, const void* __restrict__ src, int bf16,
                                                float* __restrict__ dst)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    dst[i] = bf16 ? __uint_as_float((uint32_t)reinterpret_cast<const uint16_t*>(src)[i] << 16)
                  : reinterpret_cast<const float*>(src)[i];
}

// ---- training rows from a plain lift ----

// SplitMix64 (Steele, Lea, Flood 2014) of seed + index: the row sampler.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// flag[g] = 1 for Gaussians with weight whose hash falls under the threshold.
__global__ __launch_bounds__(256) void k_pick_rows(int64_t n, const float* __restrict__ den,
                                                   uint64_t seed, uint32_t thresh,
                                                   uint32_t* __restrict__ flag)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= n) return;
    const uint32_t h = (uint32_t)(splitmix64(seed + (uint64_t)g) >> 32);
    flag[g] = (den[g] > 0.0f && h < thresh) ? 1u : 0u;
}

// Row length of each picked Gaussian (rows beyond max_rows are dropped):
// the merged weight-row lengths of its pairs over the launch's views.
__global__ __launch_bounds__(256) void k_row_len(int64_t n, int nb, const uint32_t* __restrict__ flag,
                                                 const uint32_t* __restrict__ ridx,
                                                 uint32_t max_rows,
                                                 const uint32_t* __restrict__ rank,
                                                 const uint32_t* __restrict__ pair_of_m,
                                                 const uint32_t* __restrict__ blk_off, int nblk,
                                                 const uint32_t* __restrict__ wlen,
                                                 uint32_t* __restrict__ len, uint32_t* __restrict__ gid)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= n || !flag[g] || ridx[g] >= max_rows) return;
    const uint32_t q = rank[g];
    const int cb = (int)(q / GBLOCK);
    uint32_t l = 0;
    for (int v = 0; v < nb; v++) {
        // (view, block) without visible pairs: the pair map is not written there
        const int64_t bi = (int64_t)v * nblk + cb;
        if (blk_off[bi + 1] == blk_off[bi]) continue;
        const uint32_t p = pair_of_m[(int64_t)v * n + q];
        if (p != NONE) l += wlen[p];
    }
    len[ridx[g]] = l;
    gid[ridx[g]] = (uint32_t)g;
}

// Row r: entries (pool segment, w / den), row pointer, and target E[g].
__global__ __launch_bounds__(256) void k_row_gather(int64_t n, int nb, uint32_t rows,
                                                    const uint32_t* __restrict__ gid,
                                                    const uint32_t* __restrict__ off,
                                                    uint32_t nnz0, uint32_t seg0,
                                                    const uint32_t* __restrict__ rank,
                                                    const uint32_t* __restrict__ pair_of_m,
                                                    const uint32_t* __restrict__ blk_off, int nblk,
                                                    const uint32_t* __restrict__ wlen,
                                                    const uint32_t* __restrict__ part_base,
                                                    const uint2* __restrict__ wrow,
                                                    const float* __restrict__ den,
                                                    uint32_t* __restrict__ row_ptr,
                                                    uint32_t* __restrict__ col, float* __restrict__ w)
{
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= rows) return;
    const uint32_t g = gid[r], q = rank[g];
    const float inv = 1.0f / den[g];
    uint32_t o = nnz0 + off[r];
    row_ptr[r] = o;
    const int cb = (int)(q / GBLOCK);
    for (int v = 0; v < nb; v++) {
        const int64_t bi = (int64_t)v * nblk + cb;
        if (blk_off[bi + 1] == blk_off[bi]) continue;
        const uint32_t p = pair_of_m[(int64_t)v * n + q];
        if (p == NONE) continue;
        const uint32_t b = part_base[p];
        for (uint32_t j = 0; j < wlen[p]; j++) {
            const uint2 e = wrow[b + j];
            col[o] = seg0 + e.x;
            w[o] = __uint_as_float(e.y) * inv;
            o++;
        }
    }
}

__global__ __launch_bounds__(256) void k_copy_rows(uint32_t rows, int d, const uint32_t* __restrict__ gid,
                                                   const float* __restrict__ src,
                                                   float* __restrict__ dst)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)rows * d) return;
    const int64_t r = i / d;
    const int c = (int)(i - r * d);
    dst[i] = src[(int64_t)gid[r] * d + c];
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

void launch_pick_rows(int64_t n, const float* den, uint64_t seed, uint32_t thresh, uint32_t* flag,
                      hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_pick_rows, dim3(blocks(n)), dim3(256), 0, st, n, den, seed, thresh, flag);
}

void launch_row_len(int64_t n, int nb, const uint32_t* flag, const uint32_t* ridx,
                    uint32_t max_rows, const uint32_t* rank, const uint32_t* pair_of_m,
                    const uint32_t* blk_off, int nblk, const uint32_t* wlen, uint32_t* len,
                    uint32_t* gid, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_row_len, dim3(blocks(n)), dim3(256), 0, st, n, nb, flag, ridx, max_rows,
                       rank, pair_of_m, blk_off, nblk, wlen, len, gid);
}

void launch_row_gather(int64_t n, int nb, uint32_t rows, const uint32_t* gid, const uint32_t* off,
                       uint32_t nnz0, uint32_t seg0, const uint32_t* rank,
                       const uint32_t* pair_of_m, const uint32_t* blk_off, int nblk,
                       const uint32_t* wlen, const uint32_t* part_base, const uint2* wrow,
                       const float* den, uint32_t* row_ptr, uint32_t* col, float* w,
                       hipStream_t st)
{
    if (!rows) return;
    hipLaunchKernelGGL(k_row_gather, dim3(blocks(rows)), dim3(256), 0, st, n, nb, rows, gid, off,
                       nnz0, seg0, rank, pair_of_m, blk_off, nblk, wlen, part_base, wrow, den,
                       row_ptr, col, w);
}

void launch_copy_rows(uint32_t rows, int d, const uint32_t* gid, const float* src, float* dst,
                      hipStream_t st)
{
    if (!rows) return;
    hipLaunchKernelGGL(k_copy_rows, dim3(blocks((int64_t)rows * d)), dim3(256), 0, st, rows, d,
                       gid, src, dst);
}

int gemm_splits(int M, int N, int K, int* kper)
{
    const int64_t tiles = (int64_t)((M + GT - 1) / GT) * ((N + GT - 1) / GT);
    int splits = 1;
    if (tiles < 512 && K > 8 * GK) {
        splits = (int)std::min<int64_t>((K + 8 * GK - 1) / (8 * GK), (1024 + tiles - 1) / tiles);
        splits = std::max(splits, 1);
    }
    int kp = (K + splits - 1) / splits;
    kp = (kp + GK - 1) / GK * GK;
    if (kp <= 0) kp = GK;
    *kper = kp;
    return (K + kp - 1) / kp;
}

bool decode_fused_supported(int k, int H, int D)
{
    // LDS 64 (H + 8 + KP + 8) bf16 stays within the default 64 KiB
    return k >= 1 && k <= 64 && H % 64 == 0 && H <= 384 && D % 128 == 0;
}

void launch_decode_bf16(int M, int k, int H, int D, const float* code, const float* W3,
                        const float* b3, const float* W4, const float* b4, const float* rowmask,
                        float* y, hipStream_t st)
{
    if (M <= 0) return;
    const int KP = k <= 32 ? 32 : 64;
    const size_t lds = (size_t)64 * ((H + 8) + (KP + 8)) * 2;
    const dim3 grid((unsigned)((M + 63) / 64));
    if (KP == 32)
        hipLaunchKernelGGL((k_decode_bf16<32>), grid, dim3(256), lds, st, M, k, H, D, code, W3, b3,
                           W4, b4, rowmask, y);
    else
        hipLaunchKernelGGL((k_decode_bf16<64>), grid, dim3(256), lds, st, M, k, H, D, code, W3, b3,
                           W4, b4, rowmask, y);
}

void launch_gemm(bool bf16, bool a_bf16, int M, int N, int K, const void* A, int64_t sam,
                 int64_t sak, const float* B, int64_t sbk, int64_t sbn, float* C, int64_t ldc,
                 const GemmEpi& epi, float* part, hipStream_t st)
{
    if (M <= 0 || N <= 0) return;
    int kper = GK;
    const int splits = K > 0 ? gemm_splits(M, N, K, &kper) : 1;
    const dim3 grid((unsigned)((N + GT - 1) / GT), (unsigned)((M + GT - 1) / GT), (unsigned)splits);
    float* out = splits > 1 ? part : C;
#define SLAG_GEMM(BF, TA)                                                                          \
    hipLaunchKernelGGL((k_gemm<BF, TA>), grid, dim3(256), 0, st, M, N, K,                          \
                       reinterpret_cast<const TA*>(A), sam, sak, B, sbk, sbn, kper, out, ldc, epi)
    if (bf16) {
        if (a_bf16) SLAG_GEMM(true, uint16_t);
        else SLAG_GEMM(true, float);
    } else {
        if (a_bf16) SLAG_GEMM(false, uint16_t);
        else SLAG_GEMM(false, float);
    }
#undef SLAG_GEMM
    if (splits > 1)
        hipLaunchKernelGGL(k_gemm_reduce, dim3(blocks((int64_t)M * N)), dim3(256), 0, st, M, N,
                           splits, part, C, ldc, epi);
}

size_t gemm_part_floats(int M, int N, int K)
{
    if (M <= 0 || N <= 0 || K <= 0) return 0;
    int kper;
    const int splits = gemm_splits(M, N, K, &kper);
    return splits > 1 ? (size_t)splits * M * N : 0;
}

void launch_colsum(int R, int N, const float* X, float* out, float* part, hipStream_t st)
{
    if (N <= 0) return;
    const int rows_per = 512;
    const int slices = std::max(1, (R + rows_per - 1) / rows_per);
    hipLaunchKernelGGL(k_colsum_part, dim3(blocks(N), slices), dim3(256), 0, st, R, N, X, rows_per,
                       part);
    hipLaunchKernelGGL(k_colsum_fin, dim3(blocks(N)), dim3(256), 0, st, N, slices, part, out);
}

size_t colsum_part_floats(int R, int N) { return (size_t)std::max(1, (R + 511) / 512) * N; }

void launch_mix(int R, int k, const uint32_t* row_ptr, const uint32_t* col, const float* w,
                const float* C, float* code, hipStream_t st)
{
    if (R <= 0) return;
    hipLaunchKernelGGL(k_mix, dim3(blocks((int64_t)R * k)), dim3(256), 0, st, R, k, row_ptr, col,
                       w, C, code);
}

void launch_mix_bwd(int NS, int k, const uint32_t* rp, int R, int64_t row0, const uint32_t* cbeg,
                    const uint32_t* cend, const uint32_t* csc_j, const uint32_t* csc_row,
                    const float* w, const float* dcode, float* dC, hipStream_t st)
{
    if (NS <= 0) return;
    hipLaunchKernelGGL(k_mix_bwd, dim3(blocks((int64_t)NS * k)), dim3(256), 0, st, NS, k, rp, R,
                       row0, cbeg, cend, csc_j, csc_row, w, dcode, dC);
}

void launch_row_of(uint32_t R, const uint32_t* row_ptr, const uint32_t* col, uint32_t* row_of,
                   uint32_t* key, uint32_t* ent, hipStream_t st)
{
    if (!R) return;
    hipLaunchKernelGGL(k_row_of, dim3(blocks(R)), dim3(256), 0, st, R, row_ptr, row_of, key, ent, col);
}

void launch_csc_ranges(uint32_t nnz, const uint32_t* key, const uint32_t* csc_j,
                       const uint32_t* row_of, uint32_t* cbeg, uint32_t* cend, uint32_t* csc_row,
                       hipStream_t st)
{
    if (!nnz) return;
    hipLaunchKernelGGL(k_csc_ranges, dim3(blocks(nnz)), dim3(256), 0, st, nnz, key, csc_j, row_of,
                       cbeg, cend, csc_row);
}

void launch_cos_loss(int R, int d, const float* y, const float* tg, float* dy, float* loss_part,
                     float* loss, hipStream_t st)
{
    if (R <= 0) return;
    const int nb = (R + 3) / 4;
    const float inv_r = 1.0f / (float)R;
    hipLaunchKernelGGL(k_cos_loss, dim3(nb), dim3(256), 0, st, R, d, y, tg, inv_r, dy, loss_part);
    hipLaunchKernelGGL(k_loss_fin, dim3(1), dim3(256), 0, st, nb, loss_part, inv_r, loss);
}

void launch_adam(int64_t n, float* p, const float* g, float* m, float* v, float lr, float b1,
                 float b2, float eps, int64_t step, hipStream_t st)
{
    if (n <= 0) return;
    const float c1 = 1.0f - (float)std::pow((double)b1, (double)step);
    const float c2 = 1.0f - (float)std::pow((double)b2, (double)step);
    hipLaunchKernelGGL(k_adam, dim3(blocks(n)), dim3(256), 0, st, n, p, g, m, v, lr, b1, b2, eps,
                       c1, c2);
}

void launch_to_f32(int64_t n, const void* src, bool bf16, float* dst, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_to_f32, dim3(blocks(n)), dim3(256), 0, st, n, src, (int)bf16, dst);
}

}  // namespace slag
