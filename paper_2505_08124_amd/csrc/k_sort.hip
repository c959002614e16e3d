// Prefix scans, stable LSD radix sort and the tile binning of visible pairs.
//
// Tile lists must visit Gaussians front to back with ties broken by the
// Gaussian index.  Pairs are compacted in (view, Gaussian) order, sorted
// stably by (view, depth) once, expanded into (tile, pair) entries in that
// order, and sorted stably by tile: each tile list comes out in (depth,
// Gaussian) order without ever sorting the much longer intersection array by
// depth.
#include "slag_internal.h"

namespace slag {

namespace {

constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = 256 * SCAN_ITEMS;   // elements per block
constexpr int RADIX_BITS = 8;
constexpr int RADIX = 1 << RADIX_BITS;
constexpr int RADIX_ITEMS = 16;
constexpr int RADIX_TILE = 256 * RADIX_ITEMS;

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// Loads SCAN_ITEMS consecutive elements of thread t (zero past n).
__device__ __forceinline__ void load_items(const uint32_t* data, uint64_t base, uint64_t n,
                                           uint32_t* v)
{
    if (base + SCAN_ITEMS <= n && (base & 3) == 0) {
        const uint4* p = reinterpret_cast<const uint4*>(data + base);
#pragma unroll
        for (int i = 0; i < SCAN_ITEMS / 4; i++) {
            uint4 q = p[i];
            v[4 * i] = q.x; v[4 * i + 1] = q.y; v[4 * i + 2] = q.z; v[4 * i + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < SCAN_ITEMS; i++) v[i] = (base + i < n) ? data[base + i] : 0u;
    }
}

__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t* __restrict__ data, uint64_t n,
                                                     uint32_t* __restrict__ bsum,
                                                     unsigned long long* total)
{
    __shared__ uint32_t lds[4];
    uint32_t v[SCAN_ITEMS];
    load_items(data, (uint64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS, n, v);
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) s += v[i];
    s = wave_incl_scan(s);
    if ((threadIdx.x & 63) == 63) lds[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = (uint64_t)lds[0] + lds[1] + lds[2] + lds[3];
        bsum[blockIdx.x] = (uint32_t)t;
        if (total) atomicAdd(total, (unsigned long long)t);
    }
}

// Exclusive scan of one tile in place, plus the scanned block offset.
__global__ __launch_bounds__(256) void k_scan_block(uint32_t* __restrict__ data, uint64_t n,
                                                    const uint32_t* __restrict__ boff,
                                                    unsigned long long* total)
{
    __shared__ uint32_t lds[4];
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    load_items(data, base, n, v);
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) s += v[i];
    uint32_t incl = wave_incl_scan(s);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 63) lds[w] = incl;
    __syncthreads();
    uint32_t off = boff ? boff[blockIdx.x] : 0u;
    for (int i = 0; i < w; i++) off += lds[i];
    if (total && threadIdx.x == 0)
        *total = (unsigned long long)lds[0] + lds[1] + lds[2] + lds[3];
    uint32_t run = off + incl - s;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        uint32_t x = v[i];
        if (base + i < n) data[base + i] = run;
        run += x;
    }
}

// ---------------------------------------------------------------- radix sort

template <typename K>
__device__ __forceinline__ uint32_t digit_of(K k, int shift)
{
    return (uint32_t)(k >> shift) & (RADIX - 1);
}

template <typename K>
__global__ __launch_bounds__(256) void k_radix_hist(const K* __restrict__ keys, uint64_t n,
                                                    int shift, uint32_t* __restrict__ hist,
                                                    uint32_t nblk)
{
    __shared__ uint32_t cnt[RADIX];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * RADIX_TILE;
    for (int i = threadIdx.x; i < RADIX_TILE; i += 256) {
        uint64_t idx = base + i;
        if (idx < n) atomicAdd(&cnt[digit_of(keys[idx], shift)], 1u);
    }
    __syncthreads();
    hist[(uint64_t)threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter: within a block, element order is (wave, item, lane) =
// ascending index; equal digits are ranked with ballots, waves in order.
template <typename K>
__global__ __launch_bounds__(256) void k_radix_scatter(const K* __restrict__ kin,
                                                       const uint32_t* __restrict__ vin,
                                                       K* __restrict__ kout,
                                                       uint32_t* __restrict__ vout, uint64_t n,
                                                       int shift,
                                                       const uint32_t* __restrict__ hist,
                                                       uint32_t nblk)
{
    __shared__ uint32_t wcnt[4][RADIX];
    __shared__ uint32_t dbase[RADIX];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = threadIdx.x; i < 4 * RADIX; i += 256) (&wcnt[0][0])[i] = 0;
    dbase[threadIdx.x] = hist[(uint64_t)threadIdx.x * nblk + blockIdx.x];
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint64_t base = (uint64_t)blockIdx.x * RADIX_TILE + (uint64_t)w * (RADIX_ITEMS * 64);
    K key[RADIX_ITEMS];
    uint32_t val[RADIX_ITEMS];
    uint32_t rk[RADIX_ITEMS];
#pragma unroll
    for (int it = 0; it < RADIX_ITEMS; it++) {
        const uint64_t idx = base + it * 64 + lane;
        const bool valid = idx < n;
        key[it] = valid ? kin[idx] : (K)0;
        val[it] = valid ? vin[idx] : 0u;
        const uint32_t d = digit_of(key[it], shift);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < RADIX_BITS; b++) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        uint32_t before = 0;
        if (valid) before = wcnt[w][d];
        const uint32_t r = (uint32_t)__popcll(peers & lt);
        // all lanes have read the running count before the leaders update it
        __builtin_amdgcn_wave_barrier();
        if (valid && r == 0) wcnt[w][d] = before + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
        rk[it] = before + r;
    }
    __syncthreads();
    {
        // exclusive prefix of the per-wave counts, per digit
        const int d = threadIdx.x;
        uint32_t s = 0;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            uint32_t c = wcnt[k][d];
            wcnt[k][d] = s;
            s += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < RADIX_ITEMS; it++) {
        const uint64_t idx = base + it * 64 + lane;
        if (idx < n) {
            const uint32_t d = digit_of(key[it], shift);
            const uint32_t pos = dbase[d] + wcnt[w][d] + rk[it];
            kout[pos] = key[it];
            vout[pos] = val[it];
        }
    }
}

template <typename K>
bool radix_sort(K* keys, uint32_t* vals, K* keys_alt, uint32_t* vals_alt, uint64_t n, int nbits,
                uint32_t* hist, void* ws, uint64_t* tot, hipStream_t st)
{
    if (n <= 1 || nbits <= 0) return false;
    const uint32_t nblk = (uint32_t)((n + RADIX_TILE - 1) / RADIX_TILE);
    K* ka = keys;
    K* kb = keys_alt;
    uint32_t* va = vals;
    uint32_t* vb = vals_alt;
    bool alt = false;
    for (int shift = 0; shift < nbits; shift += RADIX_BITS) {
        hipLaunchKernelGGL(k_radix_hist<K>, dim3(nblk), dim3(256), 0, st, ka, n, shift, hist,
                           nblk);
        scan_u32(hist, (uint64_t)nblk * RADIX, nullptr, ws, st);
        hipLaunchKernelGGL(k_radix_scatter<K>, dim3(nblk), dim3(256), 0, st, ka, va, kb, vb, n,
                           shift, hist, nblk);
        K* tk = ka; ka = kb; kb = tk;
        uint32_t* tv = va; va = vb; vb = tv;
        alt = !alt;
    }
    return alt;
}

// ------------------------------------------------------------- tile binning

__device__ __forceinline__ void box_of(const float4& r1, int& x0, int& x1, int& y0, int& y1)
{
    const uint32_t a = __float_as_uint(r1.z), b = __float_as_uint(r1.w);
    x0 = (int)(a & 0xFFFFu); y0 = (int)(a >> 16);
    x1 = (int)(b & 0xFFFFu); y1 = (int)(b >> 16);
}

__global__ __launch_bounds__(256) void k_rank_tiles(uint64_t npairs, const uint32_t* __restrict__ order,
                                                    const float4* __restrict__ rec,
                                                    uint32_t* __restrict__ tcr)
{
    const uint64_t r = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= npairs) return;
    int x0, x1, y0, y1;
    box_of(rec[2 * (size_t)order[r] + 1], x0, x1, y0, y1);
    tcr[r] = (uint32_t)((x1 / TILE - x0 / TILE + 1) * (y1 / TILE - y0 / TILE + 1));
}

__global__ __launch_bounds__(256) void k_emit_isect(uint64_t npairs, const uint32_t* __restrict__ order,
                                                    const float4* __restrict__ rec,
                                                    const uint16_t* __restrict__ pview,
                                                    const ViewDev* __restrict__ views,
                                                    const uint32_t* __restrict__ ioff,
                                                    uint32_t* __restrict__ ikey,
                                                    uint32_t* __restrict__ ival)
{
    const uint64_t r = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= npairs) return;
    const uint32_t p = order[r];
    int x0, x1, y0, y1;
    box_of(rec[2 * (size_t)p + 1], x0, x1, y0, y1);
    const ViewDev& V = views[pview[p]];
    const uint32_t tb = V.tile_base;
    const int ntx = V.ntx;
    uint32_t o = ioff[r];
    for (int ty = y0 / TILE; ty <= y1 / TILE; ty++)
        for (int tx = x0 / TILE; tx <= x1 / TILE; tx++) {
            ikey[o] = tb + (uint32_t)(ty * ntx + tx);
            ival[o] = p;
            o++;
        }
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * 256)
        p[i] = v;
}

__global__ __launch_bounds__(256) void k_bucket_ranges(uint64_t ni, const uint32_t* __restrict__ ikey,
                                                       uint32_t* __restrict__ bstart,
                                                       uint32_t* __restrict__ bend)
{
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= ni) return;
    const uint32_t k = ikey[i];
    if (i == 0 || ikey[i - 1] != k) bstart[k] = (uint32_t)i;
    if (i + 1 == ni || ikey[i + 1] != k) bend[k] = (uint32_t)(i + 1);
}

inline unsigned grid_for(uint64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

size_t scan_workspace_bytes(uint64_t n)
{
    size_t words = 0;
    uint64_t m = n;
    while (m > (uint64_t)SCAN_TILE) {
        m = (m + SCAN_TILE - 1) / SCAN_TILE;
        words += (m + 3) & ~3ull;
    }
    return (words + 4) * sizeof(uint32_t);
}

void scan_u32(uint32_t* data, uint64_t n, uint64_t* total_dev, void* ws, hipStream_t st)
{
    auto* tot = reinterpret_cast<unsigned long long*>(total_dev);
    if (n == 0) {
        if (tot) launch_fill_u32(reinterpret_cast<uint32_t*>(tot), 2, 0u, st);
        return;
    }
    const uint64_t nblk = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nblk == 1) {
        hipLaunchKernelGGL(k_scan_block, dim3(1), dim3(256), 0, st, data, n, (const uint32_t*)nullptr,
                           tot);
        return;
    }
    uint32_t* bsum = reinterpret_cast<uint32_t*>(ws);
    uint32_t* next = bsum + ((nblk + 3) & ~3ull);
    if (tot) launch_fill_u32(reinterpret_cast<uint32_t*>(tot), 2, 0u, st);
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nblk), dim3(256), 0, st, data, n, bsum, tot);
    scan_u32(bsum, nblk, nullptr, next, st);
    hipLaunchKernelGGL(k_scan_block, dim3((unsigned)nblk), dim3(256), 0, st, data, n, bsum,
                       (unsigned long long*)nullptr);
}

size_t radix_hist_bytes(uint64_t n)
{
    return ((n + RADIX_TILE - 1) / RADIX_TILE) * RADIX * sizeof(uint32_t) + 256;
}

bool radix_sort_u64(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
                    uint64_t n, int nbits, uint32_t* hist, void* scan_ws, uint64_t* tot,
                    hipStream_t st)
{
    return radix_sort<uint64_t>(keys, vals, keys_alt, vals_alt, n, nbits, hist, scan_ws, tot, st);
}

bool radix_sort_u32(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                    uint64_t n, int nbits, uint32_t* hist, void* scan_ws, uint64_t* tot,
                    hipStream_t st)
{
    return radix_sort<uint32_t>(keys, vals, keys_alt, vals_alt, n, nbits, hist, scan_ws, tot, st);
}

void launch_rank_tiles(uint64_t npairs, const uint32_t* order, const float4* rec, uint32_t* tcr,
                       hipStream_t st)
{
    if (!npairs) return;
    hipLaunchKernelGGL(k_rank_tiles, dim3(grid_for(npairs)), dim3(256), 0, st, npairs, order, rec,
                       tcr);
}

void launch_emit_isect(uint64_t npairs, const uint32_t* order, const float4* rec,
                       const uint16_t* pview, const ViewDev* views, const uint32_t* ioff,
                       uint32_t* ikey, uint32_t* ival, hipStream_t st)
{
    if (!npairs) return;
    hipLaunchKernelGGL(k_emit_isect, dim3(grid_for(npairs)), dim3(256), 0, st, npairs, order, rec,
                       pview, views, ioff, ikey, ival);
}

void launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t st)
{
    if (!n) return;
    uint64_t g = grid_for(n);
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)g), dim3(256), 0, st, p, n, v);
}

void launch_bucket_ranges(uint64_t ni, const uint32_t* ikey, uint32_t* bstart, uint32_t* bend,
                          hipStream_t st)
{
    if (!ni) return;
    hipLaunchKernelGGL(k_bucket_ranges, dim3(grid_for(ni)), dim3(256), 0, st, ni, ikey, bstart,
                       bend);
}

}  // namespace slag
