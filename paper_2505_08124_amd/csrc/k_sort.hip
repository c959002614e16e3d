// Prefix scans, stable LSD radix sort and the tile binning of visible pairs.
//
// Tile lists must visit Gaussians front to back with ties broken by the
// caller's Gaussian index.  Pairs are compacted in (view, Morton rank) order,
// sorted stably by (view, depth) once, runs of equal depth are put in the
// caller's index order (the tie pass below), the pairs are expanded into
// (tile, pair) entries in that order, and the entries are sorted stably by
// tile: each tile list comes out in (depth, Gaussian index) order without
// ever sorting the much longer intersection array by depth.
#include "slag_internal.h"

namespace slag {

namespace {

constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = 256 * SCAN_ITEMS;   // elements per block

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

// Scans move their tiles through LDS: global loads and stores are striped
// (element t + 256 i of the tile for thread t: one coalesced row per
// instruction), the scan itself runs over SCAN_ITEMS consecutive elements
// per thread.  One pad word per 16 keeps both LDS access patterns free of
// bank conflicts.
__device__ __forceinline__ int spad(int f) { return f + (f >> 4); }
constexpr int SCAN_LDS = SCAN_TILE + SCAN_TILE / 16;

__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t* __restrict__ data, uint64_t n,
                                                     uint32_t* __restrict__ bsum,
                                                     unsigned long long* total)
{
    __shared__ uint32_t lds[4];
    const uint64_t b0 = (uint64_t)blockIdx.x * SCAN_TILE;
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        const uint64_t x = b0 + threadIdx.x + 256 * i;
        s += x < n ? data[x] : 0u;
    }
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
    __shared__ uint32_t tile[SCAN_LDS];
    const int t = threadIdx.x;
    const uint64_t b0 = (uint64_t)blockIdx.x * SCAN_TILE;
    uint32_t ld[SCAN_ITEMS];   // all loads in flight before the first LDS store
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        const uint64_t x = b0 + t + 256 * i;
        ld[i] = x < n ? data[x] : 0u;
    }
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) tile[spad(t + 256 * i)] = ld[i];
    __syncthreads();
    uint32_t v[SCAN_ITEMS];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        v[i] = tile[spad(t * SCAN_ITEMS + i)];
        s += v[i];
    }
    uint32_t incl = wave_incl_scan(s);
    const int w = t >> 6;
    if ((t & 63) == 63) lds[w] = incl;
    __syncthreads();
    uint32_t off = boff ? boff[blockIdx.x] : 0u;
    for (int i = 0; i < w; i++) off += lds[i];
    if (total && t == 0)
        *total = (unsigned long long)lds[0] + lds[1] + lds[2] + lds[3];
    uint32_t run = off + incl - s;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        tile[spad(t * SCAN_ITEMS + i)] = run;
        run += v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        const uint64_t x = b0 + t + 256 * i;
        if (x < n) data[x] = tile[spad(t + 256 * i)];
    }
}

// ---------------------------------------------------------------- radix sort
//
// One pass sorts by a digit of up to 8 bits.  Block tile: 4 waves x ITEMS
// items x 64 lanes; element order inside a block is (wave, item, lane) = ascending index,
// so ranking equal digits with ballots, wave by wave, keeps the sort stable.
// Elements are regrouped by digit in LDS before the global write, so each
// digit's run leaves the block as consecutive addresses.  An optional second
// value array rides along.

// Items per thread: 32 (8192-element blocks) for passes of 6 bits or more,
// whose many digits need long blocks to keep runs of equal digits long;
// 16 below that.  Bare 64-bit keys take 32 only in long sorts (at least
// RADIX_LONG keys): their blocks hold 64 KB of LDS, two per CU, and a
// sort of a few thousand such blocks ran faster with the smaller ones
// (measured at 2e7 keys; 3e8 keys gained from the larger).
constexpr int RADIX_ITEMS_MIN = 16;
constexpr int RADIX_TILE_MIN = 256 * RADIX_ITEMS_MIN;
constexpr int RADIX_MAXBITS = 8;
constexpr uint64_t RADIX_LONG = 1ull << 25;
constexpr int NXCD = 8;   // XCDs of the chip; workgroups are dealt to them round-robin
template <typename K, int RB, int NV>
constexpr int radix_items(bool long_sort)
{
    return (RB >= 6 && (long_sort || !(sizeof(K) == 8 && NV == 0))) ? 32 : 16;
}

// One wave counts one sort block (256 * ITEMS keys, 4 * ITEMS coalesced
// loads per lane, in flight 32 or 64 at a time), so a workgroup covers four
// blocks and each wave writes its own column of the (digit, block) matrix.
template <typename K, int RB, int ITEMS>
__global__ __launch_bounds__(256) void k_radix_hist(const K* __restrict__ keys, uint64_t n,
                                                    int shift, uint32_t* __restrict__ hist,
                                                    uint32_t nblk)
{
    // per-wave counts in LDS: one add when a wave's items share a digit
    // (common for the high digits), else one LDS atomic per item
    constexpr int R = 1 << RB;
    constexpr int TILE_N = 256 * ITEMS;
    constexpr int PER = TILE_N / 64;
    __shared__ uint32_t cnt[4][R];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = threadIdx.x; i < 4 * R; i += 256) (&cnt[0][0])[i] = 0;
    __syncthreads();
    const uint64_t sb = (uint64_t)blockIdx.x * 4 + w;
    if (sb < nblk) {
        constexpr int CH = PER > 64 ? 32 : PER;   // keys held in registers at once
        for (int c0 = 0; c0 < PER; c0 += CH) {
        const uint64_t base = sb * TILE_N + lane + (uint64_t)c0 * 64;
        K k[CH];
#pragma unroll
        for (int it = 0; it < CH; it++) {
            const uint64_t idx = base + (uint64_t)it * 64;
            k[it] = idx < n ? keys[idx] : (K)0;
        }
#pragma unroll
        for (int it = 0; it < CH; it++) {
            const bool valid = base + (uint64_t)it * 64 < n;
            const uint32_t d = (uint32_t)(k[it] >> shift) & (R - 1);
            // all valid lanes on one digit: the first adds them; else LDS atomics
            const uint32_t d0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)d);
            const uint64_t vm = __ballot(valid);
            if (__ballot(valid && d != d0) == 0) {
                if (lane == 0 && vm) cnt[w][d0] += (uint32_t)__popcll(vm);
            } else if (valid) {
                atomicAdd(&cnt[w][d], 1u);
            }
            __builtin_amdgcn_wave_barrier();
        }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 4 * R; i += 256) {
        const uint64_t b = (uint64_t)blockIdx.x * 4 + i / R;
        if (b < nblk) hist[(uint64_t)(i % R) * nblk + b] = cnt[i / R][i % R];
    }
}

template <typename K, int RB, int NV, int ITEMS>
__global__ __launch_bounds__(256) void k_radix_scatter(const K* __restrict__ kin,
                                                       const uint32_t* __restrict__ vin,
                                                       const uint32_t* __restrict__ uin,
                                                       K* __restrict__ kout,
                                                       uint32_t* __restrict__ vout,
                                                       uint32_t* __restrict__ uout, uint64_t n,
                                                       int shift,
                                                       const uint32_t* __restrict__ hist,
                                                       uint32_t nblk)
{
    constexpr int R = 1 << RB;
    constexpr int TILE_N = 256 * ITEMS;
    __shared__ uint32_t wcnt[4][R];
    __shared__ uint32_t dbase[R];     // global start of each digit for this block
    __shared__ uint32_t lbase[R];     // block-local start of each digit
    __shared__ uint32_t tmp[8];
    __shared__ K s_key[TILE_N];
    __shared__ uint32_t s_val[NV >= 1 ? TILE_N : 1];
    __shared__ uint32_t s_aux[NV >= 2 ? TILE_N : 1];
    // XCD-aware block order: the grid is a multiple of NXCD blocks and XCD x
    // (workgroups are dealt round-robin) takes logical blocks x * per ..
    // (x + 1) * per - 1, so neighbouring blocks, whose digit runs meet in
    // shared cache lines, write them through the same L2
    const uint32_t per = gridDim.x / NXCD;
    const uint32_t lb = (blockIdx.x % NXCD) * per + blockIdx.x / NXCD;
    if (lb >= nblk) return;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint64_t bbase = (uint64_t)lb * TILE_N;
    const uint64_t base = bbase + (uint64_t)w * (ITEMS * 64);
    const int nvalid = (int)min((uint64_t)TILE_N, n - bbase);
    K key[ITEMS];
    uint32_t val[NV >= 1 ? ITEMS : 1];
    uint32_t aux[NV >= 2 ? ITEMS : 1];
    uint32_t rk[ITEMS];
    // every load of the block is issued before the first is used (the
    // ranking below has wave barriers, which keep loads from moving past them)
#pragma unroll
    for (int it = 0; it < ITEMS; it++) {
        const uint64_t idx = base + it * 64 + lane;
        const bool valid = idx < n;
        key[it] = valid ? kin[idx] : (K)0;
        if constexpr (NV >= 1) val[it] = valid ? vin[idx] : 0u;
        if constexpr (NV >= 2) aux[it] = valid ? uin[idx] : 0u;
    }
    for (int i = threadIdx.x; i < 4 * R; i += 256) (&wcnt[0][0])[i] = 0;
    for (int i = threadIdx.x; i < R; i += 256) dbase[i] = hist[(uint64_t)i * nblk + lb];
    __syncthreads();
#pragma unroll
    for (int it = 0; it < ITEMS; it++) {
        const uint64_t idx = base + it * 64 + lane;
        const bool valid = idx < n;
        const uint32_t d = (uint32_t)(key[it] >> shift) & (R - 1);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < RB; b++) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        uint32_t before = 0;
        if (valid) before = wcnt[w][d];
        const uint32_t r = (uint32_t)__popcll(peers & lt);
        // every lane has read the running count before the leaders update it
        __builtin_amdgcn_wave_barrier();
        if (valid && r == 0) wcnt[w][d] = before + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
        rk[it] = before + r;
    }
    __syncthreads();
    // per digit: exclusive prefix over waves, and the block total
    constexpr int NQ = (R + 255) / 256;
    uint32_t dtot[NQ];
#pragma unroll
    for (int q = 0; q < NQ; q++) {
        const int d = threadIdx.x + 256 * q;
        uint32_t s = 0;
        if (d < R) {
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const uint32_t c = wcnt[k][d];
                wcnt[k][d] = s;
                s += c;
            }
        }
        dtot[q] = s;
    }
    // block-local digit starts: exclusive scan of the totals over digits
    {
        uint32_t run = 0;
#pragma unroll
        for (int q = 0; q < NQ; q++) {
            // digits q*256 .. q*256+255 are owned by threads 0..255 in order
            uint32_t x = dtot[q], v = x;
#pragma unroll
            for (int dd = 1; dd < 64; dd <<= 1) {
                const uint32_t y = __shfl_up(v, dd, 64);
                if (lane >= dd) v += y;
            }
            if (lane == 63) tmp[w] = v;
            __syncthreads();
            uint32_t off = run;
            for (int i = 0; i < w; i++) off += tmp[i];
            if (threadIdx.x + 256 * q < R) lbase[threadIdx.x + 256 * q] = off + v - x;
            run += tmp[0] + tmp[1] + tmp[2] + tmp[3];
            __syncthreads();
        }
    }
    __syncthreads();
    // reorder through LDS so that equal digits sit together ...
#pragma unroll
    for (int it = 0; it < ITEMS; it++) {
        const uint64_t idx = base + it * 64 + lane;
        if (idx < n) {
            const uint32_t d = (uint32_t)(key[it] >> shift) & (R - 1);
            const uint32_t lp = lbase[d] + wcnt[w][d] + rk[it];
            s_key[lp] = key[it];
            if constexpr (NV >= 1) s_val[lp] = val[it];
            if constexpr (NV >= 2) s_aux[lp] = aux[it];
        }
    }
    __syncthreads();
    // ... and write them out in runs: consecutive threads, consecutive addresses
    for (int lp = threadIdx.x; lp < nvalid; lp += 256) {
        const K k = s_key[lp];
        const uint32_t d = (uint32_t)(k >> shift) & (R - 1);
        const uint32_t pos = dbase[d] + (uint32_t)lp - lbase[d];
        kout[pos] = k;
        if constexpr (NV >= 1) vout[pos] = s_val[lp];
        if constexpr (NV >= 2) uout[pos] = s_aux[lp];
    }
}

template <typename K, int RB, int NV, int ITEMS>
void radix_pass_items(const K* ka, const uint32_t* va, const uint32_t* ua, K* kb, uint32_t* vb,
                      uint32_t* ub, uint64_t n, int shift, uint32_t* hist, void* ws, hipStream_t st)
{
    constexpr int TILE_N = 256 * ITEMS;
    const uint32_t nblk = (uint32_t)((n + TILE_N - 1) / TILE_N);
    hipLaunchKernelGGL((k_radix_hist<K, RB, ITEMS>), dim3((nblk + 3) / 4), dim3(256), 0, st, ka, n,
                       shift, hist, nblk);
    scan_u32(hist, (uint64_t)nblk << RB, nullptr, ws, st);
    const uint32_t grid = (nblk + NXCD - 1) / NXCD * NXCD;   // whole rounds over the XCDs
    hipLaunchKernelGGL((k_radix_scatter<K, RB, NV, ITEMS>), dim3(grid), dim3(256), 0, st, ka, va, ua,
                       kb, vb, ub, n, shift, hist, nblk);
}

template <typename K, int RB, int NV>
void radix_pass(const K* ka, const uint32_t* va, const uint32_t* ua, K* kb, uint32_t* vb,
                uint32_t* ub, uint64_t n, int shift, uint32_t* hist, void* ws, hipStream_t st)
{
    constexpr int IS = radix_items<K, RB, NV>(false), IL = radix_items<K, RB, NV>(true);
    if (IL != IS && n >= RADIX_LONG)
        radix_pass_items<K, RB, NV, IL>(ka, va, ua, kb, vb, ub, n, shift, hist, ws, st);
    else
        radix_pass_items<K, RB, NV, IS>(ka, va, ua, kb, vb, ub, n, shift, hist, ws, st);
}

// Stable LSD sort of (key[, value[, aux]]) by bits [bit0, bit0 + nbits): the
// fewest passes of at most 8 bits, the bits split evenly over them (fewer
// digits per pass give longer runs of equal digits, so fuller write lines).
template <typename K, int NV>
bool radix_sort(K* keys, uint32_t* vals, uint32_t* aux, K* keys_alt, uint32_t* vals_alt,
                uint32_t* aux_alt, uint64_t n, int bit0, int nbits, uint32_t* hist, void* ws,
                hipStream_t st)
{
    if (n <= 1 || nbits <= 0) return false;
    const int passes = (nbits + RADIX_MAXBITS - 1) / RADIX_MAXBITS;
    const int rb = (nbits + passes - 1) / passes;
    K* ka = keys;
    K* kb = keys_alt;
    uint32_t *va = vals, *vb = vals_alt, *ua = aux, *ub = aux_alt;
    bool alt = false;
    for (int shift = bit0; shift < bit0 + nbits; shift += rb) {
        switch (rb) {
        case 1: radix_pass<K, 1, NV>(ka, va, ua, kb, vb, ub, n, shift, hist, ws, st); break;
        case 2: radix_pass<K, 2, NV>(ka, va, ua, kb, vb, ub, n, shift, hist, ws, st); break;
        case 3: radix_pass<K, 3, NV>(ka, va, ua, kb, vb, ub, n, shift, hist, ws, st); break;
        case 4: radix_pass<K, 4, NV>(ka, va, ua, kb, vb, ub, n, shift, hist, ws, st); break;
        case 5: radix_pass<K, 5, NV>(ka, va, ua, kb, vb, ub, n, shift, hist, ws, st); break;
        case 6: radix_pass<K, 6, NV>(ka, va, ua, kb, vb, ub, n, shift, hist, ws, st); break;
        case 7: radix_pass<K, 7, NV>(ka, va, ua, kb, vb, ub, n, shift, hist, ws, st); break;
        default: radix_pass<K, 8, NV>(ka, va, ua, kb, vb, ub, n, shift, hist, ws, st); break;
        }
        K* tk = ka; ka = kb; kb = tk;
        uint32_t* tv = va; va = vb; vb = tv;
        uint32_t* tu = ua; ua = ub; ub = tu;
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

// The depth order is either a pair-index array or, packed, the low bits of
// the sorted 64-bit depth keys.
__device__ __forceinline__ uint32_t pair_at_rank(const uint32_t* __restrict__ order,
                                                 const uint64_t* __restrict__ okey, uint64_t pmask,
                                                 uint64_t r)
{
    return okey ? (uint32_t)(okey[r] & pmask) : order[r];
}

// Four ranks per thread (strided by 256, coalesced): the four depth-order
// loads, then the four rectangle gathers, each group in flight together
// (clamped indices, so no branch separates them).  Workgroups go to the
// eight XCDs round-robin; XCD x is given the x-th eighth of the ranks, in
// order, so its gathers stay within about one view's records at a time
// (a view's pairs are contiguous in depth order and their records fit its
// L2), instead of every XCD touching every view.
constexpr int RANK_ITEMS = 4;

__global__ __launch_bounds__(256) void k_rank_tiles(uint64_t npairs, const uint32_t* __restrict__ order,
                                                    const uint64_t* __restrict__ okey, uint64_t pmask,
                                                    const uint2* __restrict__ prect,
                                                    uint32_t* __restrict__ tcr,
                                                    uint2* __restrict__ prank)
{
    // the grid is a multiple of NXCD blocks: b -> (b % NXCD) * per + b / NXCD
    // is a permutation of [0, gridDim.x)
    const uint32_t per = gridDim.x / NXCD;
    const uint32_t lb = (blockIdx.x % NXCD) * per + blockIdx.x / NXCD;
    const uint64_t r0 = (uint64_t)lb * (256 * RANK_ITEMS) + threadIdx.x;
    if (r0 - threadIdx.x >= npairs) return;
    uint32_t p[RANK_ITEMS];
    if (okey) {
#pragma unroll
        for (int i = 0; i < RANK_ITEMS; i++) {
            const uint64_t r = r0 + 256 * i;
            p[i] = (uint32_t)(okey[r < npairs ? r : npairs - 1] & pmask);
        }
    } else {
#pragma unroll
        for (int i = 0; i < RANK_ITEMS; i++) {
            const uint64_t r = r0 + 256 * i;
            p[i] = order[r < npairs ? r : npairs - 1];
        }
    }
    uint2 q[RANK_ITEMS];
#pragma unroll
    for (int i = 0; i < RANK_ITEMS; i++) q[i] = prect[p[i]];
#pragma unroll
    for (int i = 0; i < RANK_ITEMS; i++) {
        const uint64_t r = r0 + 256 * i;
        if (r < npairs) {
            tcr[r] = (q[i].y & 0xFFFFu) * (q[i].y >> 16);
            prank[r] = q[i];   // the rectangle in depth order, for the emission
        }
    }
}

// (tile, pair) entries of every pair in depth order, tiles of a
// pair in row-major order; the tile key is (view in launch << lbits) | tile in
// view.  Pairs come view-major, so a stable sort on the low lbits alone
// leaves each (view, tile) list contiguous and in depth order.  A wave emits the consecutive output range of its 64 pairs
// together: output slot e finds its pair among the wave's 64 offsets, so the
// stores are coalesced.
__global__ __launch_bounds__(256) void k_emit_isect(uint64_t npairs, const uint32_t* __restrict__ order,
                                                    const uint64_t* __restrict__ okey, uint64_t pmask,
                                                    const uint2* __restrict__ prank,
                                                    const ViewDev* __restrict__ views,
                                                    const uint32_t* __restrict__ ioff,
                                                    int lbits,
                                                    uint32_t* __restrict__ ikey,
                                                    uint32_t* __restrict__ ival)
{
    __shared__ uint32_t s_off[4][65];
    __shared__ uint32_t s_p[4][64];
    __shared__ uint32_t s_r[4][64][3];   // tile key base, tiles per row of the rect, ntx
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t r0 = (uint64_t)blockIdx.x * 256 + (uint64_t)w * 64;
    if (r0 >= npairs) return;
    const uint64_t r = r0 + lane;
    const int nw = (int)min((uint64_t)64, npairs - r0);
    uint32_t o = 0, tc = 0;
    // clamped loads, all three in flight together
    const uint64_t rc = lane < nw ? r : r0;
    const uint2 ql = prank[rc];
    const uint32_t ol = ioff[rc];
    const uint32_t pl = okey ? (uint32_t)(okey[rc] & pmask) : order[rc];
    if (lane < nw) {
        const uint32_t p = pl;
        const uint2 q = ql;
        o = ol;
        tc = (q.y & 0xFFFFu) * (q.y >> 16);
        s_p[w][lane] = p;
        s_r[w][lane][0] = q.x;
        s_r[w][lane][1] = q.y & 0xFFFFu;
        s_r[w][lane][2] = (uint32_t)views[q.x >> lbits].ntx;
        s_off[w][lane] = o;
    }
    const uint32_t o0 = __builtin_amdgcn_readfirstlane(o);
    const uint32_t last_end = (uint32_t)__builtin_amdgcn_readlane((int)(o + tc), nw - 1);
    if (lane == 0) s_off[w][nw] = last_end;
    __builtin_amdgcn_wave_barrier();
    for (uint32_t e = o0 + lane; e < last_end; e += 64) {
        // the pair owning slot e: largest j with s_off[j] <= e
        int lo = 0, hi = nw - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_off[w][mid] <= e) lo = mid; else hi = mid - 1;
        }
        const uint32_t k = e - s_off[w][lo];
        const uint32_t rw = s_r[w][lo][1], ntx = s_r[w][lo][2];
        const uint32_t dy = k / rw, dx = k % rw;
        ikey[e] = s_r[w][lo][0] + dy * ntx + dx;
        ival[e] = s_p[w][lo];
    }
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * 256)
        p[i] = v;
}

// Keys are (view in launch << lbits) | tile in view; bucket = the view's tile
// base + tile.  Four consecutive keys per thread (one 16-byte load) and
// their two outer neighbours; a run's first and last positions set its range.
__global__ __launch_bounds__(256) void k_bucket_ranges(uint64_t ni, const uint32_t* __restrict__ ikey,
                                                       const ViewDev* __restrict__ views, int lbits,
                                                       uint32_t* __restrict__ bstart,
                                                       uint32_t* __restrict__ bend)
{
    const uint64_t i0 = ((uint64_t)blockIdx.x * 256 + threadIdx.x) * 4;
    if (i0 >= ni) return;
    uint32_t k[4];
    if (i0 + 4 <= ni) {
        const uint4 q = reinterpret_cast<const uint4*>(ikey)[i0 >> 2];
        k[0] = q.x; k[1] = q.y; k[2] = q.z; k[3] = q.w;
    } else {
#pragma unroll
        for (int j = 0; j < 4; j++) k[j] = i0 + j < ni ? ikey[i0 + j] : 0u;
    }
    const uint32_t prev = i0 > 0 ? ikey[i0 - 1] : 0u, next = i0 + 4 < ni ? ikey[i0 + 4] : 0u;
    const uint32_t lmask = (1u << lbits) - 1u;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const uint64_t i = i0 + j;
        if (i >= ni) break;
        const bool first = i == 0 || (j == 0 ? prev : k[j - 1]) != k[j];
        const bool lastk = i + 1 == ni || (j == 3 ? next : k[j + 1]) != k[j];
        if (!first && !lastk) continue;
        const uint32_t b = views[k[j] >> lbits].tile_base + (k[j] & lmask);
        if (first) bstart[b] = (uint32_t)i;
        if (lastk) bend[b] = (uint32_t)(i + 1);
    }
}

// Dispatch-order keys: longer tile lists first (key = 0xFFFF - min(len, 0xFFFF)
// sorts ascending into descending length; equal keys keep tile order).
__global__ __launch_bounds__(256) void k_bucket_keys(uint32_t nb,
                                                     const uint32_t* __restrict__ bucket_view,
                                                     const uint8_t* __restrict__ view_cls,
                                                     const uint32_t* __restrict__ bstart,
                                                     const uint32_t* __restrict__ bend,
                                                     uint32_t* __restrict__ key,
                                                     uint32_t* __restrict__ val)
{
    const uint32_t b = blockIdx.x * 256 + threadIdx.x;
    if (b >= nb) return;
    const uint32_t len = bend[b] - bstart[b];
    const uint32_t cls = view_cls ? (uint32_t)view_cls[bucket_view[b]] : 0u;
    key[b] = (cls << 16) | (0xFFFFu - min(len, 0xFFFFu));
    val[b] = b;
}

// Depth order from keys that carry each pair's index within its view.
__global__ __launch_bounds__(256) void k_pairs_from_keys(uint64_t npairs,
                                                         const uint64_t* __restrict__ keys,
                                                         int vshift, uint64_t pmask,
                                                         const uint32_t* __restrict__ blk_off,
                                                         int cbv, uint32_t* __restrict__ order)
{
    for (uint64_t r = (uint64_t)blockIdx.x * 256 + threadIdx.x; r < npairs;
         r += (uint64_t)gridDim.x * 256) {
        const uint64_t k = keys[r];
        const uint64_t v = k >> vshift;
        order[r] = blk_off[v * (uint64_t)cbv] + (uint32_t)(k & pmask);
    }
}

// ----------------------------------------------------------- depth ties
//
// After the depth sort, pairs of one view with bitwise-equal depth keep the
// order of their pair indices, i.e. of the Morton order the Gaussians are
// stored in; the depth order breaks such ties by the caller's Gaussian index
// instead.  Exact FP32 depth ties are frequent in large scenes (mostly
// pairs and triples), and a run can be as long as a view (a plane facing the
// camera).  Runs of up to TIE_SHORT pairs are sorted in registers by the
// thread at their head; longer ones are compacted, sorted by (run, Gaussian
// index) with the radix sort and written back into their positions.
// hi(i) = keys[i] >> shift is the key without its pair field; only the pair
// field (or order[]) is ever rewritten, so concurrent readers of hi see
// unchanged values.

constexpr int TIE_SHORT = 8;

__device__ __forceinline__ uint64_t tie_hi(const uint64_t* __restrict__ keys, int shift, uint64_t i)
{
    return keys[i] >> shift;
}

// Is position i inside a run of more than TIE_SHORT equal keys?  (Some window
// of TIE_SHORT + 1 consecutive positions around i has equal ends.)
__device__ __forceinline__ bool in_long_run(const uint64_t* __restrict__ keys, int shift,
                                            uint64_t n, uint64_t i)
{
    const uint64_t h = tie_hi(keys, shift, i);
    const bool nb = (i > 0 && tie_hi(keys, shift, i - 1) == h) ||
                    (i + 1 < n && tie_hi(keys, shift, i + 1) == h);
    if (!nb) return false;
    for (uint64_t a = 0; a <= (uint64_t)TIE_SHORT; a++) {
        if (a > i || i - a + TIE_SHORT >= n) continue;
        if (tie_hi(keys, shift, i - a) == h && tie_hi(keys, shift, i - a + TIE_SHORT) == h)
            return true;
    }
    return false;
}

__device__ __forceinline__ uint32_t pair_of(const uint64_t* __restrict__ keys,
                                            const uint32_t* __restrict__ order, uint64_t pmask,
                                            uint64_t i)
{
    return order ? order[i] : (uint32_t)(keys[i] & pmask);
}

__device__ __forceinline__ void cmp_swap(uint32_t& ga, uint32_t& pa, uint32_t& gb, uint32_t& pb)
{
    const bool sw = ga > gb;
    const uint32_t g0 = sw ? gb : ga, g1 = sw ? ga : gb;
    const uint32_t p0 = sw ? pb : pa, p1 = sw ? pa : pb;
    ga = g0; gb = g1; pa = p0; pb = p1;
}

// Short runs sorted by their head thread; positions in long runs counted
// into *nlong.  A block covers TIE_BLOCK positions, four per thread (strided,
// so global accesses stay coalesced); its keys and TIE_SHORT on each side are
// staged in LDS once, all loads in flight together.  A tied position reads its
// window of 2 TIE_SHORT + 1 keys there (the window decides both the long-run
// test and the run's extent); a head then loads its pairs' Gaussian indices
// at once and sorts them with a fixed 19-comparator network (padding sorts
// last).  Writes change only pair fields, so other blocks' halo copies keep
// valid depths, and a run has one head, so no two threads write one position.
constexpr int TIE_BLOCK = 1024;

__global__ __launch_bounds__(256) void k_tie_short(uint64_t n, uint64_t* __restrict__ keys, int shift,
                                                   uint32_t* __restrict__ order, uint64_t pmask,
                                                   const uint32_t* __restrict__ gidx,
                                                   unsigned long long* __restrict__ nlong)
{
    static_assert(TIE_SHORT == 8, "the sorting network is for 8 entries");
    constexpr int WN = 2 * TIE_SHORT + 1;
    constexpr int SN = TIE_BLOCK + 2 * TIE_SHORT;
    constexpr int NL = (SN + 255) / 256;
    __shared__ uint64_t sk[SN];          // keys b0 - TIE_SHORT .. b0 + TIE_BLOCK + TIE_SHORT
    __shared__ uint32_t wl[4];
    const uint64_t b0 = (uint64_t)blockIdx.x * TIE_BLOCK;
    uint64_t ld[NL];
#pragma unroll
    for (int j = 0; j < NL; j++) {
        const int a = threadIdx.x + 256 * j;
        const int64_t x = (int64_t)b0 - TIE_SHORT + a;
        ld[j] = (a < SN && x >= 0 && (uint64_t)x < n) ? keys[x] : 0ull;
    }
#pragma unroll
    for (int j = 0; j < NL; j++) {
        const int a = threadIdx.x + 256 * j;
        if (a < SN) sk[a] = ld[j];
    }
    __syncthreads();
    uint32_t nlng = 0;
#pragma unroll 1
    for (int k = 0; k < TIE_BLOCK / 256; k++) {
        const int lo = threadIdx.x + 256 * k;
        const uint64_t i = b0 + lo;
        const int li = lo + TIE_SHORT;   // i's slot in sk
        if (i >= n) break;
        const uint64_t h = sk[li] >> shift;
        const bool tp = i > 0 && (sk[li - 1] >> shift) == h;
        const bool tn = i + 1 < n && (sk[li + 1] >> shift) == h;
        if (!(tp || tn)) continue;
        bool eq[WN];
#pragma unroll
        for (int a = 0; a < WN; a++) {
            const int64_t x = (int64_t)i - TIE_SHORT + a;
            eq[a] = x >= 0 && (uint64_t)x < n && (sk[li - TIE_SHORT + a] >> shift) == h;
        }
        bool lng = false;
#pragma unroll
        for (int a = 0; a <= TIE_SHORT; a++) lng = lng || (eq[TIE_SHORT - a] && eq[WN - 1 - a]);
        nlng += lng;
        if (tp || lng) continue;
        // head of a short run: positions i .. i + len - 1, len <= 8
        uint32_t pv[TIE_SHORT], gv[TIE_SHORT];
#pragma unroll
        for (int a = 0; a < TIE_SHORT; a++) {
            const bool in = eq[TIE_SHORT + a];
            // positions past the run take the head's pair: their Gaussian
            // index is not used, and the head's is already being loaded
            pv[a] = order ? order[in ? i + a : i] : (uint32_t)(sk[li + (in ? a : 0)] & pmask);
        }
#pragma unroll
        for (int a = 0; a < TIE_SHORT; a++) {
            const uint32_t g = gidx[pv[a]];
            gv[a] = eq[TIE_SHORT + a] ? g : 0xFFFFFFFFu;
        }
        cmp_swap(gv[0], pv[0], gv[1], pv[1]); cmp_swap(gv[2], pv[2], gv[3], pv[3]);
        cmp_swap(gv[4], pv[4], gv[5], pv[5]); cmp_swap(gv[6], pv[6], gv[7], pv[7]);
        cmp_swap(gv[0], pv[0], gv[2], pv[2]); cmp_swap(gv[1], pv[1], gv[3], pv[3]);
        cmp_swap(gv[4], pv[4], gv[6], pv[6]); cmp_swap(gv[5], pv[5], gv[7], pv[7]);
        cmp_swap(gv[1], pv[1], gv[2], pv[2]); cmp_swap(gv[5], pv[5], gv[6], pv[6]);
        cmp_swap(gv[0], pv[0], gv[4], pv[4]); cmp_swap(gv[1], pv[1], gv[5], pv[5]);
        cmp_swap(gv[2], pv[2], gv[6], pv[6]); cmp_swap(gv[3], pv[3], gv[7], pv[7]);
        cmp_swap(gv[2], pv[2], gv[4], pv[4]); cmp_swap(gv[3], pv[3], gv[5], pv[5]);
        cmp_swap(gv[1], pv[1], gv[2], pv[2]); cmp_swap(gv[3], pv[3], gv[4], pv[4]);
        cmp_swap(gv[5], pv[5], gv[6], pv[6]);
#pragma unroll
        for (int a = 0; a < TIE_SHORT; a++) {
            if (!eq[TIE_SHORT + a]) continue;
            if (order) order[i + a] = pv[a];
            else keys[i + a] = (sk[li + a] & ~pmask) | pv[a];
        }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) nlng += (uint32_t)__shfl_xor((int)nlng, d, 64);
    if ((threadIdx.x & 63) == 0) wl[threadIdx.x >> 6] = nlng;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t t = wl[0] + wl[1] + wl[2] + wl[3];
        if (t) atomicAdd(nlong, (unsigned long long)t);
    }
}

__global__ __launch_bounds__(256) void k_tie_flags(uint64_t n, const uint64_t* __restrict__ keys,
                                                   int shift, uint32_t* __restrict__ flag)
{
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) flag[i] = in_long_run(keys, shift, n, i) ? 1u : 0u;
}

// fpos: exclusive scan of the long-run flags; per long-run position j (in
// position order): its position, pair index and caller's Gaussian index
__global__ __launch_bounds__(256) void k_tie_gather(uint64_t n, const uint64_t* __restrict__ keys,
                                                    int shift, const uint32_t* __restrict__ order,
                                                    uint64_t pmask,
                                                    const uint32_t* __restrict__ fpos,
                                                    const uint32_t* __restrict__ gidx,
                                                    uint32_t* __restrict__ tpos,
                                                    uint32_t* __restrict__ tv,
                                                    uint32_t* __restrict__ tg)
{
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n || !in_long_run(keys, shift, n, i)) return;
    const uint32_t j = fpos[i];
    const uint32_t p = pair_of(keys, order, pmask, i);
    tpos[j] = (uint32_t)i;
    tv[j] = p;
    tg[j] = gidx[p];
}

__device__ __forceinline__ uint32_t tie_head(const uint64_t* __restrict__ keys, int shift,
                                             const uint32_t* __restrict__ tpos, uint32_t j)
{
    return (j == 0 || tie_hi(keys, shift, tpos[j - 1]) != tie_hi(keys, shift, tpos[j])) ? 1u : 0u;
}

__global__ __launch_bounds__(256) void k_tie_heads(uint32_t m, const uint64_t* __restrict__ keys,
                                                   int shift, const uint32_t* __restrict__ tpos,
                                                   uint32_t* __restrict__ head)
{
    const uint32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j < m) head[j] = tie_head(keys, shift, tpos, j);
}

// hs: exclusive scan of the run heads; sort key (run ordinal, Gaussian index)
__global__ __launch_bounds__(256) void k_tie_keys(uint32_t m, const uint64_t* __restrict__ keys,
                                                  int shift, const uint32_t* __restrict__ tpos,
                                                  const uint32_t* __restrict__ hs,
                                                  const uint32_t* __restrict__ tg, int gbits,
                                                  uint64_t* __restrict__ tk)
{
    const uint32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j >= m) return;
    const uint32_t run = hs[j] + tie_head(keys, shift, tpos, j) - 1u;
    tk[j] = ((uint64_t)run << gbits) | tg[j];
}

// the j-th pair of the sorted runs goes to the j-th long-run position: runs
// keep their positions, their pairs come in Gaussian-index order
__global__ __launch_bounds__(256) void k_tie_scatter(uint32_t m, const uint32_t* __restrict__ tpos,
                                                     const uint32_t* __restrict__ tv,
                                                     uint64_t* __restrict__ keys,
                                                     uint32_t* __restrict__ order, uint64_t pmask)
{
    const uint32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j >= m) return;
    const uint32_t i = tpos[j];
    if (order) order[i] = tv[j];
    else keys[i] = (keys[i] & ~pmask) | tv[j];
}

inline unsigned grid_for(uint64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

void launch_tie_short(uint64_t n, uint64_t* keys, int shift, uint32_t* order, uint64_t pmask,
                      const uint32_t* gidx, unsigned long long* nlong, hipStream_t st)
{
    if (!n) return;
    hipLaunchKernelGGL(k_tie_short, dim3((unsigned)((n + TIE_BLOCK - 1) / TIE_BLOCK)), dim3(256), 0,
                       st, n, keys, shift, order, pmask, gidx, nlong);
}

void launch_tie_flags(uint64_t n, const uint64_t* keys, int shift, uint32_t* flag, hipStream_t st)
{
    if (!n) return;
    hipLaunchKernelGGL(k_tie_flags, dim3(grid_for(n)), dim3(256), 0, st, n, keys, shift, flag);
}

void launch_tie_fix(uint64_t n, uint32_t m, uint64_t* keys, int shift, uint32_t* order,
                    uint64_t pmask, const uint32_t* fpos, const uint32_t* gidx, int gbits,
                    uint32_t* tpos, uint32_t* tv, uint32_t* tv_alt, uint32_t* tg, uint32_t* head,
                    uint64_t* tk, uint64_t* tk_alt, uint32_t* hist, void* scan_ws, hipStream_t st)
{
    if (!n || !m) return;
    hipLaunchKernelGGL(k_tie_gather, dim3(grid_for(n)), dim3(256), 0, st, n, keys, shift, order,
                       pmask, fpos, gidx, tpos, tv, tg);
    hipLaunchKernelGGL(k_tie_heads, dim3(grid_for(m)), dim3(256), 0, st, m, keys, shift, tpos, head);
    scan_u32(head, m, nullptr, scan_ws, st);
    hipLaunchKernelGGL(k_tie_keys, dim3(grid_for(m)), dim3(256), 0, st, m, keys, shift, tpos, head,
                       tg, gbits, tk);
    // runs <= m / 2 + 1: their ordinals fit in bit_length(m) bits
    int rbits = 0;
    while (rbits < 32 && ((uint64_t)1 << rbits) <= (uint64_t)m) rbits++;
    const bool alt = radix_sort_u64(tk, tv, tk_alt, tv_alt, m, rbits + gbits, hist, scan_ws,
                                    nullptr, st);
    hipLaunchKernelGGL(k_tie_scatter, dim3(grid_for(m)), dim3(256), 0, st, m, tpos,
                       alt ? tv_alt : tv, keys, order, pmask);
}

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
    return ((n + RADIX_TILE_MIN - 1) / RADIX_TILE_MIN) * ((size_t)1 << RADIX_MAXBITS) * sizeof(uint32_t) +
           256;
}

bool radix_sort_u64(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
                    uint64_t n, int nbits, uint32_t* hist, void* scan_ws, uint64_t* tot,
                    hipStream_t st)
{
    (void)tot;
    return radix_sort<uint64_t, 1>(keys, vals, nullptr, keys_alt, vals_alt, nullptr, n, 0, nbits,
                                   hist, scan_ws, st);
}

bool radix_sort_u64_keys(uint64_t* keys, uint64_t* keys_alt, uint64_t n, int bit0, int nbits,
                         uint32_t* hist, void* scan_ws, hipStream_t st)
{
    return radix_sort<uint64_t, 0>(keys, nullptr, nullptr, keys_alt, nullptr, nullptr, n, bit0,
                                   nbits, hist, scan_ws, st);
}

bool radix_sort_u32(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                    uint64_t n, int nbits, uint32_t* hist, void* scan_ws, uint64_t* tot,
                    hipStream_t st)
{
    (void)tot;
    return radix_sort<uint32_t, 1>(keys, vals, nullptr, keys_alt, vals_alt, nullptr, n, 0, nbits,
                                   hist, scan_ws, st);
}

void launch_rank_tiles(uint64_t npairs, const uint32_t* order, const uint64_t* okey,
                       uint64_t pmask, const uint2* prect, uint32_t* tcr, uint2* prank,
                       hipStream_t st)
{
    if (!npairs) return;
    const uint64_t per = 256 * RANK_ITEMS;
    const uint64_t nblk = (npairs + per - 1) / per;
    const uint64_t grid = (nblk + NXCD - 1) / NXCD * NXCD;   // whole rounds over the XCDs
    hipLaunchKernelGGL(k_rank_tiles, dim3((unsigned)grid), dim3(256), 0, st, npairs, order, okey,
                       pmask, prect, tcr, prank);
}

void launch_emit_isect(uint64_t npairs, const uint32_t* order, const uint64_t* okey,
                       uint64_t pmask, const uint2* prank, const ViewDev* views,
                       const uint32_t* ioff, int lbits, uint32_t* ikey, uint32_t* ival,
                       hipStream_t st)
{
    if (!npairs) return;
    hipLaunchKernelGGL(k_emit_isect, dim3(grid_for(npairs)), dim3(256), 0, st, npairs, order, okey,
                       pmask, prank, views, ioff, lbits, ikey, ival);
}

void launch_pairs_from_keys(uint64_t npairs, const uint64_t* keys, int vshift, uint64_t pmask,
                            const uint32_t* blk_off, int cbv, uint32_t* order, hipStream_t st)
{
    if (!npairs) return;
    hipLaunchKernelGGL(k_pairs_from_keys, dim3(grid_for(npairs)), dim3(256), 0, st, npairs, keys,
                       vshift, pmask, blk_off, cbv, order);
}

void launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t st)
{
    if (!n) return;
    uint64_t g = grid_for(n);
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)g), dim3(256), 0, st, p, n, v);
}

void launch_bucket_ranges(uint64_t ni, const uint32_t* ikey, const ViewDev* views, int lbits,
                          uint32_t* bstart, uint32_t* bend, hipStream_t st)
{
    if (!ni) return;
    hipLaunchKernelGGL(k_bucket_ranges, dim3(grid_for((ni + 3) / 4)), dim3(256), 0, st, ni, ikey, views,
                       lbits, bstart, bend);
}

void launch_bucket_keys(uint32_t nb, const uint32_t* bucket_view, const uint8_t* view_cls,
                        const uint32_t* bstart, const uint32_t* bend, uint32_t* key,
                        uint32_t* val, hipStream_t st)
{
    if (!nb) return;
    hipLaunchKernelGGL(k_bucket_keys, dim3(grid_for(nb)), dim3(256), 0, st, nb, bucket_view,
                       view_cls, bstart, bend, key, val);
}

}  // namespace slag
