// Internal declarations shared by the host library and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace slag {

constexpr int TILE = 16;                 // default tile edge in pixels (16 x 16 = 4 waves of 8 x 8;
                                         // 8 x 8 tiles, one wave, are the other choice)
constexpr int TILE_PIX = TILE * TILE;    // the most pixels (and tile segments) of a tile
constexpr int NS_CAP = 4;                // tile segments accumulated per compositing pass
constexpr int BATCH = 64;                // tile-list entries staged in LDS per step
constexpr int MAX_LABELS = 4;            // masks one pixel may lie in (overlapping masks)
constexpr uint32_t NONE = 0xFFFFFFFFu;

// One view of the current launch, with everything its kernels need.
struct ViewDev {
    float fx, fy, cx, cy;
    float R[9];
    float t[3];
    int32_t W, H;
    float limx, limy;        // guard clamp of x/z, y/z (1.3 x half-FOV tangent, FP32)
    int32_t ntx, nty;        // tiles per row / column
    int32_t tsh;             // log2 of the tile edge (3 or 4)
    uint32_t tile_base;      // first bucket (tile) of this view in the launch
    uint32_t sat_off;        // first entry of this view's summed-area table
    uint64_t pix_off;        // first pixel of this view in the id array
    uint32_t seg_off;        // first feature row of this view
    uint32_t nseg;           // segments of this view
    // rasterizer constants of the context (FP32 decision values; the FP64
    // values of the compositing records)
    float near_z, dil, rho2;         // near plane, dilation (px^2), pixel-box q bound
    float amin, amax, tmin, l2amin;  // alpha bounds, transmittance stop, log2(alpha_min)
    double guard_d, dil_d;           // Jacobian clamp (half-FOV tangents), dilation
};

// Pair record (one visible (view, Gaussian) pair), two float4, with the
// inverse covariance prescaled so that alpha = o exp(-q/2) = 2^(log2(o) +
// A dx^2 + B dx dy + C dy^2), formed in FP64 and rounded once:
//   r0 = (u - x0, v - y0, A, B)   screen mean as an offset from the box corner,
//        A = -log2(e)/2 conic_xx, B = -log2(e) conic_xy
//   r1 = (C, log2(o), x0 | y0 << 16, x1 | y1 << 16)   C = -log2(e)/2 conic_yy;
//        pixel box (inclusive)
constexpr float NHALF_LOG2E = -0.72134752044448170368f;   // -log2(e) / 2
constexpr float NLOG2E = -1.44269504088896340736f;        // -log2(e)

// ---- launchers (each enqueues on `st`) ----
// Validation, FP32 world covariance cov3 [6][n] (decision path), FP64 world
// covariance covd [6][n] and lo2 = log2(opacity) (compositing records).
void launch_prep_gauss(int64_t n, const float* means, const float* scales, const float* quats,
                       const float* opac, float* cov3, double* covd, float* lo2, uint32_t* err,
                       hipStream_t st);
// Segment ids of npix pixels, lpp labels each: every id in [-1, nseg) and a
// pixel's non-negative labels distinct, else err |= 2.
void launch_validate_ids(int64_t npix, const int32_t* ids, int lpp, int32_t nseg, uint32_t* err,
                         hipStream_t st);
// dst[p][l] = l < lin ? src[p][l] : -1 for l < lout (label layers widened).
void launch_expand_labels(int64_t npix, const int32_t* src, int lin, int32_t* dst, int lout,
                          hipStream_t st);
// Gaussian blocks of the projection grid: GBLOCK consecutive (Morton-order)
// Gaussians.  Per block, the bounding box of the means and the largest
// covariance trace (geo [nblk][8]), from which the counting pass rules out
// whole blocks outside a view.
constexpr int GBLOCK = 2048;
void launch_block_geo(int64_t n, const float* means, const float* cov3, float* geo, hipStream_t st);
// Pass 1 over a (view, Gaussian block) grid: tile count of each pair (0 = not
// visible), visible pairs per block (blk_vis), depth range per block.  Blocks
// ruled out by their geometry get blk_vis = 0 and leave tcnt unwritten.
void launch_count(int nb, int64_t n, const ViewDev* views, const float* means, const float* cov3,
                  const float* geo, uint32_t* tcnt, uint32_t* blk_vis, uint32_t* zrange,
                  hipStream_t st);
int count_blocks_per_view(int64_t n);
// Pass 2 over the same (view, Gaussian block) grid: visible pairs compacted
// in (view, Morton rank) order with their records, depth keys (the pair
// index -- or, plocal, its index within its view -- in the low pbits bits
// when pbits > 0, else the pair index in dval), part-list capacities
// psz, packed tile rectangles prect (entry key base for lbits), the caller's
// Gaussian index pgauss[pair] = perm[g], the view pview, and the (view, rank)
// -> pair map pair_of_m (NONE where not visible); pz only when non-null.
// blk_off = exclusive scan of blk_vis over nb * nblk + 1 entries (a block
// with no visible pair reads no tile count).
void launch_emit_pairs(int nb, int64_t n, const ViewDev* views, const float* means,
                       const float* cov3, const double* covd, const float* lo2,
                       uint32_t* tcnt_pairof,
                       const uint32_t* blk_off, float4* rec, uint32_t* pgauss, uint16_t* pview,
                       uint64_t* dkey, uint32_t* dval, uint32_t* psz, uint32_t* pz,
                       const uint32_t* sat, uint32_t zmin, int zbits, int pbits, int plocal,
                       uint32_t* blk_tot, const uint32_t* perm, uint32_t* pair_of_m, uint2* prect,
                       int lbits, hipStream_t st);
// out[0..1] = (min of even, max of odd) entries of in[2 * npairs], or their
// 64-bit sums in sum mode; one block
void launch_reduce_pairs(const uint32_t* in, uint64_t npairs, bool sum_mode,
                         unsigned long long* out, hipStream_t st);
// Morton order of the Gaussian means: bounding box (order-preserving integer
// images in box6[0..2] = min, [3..5] = max), 63-bit keys, inverse permutation
void launch_bbox(int64_t n, const float* means, uint32_t* box6, hipStream_t st);
void launch_morton(int64_t n, const float* means, const float* lo_scale, uint64_t* keys,
                   uint32_t* vals, hipStream_t st);
void launch_invert(int64_t n, const uint32_t* perm, uint32_t* rank, hipStream_t st);
// Gaussians into Morton order: q-th output = input perm[q] (means [n][3],
// covariances [6][n] FP32 and FP64, log2 opacities [n]).
void launch_gather_gauss(int64_t n, const uint32_t* perm, const float* means, const float* cov3,
                         const double* covd, const float* lo2, float* means_o, float* cov3_o,
                         double* covd_o, float* lo2_o, hipStream_t st);

// scans: exclusive prefix sum in place; the 64-bit total goes to *total_dev
size_t scan_workspace_bytes(uint64_t n);
void scan_u32(uint32_t* data, uint64_t n, uint64_t* total_dev, void* ws, hipStream_t st);

// stable LSD radix sort of (key, value) by bits [0, nbits); returns true when
// the result ended in the *_alt buffers
size_t radix_hist_bytes(uint64_t n);
bool radix_sort_u64(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
                    uint64_t n, int nbits, uint32_t* hist, void* scan_ws, uint64_t* tot,
                    hipStream_t st);
bool radix_sort_u32(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                    uint64_t n, int nbits, uint32_t* hist, void* scan_ws, uint64_t* tot,
                    hipStream_t st);

// keys only, by bits [bit0, bit0 + nbits) (stable)
bool radix_sort_u64_keys(uint64_t* keys, uint64_t* keys_alt, uint64_t n, int bit0, int nbits,
                         uint32_t* hist, void* scan_ws, hipStream_t st);

// Depth ties: runs of equal sorted keys (without their low `shift` bits) get
// their pairs in the caller's Gaussian order gidx[pair]; pairs are order[i],
// or the low bits of keys[i] (pmask) when order is null.  launch_tie_short
// reorders the runs of at most 8 pairs and adds the number of positions in
// longer runs to *nlong; for those, launch_tie_flags marks them (flag[i] = 1)
// and launch_tie_fix, given fpos = exclusive scan of the flags and their
// count m, sorts them (gbits: bits of the Gaussian index).  Work arrays: m
// entries each (tk, tk_alt: 64-bit); hist and scan_ws sized for n.
void launch_tie_short(uint64_t n, uint64_t* keys, int shift, uint32_t* order, uint64_t pmask,
                      const uint32_t* gidx, unsigned long long* nlong, hipStream_t st);
void launch_tie_flags(uint64_t n, const uint64_t* keys, int shift, uint32_t* flag, hipStream_t st);
void launch_tie_fix(uint64_t n, uint32_t m, uint64_t* keys, int shift, uint32_t* order,
                    uint64_t pmask, const uint32_t* fpos, const uint32_t* gidx, int gbits,
                    uint32_t* tpos, uint32_t* tv, uint32_t* tv_alt, uint32_t* tg, uint32_t* head,
                    uint64_t* tk, uint64_t* tk_alt, uint32_t* hist, void* scan_ws, hipStream_t st);

// depth order: order[r], or (okey non-null) okey[r] & pmask; prect[p] = (entry
// key of the pair's top-left tile, rectangle width | height << 16).
// launch_rank_tiles writes the tile count tcr[r] and the rectangle prank[r]
// of the pair of depth rank r; launch_emit_isect reads prank.
void launch_rank_tiles(uint64_t npairs, const uint32_t* order, const uint64_t* okey,
                       uint64_t pmask, const uint2* prect, uint32_t* tcr, uint2* prank,
                       hipStream_t st);
void launch_emit_isect(uint64_t npairs, const uint32_t* order, const uint64_t* okey,
                       uint64_t pmask, const uint2* prank, const ViewDev* views,
                       const uint32_t* ioff, int lbits, uint32_t* ikey, uint32_t* ival,
                       hipStream_t st);
void launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t st);
// Depth order of pairs from sorted depth keys that carry each pair's index
// within its view in the low bits (pmask): order[r] = the view's first pair
// blk_off[view * cbv] + key & pmask, with view = key >> vshift (cbv Gaussian
// blocks per view).
void launch_pairs_from_keys(uint64_t npairs, const uint64_t* keys, int vshift, uint64_t pmask,
                            const uint32_t* blk_off, int cbv, uint32_t* order, hipStream_t st);
// Dispatch keys: (resolution class << 16) | (0xFFFF - min(list length, 0xFFFF)),
// class 0 for every view when view_cls is null.
void launch_bucket_keys(uint32_t nb, const uint32_t* bucket_view, const uint8_t* view_cls,
                        const uint32_t* bstart, const uint32_t* bend, uint32_t* key,
                        uint32_t* val, hipStream_t st);
void launch_bucket_ranges(uint64_t ni, const uint32_t* ikey, const ViewDev* views, int lbits,
                          uint32_t* bstart, uint32_t* bend, hipStream_t st);

// Distinct segment ids of each ts x ts tile over the lpp label layers of its
// pixels (ids [pixels][lpp], -1 = none), ascending in segl[bucket][ts^2];
// more than ts^2 in one tile sets bit 4 of *err.
void launch_tile_segs(int ts, uint32_t nbuckets, const uint32_t* bucket_view, const ViewDev* views,
                      const int32_t* ids, int lpp, uint32_t* ns_tile, uint16_t* segl,
                      unsigned long long* err, hipStream_t st);
void launch_sat(int nb, const ViewDev* views, const uint32_t* ns_tile, uint32_t* sat,
                hipStream_t st);
// Compositing variants (bitwise-equal results; register budgets, group
// padding, one workgroup per bucket or a persistent queue).
int composite_variants();
const char* composite_variant_name(int v);
// Part lists: pinfo[p] = (base, fill), pinfo[npairs] = (total, 0); pair p
// owns part[base .. next base); compositing appends (tile-in-rect << 16 |
// view-local segment, weight) entries for its non-zero sums, counting them
// in the fill field (zeroed by launch_init_pinfo).
void launch_init_pinfo(uint64_t npairs, const uint32_t* base, uint32_t total, uint2* pinfo,
                       hipStream_t st);
// counters: [0] accepted blends, [1] in-box tests, [2] tile-list tests (count
// mode), [3] part-list entries lost to a capacity error (always; 0 by
// construction).  pix_t / pix_w / pix_n (count mode, may be null): final
// transmittance, sum of accepted weights and accepted blends of every pixel
// walked (indexed like the id maps).  The persistent variants (4, 5) run
// min(nbuckets, pgrid) workgroups that take buckets from *queue (zeroed here
// by a fill kernel); the others ignore queue and pgrid.
void launch_composite(bool count, int variant, int ts, uint32_t nbuckets, const uint32_t* order,
                      uint32_t obase, const uint32_t* bucket_view, const ViewDev* views,
                      const uint32_t* bstart, const uint32_t* bend, const uint32_t* ival,
                      uint2* pinfo, const float4* rec, const uint32_t* ns_tile,
                      const uint16_t* segl, const int32_t* ids, int lpp, bool kernel_w,
                      uint2* part, unsigned long long* counters, float* pix_t, float* pix_w,
                      uint32_t* pix_n, uint32_t* queue, uint32_t pgrid, hipStream_t st);
// Render-back of attr [N][C] (caller's Gaussian order) into view vi of the
// last launch: out [H][W][C] = sum w a / sum w per pixel (0 where no weight),
// wsum [H][W] (may be null); ntiles = the view's tile count.
void launch_render(bool kernel_w, int ts, int ntiles, const ViewDev* views, int vi, const uint32_t* bstart,
                   const uint32_t* bend, const uint32_t* ival, const float4* rec,
                   const uint32_t* pgauss, const float* attr, int C, float* out, float* wsum,
                   hipStream_t st);
// out[i] = bfloat16(in[i]) (round to nearest even), as bit patterns
void launch_f32_to_bf16(uint64_t n, const float* in, uint16_t* out, hipStream_t st);
void launch_merge(uint64_t npairs, const uint16_t* pview, const ViewDev* views, const uint2* pinfo,
                  const uint2* part, uint2* wrow, uint32_t* wlen, unsigned long long* nnz,
                  hipStream_t st);

bool contract_supported(int d);
// code tables of the codec: d in {16, 32, 48} besides the feature sizes
bool contract_supported_codes(int d);
// Per Gaussian block, the views of the launch in which it has visible pairs
// (ascending; vlist [nblk][nb], vcnt [nblk]) from the scanned visible counts;
// the contraction walks only those views.  With wkey/gidx (nblk entries
// each): the dispatch keys of the blocks for a contraction over Gaussian
// blocks [gb0, gb1) (sorting them over 28 bits gives the blocks in range,
// heaviest first, then the others).
void launch_view_lists(int nb, int nblk, const uint32_t* blk_off, uint16_t* vlist, uint32_t* vcnt,
                       int64_t gb0, int64_t gb1, uint32_t* wkey, uint32_t* gidx, hipStream_t st);
// The walk-only contraction's output (BF16 features, D >= 768): per block
// of 16 Gaussians of the range, a list of chunks of 32 columns.
struct ChunkOut {
    uint32_t* cks;       // [cap][32] feature row of each column, NONE past a round's end
    float* cA;           // [cap][16][32] the 16 rows' weights of each column
    uint32_t* cnext;     // [cap] next chunk of the block, NONE after its last
    uint32_t* head;      // [blocks] first chunk of each block, NONE if it has none
    const float* rowden_in;   // [blocks][16] the rows' weight sums of the earlier launches
    float* rowden;       // [blocks][16] the same after this launch (den after the last)
    uint32_t* counter;   // chunks taken (zeroed by the caller); may exceed cap,
    uint32_t cap;        //   and then nothing past cap is written
};
// Whether a contraction of width d runs as walk + chunk multiply.
bool contract_split(int d, bool bf16);
// Contraction of the Gaussians of Morton ranks [q_begin, q_end) (q_begin a
// multiple of 16): output row of rank q is perm[q] (the caller's order), or
// q - q_begin when `local` (one chunk of a streamed lift).  gorder: the
// Gaussian blocks met by the range in dispatch order (its first entries).
void launch_contract(int64_t n, int nb, int d, bool bf16, const uint32_t* perm,
                     const uint32_t* pair_of_m, const ViewDev* views, const uint16_t* vlist,
                     const uint32_t* vcnt, const uint2* pinfo, const uint2* part, const void* feats,
                     float* num, float* den, bool first, bool last, int64_t q_begin, int64_t q_end,
                     bool local, const uint32_t* gorder, hipStream_t st);
// The same split in two (contract_split(d, bf16)): each view launch's walk
// appends to co (heads at co.head, its rows' running sums in co.rowden,
// starting from zero when `first`); after the last one (and after the caller
// has checked co.counter <= co.cap), one chunk multiply over the nlists
// launches' lists (heads co.head[l][block]) writes E and den.
void launch_contract_walk(int64_t n, int nb, int d, const uint32_t* perm, const uint32_t* pair_of_m,
                          const ViewDev* views, const uint16_t* vlist, const uint32_t* vcnt,
                          const uint2* pinfo, const uint2* part, const float* den, bool first,
                          int64_t q_begin, int64_t q_end, bool local, const uint32_t* gorder,
                          const ChunkOut& co, hipStream_t st);
void launch_contract_chunks(int64_t n, int d, const uint32_t* perm, const ChunkOut& co, int nlists,
                            const void* feats, float* num, float* den, int64_t q_begin,
                            int64_t q_end, bool local, const uint32_t* gorder, hipStream_t st);

// ---- codec ----
enum { GEMM_NONE = 0, GEMM_GELU = 1, GEMM_GELU_BWD = 2 };
// Epilogue of a product, per output element (row, col) at index idx:
// v += bias[col]; zsave[idx] = v; v = gelu(v) (GEMM_GELU) or
// v *= gelu'(aux[idx]) (GEMM_GELU_BWD); v = 0 where rowmask[row] <= 0.
struct GemmEpi {
    const float* bias = nullptr;
    int act = GEMM_NONE;
    float* zsave = nullptr;
    const float* aux = nullptr;
    const float* rowmask = nullptr;
};
int gemm_splits(int M, int N, int K, int* kper);
size_t gemm_part_floats(int M, int N, int K);
// Decoder y = (gelu(code W3^T + b3)) W4^T + b4 with BF16 products in one
// kernel (the hidden layer stays in LDS); y rows with rowmask <= 0 are zero.
// W3 [H][k], W4 [D][H] FP32 (rounded to bf16 like the staged products).
bool decode_fused_supported(int k, int H, int D);
void launch_decode_bf16(int M, int k, int H, int D, const float* code, const float* W3,
                        const float* b3, const float* W4, const float* b4, const float* rowmask,
                        float* y, hipStream_t st);
void launch_gemm(bool bf16, bool a_bf16, int M, int N, int K, const void* A, int64_t sam,
                 int64_t sak, const float* B, int64_t sbk, int64_t sbn, float* C, int64_t ldc,
                 const GemmEpi& epi, float* part, hipStream_t st);
size_t colsum_part_floats(int R, int N);
void launch_colsum(int R, int N, const float* X, float* out, float* part, hipStream_t st);
void launch_mix(int R, int k, const uint32_t* row_ptr, const uint32_t* col, const float* w,
                const float* C, float* code, hipStream_t st);
// Gradient of the mixing through the pool's column grouping (no atomics):
// the batch is rows row0 .. row0 + R - 1 (row pointers rp from row0, so its
// entries are [rp[0], rp[R])); cbeg/cend
// the column ranges of csc_j (entry indices, ascending per column), csc_row
// the row of each grouped entry.  launch_row_of writes the row of every
// entry plus (column, entry) sort pairs; launch_csc_ranges the column ranges
// and rows from the column-sorted pairs (cbeg/cend zero-filled first).
void launch_mix_bwd(int NS, int k, const uint32_t* rp, int R, int64_t row0, const uint32_t* cbeg,
                    const uint32_t* cend, const uint32_t* csc_j, const uint32_t* csc_row,
                    const float* w, const float* dcode, float* dC, hipStream_t st);
void launch_row_of(uint32_t R, const uint32_t* row_ptr, const uint32_t* col, uint32_t* row_of,
                   uint32_t* key, uint32_t* ent, hipStream_t st);
void launch_csc_ranges(uint32_t nnz, const uint32_t* key, const uint32_t* csc_j,
                       const uint32_t* row_of, uint32_t* cbeg, uint32_t* cend, uint32_t* csc_row,
                       hipStream_t st);
void launch_cos_loss(int R, int d, const float* y, const float* tg, float* dy, float* loss_part,
                     float* loss, hipStream_t st);
void launch_adam(int64_t n, float* p, const float* g, float* m, float* v, float lr, float b1,
                 float b2, float eps, int64_t step, hipStream_t st);
void launch_to_f32(int64_t n, const void* src, bool bf16, float* dst, hipStream_t st);
void launch_pick_rows(int64_t n, const float* den, uint64_t seed, uint32_t thresh, uint32_t* flag,
                      hipStream_t st);
// (the pair map is read only in (view, block)s with visible pairs, by blk_off,
// the scanned per-(view, block) counts, nblk blocks per view)
void launch_row_len(int64_t n, int nb, const uint32_t* flag, const uint32_t* ridx,
                    uint32_t max_rows, const uint32_t* rank, const uint32_t* pair_of_m,
                    const uint32_t* blk_off, int nblk, const uint32_t* wlen, uint32_t* len,
                    uint32_t* gid, hipStream_t st);
void launch_row_gather(int64_t n, int nb, uint32_t rows, const uint32_t* gid, const uint32_t* off,
                       uint32_t nnz0, uint32_t seg0, const uint32_t* rank,
                       const uint32_t* pair_of_m, const uint32_t* blk_off, int nblk,
                       const uint32_t* wlen, const uint32_t* part_base, const uint2* wrow,
                       const float* den, uint32_t* row_ptr, uint32_t* col, float* w,
                       hipStream_t st);
void launch_copy_rows(uint32_t rows, int d, const uint32_t* gid, const float* src, float* dst,
                      hipStream_t st);

// cosine-similarity search (k_query.hip): unit queries transposed to
// qt[d][qp] (qp = nq rounded up to 16; err |= 1 for a zero or non-finite
// query); scores of every (query, Gaussian) with per-query counts of
// scores >= thr (counts zeroed by the caller) and, if keys != null, sort keys
// and indices at [q n + g]; the class of highest score per Gaussian; the
// first k entries of each query's sorted list
void launch_qprep(int nq, int qp, int d, const float* q, float* qt, uint32_t* err, hipStream_t st);
void launch_scores(int nq, int64_t n, int d, const float* E, const float* qt, float thr,
                   uint32_t* keys, uint32_t* vals, unsigned long long* counts, hipStream_t st);
void launch_classify(int nc, int64_t n, int d, const float* E, const float* qt, int32_t* label,
                     float* best, hipStream_t st);
void launch_topk_out(int nq, int k, int64_t n, const uint32_t* keys, const uint32_t* vals,
                     uint32_t* idx, float* cosv, hipStream_t st);
// Device address of the search's static work area on `device` (current when
// query_scratch_init is called, once per device, at context creation);
// null before that.
hipError_t query_scratch_init(int device);
void* query_scratch(int device);

}  // namespace slag
