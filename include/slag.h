/*
 * slag.h -- C interface of the MI355X (gfx950) lift of per-view segment
 * embeddings into per-Gaussian embeddings.
 *
 * The operation (paper, Method section, "Semantic Embedding"):
 *   1. every Gaussian G_k of the scene is rasterized with each training
 *      camera (K_i, R_i, t_i); the rasterizer yields, for every pixel p, the
 *      weights w_kp of the Gaussians contributing to p (the rasterizer
 *      equation); here w_kp = alpha_kp * T_kp, the front-to-back blend weight;
 *   2. the weights are masked by the segment that owns the pixel (parameter
 *      masking, w'_kp = w_kp * M_j(p));
 *   3. each Gaussian's embedding is the weight-normalised sum of the segment
 *      features over all views, segments and pixels (the aggregation
 *      equation): E_k = sum w'_kp E_ij / sum w'_kp, and E_k = 0 when the sum
 *      of weights is 0.
 *
 * Conventions the paper does not fix (3D Gaussian splatting's):
 *   alpha = min(0.99, o exp(-q/2)) with q = d^T Sigma2^{-1} d, d = pixel
 *   centre (u+0.5, v+0.5) minus the projected mean; blends with alpha < 1/255
 *   are skipped; a pixel stops before the Gaussian that would take its
 *   transmittance below 1e-4; Sigma2 is the EWA projection with the Jacobian
 *   at x/z, y/z clamped to 1.3 x the half-FOV tangent, plus 0.3 px^2 on the
 *   diagonal; Gaussians with camera depth <= 0.01 are culled.  Per pixel the
 *   Gaussians are visited by ascending FP32 camera depth, ties by ascending
 *   Gaussian index.  Depth, culling and the conservative pixel box are
 *   evaluated by a fixed FP32 operation sequence (see the library's
 *   projection source), so they are reproducible bit for bit on the CPU.
 *
 * Threading: a context is used by one host thread at a time.  All calls are
 * ordered on the context's HIP stream.  No call aborts or throws; every call
 * returns a slag_status and, on failure, slag_last_error() describes it.
 */
#ifndef SLAG_H
#define SLAG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SLAG_OK = 0,
    SLAG_E_INVALID_ARG = 1,     /* bad pointer, size, id or parameter value */
    SLAG_E_OUT_OF_MEMORY = 2,   /* device allocation failed */
    SLAG_E_DEVICE = 3,          /* HIP runtime error; destroy the context */
    SLAG_E_STATE = 4,           /* call out of order (e.g. lift before inputs) */
    SLAG_E_CAPACITY = 5,        /* a size limit of the implementation was hit */
    SLAG_E_NOT_SUPPORTED = 6
} slag_status;

typedef enum { SLAG_HOST = 0, SLAG_DEVICE = 1 } slag_mem;
typedef enum { SLAG_F32 = 0, SLAG_BF16 = 1 } slag_dtype;

/* One pinhole camera (OpenCV axes: x right, y down, z forward).
 * Intrinsics K = [[fx,0,cx],[0,fy,cy],[0,0,1]]; R (row-major) and t map
 * world points to camera space: X_cam = R X_world + t.  72 bytes. */
typedef struct {
    float fx, fy, cx, cy;
    float R[9];
    float t[3];
    int32_t width, height;
} slag_camera;

enum {
    SLAG_FLAG_PROFILE = 1,      /* record per-stage HIP events (slag_get_stats; eager
                                   lifts only: a graph replay reports ms_total alone) */
    SLAG_FLAG_COUNT = 2,        /* count blends and tests (slag_get_stats) */
    SLAG_FLAG_KEEP_DEBUG = 4,   /* keep the last view batch's tile lists and W rows */
    SLAG_FLAG_GRAPH = 8,        /* replay the lift as one HIP graph while the inputs are
                                   unchanged: the first lift after an input change runs
                                   eagerly (sizing every buffer) and captures its launch
                                   sequence; later lifts launch the graph.  Replays record
                                   ms_total but no per-stage times. */
    SLAG_FLAG_AUTOTUNE = 16     /* eager lifts time every compositing variant once per image
                                   size (all give bitwise-equal results); a launch then
                                   composites all its views in one kernel with the variant of
                                   least summed time over its image sizes.  Tuned sizes are
                                   kept for later lifts of this context and, if the
                                   environment variable SLAG_TUNE_CACHE names a file, read
                                   from it at slag_create and written back after tuning
                                   (text, one line per device kind and image size; lines of
                                   other devices or variant sets are kept, unreadable lines
                                   ignored; the file is replaced by rename, so processes that
                                   tune at once never leave it half written, and the last
                                   writer's table wins) */
};

typedef struct {
    int32_t max_views_per_launch;   /* 0 = as many as fit (all views if possible) */
    int32_t flags;                  /* SLAG_FLAG_* */
    /* Cap on the tile intersections and on the part slots of one launch
     * (0 = 2^32 - 16, the limit of the 32-bit list positions).  An eager lift
     * whose launch would exceed it re-plans with half the views per launch
     * and starts over, until every launch fits (a launch of one view that
     * does not fit is SLAG_E_CAPACITY); the context keeps the smaller plan
     * until the Gaussians or cameras change.  Results do not depend on the
     * plan beyond FP32 rounding of the contraction. */
    int64_t max_launch_entries;
    /* Rasterizer constants, which the paper leaves to the rasterizer (0 =
     * 3D Gaussian splatting's value, in brackets): alpha_max [0.99] caps
     * alpha; blends with alpha < alpha_min [1/255] are skipped (and the
     * conservative pixel box is sized for it: rho^2 = 2 ln(1 / alpha_min));
     * a pixel stops before the blend that would take its transmittance below
     * t_min [1e-4]; dilation [0.3 px^2] is added to the projected covariance's
     * diagonal; Gaussians at camera depth <= near_z [0.01] are culled; guard
     * [1.3] clamps x/z and y/z of the Jacobian at that many half-FOV
     * tangents.  Need 0 < alpha_min < alpha_max <= 1, 0 < t_min < 1, else
     * slag_create fails with SLAG_E_INVALID_ARG. */
    float alpha_max, alpha_min, t_min, dilation, near_z, guard;
    int32_t tile_size;              /* binning and compositing tile edge in pixels: 0 (=
                                       16), 16 (four waves of 8 x 8 per tile) or 8 (one
                                       wave); others are SLAG_E_NOT_SUPPORTED.  Contributing
                                       sets and per-pixel weights do not depend on it; W,
                                       den and E only through the order of FP32 sums */
    int32_t deterministic;          /* 0 or 1: every lift is deterministic (bitwise-equal
                                       results for equal inputs and options, whatever the
                                       launch order or atomics' timing); 1 asks for it */
    int32_t labels_per_pixel;       /* masks one pixel may lie in (overlapping masks): 0 or 1
                                       (one id per pixel), up to 4; see
                                       slag_set_segments_multi */
    int32_t weight_mode;            /* the weight w_kp a pixel gives each Gaussian the
                                       front-to-back walk blends: 0 = the blend weight
                                       alpha T (default), 1 = the Gaussian kernel
                                       exp(-q/2) itself (the paper's weight equation,
                                       with the contributing set of the walk) */
    int32_t composite_variant;      /* 0: the tuned variant (SLAG_FLAG_AUTOTUNE) or variant
                                       0; v + 1 forces compositing variant v (0 <= v <
                                       slag_variant_count(), names from slag_variant_name);
                                       every variant gives bitwise-equal results.  Kernel
                                       weights (weight_mode 1) have one shape and ignore it */
    int32_t reserved;
} slag_options;

typedef struct {
    int64_t n_views, n_batches;
    int64_t n_visible_pairs;        /* (view, Gaussian) pairs with a non-empty box */
    int64_t n_intersections;        /* (pair, tile) entries */
    int64_t n_part_slots;           /* per-(intersection, tile segment) partial sums */
    int64_t n_weights;              /* non-zero (pair, tile, segment) weights */
    int64_t n_contrib;              /* accepted blends, all pixels (SLAG_FLAG_COUNT) */
    int64_t n_tests;                /* in-box tests before termination (SLAG_FLAG_COUNT) */
    int64_t n_tile_tests;           /* tile-list tests executed (SLAG_FLAG_COUNT) */
    double ms_total;                /* last lift, HIP events (SLAG_FLAG_PROFILE) */
    double ms_stage[16];            /* per stage, see slag_stage_name() */
    int32_t n_stages;
    int32_t reserved;
    int64_t n_lost;                 /* part-list entries lost to a capacity error (0 by
                                       construction; non-zero fails slag_get_embeddings) */
} slag_stats;

typedef struct slag_ctx slag_ctx;

/* Create a context on HIP device `device`.  `hip_stream` (a hipStream_t) is
 * borrowed and must outlive the context; NULL makes the context create and
 * own a stream.  `opt` may be NULL (defaults). */
slag_status slag_create(int32_t device, void* hip_stream, const slag_options* opt,
                        slag_ctx** out);
void slag_destroy(slag_ctx* ctx);
/* Context-owned message of the last failed call; valid until the next call. */
const char* slag_last_error(const slag_ctx* ctx);

/* The Gaussian set G = {G_1..G_N} (paper: the rasterizer's first argument).
 * means_xyz[N][3], scales_xyz[N][3] (linear standard deviations, > 0),
 * quats_wxyz[N][4] (rotation, any non-zero norm), opacity[N] in (0, 1].
 * All FP32.  Pointers are `where`-resident and are copied before return.
 * n = 0 is valid; more than 65535 x 2048 Gaussians is SLAG_E_CAPACITY.
 * Non-finite or out-of-range values are rejected here with
 * SLAG_E_INVALID_ARG (a validation kernel and one synchronisation). */
slag_status slag_set_gaussians(slag_ctx* ctx, int64_t n, const float* means_xyz,
                               const float* scales_xyz, const float* quats_wxyz,
                               const float* opacity, slag_mem where);

/* The training cameras (K_i, R_i, t_i) and image sizes; host memory, copied.
 * Setting cameras discards previously set segment maps. */
slag_status slag_set_cameras(slag_ctx* ctx, int32_t n_views, const slag_camera* cams);

/* The masks M_j of view `view` as one segment id per pixel: ids[H][W]
 * row-major int32, -1 = pixel in no mask, else 0 <= id < n_seg.  Copied.
 * Ids out of range are rejected here with SLAG_E_INVALID_ARG. */
slag_status slag_set_segments(slag_ctx* ctx, int32_t view, const int32_t* ids, int32_t n_seg,
                              slag_mem where);

/* Overlapping masks (the paper's masks M_j are per-object binary masks, and
 * one pixel may lie in several): ids[H][W][n_labels] row-major int32, the
 * masks containing each pixel (distinct, in any order), -1 for unused
 * entries; 1 <= n_labels <= the context's labels_per_pixel option.  Every
 * label of a pixel receives the pixel's blend weights (parameter masking per
 * mask), and the aggregation sums over every mask and its pixels.  Copied;
 * ids out of range or repeated within a pixel are SLAG_E_INVALID_ARG.  With
 * n_labels = 1 this is slag_set_segments. */
slag_status slag_set_segments_multi(slag_ctx* ctx, int32_t view, const int32_t* ids,
                                    int32_t n_labels, int32_t n_seg, slag_mem where);

/* The segment embeddings E_ij: table[sum_v n_seg_v][d], view-major (all
 * segments of view 0, then view 1, ...), FP32 or BF16.  Copied.  d is 64,
 * 128, 256, 512, 768 or 1024 (else SLAG_E_NOT_SUPPORTED); a BF16 table is at
 * most 4 GiB (else SLAG_E_CAPACITY). */
slag_status slag_set_features(slag_ctx* ctx, int32_t d, slag_dtype dtype, const void* table,
                              slag_mem where);

/* Run the lift over every view.  Stream-ordered; returns once the work is
 * enqueued (and after any host synchronisation needed for sizing: two per
 * view batch in an eager lift, none in a graph replay). */
slag_status slag_lift(slag_ctx* ctx);

/* The lifted embeddings E_GAUSSIAN[N][d] (the aggregation equation's
 * normalised sums, paper Method "Semantic Embedding"), in input Gaussian
 * order: `out` (may be NULL) receives FP32 values (dtype SLAG_F32, 4 d bytes
 * per row) or their bfloat16 roundings, nearest even (SLAG_BF16, 2 d bytes
 * per row); `den` (may be NULL) receives the weight sums den[N] (FP32).  Rows
 * with den = 0 are 0.  Both are `where`-resident and caller-owned.
 * Synchronises the stream.  Fails with SLAG_E_CAPACITY (and the result must
 * not be used) if the last lift lost weights to a capacity error. */
slag_status slag_get_embeddings(slag_ctx* ctx, void* out, slag_dtype dtype, float* den,
                                slag_mem where);

/* The lift with E_GAUSSIAN streamed to host memory in chunks of
 * `chunk_rows` Gaussians (the paper runs the aggregation in several
 * iterations when the embedding tensor does not fit on the GPU: Method,
 * multi-GPU scaling; Experiments, the large aerial scene): the device holds
 * one chunk of the output (chunk_rows (d + 1) floats) instead of N (d + 1).
 * out[N][d] (FP32, or BF16 rounded nearest-even) and den[N] (FP32) are host
 * memory in the caller's Gaussian order; either may be NULL.  chunk_rows is
 * a positive multiple of 16.  With one view launch the compositing runs
 * once and only the contraction repeats per chunk; with several launches
 * each chunk repeats the whole lift.  Results equal slag_lift followed by
 * slag_get_embeddings bit for bit.  Synchronous; afterwards the context holds
 * no lift result (slag_get_embeddings fails with SLAG_E_STATE) and
 * slag_get_stats reports the first chunk's lift. */
slag_status slag_lift_chunked(slag_ctx* ctx, int64_t chunk_rows, void* out, slag_dtype dtype,
                              float* den);

/* Render per-Gaussian attributes into one view with the weights of the
 * lift (Method, the rendering equation: the Gaussians covering a pixel are
 * alpha-composited front to back; with the lift's weight w = alpha T, or
 * the kernel weight when weight_mode = 1; every pixel, no masking):
 *   out[y][x][c] = sum_k w_k attr[g_k][c] / sum_k w_k   (0 where nothing blends)
 *   wsum[y][x]   = sum_k w_k
 * attr [N][C] FP32 in the caller's Gaussian order, C = 1 .. 1024 (for
 * example E_GAUSSIAN rendered back into a view as a feature map, or a
 * per-Gaussian query score), in host or device memory as attr_where says;
 * out [H][W][C] and wsum [H][W] (may be NULL) FP32 where out_where says,
 * H x W the view's camera.  Needs the Gaussians and cameras only (segments
 * and features need not be set).  The view is projected, sorted and binned
 * anew in the lift's buffers: the last lift's debug exports fail with
 * SLAG_E_STATE afterwards; its embeddings and statistics stay.  Synchronous.
 * Errors: SLAG_E_INVALID_ARG (view or C out of range, null pointers, bad
 * memory kind), SLAG_E_STATE (no Gaussians or cameras), SLAG_E_CAPACITY
 * (the view's tile intersections exceed max_launch_entries), device errors. */
slag_status slag_render(slag_ctx* ctx, int32_t view, const float* attr, int32_t C,
                        slag_mem attr_where, float* out, float* wsum, slag_mem out_where);

slag_status slag_get_stats(slag_ctx* ctx, slag_stats* stats);
const char* slag_stage_name(int32_t stage);

/* Compositing variant chosen per image size (SLAG_FLAG_AUTOTUNE), with the
 * time of each variant on the lift that tuned it (or as read from the tuning
 * cache). */
typedef struct {
    int32_t width, height;
    int32_t variant;                /* index of the fastest, see slag_variant_name() */
    int32_t n_variants;
    float ms[8];                    /* per variant, compositing of this image size */
} slag_tuning;
/* Copies up to `cap` entries to out; *n receives the number of tuned sizes. */
slag_status slag_get_tuning(slag_ctx* ctx, slag_tuning* out, int32_t cap, int32_t* n);
const char* slag_variant_name(int32_t variant);
/* Number of compositing variants (at most 8). */
int32_t slag_variant_count(void);

/* Debug exports for the last view batch (needs SLAG_FLAG_KEEP_DEBUG).
 * Tile lists of view `view`: entries ordered by (tile, depth, Gaussian) with
 * tile = ty * ceil(W/T) + tx for tiles of T x T pixels; three host arrays of capacity `cap`.  *len
 * receives the count (also when it exceeds cap, then nothing is written). */
slag_status slag_debug_tile_lists(slag_ctx* ctx, int32_t view, uint32_t* tile,
                                  uint32_t* depth_bits, uint32_t* gauss, int64_t cap,
                                  int64_t* len);
/* Masked weight sums of view `view` as (Gaussian, view-local segment, weight)
 * entries, one per (Gaussian, tile, segment) with non-zero weight (a segment
 * may repeat across the tiles of one Gaussian).  Host arrays. */
slag_status slag_debug_weights(slag_ctx* ctx, int32_t view, uint32_t* gauss, uint32_t* seg,
                               float* w, int64_t cap, int64_t* len);

/* Debug exports of the last lift (SLAG_FLAG_KEEP_DEBUG; the view must be in
 * the last view batch).  `out` is a host buffer of `cap` bytes; *len receives
 * the byte size of the export (also when it exceeds cap: then nothing is
 * written).  Layouts (little-endian, row-major):
 *   SLAG_DEBUG_KEYS          uint32 [entries][3]: (tile, FP32 depth bits, caller's Gaussian
 *                            index) of the view's tile lists, ordered by (tile, depth,
 *                            Gaussian); tile = ty * ceil(W / 16) + tx
 *   SLAG_DEBUG_TILE_RANGES   uint32 [tiles][2]: [start, end) of each tile's rows in KEYS
 *   SLAG_DEBUG_W_VIEW        uint32 [entries][3]: (Gaussian, view-local segment, FP32 weight
 *                            bits), one per (Gaussian, tile, segment) with non-zero masked
 *                            weight (the per-view sums of the aggregation equation, by tile)
 *   SLAG_DEBUG_PIXEL_T_FINAL float [H][W]: transmittance after each pixel's front-to-back walk
 *   SLAG_DEBUG_PIXEL_WSUM    float [H][W]: sum of the pixel's accepted blend weights (all
 *                            pixels, masked or not); front-to-back compositing telescopes, so
 *                            WSUM = 1 - T_FINAL up to rounding
 *   SLAG_DEBUG_PIXEL_COUNT   uint32 [H][W]: accepted blends of the pixel
 *   SLAG_DEBUG_COUNTERS      int64 [4]: accepted blends, in-box tests, tile-list tests, lost
 *                            part-list entries (view ignored)
 * The PIXEL_* exports need a lift with SLAG_FLAG_COUNT as well (the counting pass walks every
 * pixel, background included); else SLAG_E_STATE. */
typedef enum {
    SLAG_DEBUG_KEYS = 0,
    SLAG_DEBUG_TILE_RANGES = 1,
    SLAG_DEBUG_W_VIEW = 2,
    SLAG_DEBUG_PIXEL_T_FINAL = 3,
    SLAG_DEBUG_PIXEL_WSUM = 4,
    SLAG_DEBUG_PIXEL_COUNT = 5,
    SLAG_DEBUG_COUNTERS = 6
} slag_debug;
slag_status slag_get_debug(slag_ctx* ctx, slag_debug what, int32_t view, void* out, int64_t cap,
                           int64_t* len);

#ifdef __cplusplus
}
#endif
#endif /* SLAG_H */
