// Host-side state of a lift context, shared by the lift and the codec
// entry points (private to the library).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/slag.h"
#include "../../include/slag_codec.h"
#include "slag_internal.h"

namespace slag_host {

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    template <typename T>
    T* as() const { return reinterpret_cast<T*>(p); }
};

enum Stage {
    ST_TILES = 0, ST_PROJECT, ST_DEPTH_SORT, ST_BIN, ST_TILE_SORT, ST_PART_PREP, ST_COMPOSITE,
    ST_MERGE, ST_CONTRACT, ST_ENCODE, ST_DECODE, ST_COUNT_
};

struct Batch {
    int v0 = 0, nb = 0;
    uint32_t nbuckets = 0, nsat = 0;
    DevBuf views, bucket_view;
    // sizes read back by the last eager lift (reused while capturing a graph)
    uint64_t npairs = 0, ni = 0, nparts = 0, ntie = 0;
    uint64_t nchunks = 0;   // chunks the contraction's walk took (whole range)
    uint32_t zmin = 0, zmax = 0;
    // resolution classes (distinct image sizes, first appearance order): the
    // tuner times each class alone; the compositing runs one launch over all
    int ncls = 0;
    int lbits = 0;     // bits of the largest view's tile count (tile-sort key width)
    std::vector<uint32_t> cls_w, cls_h, cls_nb, cls_off;
    DevBuf view_cls;   // [nb] uint8 class of each view
};

struct TuneEntry {
    int variant = 0;
    int n_variants = 0;
    float ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};
};

struct TimedEvent {
    int stage;
    hipEvent_t a, b;
};

// The learned codec: parameters, Adam state, training pool and work arrays.
struct CodecState {
    int d = 0, h = 0, k = 0;
    bool bf16 = true;
    bool ready = false;
    int64_t nparam = 0;
    DevBuf params, grad, adam_m, adam_v;
    int64_t step = 0;
    // training pool: segment features (FP32), rows (Gaussians) as CSR over
    // pool segments with normalised weights, and target embeddings
    int64_t pool_seg = 0, pool_rows = 0, pool_nnz = 0;
    DevBuf pF, prow, pcol, pw, ptgt;
    // work arrays
    DevBuf a1, h1, C, dC, code, dcode, a3, h2, y, dy, gpart, cpart, lpart, loss;
    // training-row extraction
    DevBuf rflag, ridx, rlen, roff, rgid;
    // the pool's entries grouped by column (gradient of the mixing without
    // atomics), rebuilt when the pool changes
    DevBuf csc_key, csc_j, csc_key_alt, csc_j_alt, csc_row, row_of, cbeg, cend, csc_hist, csc_ws;
    bool csc_valid = false;
    // codec lift
    DevBuf codes, hid;
    bool have_codes = false;
};

// Rasterizer constants of a context (slag_options, defaults filled in).
struct RasterConsts {
    float amax, amin, tmin, rho2, l2amin, dil, near_z, guard;
    double dil_d, guard_d;
};

// Work arrays of the cosine-similarity search (library-allocated; kept
// between calls).
struct QueryState {
    DevBuf emb, q, qt, counts, keys, vals, keys_alt, vals_alt, hist, scan_ws;
};

}  // namespace slag_host

struct slag_ctx {
    int device = 0;
    hipStream_t st = nullptr;
    bool own_stream = false;
    slag_options opt{};
    slag_host::RasterConsts rc{};
    std::string err;

    int64_t n = -1;
    slag_host::DevBuf means, scales, quats, opac, cov3;
    slag_host::DevBuf covd, lo2;    // FP64 world covariance [6][N], log2 opacity [N]
    slag_host::DevBuf perm, rank;   // Morton order of the Gaussians (rank -> input index, inverse)
    slag_host::DevBuf bgeo;         // per Gaussian block: bounding box, largest covariance trace
    slag_host::DevBuf vlist, vcnt;  // per Gaussian block: views with visible pairs (this launch)

    int nviews = -1;
    std::vector<slag_camera> cams;
    std::vector<uint64_t> pix_off;
    std::vector<int32_t> nseg;
    std::vector<char> seg_set;
    slag_host::DevBuf ids;            // [pixels][lpp] segment ids, -1 = none
    slag_host::DevBuf idstage;        // host ids staged for widening to lpp labels
    int lpp = 1;                      // labels per pixel (slag_options.labels_per_pixel)
    bool kernel_w = false;            // weights are Gaussian kernel values (slag_options.weight_mode)

    int d = 0;
    slag_dtype fdt = SLAG_F32;
    slag_host::DevBuf feats;
    bool feats_set = false;
    uint64_t feat_rows = 0;

    slag_host::DevBuf num, den;
    bool have_out = false;
    bool out_is_codec = false;

    std::vector<slag_host::Batch> plan;
    int plan_views = -1;
    int auto_maxv = 0;                // views per launch found by a re-plan (0 = no limit)
    int replan_views = 0;             // set by a launch that overflowed: views to try instead

    // workspace
    slag_host::DevBuf ns_tile, segl, sat, tcnt, blk_vis, small, scan_ws, hist;
    slag_host::DevBuf rec, pgauss, pview, dkey, dkey_alt, dval, dval_alt, psz, pz, tcr, wlen,
        pair_of_m;
    slag_host::DevBuf ikey, ikey_alt, ival, ival_alt, bstart, bend, part, wrow, pinfo;
    slag_host::DevBuf prect, prank, blk_aux, bkey, bkey_alt, bord, bord_alt;
    slag_host::DevBuf tflag, tpos, tv, tv_alt, tg, thead, tk, tk_alt;   // depth ties
    slag_host::DevBuf pixdbg;         // per-pixel T_final, weight sum, blend count (debug)
    slag_host::DevBuf outbf;          // BF16 copy of the output for host fetches
    slag_host::DevBuf cnum, cden, cbf;  // one chunk of a streamed lift's output (Morton rows)
    void* chost = nullptr;            // pinned staging of one chunk
    size_t chost_cap = 0;
    uint64_t* host_small = nullptr;   // pinned read-back area

    slag_host::CodecState codec;
    slag_host::QueryState query;

    // compositing variant per image size (SLAG_FLAG_AUTOTUNE), and the events that time them
    std::map<uint64_t, slag_host::TuneEntry> tune;
    hipEvent_t tune_ev[2] = {nullptr, nullptr};
    std::string tune_cache;   // file named by SLAG_TUNE_CACHE ("" = none)
    std::string dev_kind;     // architecture name and compute-unit count
    uint32_t pgrid = 0;       // workgroups of a persistent compositing launch
    int ts = 16, tsh = 4;     // tile edge in pixels (16 or 8) and its log2

    // graph replay of the lift (SLAG_FLAG_GRAPH)
    uint64_t gen = 1;                 // bumped by every input change
    uint64_t graph_gen = 0;           // generation the graph was captured for
    int graph_mode = -1;              // 0 plain, 1 codec
    bool capturing = false;
    // render-back: the launch runs projection through the tile ranges only
    bool front_only = false;
    bool lists_valid = false;                // the last lift's pair lists are still in the buffers
    const uint32_t* front_ival = nullptr;   // its sorted list entries (pairs)
    slag_host::Batch rbatch;                 // its one-view launch
    slag_host::DevBuf rattr, rout;           // staged host attributes / outputs
    // contraction dispatch order: per Gaussian block a work key and its index
    slag_host::DevBuf gkey, gkey_alt, gval, gval_alt;
    // walk + chunk multiply (D >= 768 BF16): chunk lists of the blocks
    slag_host::DevBuf cks, cA, cnext, chead, rowden;
    uint64_t chunk_cap = 0;    // chunks the buffers hold
    uint64_t chunk_used = 0;   // chunks of the lift's earlier view launches (eager)
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    slag_stats graph_stats{};

    // results of the last lift
    slag_stats stats{};
    std::vector<slag_host::TimedEvent> events;
    std::vector<hipEvent_t> free_events;
    // last batch (debug exports, training rows)
    int last_v0 = -1, last_nb = 0;
    bool last_pix = false;            // the last batch wrote the per-pixel outputs
    uint64_t last_npairs = 0, last_ni = 0;
    const uint32_t* last_ikey = nullptr;
    const uint32_t* last_ival = nullptr;
};

namespace slag_host {

// small device area layout (uint64 words)
enum { SM_TOT = 0, SM_ZRANGE = 2, SM_TOTALS = 4, SM_COUNTERS = 8, SM_NNZ = 12, SM_ERR = 14,
       SM_TIES = 16, SM_LERR = 18, SM_CHUNKS = 20, SM_QUEUE = 22, SM_WORDS = 24 };

#define FAIL(ctx, code, msg)                 \
    do {                                     \
        (ctx)->err = (msg);                  \
        return (code);                       \
    } while (0)

#define HC(ctx, expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) {                                                          \
            (ctx)->err = std::string(#expr) + ": " + hipGetErrorString(e_);              \
            return SLAG_E_DEVICE;                                                        \
        }                                                                                \
    } while (0)

#define CK(expr)                          \
    do {                                  \
        slag_status s_ = (expr);          \
        if (s_ != SLAG_OK) return s_;     \
    } while (0)

// Device buffer of at least `bytes` (contents not kept when it grows).
slag_status ensure(slag_ctx* c, DevBuf& b, size_t bytes);
// Device buffer of at least `bytes`, keeping the first `keep` bytes.
slag_status grow_keep(slag_ctx* c, DevBuf& b, size_t bytes, size_t keep);
void release(DevBuf& b);
slag_status copy_in(slag_ctx* c, DevBuf& dst, const void* src, size_t bytes, slag_mem where);
slag_status ensure_scan(slag_ctx* c, uint64_t len);
// Copy `words` uint64 words of the small device area to host_small (synchronous).
slag_status read_small(slag_ctx* c, int off, int words);
slag_status stage_begin(slag_ctx* c, int stage, hipEvent_t* a);
slag_status stage_end(slag_ctx* c, int stage, hipEvent_t a);
int bit_length(uint64_t x);

// The lift (plain or codec) on the context's inputs.
slag_status run_lift(slag_ctx* c, bool codec);
// SLAG_E_CAPACITY if the last lift's kernels flagged an error.
slag_status check_lift_errors(slag_ctx* c);
// Codec pieces used by the lift: codes of the context's feature table into
// codec.C, and decoding of codec.codes into the context's output.
slag_status codec_encode_table(slag_ctx* c);
slag_status codec_decode_codes(slag_ctx* c);
// Release the codec's device memory.
void codec_release(slag_ctx* c);
// Mark the captured lift graph stale (any input change), or destroy it.
void invalidate_graph(slag_ctx* c);
void destroy_graph(slag_ctx* c);

}  // namespace slag_host
