// Host side of the C interface: input upload and validation, the per-launch
// view plan, workspace management, and the stream-ordered lift pipeline.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cctype>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <unistd.h>
#include <vector>

#include "slag_ctx.h"

using namespace slag;
using namespace slag_host;

namespace {

const char* kStageNames[ST_COUNT_] = {"tile_segments", "project", "depth_sort", "bin",
                                      "tile_sort", "part_prep", "composite", "merge",
                                      "contract", "encode", "decode"};

}  // namespace

namespace slag_host {

slag_status ensure(slag_ctx* c, DevBuf& b, size_t bytes)
{
    if (bytes <= b.cap && b.p) return SLAG_OK;
    if (b.p) {
        (void)hipStreamSynchronize(c->st);
        (void)hipFree(b.p);
        b.p = nullptr;
        b.cap = 0;
        c->gen++;   // a recorded graph may hold the old address
    }
    size_t want = bytes + bytes / 8 + 256;
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();
        c->err = "device allocation of " + std::to_string(want) + " bytes failed";
        return SLAG_E_OUT_OF_MEMORY;
    }
    b.cap = want;
    return SLAG_OK;
}

void release(DevBuf& b)
{
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
}

slag_status grow_keep(slag_ctx* c, DevBuf& b, size_t bytes, size_t keep)
{
    if (bytes <= b.cap && b.p) return SLAG_OK;
    DevBuf nb;
    CK(ensure(c, nb, bytes));
    if (keep && b.p) {
        const hipError_t e = hipMemcpyAsync(nb.p, b.p, std::min(keep, b.cap), hipMemcpyDeviceToDevice,
                                            c->st);
        if (e != hipSuccess) {
            release(nb);
            c->err = std::string("grow_keep copy: ") + hipGetErrorString(e);
            return SLAG_E_DEVICE;
        }
        (void)hipStreamSynchronize(c->st);
    }
    release(b);
    b = nb;
    return SLAG_OK;
}

slag_status copy_in(slag_ctx* c, DevBuf& dst, const void* src, size_t bytes, slag_mem where)
{
    CK(ensure(c, dst, bytes));
    if (bytes == 0) return SLAG_OK;
    HC(c, hipMemcpyAsync(dst.p, src, bytes,
                         where == SLAG_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                         c->st));
    return SLAG_OK;
}

slag_status ensure_scan(slag_ctx* c, uint64_t len)
{
    return ensure(c, c->scan_ws, scan_workspace_bytes(std::max<uint64_t>(len, 1)));
}

int bit_length(uint64_t x)
{
    int b = 0;
    while (x) { b++; x >>= 1; }
    return b;
}

// stage timing
slag_status stage_begin(slag_ctx* c, int stage, hipEvent_t* a)
{
    *a = nullptr;
    if (!(c->opt.flags & SLAG_FLAG_PROFILE) || c->capturing) return SLAG_OK;
    hipEvent_t e;
    if (!c->free_events.empty()) { e = c->free_events.back(); c->free_events.pop_back(); }
    else HC(c, hipEventCreate(&e));
    HC(c, hipEventRecord(e, c->st));
    *a = e;
    (void)stage;
    return SLAG_OK;
}

slag_status stage_end(slag_ctx* c, int stage, hipEvent_t a)
{
    if (!a) return SLAG_OK;
    hipEvent_t e;
    if (!c->free_events.empty()) { e = c->free_events.back(); c->free_events.pop_back(); }
    else HC(c, hipEventCreate(&e));
    HC(c, hipEventRecord(e, c->st));
    c->events.push_back({stage, a, e});
    return SLAG_OK;
}

slag_status read_small(slag_ctx* c, int off, int words)
{
    HC(c, hipMemcpyAsync(c->host_small + off, c->small.as<uint64_t>() + off, words * 8,
                         hipMemcpyDeviceToHost, c->st));
    HC(c, hipStreamSynchronize(c->st));
    return SLAG_OK;
}

}  // namespace slag_host

// Morton order of the Gaussian means: the Gaussians are stored in this
// order (pairs of nearby Gaussians get nearby pair indices, and the
// contraction takes Gaussians in blocks of 16 consecutive along the curve).
// Ties (equal 63-bit codes) keep input order.  perm[q] = input index of the
// q-th Gaussian, rank = its inverse.
static float from_ord(uint32_t o)
{
    uint32_t u = (o & 0x80000000u) ? (o ^ 0x80000000u) : ~o;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

static slag_status morton_order(slag_ctx* c, int64_t n)
{
    const uint64_t nn = (uint64_t)std::max<int64_t>(n, 1);
    CK(ensure(c, c->perm, nn * 4));
    CK(ensure(c, c->rank, nn * 4));
    if (n == 0) return SLAG_OK;
    CK(ensure(c, c->dkey, nn * 8));
    CK(ensure(c, c->dkey_alt, nn * 8));
    CK(ensure(c, c->dval, nn * 4));
    CK(ensure(c, c->dval_alt, nn * 4));
    CK(ensure(c, c->hist, radix_hist_bytes(nn)));
    CK(ensure_scan(c, nn / 2 + 4096));
    uint32_t* box = reinterpret_cast<uint32_t*>(c->small.as<uint64_t>() + SM_TOTALS);
    launch_fill_u32(box, 3, 0xFFFFFFFFu, c->st);
    launch_fill_u32(box + 3, 3, 0u, c->st);
    launch_bbox(n, c->means.as<float>(), box, c->st);
    CK(read_small(c, SM_TOTALS, 3));
    uint32_t b6[6];
    std::memcpy(b6, c->host_small + SM_TOTALS, sizeof(b6));
    float ls[6];
    for (int k = 0; k < 3; k++) {
        const float lo = from_ord(b6[k]), hi = from_ord(b6[3 + k]);
        const float ext = hi - lo;
        ls[k] = lo;
        ls[3 + k] = ext > 0.0f ? 2097151.0f / ext : 0.0f;
    }
    float* dls = reinterpret_cast<float*>(c->small.as<uint64_t>() + SM_TOTALS);
    HC(c, hipMemcpyAsync(dls, ls, sizeof(ls), hipMemcpyHostToDevice, c->st));
    launch_morton(n, c->means.as<float>(), dls, c->dkey.as<uint64_t>(), c->dval.as<uint32_t>(),
                  c->st);
    const bool alt = radix_sort_u64(c->dkey.as<uint64_t>(), c->dval.as<uint32_t>(),
                                    c->dkey_alt.as<uint64_t>(), c->dval_alt.as<uint32_t>(),
                                    (uint64_t)n, 63, c->hist.as<uint32_t>(), c->scan_ws.p,
                                    nullptr, c->st);
    const uint32_t* sorted = alt ? c->dval_alt.as<uint32_t>() : c->dval.as<uint32_t>();
    HC(c, hipMemcpyAsync(c->perm.p, sorted, (size_t)n * 4, hipMemcpyDeviceToDevice, c->st));
    launch_invert(n, c->perm.as<uint32_t>(), c->rank.as<uint32_t>(), c->st);
    DevBuf m2, c2, d2, l2;
    CK(ensure(c, m2, nn * 12));
    CK(ensure(c, c2, nn * 24));
    CK(ensure(c, d2, nn * 48));
    CK(ensure(c, l2, nn * 4));
    launch_gather_gauss(n, c->perm.as<uint32_t>(), c->means.as<float>(), c->cov3.as<float>(),
                        c->covd.as<double>(), c->lo2.as<float>(), m2.as<float>(), c2.as<float>(),
                        d2.as<double>(), l2.as<float>(), c->st);
    HC(c, hipStreamSynchronize(c->st));
    std::swap(c->means, m2);
    std::swap(c->cov3, c2);
    std::swap(c->covd, d2);
    std::swap(c->lo2, l2);
    release(m2);
    release(c2);
    release(d2);
    release(l2);
    // per Gaussian block: bounding box and largest covariance trace
    CK(ensure(c, c->bgeo, (size_t)count_blocks_per_view(n) * 32));
    launch_block_geo(n, c->means.as<float>(), c->cov3.as<float>(), c->bgeo.as<float>(), c->st);
    return SLAG_OK;
}

// ---------------------------------------------------------------- view plan

// One launch of views [v0, v0 + nb): per-view constants, tile buckets and
// resolution classes, uploaded.  seg_off[v] = the first segment of view v.
static slag_status make_batch(slag_ctx* c, int v0, int nb, int lbits,
                              const std::vector<uint64_t>& seg_off, Batch& b)
{
    b.v0 = v0;
    b.nb = nb;
    b.lbits = lbits;
    std::vector<ViewDev> vd(b.nb);
    std::vector<uint32_t> bv;
    uint32_t tb = 0, so = 0;
    for (int i = 0; i < b.nb; i++) {
        const slag_camera& cam = c->cams[v0 + i];
        ViewDev& x = vd[i];
        x.fx = cam.fx; x.fy = cam.fy; x.cx = cam.cx; x.cy = cam.cy;
        std::memcpy(x.R, cam.R, sizeof(x.R));
        std::memcpy(x.t, cam.t, sizeof(x.t));
        x.W = cam.width; x.H = cam.height;
        // guard clamp, same FP32 operations as the CPU decision path
        const RasterConsts& K = c->rc;
        volatile float hw = 0.5f * (float)cam.width, hh = 0.5f * (float)cam.height;
        volatile float tanx = hw / cam.fx, tany = hh / cam.fy;
        x.limx = K.guard * tanx;
        x.limy = K.guard * tany;
        x.near_z = K.near_z;
        x.dil = K.dil;
        x.rho2 = K.rho2;
        x.amin = K.amin;
        x.amax = K.amax;
        x.tmin = K.tmin;
        x.l2amin = K.l2amin;
        x.guard_d = K.guard_d;
        x.dil_d = K.dil_d;
        x.ntx = (cam.width + c->ts - 1) / c->ts;
        x.nty = (cam.height + c->ts - 1) / c->ts;
        x.tsh = c->tsh;
        x.tile_base = tb;
        x.sat_off = so;
        x.pix_off = c->pix_off[v0 + i];
        x.seg_off = (uint32_t)seg_off[v0 + i];
        x.nseg = (uint32_t)c->nseg[v0 + i];
        const uint32_t nt = (uint32_t)(x.ntx * x.nty);
        bv.insert(bv.end(), nt, (uint32_t)i);
        tb += nt;
        so += (uint32_t)((x.ntx + 1) * (x.nty + 1));
    }
    b.nbuckets = tb;
    b.nsat = so;
    // resolution classes
    std::vector<uint8_t> vcls(b.nb);
    for (int i = 0; i < b.nb; i++) {
        const uint32_t W = (uint32_t)vd[i].W, H = (uint32_t)vd[i].H;
        int k = 0;
        while (k < b.ncls && !(b.cls_w[k] == W && b.cls_h[k] == H)) k++;
        if (k == b.ncls) {
            if (b.ncls < 256) {
                b.cls_w.push_back(W);
                b.cls_h.push_back(H);
                b.cls_nb.push_back(0);
                b.ncls++;
            } else {
                k = 255;   // beyond 256 sizes: share the last class
            }
        }
        vcls[i] = (uint8_t)k;
        b.cls_nb[k] += (uint32_t)(vd[i].ntx * vd[i].nty);
    }
    b.cls_off.assign(b.ncls + 1, 0);
    for (int k = 0; k < b.ncls; k++) b.cls_off[k + 1] = b.cls_off[k] + b.cls_nb[k];
    CK(ensure(c, b.view_cls, vcls.size() + 16));
    HC(c, hipMemcpy(b.view_cls.p, vcls.data(), vcls.size(), hipMemcpyHostToDevice));
    CK(ensure(c, b.views, vd.size() * sizeof(ViewDev)));
    CK(ensure(c, b.bucket_view, bv.size() * sizeof(uint32_t)));
    HC(c, hipMemcpy(b.views.p, vd.data(), vd.size() * sizeof(ViewDev), hipMemcpyHostToDevice));
    if (!bv.empty())
        HC(c, hipMemcpy(b.bucket_view.p, bv.data(), bv.size() * sizeof(uint32_t),
                        hipMemcpyHostToDevice));
    return SLAG_OK;
}

static slag_status build_plan(slag_ctx* c)
{
    for (auto& b : c->plan) { release(b.views); release(b.bucket_view); release(b.view_cls); }
    c->plan.clear();
    const int V = c->nviews;
    int maxv = c->opt.max_views_per_launch > 0 ? c->opt.max_views_per_launch : V;
    if (c->auto_maxv > 0) maxv = std::min(maxv, c->auto_maxv);   // set by an earlier re-plan
    maxv = std::min(maxv, 65535);
    // keep (view, Gaussian) indices and tile-list positions in 32 bits
    const int64_t n = std::max<int64_t>(c->n, 1);
    const int64_t cap_pairs = (int64_t)1 << 31;
    maxv = (int)std::max<int64_t>(1, std::min<int64_t>(maxv, cap_pairs / n));
    // tile-sort keys are (view in launch << lbits) | tile in view, 32 bits
    int lbits = 0;
    for (int v = 0; v < V; v++) {
        const int64_t nt = (int64_t)((c->cams[v].width + c->ts - 1) / c->ts) *
                           ((c->cams[v].height + c->ts - 1) / c->ts);
        lbits = std::max(lbits, bit_length((uint64_t)std::max<int64_t>(nt - 1, 0)));
    }
    lbits = std::max(lbits, 1);
    if (lbits > 31) FAIL(c, SLAG_E_CAPACITY, "image too large for 32-bit tile keys");
    maxv = (int)std::min<int64_t>(maxv, (int64_t)1 << (32 - lbits));
    std::vector<uint64_t> seg_off(V + 1, 0);
    for (int v = 0; v < V; v++) seg_off[v + 1] = seg_off[v] + (uint64_t)c->nseg[v];
    for (int v0 = 0; v0 < V; v0 += maxv) {
        Batch b;
        CK(make_batch(c, v0, std::min(maxv, V - v0), lbits, seg_off, b));
        c->plan.push_back(b);
    }
    c->plan_views = V;
    return SLAG_OK;
}

// ------------------------------------------------------------------ the lift

// Tuning cache (SLAG_TUNE_CACHE): one text line per device kind and image
// size, "slag-tune <device kind> <variants> <width> <height> <variant> <ms>...".
// Lines of other device kinds or variant sets are kept when the file is
// rewritten; lines that do not parse are ignored (and dropped on rewrite).
static const char* kTuneTag = "slag-tune";

static bool parse_tune_line(const std::string& line, std::string& kind, int& nvar, uint32_t& w,
                            uint32_t& h, TuneEntry& te)
{
    std::istringstream is(line);
    std::string tag;
    long long W = 0, H = 0;
    if (!(is >> tag >> kind >> nvar >> W >> H >> te.variant) || tag != kTuneTag) return false;
    if (nvar < 1 || nvar > 8 || W < 1 || H < 1 || W > 0xFFFFFFFFll || H > 0xFFFFFFFFll ||
        te.variant < 0 || te.variant >= nvar)
        return false;
    for (int v = 0; v < nvar; v++)
        if (!(is >> te.ms[v]) || !std::isfinite(te.ms[v])) return false;
    te.n_variants = nvar;
    w = (uint32_t)W;
    h = (uint32_t)H;
    return true;
}

static void load_tune_cache(slag_ctx* c)
{
    if (c->tune_cache.empty()) return;
    std::ifstream f(c->tune_cache);
    std::string line, kind;
    while (std::getline(f, line)) {
        TuneEntry te;
        int nvar = 0;
        uint32_t w = 0, h = 0;
        if (parse_tune_line(line, kind, nvar, w, h, te) && kind == c->dev_kind &&
            nvar == composite_variants())
            c->tune[((uint64_t)w << 32) | h] = te;
    }
}

// Best effort: a cache that cannot be written leaves the lift unaffected.
static void save_tune_cache(slag_ctx* c)
{
    if (c->tune_cache.empty()) return;
    std::vector<std::string> keep;
    {
        std::ifstream f(c->tune_cache);
        std::string line, kind;
        while (std::getline(f, line)) {
            TuneEntry te;
            int nvar = 0;
            uint32_t w = 0, h = 0;
            if (!parse_tune_line(line, kind, nvar, w, h, te)) continue;
            if (kind == c->dev_kind && nvar == composite_variants() &&
                c->tune.count(((uint64_t)w << 32) | h))
                continue;   // replaced by this context's entry
            keep.push_back(line);
        }
    }
    const std::string tmp = c->tune_cache + ".tmp" + std::to_string((long long)getpid());
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    for (const auto& l : keep) std::fprintf(f, "%s\n", l.c_str());
    for (const auto& kv : c->tune) {
        const TuneEntry& te = kv.second;
        if (te.n_variants != composite_variants()) continue;
        std::fprintf(f, "%s %s %d %u %u %d", kTuneTag, c->dev_kind.c_str(), te.n_variants,
                     (unsigned)(kv.first >> 32), (unsigned)(kv.first & 0xFFFFFFFFu), te.variant);
        for (int v = 0; v < te.n_variants; v++) std::fprintf(f, " %.9g", (double)te.ms[v]);
        std::fprintf(f, "\n");
    }
    const bool ok = std::fclose(f) == 0;
    if (!ok || std::rename(tmp.c_str(), c->tune_cache.c_str()) != 0) std::remove(tmp.c_str());
}

// Time every compositing variant on one resolution class (second of two
// runs each, so caches are warm) and keep the fastest.
template <typename F>
static slag_status tune_class(slag_ctx* c, TuneEntry& te, F&& launch)
{
    for (int i = 0; i < 2; i++)
        if (!c->tune_ev[i]) HC(c, hipEventCreate(&c->tune_ev[i]));
    float best = 0.0f;
    for (int v = 0; v < te.n_variants; v++) {
        launch(v);
        HC(c, hipEventRecord(c->tune_ev[0], c->st));
        launch(v);
        HC(c, hipEventRecord(c->tune_ev[1], c->st));
        HC(c, hipEventSynchronize(c->tune_ev[1]));
        float ms = 0.0f;
        HC(c, hipEventElapsedTime(&ms, c->tune_ev[0], c->tune_ev[1]));
        te.ms[v] = ms;
        if (v == 0 || ms < best) { best = ms; te.variant = v; }
    }
    return SLAG_OK;
}

// What the contraction multiplies the weights with, and where it writes.
struct ContractTarget {
    const void* table;   // [rows][d] FP32 or BF16
    int d;
    bool bf16;
    float* out;          // [N][d], or [q_end - q_begin][d] rows in Morton order when local
    float* den;          // [N], or [q_end - q_begin] when local
    int64_t q_begin = 0, q_end = -1;   // Morton ranks contracted (q_end < 0: all)
    bool local = false;
};

// The contraction of one view batch whose part lists are on the device.
// Room for `want` contraction chunks, keeping the first chunk_used chunks
// (the lists of the lift's earlier view launches).
static slag_status grow_chunks(slag_ctx* c, uint64_t want)
{
    if (want <= c->chunk_cap && c->cks.p) return SLAG_OK;
    const uint64_t cap = std::max<uint64_t>(want + want / 8, 1024);
    CK(grow_keep(c, c->cks, cap * 128 + 16, c->chunk_used * 128));
    CK(grow_keep(c, c->cA, cap * 2048 + 16, c->chunk_used * 2048));
    CK(grow_keep(c, c->cnext, cap * 4 + 16, c->chunk_used * 4));
    c->chunk_cap = cap;
    c->gen++;   // a recorded graph may hold the old addresses
    return SLAG_OK;
}

static slag_status contract_batch(slag_ctx* c, Batch& B, bool first, bool last,
                                  const ContractTarget& ct)
{
    hipEvent_t ev;
    const int cbv = count_blocks_per_view(c->n);
    const int64_t q_end = ct.q_end < 0 ? c->n : ct.q_end;
    CK(stage_begin(c, ST_CONTRACT, &ev));
    // view lists, and the Gaussian blocks of the range heaviest first
    const size_t gb = (size_t)cbv * 4 + 16;
    CK(ensure(c, c->gkey, gb));
    CK(ensure(c, c->gkey_alt, gb));
    CK(ensure(c, c->gval, gb));
    CK(ensure(c, c->gval_alt, gb));
    CK(ensure(c, c->hist, radix_hist_bytes((uint64_t)cbv)));
    CK(ensure_scan(c, (uint64_t)cbv));
    launch_view_lists(B.nb, cbv, c->blk_vis.as<uint32_t>(), c->vlist.as<uint16_t>(),
                      c->vcnt.as<uint32_t>(), ct.q_begin / GBLOCK, (q_end + GBLOCK - 1) / GBLOCK,
                      c->gkey.as<uint32_t>(), c->gval.as<uint32_t>(), c->st);
    const bool alt = radix_sort_u32(c->gkey.as<uint32_t>(), c->gval.as<uint32_t>(),
                                    c->gkey_alt.as<uint32_t>(), c->gval_alt.as<uint32_t>(),
                                    (uint64_t)cbv, 28, c->hist.as<uint32_t>(), c->scan_ws.p,
                                    nullptr, c->st);
    const uint32_t* gorder = alt ? c->gval_alt.as<uint32_t>() : c->gval.as<uint32_t>();
    if (!contract_split(ct.d, ct.bf16)) {
        launch_contract(c->n, B.nb, ct.d, ct.bf16, c->perm.as<uint32_t>(),
                        c->pair_of_m.as<uint32_t>(), B.views.as<ViewDev>(), c->vlist.as<uint16_t>(),
                        c->vcnt.as<uint32_t>(), c->pinfo.as<uint2>(), c->part.as<uint2>(), ct.table,
                        ct.out, ct.den, first, last, ct.q_begin, q_end, ct.local, gorder, c->st);
    } else if (q_end > ct.q_begin && c->n > 0) {
        // Each view launch's walk appends its blocks' chunk lists to one
        // buffer (and carries the rows' weight sums in rowden); after the
        // last launch one multiply takes every launch's lists.  An eager
        // walk reads the chunk count back: one that ran out of room is run
        // again after the buffer has grown (the earlier launches' chunks
        // copied over); a recorded graph reuses the sizes.
        const bool whole = ct.q_begin == 0 && q_end == c->n;
        const uint64_t nblocks = (uint64_t)((q_end - ct.q_begin + 15) / 16);
        const int nbat = (int)c->plan.size();
        const int bi = (int)(&B - c->plan.data());
        if (bi < 0 || bi >= nbat) FAIL(c, SLAG_E_STATE, "contraction of a launch outside the plan");
        CK(ensure(c, c->chead, (uint64_t)nbat * nblocks * 4 + 16));
        CK(ensure(c, c->rowden, 2 * nblocks * 64 + 16));   // two halves: in, out by launch parity
        uint64_t* small = c->small.as<uint64_t>();
        uint32_t* counter = reinterpret_cast<uint32_t*>(small + SM_CHUNKS);
        if (first) {
            c->chunk_used = 0;
            launch_fill_u32(counter, 2, 0u, c->st);
        }
        if (!c->capturing) {
            // first guess one chunk per block: most first lifts outgrow it
            // once (so the re-run path is the common one, not a rare one)
            const uint64_t want = c->chunk_used + ((whole && B.nchunks) ? B.nchunks : nblocks + 1024);
            CK(grow_chunks(c, want));
        }
        for (;;) {
            float* rd = c->rowden.as<float>();
            ChunkOut co{c->cks.as<uint32_t>(), c->cA.as<float>(), c->cnext.as<uint32_t>(),
                        c->chead.as<uint32_t>() + (uint64_t)bi * nblocks,
                        rd + (uint64_t)((bi + 1) & 1) * nblocks * 16, rd + (uint64_t)(bi & 1) * nblocks * 16,
                        counter, (uint32_t)std::min<uint64_t>(c->chunk_cap, 0xFFFFFFF0ull)};
            launch_contract_walk(c->n, B.nb, ct.d, c->perm.as<uint32_t>(),
                                 c->pair_of_m.as<uint32_t>(), B.views.as<ViewDev>(),
                                 c->vlist.as<uint16_t>(), c->vcnt.as<uint32_t>(),
                                 c->pinfo.as<uint2>(), c->part.as<uint2>(), ct.den, first,
                                 ct.q_begin, q_end, ct.local, gorder, co, c->st);
            if (c->capturing) break;
            CK(read_small(c, SM_CHUNKS, 1));
            const uint64_t used = c->host_small[SM_CHUNKS] & 0xFFFFFFFFull;
            if (used > c->chunk_cap) {
                // nothing past the buffer was written, and the walk reads
                // only its inputs: grow, rewind the count, walk again
                if (used > 0xFFFFFFF0ull) FAIL(c, SLAG_E_CAPACITY, "too many contraction chunks");
                CK(grow_chunks(c, used));
                launch_fill_u32(counter, 1, (uint32_t)c->chunk_used, c->st);
                continue;
            }
            if (whole) B.nchunks = used - c->chunk_used;
            c->chunk_used = used;
            break;
        }
        if (last) {
            float* rd = c->rowden.as<float>();
            ChunkOut co{c->cks.as<uint32_t>(), c->cA.as<float>(), c->cnext.as<uint32_t>(),
                        c->chead.as<uint32_t>(), rd, rd + (uint64_t)(bi & 1) * nblocks * 16, counter,
                        (uint32_t)std::min<uint64_t>(c->chunk_cap, 0xFFFFFFF0ull)};
            launch_contract_chunks(c->n, ct.d, c->perm.as<uint32_t>(), co, bi + 1, ct.table, ct.out,
                                   ct.den, ct.q_begin, q_end, ct.local, gorder, c->st);
        }
    }
    CK(stage_end(c, ST_CONTRACT, ev));
    return SLAG_OK;
}

static slag_status lift_batch(slag_ctx* c, Batch& B, bool first, bool last,
                              const ContractTarget& ct)
{
    hipStream_t st = c->st;
    const int64_t n = c->n;
    const int nb = B.nb;
    const ViewDev* views = B.views.as<ViewDev>();
    uint64_t* small = c->small.as<uint64_t>();
    const bool count = (c->opt.flags & SLAG_FLAG_COUNT) != 0;
    const bool debug = (c->opt.flags & SLAG_FLAG_KEEP_DEBUG) != 0;
    hipEvent_t ev;

    // tile segment tables and their summed-area tables
    CK(stage_begin(c, ST_TILES, &ev));
    CK(ensure(c, c->ns_tile, (size_t)B.nbuckets * 4));
    CK(ensure(c, c->segl, (size_t)B.nbuckets * (size_t)(c->ts * c->ts) * 2));
    CK(ensure(c, c->sat, (size_t)B.nsat * 4));
    if (c->front_only) {
        // render-back: no segments, so no part slots
        launch_fill_u32(c->sat.as<uint32_t>(), B.nsat, 0u, st);
    } else {
        launch_tile_segs(c->ts, B.nbuckets, B.bucket_view.as<uint32_t>(), views, c->ids.as<int32_t>(),
                         c->lpp, c->ns_tile.as<uint32_t>(), c->segl.as<uint16_t>(),
                         reinterpret_cast<unsigned long long*>(small + SM_LERR), st);
        launch_sat(nb, views, c->ns_tile.as<uint32_t>(), c->sat.as<uint32_t>(), st);
    }
    CK(stage_end(c, ST_TILES, ev));

    // projection: count, compact, records
    CK(stage_begin(c, ST_PROJECT, &ev));
    const uint64_t npq = (uint64_t)nb * (uint64_t)n;
    const int cbv = count_blocks_per_view(n);
    const uint64_t nblk = (uint64_t)cbv * nb;
    CK(ensure(c, c->tcnt, npq * 4));
    CK(ensure(c, c->blk_vis, nblk * 4 + 16));
    CK(ensure(c, c->vlist, nblk * 2 + 16));
    CK(ensure(c, c->vcnt, (size_t)cbv * 4 + 16));
    CK(ensure(c, c->blk_aux, nblk * 8 + 16));
    CK(ensure_scan(c, nblk + 1));
    launch_count(nb, n, views, c->means.as<float>(), c->cov3.as<float>(), c->bgeo.as<float>(),
                 c->tcnt.as<uint32_t>(), c->blk_vis.as<uint32_t>(), c->blk_aux.as<uint32_t>(), st);
    launch_reduce_pairs(c->blk_aux.as<uint32_t>(), nblk, false,
                        reinterpret_cast<unsigned long long*>(small + SM_ZRANGE), st);
    // one extra zero entry: after the scan it holds the total, so every
    // block's count is the difference of two neighbours
    launch_fill_u32(c->blk_vis.as<uint32_t>() + nblk, 1, 0u, st);
    scan_u32(c->blk_vis.as<uint32_t>(), nblk + 1, small + SM_TOT, c->scan_ws.p, st);
    if (!c->capturing) {
        CK(read_small(c, 0, 4));
        B.npairs = c->host_small[SM_TOT];
        B.zmin = (uint32_t)c->host_small[SM_ZRANGE];
        B.zmax = (uint32_t)c->host_small[SM_ZRANGE + 1];
    }
    const uint64_t npairs = B.npairs;
    const uint32_t zmin = B.zmin, zmax = B.zmax;
    if (npairs > 0xFFFFFFF0ull) FAIL(c, SLAG_E_CAPACITY, "too many visible pairs in one launch");
    const int zbits = (npairs && zmax >= zmin) ? bit_length((uint64_t)(zmax - zmin)) : 0;
    const int vbits = bit_length((uint64_t)(nb > 0 ? nb - 1 : 0));
    // depth keys carry the pair index in their low bits when everything fits
    // in 64 bits (one 8-byte array to sort instead of 8 + 4 bytes); else the
    // pair's index within its view (a view has at most n pairs), turned back
    // into pair indices after the sort
    const int pneed = std::max(1, bit_length(npairs > 0 ? npairs - 1 : 0));
    const int lneed = std::max(1, bit_length((uint64_t)std::max<int64_t>(n - 1, 0)));
    const bool pglobal = vbits + zbits + pneed <= 64;
    const bool plocal = !pglobal && vbits + zbits + lneed <= 64;
    const int pbits = pglobal ? pneed : plocal ? lneed : 0;
    const uint64_t np = std::max<uint64_t>(npairs, 1);
    CK(ensure(c, c->rec, np * 32));
    CK(ensure(c, c->pgauss, np * 4));
    CK(ensure(c, c->pview, np * 2));
    CK(ensure(c, c->dkey, np * 8));
    CK(ensure(c, c->dkey_alt, np * 8));
    CK(ensure(c, c->dval, np * 4));
    CK(ensure(c, c->dval_alt, np * 4));
    CK(ensure(c, c->psz, np * 4 + 16));
    CK(ensure(c, c->pz, np * 4));
    CK(ensure(c, c->prect, np * 8));
    CK(ensure(c, c->tcr, np * 4 + 16));
    CK(ensure(c, c->wlen, np * 4));
    CK(ensure(c, c->pair_of_m, npq * 4));
    launch_emit_pairs(nb, n, views, c->means.as<float>(), c->cov3.as<float>(),
                      c->covd.as<double>(), c->lo2.as<float>(),
                      c->tcnt.as<uint32_t>(), c->blk_vis.as<uint32_t>(), c->rec.as<float4>(),
                      c->pgauss.as<uint32_t>(), c->pview.as<uint16_t>(),
                      c->dkey.as<uint64_t>(), c->dval.as<uint32_t>(), c->psz.as<uint32_t>(),
                      debug ? c->pz.as<uint32_t>() : nullptr,
                      c->sat.as<uint32_t>(), zmin, zbits, pbits, plocal ? 1 : 0,
                      c->blk_aux.as<uint32_t>(),
                      c->perm.as<uint32_t>(), c->pair_of_m.as<uint32_t>(), c->prect.as<uint2>(), B.lbits,
                      st);
    launch_reduce_pairs(c->blk_aux.as<uint32_t>(), nblk, true,
                        reinterpret_cast<unsigned long long*>(small + SM_TOTALS), st);
    CK(stage_end(c, ST_PROJECT, ev));

    uint64_t ni = 0, nparts = 0;
    if (npairs) {
        if (!c->capturing) {
            CK(read_small(c, SM_TOTALS, 2));
            B.ni = c->host_small[SM_TOTALS];
            B.nparts = c->host_small[SM_TOTALS + 1];
        }
        ni = B.ni;
        nparts = B.nparts;
        const uint64_t cap = c->opt.max_launch_entries > 0
                                 ? std::min<uint64_t>((uint64_t)c->opt.max_launch_entries, 0xFFFFFFF0ull)
                                 : 0xFFFFFFF0ull;
        if (ni > cap || nparts > cap) {
            // 32-bit list positions would overflow: an eager lift re-plans
            // with fewer views per launch (run_lift halves the batch and
            // starts over); nothing has been written to the outputs yet
            // that the restart does not overwrite
            c->replan_views = nb > 1 ? (nb + 1) / 2 : 0;
            FAIL(c, SLAG_E_CAPACITY, "too many tile intersections in one launch of " +
                                         std::to_string(nb) + " views");
        }
    }
    c->stats.n_visible_pairs += (int64_t)npairs;
    c->stats.n_intersections += (int64_t)ni;
    c->stats.n_part_slots += (int64_t)nparts;

    const uint32_t* skey = nullptr;
    const uint32_t* sval = nullptr;
    if (c->front_only && !npairs) {
        c->front_ival = nullptr;   // nothing visible: no lists
        return SLAG_OK;
    }
    if (npairs) {
        // depth order of pairs within each view
        CK(stage_begin(c, ST_DEPTH_SORT, &ev));
        CK(ensure(c, c->hist, std::max(radix_hist_bytes(npairs), radix_hist_bytes(ni))));
        CK(ensure_scan(c, std::max<uint64_t>(npairs, ni / 2 + 4096)));
        const uint32_t* order = nullptr;
        const uint64_t* okey = nullptr;
        uint64_t* skeys = nullptr;   // the sorted depth keys
        const uint64_t pmask = pbits ? ((1ull << pbits) - 1ull) : 0ull;
        if (pbits) {
            const bool alt = radix_sort_u64_keys(c->dkey.as<uint64_t>(), c->dkey_alt.as<uint64_t>(),
                                                 npairs, pbits, zbits + vbits,
                                                 c->hist.as<uint32_t>(), c->scan_ws.p, st);
            skeys = alt ? c->dkey_alt.as<uint64_t>() : c->dkey.as<uint64_t>();
            if (plocal) {
                // view-local indices: the depth order as pair indices
                launch_pairs_from_keys(npairs, skeys, pbits + zbits, pmask,
                                       c->blk_vis.as<uint32_t>(), cbv, c->dval.as<uint32_t>(), st);
                order = c->dval.as<uint32_t>();
            } else {
                okey = skeys;
            }
        } else {
            const bool alt = radix_sort_u64(c->dkey.as<uint64_t>(), c->dval.as<uint32_t>(),
                                            c->dkey_alt.as<uint64_t>(), c->dval_alt.as<uint32_t>(),
                                            npairs, zbits + vbits, c->hist.as<uint32_t>(),
                                            c->scan_ws.p, nullptr, st);
            order = alt ? c->dval_alt.as<uint32_t>() : c->dval.as<uint32_t>();
            skeys = alt ? c->dkey_alt.as<uint64_t>() : c->dkey.as<uint64_t>();
        }
        // equal depths: the caller's Gaussian index decides (pairs follow the
        // storage order, the Morton order, until here)
        {
            uint64_t* tkeys = skeys;
            launch_fill_u32(reinterpret_cast<uint32_t*>(small + SM_TIES), 2, 0u, st);
            launch_tie_short(npairs, tkeys, pbits, const_cast<uint32_t*>(order), pmask,
                             c->pgauss.as<uint32_t>(),
                             reinterpret_cast<unsigned long long*>(small + SM_TIES), st);
            if (!c->capturing) {
                CK(read_small(c, SM_TIES, 1));
                B.ntie = c->host_small[SM_TIES];
            }
            const uint64_t m = B.ntie;   // positions in runs of more than 8 pairs
            if (m) {
                CK(ensure(c, c->tflag, np * 4));
                launch_tie_flags(npairs, tkeys, pbits, c->tflag.as<uint32_t>(), st);
                scan_u32(c->tflag.as<uint32_t>(), npairs, nullptr, c->scan_ws.p, st);
                CK(ensure(c, c->tpos, m * 4));
                CK(ensure(c, c->tv, m * 4));
                CK(ensure(c, c->tv_alt, m * 4));
                CK(ensure(c, c->tg, m * 4));
                CK(ensure(c, c->thead, m * 4));
                CK(ensure(c, c->tk, m * 8));
                CK(ensure(c, c->tk_alt, m * 8));
                launch_tie_fix(npairs, (uint32_t)m, tkeys, pbits, const_cast<uint32_t*>(order),
                               pmask, c->tflag.as<uint32_t>(), c->pgauss.as<uint32_t>(),
                               std::max(1, bit_length((uint64_t)std::max<int64_t>(n - 1, 0))),
                               c->tpos.as<uint32_t>(), c->tv.as<uint32_t>(),
                               c->tv_alt.as<uint32_t>(), c->tg.as<uint32_t>(),
                               c->thead.as<uint32_t>(), c->tk.as<uint64_t>(),
                               c->tk_alt.as<uint64_t>(), c->hist.as<uint32_t>(), c->scan_ws.p,
                               st);
            }
        }
        CK(stage_end(c, ST_DEPTH_SORT, ev));

        // (tile, pair) entries in depth order; part-list bases (pair-major) by scan
        CK(stage_begin(c, ST_BIN, &ev));
        scan_u32(c->psz.as<uint32_t>(), npairs, nullptr, c->scan_ws.p, st);
        CK(ensure(c, c->ikey, ni * 4));
        CK(ensure(c, c->ikey_alt, ni * 4));
        CK(ensure(c, c->ival, ni * 4));
        CK(ensure(c, c->ival_alt, ni * 4));
        CK(ensure(c, c->prank, np * 8));
        launch_rank_tiles(npairs, order, okey, pmask, c->prect.as<uint2>(), c->tcr.as<uint32_t>(),
                          c->prank.as<uint2>(), st);
        scan_u32(c->tcr.as<uint32_t>(), npairs, nullptr, c->scan_ws.p, st);
        launch_emit_isect(npairs, order, okey, pmask, c->prank.as<uint2>(), views,
                          c->tcr.as<uint32_t>(), B.lbits, c->ikey.as<uint32_t>(),
                          c->ival.as<uint32_t>(), st);
        CK(stage_end(c, ST_BIN, ev));

        // stable sort by tile -> per-tile lists in (depth, Gaussian) order
        CK(stage_begin(c, ST_TILE_SORT, &ev));
        const bool alt2 = radix_sort_u32(c->ikey.as<uint32_t>(), c->ival.as<uint32_t>(),
                                         c->ikey_alt.as<uint32_t>(), c->ival_alt.as<uint32_t>(), ni,
                                         B.lbits, c->hist.as<uint32_t>(), c->scan_ws.p, nullptr, st);
        skey = alt2 ? c->ikey_alt.as<uint32_t>() : c->ikey.as<uint32_t>();
        sval = alt2 ? c->ival_alt.as<uint32_t>() : c->ival.as<uint32_t>();
        CK(ensure(c, c->bstart, (size_t)B.nbuckets * 4 + 4));
        CK(ensure(c, c->bend, (size_t)B.nbuckets * 4 + 4));
        launch_fill_u32(c->bstart.as<uint32_t>(), B.nbuckets, 0u, st);
        launch_fill_u32(c->bend.as<uint32_t>(), B.nbuckets, 0u, st);
        launch_bucket_ranges(ni, skey, views, B.lbits, c->bstart.as<uint32_t>(),
                             c->bend.as<uint32_t>(), st);
        if (c->front_only) {
            CK(stage_end(c, ST_TILE_SORT, ev));
            c->front_ival = sval;
            return SLAG_OK;
        }
        // dispatch order of the compositing workgroups: longest lists first
        // over all views of the launch (by_class: image size first, for the
        // tuner, which times each size alone)
        CK(ensure(c, c->bkey, (size_t)B.nbuckets * 4 + 4));
        CK(ensure(c, c->bkey_alt, (size_t)B.nbuckets * 4 + 4));
        CK(ensure(c, c->bord, (size_t)B.nbuckets * 4 + 4));
        CK(ensure(c, c->bord_alt, (size_t)B.nbuckets * 4 + 4));
        CK(ensure(c, c->hist, radix_hist_bytes(B.nbuckets)));
        CK(ensure_scan(c, B.nbuckets));
        auto sort_buckets = [&](bool by_class) -> const uint32_t* {
            launch_bucket_keys(B.nbuckets, B.bucket_view.as<uint32_t>(),
                               by_class ? B.view_cls.as<uint8_t>() : nullptr,
                               c->bstart.as<uint32_t>(), c->bend.as<uint32_t>(),
                               c->bkey.as<uint32_t>(), c->bord.as<uint32_t>(), st);
            const int kbits = 16 + (by_class ? bit_length((uint64_t)(B.ncls - 1)) : 0);
            const bool alt = radix_sort_u32(c->bkey.as<uint32_t>(), c->bord.as<uint32_t>(),
                                            c->bkey_alt.as<uint32_t>(), c->bord_alt.as<uint32_t>(),
                                            B.nbuckets, kbits, c->hist.as<uint32_t>(),
                                            c->scan_ws.p, nullptr, st);
            return alt ? c->bord_alt.as<uint32_t>() : c->bord.as<uint32_t>();
        };
        const uint32_t* border = sort_buckets(false);
        CK(stage_end(c, ST_TILE_SORT, ev));

        // part lists: pinfo[p] = (base psz[p] (scanned), fill 0), sentinel (total, 0)
        CK(stage_begin(c, ST_PART_PREP, &ev));
        CK(ensure(c, c->part, std::max<uint64_t>(nparts, 1) * 8));
        CK(ensure(c, c->pinfo, (np + 1) * 8));
        launch_init_pinfo(npairs, c->psz.as<uint32_t>(), (uint32_t)nparts, c->pinfo.as<uint2>(), st);
        CK(stage_end(c, ST_PART_PREP, ev));

        // per-pixel debug outputs (counting lifts with debug exports): pixels
        // of tiles without list entries keep T = 1, no weight, no blend
        float* pix_t = nullptr;
        float* pix_w = nullptr;
        uint32_t* pix_n = nullptr;
        if (count && debug) {
            const uint64_t P = c->pix_off[c->nviews];
            const uint64_t p0 = c->pix_off[B.v0], p1 = c->pix_off[B.v0 + nb];
            CK(ensure(c, c->pixdbg, P * 12 + 16));
            pix_t = c->pixdbg.as<float>();
            pix_w = pix_t + P;
            pix_n = reinterpret_cast<uint32_t*>(pix_w + P);
            launch_fill_u32(reinterpret_cast<uint32_t*>(pix_t) + p0, p1 - p0, 0x3F800000u, st);
            launch_fill_u32(reinterpret_cast<uint32_t*>(pix_w) + p0, p1 - p0, 0u, st);
            launch_fill_u32(pix_n + p0, p1 - p0, 0u, st);
        }
        CK(stage_begin(c, ST_COMPOSITE, &ev));
        auto clear_lists = [&]() {
            launch_init_pinfo(npairs, c->psz.as<uint32_t>(), (uint32_t)nparts,
                              c->pinfo.as<uint2>(), st);
        };
        // tuning: time every variant of each untuned size alone (each run
        // starts from empty part lists), then composite the launch for real
        uint32_t* queue = reinterpret_cast<uint32_t*>(small + SM_QUEUE);
        const bool tuning = (c->opt.flags & SLAG_FLAG_AUTOTUNE) && !c->capturing && !count &&
                            !c->kernel_w && c->opt.composite_variant == 0;
        bool untuned = false;
        for (int k = 0; k < B.ncls; k++)
            untuned = untuned ||
                      (B.cls_nb[k] && !c->tune.count(((uint64_t)B.cls_w[k] << 32) | B.cls_h[k]));
        if (tuning && untuned) {
            const uint32_t* corder = sort_buckets(true);
            for (int k = 0; k < B.ncls; k++) {
                if (!B.cls_nb[k]) continue;
                const uint64_t key = ((uint64_t)B.cls_w[k] << 32) | B.cls_h[k];
                if (c->tune.count(key)) continue;
                auto launch = [&](int var) {
                    clear_lists();
                    launch_composite(false, var, c->ts, B.cls_nb[k], corder, B.cls_off[k],
                                     B.bucket_view.as<uint32_t>(), views, c->bstart.as<uint32_t>(),
                                     c->bend.as<uint32_t>(), sval, c->pinfo.as<uint2>(),
                                     c->rec.as<float4>(), c->ns_tile.as<uint32_t>(),
                                     c->segl.as<uint16_t>(), c->ids.as<int32_t>(), c->lpp,
                                     c->kernel_w, c->part.as<uint2>(),
                                     reinterpret_cast<unsigned long long*>(small + SM_COUNTERS),
                                     nullptr, nullptr, nullptr, queue, c->pgrid, st);
                };
                TuneEntry te;
                te.n_variants = std::min(composite_variants(), 8);
                CK(tune_class(c, te, launch));
                c->tune.emplace(key, te);
            }
            clear_lists();
            border = sort_buckets(false);
            save_tune_cache(c);
        }
        int var = 0;
        if (c->opt.composite_variant > 0) {
            var = c->opt.composite_variant - 1;
        } else {
            // the variant of least summed time over the launch's image sizes
            // (variant 0 while a size is untuned)
            double tot[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            bool all = true;
            for (int k = 0; k < B.ncls && all; k++) {
                if (!B.cls_nb[k]) continue;
                auto it = c->tune.find(((uint64_t)B.cls_w[k] << 32) | B.cls_h[k]);
                all = it != c->tune.end() && it->second.n_variants == composite_variants();
                for (int v = 0; all && v < it->second.n_variants; v++) tot[v] += it->second.ms[v];
            }
            if (all)
                for (int v = 1; v < std::min(composite_variants(), 8); v++)
                    if (tot[v] < tot[var]) var = v;
        }
        launch_composite(count, var, c->ts, B.nbuckets, border, 0, B.bucket_view.as<uint32_t>(), views,
                         c->bstart.as<uint32_t>(), c->bend.as<uint32_t>(), sval,
                         c->pinfo.as<uint2>(), c->rec.as<float4>(), c->ns_tile.as<uint32_t>(),
                         c->segl.as<uint16_t>(), c->ids.as<int32_t>(), c->lpp, c->kernel_w,
                         c->part.as<uint2>(),
                         reinterpret_cast<unsigned long long*>(small + SM_COUNTERS), pix_t, pix_w,
                         pix_n, queue, c->pgrid, st);
        CK(stage_end(c, ST_COMPOSITE, ev));

        if (c->opt.flags & SLAG_FLAG_KEEP_DEBUG) {
            // per-pair weight rows, only for the debug export
            CK(stage_begin(c, ST_MERGE, &ev));
            CK(ensure(c, c->wrow, std::max<uint64_t>(nparts, 1) * 8));
            launch_merge(npairs, c->pview.as<uint16_t>(), views, c->pinfo.as<uint2>(),
                         c->part.as<uint2>(), c->wrow.as<uint2>(),
                         c->wlen.as<uint32_t>(),
                         reinterpret_cast<unsigned long long*>(small + SM_NNZ), st);
            CK(stage_end(c, ST_MERGE, ev));
        }
    }

    CK(contract_batch(c, B, first, last, ct));

    c->last_v0 = B.v0;
    c->last_nb = nb;
    c->last_pix = count && debug;
    c->last_npairs = npairs;
    c->last_ni = ni;
    c->last_ikey = skey;
    c->last_ival = sval;
    return SLAG_OK;
}

// ------------------------------------------------------------------ C API

extern "C" {

slag_status slag_create(int32_t device, void* hip_stream, const slag_options* opt, slag_ctx** out)
{
    if (!out) return SLAG_E_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return SLAG_E_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess) return SLAG_E_DEVICE;
    // the search's static work area on this device (slag_query_static)
    if (slag::query_scratch_init(device) != hipSuccess) return SLAG_E_DEVICE;
    slag_ctx* c = new (std::nothrow) slag_ctx();
    if (!c) return SLAG_E_OUT_OF_MEMORY;
    c->device = device;
    if (opt) c->opt = *opt;
    {
        // rasterizer constants: 0 = 3D Gaussian splatting's default; the FP64
        // values are the option floats widened, rho^2 = 2 ln(1 / alpha_min)
        // rounded once (the defaults keep their exact literals)
        const slag_options& o = c->opt;
        const float amax = o.alpha_max > 0.0f ? o.alpha_max : 0.99f;
        const float amin = o.alpha_min > 0.0f ? o.alpha_min : 1.0f / 255.0f;
        const float tmin = o.t_min > 0.0f ? o.t_min : 1e-4f;
        const bool ok = std::isfinite(o.alpha_max) && std::isfinite(o.alpha_min) &&
                        std::isfinite(o.t_min) && std::isfinite(o.dilation) &&
                        std::isfinite(o.near_z) && std::isfinite(o.guard) && o.alpha_max >= 0.0f &&
                        o.alpha_min >= 0.0f && o.t_min >= 0.0f && o.dilation >= 0.0f &&
                        o.near_z >= 0.0f && o.guard >= 0.0f && amin < amax && amax <= 1.0f &&
                        tmin < 1.0f && (o.deterministic == 0 || o.deterministic == 1);
        if (!ok) {
            delete c;
            return SLAG_E_INVALID_ARG;
        }
        if (o.tile_size != 0 && o.tile_size != 16 && o.tile_size != 8) {
            delete c;
            return SLAG_E_NOT_SUPPORTED;
        }
        c->ts = o.tile_size == 8 ? 8 : TILE;
        c->tsh = c->ts == 8 ? 3 : 4;
        if (o.labels_per_pixel < 0 || o.labels_per_pixel > MAX_LABELS) {
            delete c;
            return SLAG_E_INVALID_ARG;
        }
        c->lpp = o.labels_per_pixel > 0 ? o.labels_per_pixel : 1;
        if (o.weight_mode != 0 && o.weight_mode != 1) {
            delete c;
            return SLAG_E_INVALID_ARG;
        }
        c->kernel_w = o.weight_mode == 1;
        if (o.composite_variant < 0 || o.composite_variant > composite_variants()) {
            delete c;
            return SLAG_E_INVALID_ARG;
        }
        RasterConsts& K = c->rc;
        K.amax = amax;
        K.amin = amin;
        K.tmin = tmin;
        K.rho2 = o.alpha_min > 0.0f ? (float)(2.0 * std::log(1.0 / (double)o.alpha_min))
                                    : 0x1.62a41p+3f;
        K.l2amin = o.alpha_min > 0.0f ? (float)std::log2((double)o.alpha_min)
                                      : -7.99435343685885793770f;
        K.dil = o.dilation > 0.0f ? o.dilation : 0.3f;
        K.dil_d = o.dilation > 0.0f ? (double)o.dilation : 0.3;
        K.near_z = o.near_z > 0.0f ? o.near_z : 0.01f;
        K.guard = o.guard > 0.0f ? o.guard : 1.3f;
        K.guard_d = o.guard > 0.0f ? (double)o.guard : 1.3;
    }
    if (hip_stream) {
        c->st = reinterpret_cast<hipStream_t>(hip_stream);
    } else {
        if (hipStreamCreateWithFlags(&c->st, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return SLAG_E_DEVICE;
        }
        c->own_stream = true;
    }
    if (ensure(c, c->small, SM_WORDS * 8) != SLAG_OK ||
        hipHostMalloc((void**)&c->host_small, SM_WORDS * 8, hipHostMallocDefault) != hipSuccess) {
        slag_destroy(c);
        return SLAG_E_OUT_OF_MEMORY;
    }
    std::memset(c->host_small, 0, SM_WORDS * 8);
    if (hipMemset(c->small.p, 0, SM_WORDS * 8) != hipSuccess) {
        slag_destroy(c);
        return SLAG_E_DEVICE;
    }
    {
        // persistent compositing: eight resident workgroups per compute unit;
        // the tuning cache is keyed by the device kind
        hipDeviceProp_t pr;
        if (hipGetDeviceProperties(&pr, device) != hipSuccess) {
            slag_destroy(c);
            return SLAG_E_DEVICE;
        }
        c->pgrid = (uint32_t)std::max(pr.multiProcessorCount, 1) * 8u;
        std::string arch(pr.gcnArchName);
        for (auto& ch : arch)
            if (std::isspace((unsigned char)ch)) ch = '_';
        c->dev_kind = arch + "/" + std::to_string(pr.multiProcessorCount) + "/tile" +
                      std::to_string(c->ts);
        const char* path = std::getenv("SLAG_TUNE_CACHE");
        c->tune_cache = path ? path : "";
        load_tune_cache(c);
    }
    *out = c;
    return SLAG_OK;
}

void slag_destroy(slag_ctx* c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->st) (void)hipStreamSynchronize(c->st);
    DevBuf* bufs[] = {&c->means, &c->scales, &c->quats, &c->opac, &c->cov3, &c->covd, &c->lo2,
                      &c->ids, &c->feats,
                      &c->num, &c->den, &c->ns_tile, &c->segl, &c->sat, &c->tcnt, &c->blk_vis,
                      &c->small, &c->scan_ws, &c->hist, &c->rec, &c->pgauss, &c->pview, &c->dkey,
                      &c->dkey_alt, &c->dval, &c->dval_alt, &c->psz, &c->pz, &c->tcr, &c->wlen,
                      &c->ikey, &c->ikey_alt, &c->ival, &c->ival_alt, &c->bstart, &c->bend,
                      &c->part, &c->wrow, &c->perm, &c->rank, &c->pair_of_m,
                      &c->pinfo, &c->prect, &c->prank, &c->blk_aux, &c->bkey,
                      &c->bkey_alt, &c->bord, &c->bord_alt, &c->tflag, &c->tpos, &c->tv,
                      &c->tv_alt, &c->tg, &c->thead, &c->tk, &c->tk_alt, &c->pixdbg,
                      &c->outbf, &c->idstage, &c->bgeo, &c->vlist, &c->vcnt, &c->cnum, &c->cden, &c->cbf,
                      &c->query.emb, &c->query.q, &c->query.qt, &c->query.counts,
                      &c->query.keys, &c->query.vals, &c->query.keys_alt, &c->query.vals_alt,
                      &c->query.hist, &c->query.scan_ws, &c->rattr, &c->rout, &c->gkey,
                      &c->gkey_alt, &c->gval, &c->gval_alt, &c->cks, &c->cA, &c->cnext,
                      &c->chead, &c->rowden,
                      &c->rbatch.views, &c->rbatch.bucket_view, &c->rbatch.view_cls};
    destroy_graph(c);
    for (DevBuf* b : bufs) release(*b);
    codec_release(c);
    for (auto& b : c->plan) { release(b.views); release(b.bucket_view); release(b.view_cls); }
    for (auto& e : c->events) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
    for (auto e : c->tune_ev)
        if (e) (void)hipEventDestroy(e);
    for (auto e : c->free_events) (void)hipEventDestroy(e);
    if (c->host_small) (void)hipHostFree(c->host_small);
    if (c->chost) (void)hipHostFree(c->chost);
    if (c->own_stream && c->st) (void)hipStreamDestroy(c->st);
    delete c;
}

const char* slag_last_error(const slag_ctx* c) { return c ? c->err.c_str() : "null context"; }

slag_status slag_get_tuning(slag_ctx* c, slag_tuning* out, int32_t cap, int32_t* n)
{
    if (!c || !n || cap < 0 || (cap > 0 && !out)) return SLAG_E_INVALID_ARG;
    c->err.clear();
    *n = (int32_t)c->tune.size();
    int32_t i = 0;
    for (const auto& kv : c->tune) {
        if (i >= cap) break;
        slag_tuning& t = out[i++];
        t.width = (int32_t)(kv.first >> 32);
        t.height = (int32_t)(kv.first & 0xFFFFFFFFu);
        t.variant = kv.second.variant;
        t.n_variants = kv.second.n_variants;
        for (int v = 0; v < 8; v++) t.ms[v] = kv.second.ms[v];
    }
    return SLAG_OK;
}

const char* slag_variant_name(int32_t v) { return composite_variant_name(v); }

int32_t slag_variant_count(void) { return composite_variants(); }

const char* slag_stage_name(int32_t s)
{
    return (s >= 0 && s < ST_COUNT_) ? kStageNames[s] : "";
}

slag_status slag_set_gaussians(slag_ctx* c, int64_t n, const float* means, const float* scales,
                               const float* quats, const float* opacity, slag_mem where)
{
    if (!c) return SLAG_E_INVALID_ARG;
    c->err.clear();
    invalidate_graph(c);
    if (n < 0 || (n > 0 && (!means || !scales || !quats || !opacity)))
        FAIL(c, SLAG_E_INVALID_ARG, "null pointer or negative Gaussian count");
    // the projection grid holds one row of workgroups per 2048 Gaussians
    if (n >= ((int64_t)1 << 31) || count_blocks_per_view(n) > 65535)
        FAIL(c, SLAG_E_CAPACITY, "at most 65535 x 2048 Gaussians");
    if (where != SLAG_HOST && where != SLAG_DEVICE) FAIL(c, SLAG_E_INVALID_ARG, "bad memory kind");
    HC(c, hipSetDevice(c->device));
    CK(copy_in(c, c->means, means, (size_t)n * 12, where));
    CK(copy_in(c, c->scales, scales, (size_t)n * 12, where));
    CK(copy_in(c, c->quats, quats, (size_t)n * 16, where));
    CK(copy_in(c, c->opac, opacity, (size_t)n * 4, where));
    CK(ensure(c, c->cov3, (size_t)std::max<int64_t>(n, 1) * 24));
    CK(ensure(c, c->covd, (size_t)std::max<int64_t>(n, 1) * 48));
    CK(ensure(c, c->lo2, (size_t)std::max<int64_t>(n, 1) * 4));
    uint32_t* err = reinterpret_cast<uint32_t*>(c->small.as<uint64_t>() + SM_ERR);
    launch_fill_u32(err, 1, 0u, c->st);
    launch_prep_gauss(n, c->means.as<float>(), c->scales.as<float>(), c->quats.as<float>(),
                      c->opac.as<float>(), c->cov3.as<float>(), c->covd.as<double>(),
                      c->lo2.as<float>(), err, c->st);
    CK(read_small(c, SM_ERR, 1));
    c->n = -1;
    c->have_out = false;
    if (c->host_small[SM_ERR] & 1)
        FAIL(c, SLAG_E_INVALID_ARG, "Gaussian parameters must be finite, scales > 0, quaternions "
                                    "non-zero and opacity in (0, 1]");
    CK(morton_order(c, n));
    c->n = n;
    c->plan_views = -1;   // launch sizes depend on n
    c->auto_maxv = 0;
    return SLAG_OK;
}

slag_status slag_set_cameras(slag_ctx* c, int32_t n_views, const slag_camera* cams)
{
    if (!c) return SLAG_E_INVALID_ARG;
    c->err.clear();
    invalidate_graph(c);
    if (n_views < 0 || (n_views > 0 && !cams)) FAIL(c, SLAG_E_INVALID_ARG, "bad camera array");
    uint64_t tot = 0;
    std::vector<uint64_t> off(n_views + 1, 0);
    for (int v = 0; v < n_views; v++) {
        const slag_camera& k = cams[v];
        if (k.width <= 0 || k.height <= 0 || k.width > 65535 || k.height > 65535)
            FAIL(c, SLAG_E_INVALID_ARG, "camera " + std::to_string(v) + ": image size out of range");
        bool fin = std::isfinite(k.fx) && std::isfinite(k.fy) && std::isfinite(k.cx) &&
                   std::isfinite(k.cy) && k.fx > 0 && k.fy > 0;
        for (int i = 0; i < 9; i++) fin = fin && std::isfinite(k.R[i]);
        for (int i = 0; i < 3; i++) fin = fin && std::isfinite(k.t[i]);
        if (!fin) FAIL(c, SLAG_E_INVALID_ARG, "camera " + std::to_string(v) + ": non-finite or "
                                              "non-positive intrinsics/extrinsics");
        off[v] = tot;
        tot += (uint64_t)k.width * (uint64_t)k.height;
    }
    off[n_views] = tot;
    HC(c, hipSetDevice(c->device));
    CK(ensure(c, c->ids, std::max<uint64_t>(tot, 1) * 4 * (uint64_t)c->lpp));
    c->cams.assign(cams, cams + n_views);
    c->pix_off = off;
    c->nviews = n_views;
    c->nseg.assign(n_views, 0);
    c->seg_set.assign(n_views, 0);
    c->feats_set = false;
    c->have_out = false;
    c->plan_views = -1;
    c->auto_maxv = 0;
    return SLAG_OK;
}

slag_status slag_set_segments(slag_ctx* c, int32_t view, const int32_t* ids, int32_t n_seg,
                              slag_mem where)
{
    return slag_set_segments_multi(c, view, ids, 1, n_seg, where);
}

slag_status slag_set_segments_multi(slag_ctx* c, int32_t view, const int32_t* ids, int32_t nl,
                                    int32_t n_seg, slag_mem where)
{
    if (!c) return SLAG_E_INVALID_ARG;
    c->err.clear();
    invalidate_graph(c);
    if (c->nviews < 0) FAIL(c, SLAG_E_STATE, "set cameras before segments");
    if (view < 0 || view >= c->nviews) FAIL(c, SLAG_E_INVALID_ARG, "view index out of range");
    if (!ids || n_seg < 0) FAIL(c, SLAG_E_INVALID_ARG, "null ids or negative segment count");
    if (nl < 1 || nl > c->lpp)
        FAIL(c, SLAG_E_INVALID_ARG, "labels per pixel must be in [1, labels_per_pixel = " +
                                        std::to_string(c->lpp) + "]");
    if (where != SLAG_HOST && where != SLAG_DEVICE) FAIL(c, SLAG_E_INVALID_ARG, "bad memory kind");
    if (n_seg > 65535) FAIL(c, SLAG_E_NOT_SUPPORTED, "at most 65535 segments per view");
    HC(c, hipSetDevice(c->device));
    const uint64_t npix = c->pix_off[view + 1] - c->pix_off[view];
    const int L = c->lpp;
    int32_t* dst = c->ids.as<int32_t>() + c->pix_off[view] * (uint64_t)L;
    if (nl == L) {
        HC(c, hipMemcpyAsync(dst, ids, npix * 4 * (uint64_t)L,
                             where == SLAG_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                             c->st));
    } else {
        // fewer labels than the context's layout: widened with -1
        const int32_t* src = ids;
        if (where == SLAG_HOST) {
            CK(ensure(c, c->idstage, npix * 4 * (uint64_t)nl));
            HC(c, hipMemcpyAsync(c->idstage.p, ids, npix * 4 * (uint64_t)nl, hipMemcpyHostToDevice,
                                 c->st));
            src = c->idstage.as<int32_t>();
        }
        launch_expand_labels((int64_t)npix, src, nl, dst, L, c->st);
    }
    uint32_t* err = reinterpret_cast<uint32_t*>(c->small.as<uint64_t>() + SM_ERR);
    launch_fill_u32(err, 1, 0u, c->st);
    launch_validate_ids((int64_t)npix, dst, L, n_seg, err, c->st);
    CK(read_small(c, SM_ERR, 1));
    if (c->host_small[SM_ERR] & 2) {
        c->seg_set[view] = 0;
        FAIL(c, SLAG_E_INVALID_ARG, "segment id out of range [-1, n_seg), or a mask listed "
                                    "twice for one pixel, in view " + std::to_string(view));
    }
    if (c->nseg[view] != n_seg) c->feats_set = false;
    c->nseg[view] = n_seg;
    c->seg_set[view] = 1;
    c->have_out = false;
    c->plan_views = -1;
    return SLAG_OK;
}

slag_status slag_set_features(slag_ctx* c, int32_t d, slag_dtype dtype, const void* table,
                              slag_mem where)
{
    if (!c) return SLAG_E_INVALID_ARG;
    c->err.clear();
    invalidate_graph(c);
    if (c->nviews < 0) FAIL(c, SLAG_E_STATE, "set cameras and segments before features");
    for (int v = 0; v < c->nviews; v++)
        if (!c->seg_set[v]) FAIL(c, SLAG_E_STATE, "segments of view " + std::to_string(v) + " not set");
    if (d <= 0 || (dtype != SLAG_F32 && dtype != SLAG_BF16))
        FAIL(c, SLAG_E_INVALID_ARG, "bad feature dimension or dtype");
    if (!contract_supported(d))
        FAIL(c, SLAG_E_NOT_SUPPORTED, "feature dimension must be 64, 128, 256, 512, 768 or 1024");
    uint64_t rows = 0;
    for (int v = 0; v < c->nviews; v++) rows += (uint64_t)c->nseg[v];
    if (rows > 0 && !table) FAIL(c, SLAG_E_INVALID_ARG, "null feature table");
    // the contraction addresses BF16 rows with 32-bit byte offsets
    if (dtype == SLAG_BF16 && rows * (uint64_t)d * 2u > 0xFFFFFFFFull)
        FAIL(c, SLAG_E_CAPACITY, "BF16 feature table over 4 GiB");
    HC(c, hipSetDevice(c->device));
    const size_t es = dtype == SLAG_BF16 ? 2 : 4;
    CK(copy_in(c, c->feats, table, rows * (size_t)d * es, where));
    CK(ensure(c, c->feats, std::max<size_t>(rows * (size_t)d * es, 16)));
    c->d = d;
    c->fdt = dtype;
    c->feat_rows = rows;
    c->feats_set = true;
    c->have_out = false;
    return SLAG_OK;
}

}  // extern "C"

namespace slag_host {

// The launch sequence of one lift (eager, or recorded into a graph while
// c->capturing: then no host synchronisation, allocation or event).
static slag_status lift_sequence(slag_ctx* c, bool codec)
{
    CodecState& K = c->codec;
    const int64_t n = c->n;
    uint64_t* small = c->small.as<uint64_t>();
    launch_fill_u32(reinterpret_cast<uint32_t*>(small + SM_COUNTERS), 12, 0u, c->st);
    launch_fill_u32(reinterpret_cast<uint32_t*>(small + SM_LERR), 2, 0u, c->st);
    if (n == 0) return SLAG_OK;
    ContractTarget ct{c->feats.p, c->d, c->fdt == SLAG_BF16, c->num.as<float>(), c->den.as<float>()};
    if (codec) {
        hipEvent_t ev;
        CK(stage_begin(c, ST_ENCODE, &ev));
        CK(codec_encode_table(c));
        CK(stage_end(c, ST_ENCODE, ev));
        CK(ensure(c, K.codes, (size_t)n * K.k * 4));
        ct = ContractTarget{K.C.p, K.k, false, K.codes.as<float>(), c->den.as<float>()};
    }
    if (c->plan.empty()) {
        launch_fill_u32(reinterpret_cast<uint32_t*>(ct.out), (uint64_t)n * ct.d, 0u, c->st);
        launch_fill_u32(c->den.as<uint32_t>(), (uint64_t)n, 0u, c->st);
    }
    for (size_t i = 0; i < c->plan.size(); i++)
        CK(lift_batch(c, c->plan[i], i == 0, i + 1 == c->plan.size(), ct));
    if (codec) {
        hipEvent_t ev;
        CK(stage_begin(c, ST_DECODE, &ev));
        CK(codec_decode_codes(c));
        CK(stage_end(c, ST_DECODE, ev));
    }
    return SLAG_OK;
}

static void drop_graph(slag_ctx* c)
{
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    c->graph_mode = -1;
}

// Record the launch sequence of the lift just run eagerly into a graph.
static slag_status capture_lift(slag_ctx* c, bool codec)
{
    drop_graph(c);
    HC(c, hipStreamBeginCapture(c->st, hipStreamCaptureModeRelaxed));
    c->capturing = true;
    const slag_status s = lift_sequence(c, codec);
    c->capturing = false;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->st, &g);
    if (s != SLAG_OK) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        c->err = std::string("graph capture: ") + hipGetErrorString(e);
        return SLAG_E_DEVICE;
    }
    c->graph = g;
    const hipError_t ei = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
        drop_graph(c);
        c->err = std::string("graph instantiate: ") + hipGetErrorString(ei);
        return SLAG_E_DEVICE;
    }
    c->graph_gen = c->gen;
    c->graph_mode = codec ? 1 : 0;
    return SLAG_OK;
}

static slag_status check_inputs(slag_ctx* c)
{
    if (c->n < 0) FAIL(c, SLAG_E_STATE, "Gaussians not set");
    if (c->nviews < 0) FAIL(c, SLAG_E_STATE, "cameras not set");
    for (int v = 0; v < c->nviews; v++)
        if (!c->seg_set[v]) FAIL(c, SLAG_E_STATE, "segments of view " + std::to_string(v) + " not set");
    if (!c->feats_set) FAIL(c, SLAG_E_STATE, "features not set (or segment counts changed)");
    return SLAG_OK;
}

slag_status run_lift(slag_ctx* c, bool codec)
{
    if (!c) return SLAG_E_INVALID_ARG;
    c->err.clear();
    CK(check_inputs(c));
    CodecState& K = c->codec;
    if (codec && !K.ready) FAIL(c, SLAG_E_STATE, "codec not initialised");
    if (codec && K.d != c->d) FAIL(c, SLAG_E_STATE, "codec dimension differs from the features'");
    HC(c, hipSetDevice(c->device));
    c->have_out = false;
    c->out_is_codec = false;
    K.have_codes = false;
    for (auto& e : c->events) { c->free_events.push_back(e.a); c->free_events.push_back(e.b); }
    c->events.clear();
    const bool use_graph = (c->opt.flags & SLAG_FLAG_GRAPH) != 0;
    const bool replay = use_graph && c->gexec && c->graph_gen == c->gen &&
                        c->graph_mode == (codec ? 1 : 0) && c->plan_views == c->nviews;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->opt.flags & SLAG_FLAG_PROFILE) {
        CK(stage_begin(c, -1, &e0));
    }
    if (replay) {
        HC(c, hipGraphLaunch(c->gexec, c->st));
        c->stats = c->graph_stats;
    } else {
        std::memset(&c->stats, 0, sizeof(c->stats));
        c->last_v0 = -1;
        const int64_t n = c->n;
        CK(ensure(c, c->num, (size_t)std::max<int64_t>(n, 1) * c->d * 4));
        CK(ensure(c, c->den, (size_t)std::max<int64_t>(n, 1) * 4));
        if (c->plan_views != c->nviews) CK(build_plan(c));
        for (;;) {
            c->replan_views = 0;
            const slag_status s = lift_sequence(c, codec);
            if (s == SLAG_OK) break;
            // a launch too large for 32-bit list positions: fewer views per
            // launch, then the whole sequence again (the first batch rewrites
            // the outputs)
            if (s != SLAG_E_CAPACITY || c->replan_views <= 0) return s;
            c->auto_maxv = c->replan_views;
            std::memset(&c->stats, 0, sizeof(c->stats));
            c->last_v0 = -1;
            CK(build_plan(c));
        }
        c->stats.n_views = c->nviews;
        c->stats.n_batches = (int64_t)c->plan.size();
    }
    if (e0) {
        if (!c->free_events.empty()) { e1 = c->free_events.back(); c->free_events.pop_back(); }
        else HC(c, hipEventCreate(&e1));
        HC(c, hipEventRecord(e1, c->st));
        c->events.push_back({-1, e0, e1});
    }
    if (use_graph && !replay && c->n > 0) {
        c->graph_stats = c->stats;
        for (int i = 0; i < 16; i++) c->graph_stats.ms_stage[i] = 0.0;
        // recording the launch sequence walks the batches again: keep the
        // eager lift's counts
        const slag_stats eager = c->stats;
        CK(capture_lift(c, codec));
        c->stats = eager;
    }
    c->have_out = true;
    c->out_is_codec = codec;
    c->lists_valid = true;
    K.have_codes = codec;
    return SLAG_OK;
}

// The lift with the output streamed to host memory in chunks of Morton
// ranks (slag_lift_chunked).
static slag_status chunked_lift(slag_ctx* c, int64_t R, void* out, slag_dtype dtype, float* den)
{
    const int64_t n = c->n;
    const int d = c->d;
    hipStream_t st = c->st;
    const size_t esz = dtype == SLAG_BF16 ? 2 : 4;
    CK(ensure(c, c->cnum, (size_t)R * d * 4));
    CK(ensure(c, c->cden, (size_t)R * 4));
    if (dtype == SLAG_BF16) CK(ensure(c, c->cbf, (size_t)R * d * 2));
    const size_t hbytes = (size_t)R * d * esz + (size_t)R * 4;
    if (c->chost_cap < hbytes) {
        if (c->chost) (void)hipHostFree(c->chost);
        c->chost = nullptr;
        c->chost_cap = 0;
        if (hipHostMalloc(&c->chost, hbytes, hipHostMallocDefault) != hipSuccess)
            FAIL(c, SLAG_E_OUT_OF_MEMORY, "pinned staging for a chunked lift");
        c->chost_cap = hbytes;
    }
    std::vector<uint32_t> perm((size_t)n);
    HC(c, hipMemcpyAsync(perm.data(), c->perm.p, (size_t)n * 4, hipMemcpyDeviceToHost, st));
    HC(c, hipStreamSynchronize(st));
    unsigned char* hrow = static_cast<unsigned char*>(c->chost);
    float* hden = reinterpret_cast<float*>(hrow + (size_t)R * d * esz);
    const bool single = c->plan.size() == 1;
    slag_stats first_stats{};
    for (int64_t r0 = 0; r0 < n; r0 += R) {
        const int64_t r1 = std::min<int64_t>(n, r0 + R);
        ContractTarget ct{c->feats.p, d, c->fdt == SLAG_BF16, c->cnum.as<float>(),
                          c->cden.as<float>(), r0, r1, true};
        for (size_t i = 0; i < c->plan.size(); i++) {
            const bool first = i == 0, last = i + 1 == c->plan.size();
            if (single && r0 > 0) CK(contract_batch(c, c->plan[i], first, last, ct));
            else CK(lift_batch(c, c->plan[i], first, last, ct));
        }
        if (r0 == 0) first_stats = c->stats;
        const int64_t rows = r1 - r0;
        if (out) {
            if (dtype == SLAG_BF16) {
                launch_f32_to_bf16((uint64_t)rows * d, c->cnum.as<float>(), c->cbf.as<uint16_t>(), st);
                HC(c, hipMemcpyAsync(hrow, c->cbf.p, (size_t)rows * d * 2, hipMemcpyDeviceToHost, st));
            } else {
                HC(c, hipMemcpyAsync(hrow, c->cnum.p, (size_t)rows * d * 4, hipMemcpyDeviceToHost, st));
            }
        }
        if (den) HC(c, hipMemcpyAsync(hden, c->cden.p, (size_t)rows * 4, hipMemcpyDeviceToHost, st));
        HC(c, hipStreamSynchronize(st));
        // rows arrive in Morton order: each goes to its caller index
        const size_t rb = (size_t)d * esz;
        for (int64_t q = r0; q < r1; q++) {
            const size_t g = perm[(size_t)q];
            if (out) std::memcpy(static_cast<unsigned char*>(out) + g * rb, hrow + (size_t)(q - r0) * rb, rb);
            if (den) den[g] = hden[q - r0];
        }
    }
    c->stats = first_stats;
    return SLAG_OK;
}

// Errors the last lift's kernels flagged (bit 4: a tile held more distinct
// segments than its table).
slag_status check_lift_errors(slag_ctx* c)
{
    CK(read_small(c, SM_LERR, 1));
    if (c->host_small[SM_LERR] & 4)
        FAIL(c, SLAG_E_CAPACITY, "a 16x16 tile lies in more than 256 distinct masks; the result "
                                 "is incomplete");
    return SLAG_OK;
}

void invalidate_graph(slag_ctx* c) { c->gen++; }

void destroy_graph(slag_ctx* c) { drop_graph(c); }

}  // namespace slag_host

extern "C" {

slag_status slag_lift(slag_ctx* c) { return run_lift(c, false); }

slag_status slag_lift_chunked(slag_ctx* c, int64_t chunk_rows, void* out, slag_dtype dtype,
                              float* den)
{
    if (!c) return SLAG_E_INVALID_ARG;
    c->err.clear();
    if (chunk_rows <= 0 || chunk_rows % 16) FAIL(c, SLAG_E_INVALID_ARG, "chunk_rows must be a positive multiple of 16");
    if (dtype != SLAG_F32 && dtype != SLAG_BF16) FAIL(c, SLAG_E_INVALID_ARG, "bad output dtype");
    CK(check_inputs(c));
    HC(c, hipSetDevice(c->device));
    c->have_out = false;
    c->out_is_codec = false;
    c->codec.have_codes = false;
    for (auto& e : c->events) { c->free_events.push_back(e.a); c->free_events.push_back(e.b); }
    c->events.clear();
    std::memset(&c->stats, 0, sizeof(c->stats));
    c->last_v0 = -1;
    if (c->n == 0) return SLAG_OK;
    const int64_t R = std::min<int64_t>(chunk_rows, (c->n + 15) & ~(int64_t)15);
    if (c->plan_views != c->nviews) CK(build_plan(c));
    uint64_t* small = c->small.as<uint64_t>();
    for (;;) {
        launch_fill_u32(reinterpret_cast<uint32_t*>(small + SM_COUNTERS), 12, 0u, c->st);
        launch_fill_u32(reinterpret_cast<uint32_t*>(small + SM_LERR), 2, 0u, c->st);
        c->replan_views = 0;
        const slag_status s = chunked_lift(c, R, out, dtype, den);
        if (s == SLAG_OK) break;
        if (s != SLAG_E_CAPACITY || c->replan_views <= 0) return s;
        c->auto_maxv = c->replan_views;
        std::memset(&c->stats, 0, sizeof(c->stats));
        c->last_v0 = -1;
        CK(build_plan(c));
    }
    c->stats.n_views = c->nviews;
    c->stats.n_batches = (int64_t)c->plan.size();
    CK(check_lift_errors(c));
    CK(read_small(c, SM_COUNTERS + 3, 1));
    if (c->host_small[SM_COUNTERS + 3])
        FAIL(c, SLAG_E_CAPACITY, std::to_string(c->host_small[SM_COUNTERS + 3]) +
                                     " part-list entries did not fit their capacity; the result "
                                     "is incomplete");
    return SLAG_OK;
}

slag_status slag_get_embeddings(slag_ctx* c, void* out, slag_dtype dtype, float* den,
                                slag_mem where)
{
    if (!c) return SLAG_E_INVALID_ARG;
    c->err.clear();
    if (!c->have_out) FAIL(c, SLAG_E_STATE, "no lift result");
    if (dtype != SLAG_F32 && dtype != SLAG_BF16) FAIL(c, SLAG_E_INVALID_ARG, "bad output dtype");
    if (where != SLAG_HOST && where != SLAG_DEVICE) FAIL(c, SLAG_E_INVALID_ARG, "bad memory kind");
    HC(c, hipSetDevice(c->device));
    const hipMemcpyKind k = where == SLAG_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const size_t n = (size_t)c->n;
    if (out && n) {
        if (dtype == SLAG_F32) {
            HC(c, hipMemcpyAsync(out, c->num.p, n * c->d * 4, k, c->st));
        } else if (where == SLAG_DEVICE) {
            launch_f32_to_bf16((uint64_t)n * c->d, c->num.as<float>(), static_cast<uint16_t*>(out),
                               c->st);
        } else {
            CK(ensure(c, c->outbf, n * c->d * 2));
            launch_f32_to_bf16((uint64_t)n * c->d, c->num.as<float>(), c->outbf.as<uint16_t>(),
                               c->st);
            HC(c, hipMemcpyAsync(out, c->outbf.p, n * c->d * 2, k, c->st));
        }
    }
    if (den && n) HC(c, hipMemcpyAsync(den, c->den.p, n * 4, k, c->st));
    CK(check_lift_errors(c));
    // part-list capacity errors of the last lift (none by construction)
    CK(read_small(c, SM_COUNTERS + 3, 1));
    if (c->host_small[SM_COUNTERS + 3])
        FAIL(c, SLAG_E_CAPACITY, std::to_string(c->host_small[SM_COUNTERS + 3]) +
                                     " part-list entries did not fit their capacity; the result "
                                     "is incomplete");
    return SLAG_OK;
}

slag_status slag_get_stats(slag_ctx* c, slag_stats* s)
{
    if (!c || !s) return SLAG_E_INVALID_ARG;
    c->err.clear();
    HC(c, hipSetDevice(c->device));
    HC(c, hipStreamSynchronize(c->st));
    CK(read_small(c, SM_COUNTERS, 6));
    c->stats.n_lost = (int64_t)c->host_small[SM_COUNTERS + 3];
    c->stats.n_contrib = (int64_t)c->host_small[SM_COUNTERS];
    c->stats.n_tests = (int64_t)c->host_small[SM_COUNTERS + 1];
    c->stats.n_tile_tests = (int64_t)c->host_small[SM_COUNTERS + 2];
    c->stats.n_weights = (int64_t)c->host_small[SM_NNZ];
    for (int i = 0; i < 16; i++) c->stats.ms_stage[i] = 0.0;
    c->stats.ms_total = 0.0;
    for (auto& e : c->events) {
        float ms = 0.0f;
        HC(c, hipEventElapsedTime(&ms, e.a, e.b));
        if (e.stage < 0) c->stats.ms_total += ms;
        else c->stats.ms_stage[e.stage] += ms;
    }
    c->stats.n_stages = ST_COUNT_;
    *s = c->stats;
    return SLAG_OK;
}

slag_status slag_debug_tile_lists(slag_ctx* c, int32_t view, uint32_t* tile, uint32_t* depth_bits,
                                  uint32_t* gauss, int64_t cap, int64_t* len)
{
    if (!c || !len) return SLAG_E_INVALID_ARG;
    c->err.clear();
    if (!(c->opt.flags & SLAG_FLAG_KEEP_DEBUG) || c->last_v0 < 0)
        FAIL(c, SLAG_E_STATE, "debug exports need SLAG_FLAG_KEEP_DEBUG and a lift");
    if (view < c->last_v0 || view >= c->last_v0 + c->last_nb)
        FAIL(c, SLAG_E_STATE, "view not in the last launch");
    HC(c, hipSetDevice(c->device));
    HC(c, hipStreamSynchronize(c->st));
    const uint64_t ni = c->last_ni, np = c->last_npairs;
    *len = 0;
    if (!ni) return SLAG_OK;
    std::vector<uint32_t> k(ni), v(ni), pg(np), pz(np);
    HC(c, hipMemcpy(k.data(), c->last_ikey, ni * 4, hipMemcpyDeviceToHost));
    HC(c, hipMemcpy(v.data(), c->last_ival, ni * 4, hipMemcpyDeviceToHost));
    HC(c, hipMemcpy(pg.data(), c->pgauss.p, np * 4, hipMemcpyDeviceToHost));
    HC(c, hipMemcpy(pz.data(), c->pz.p, np * 4, hipMemcpyDeviceToHost));
    const Batch* B = nullptr;
    for (auto& b : c->plan)
        if (b.v0 == c->last_v0) B = &b;
    if (!B) FAIL(c, SLAG_E_STATE, "launch plan changed since the lift");
    // keys are (view in launch << lbits) | tile in view; lists come out
    // tile-major within the key order, so sort this view's entries by tile
    // (stable: depth order within a tile is kept)
    const uint32_t vl = (uint32_t)(view - c->last_v0);
    const uint32_t mask = (1u << B->lbits) - 1u;
    std::vector<uint64_t> sel;
    for (uint64_t i = 0; i < ni; i++)
        if ((k[i] >> B->lbits) == vl) sel.push_back(((uint64_t)(k[i] & mask) << 32) | (uint64_t)i);
    std::stable_sort(sel.begin(), sel.end(),
                     [](uint64_t a, uint64_t b) { return (a >> 32) < (b >> 32); });
    const int64_t m = (int64_t)sel.size();
    *len = m;
    if (m > cap) return SLAG_OK;
    for (int64_t o = 0; o < m; o++) {
        const uint64_t i = sel[o] & 0xFFFFFFFFull;
        if (tile) tile[o] = (uint32_t)(sel[o] >> 32);
        if (depth_bits) depth_bits[o] = pz[v[i]];
        if (gauss) gauss[o] = pg[v[i]];
    }
    return SLAG_OK;
}

slag_status slag_debug_weights(slag_ctx* c, int32_t view, uint32_t* gauss, uint32_t* seg, float* w,
                               int64_t cap, int64_t* len)
{
    if (!c || !len) return SLAG_E_INVALID_ARG;
    c->err.clear();
    if (!(c->opt.flags & SLAG_FLAG_KEEP_DEBUG) || c->last_v0 < 0)
        FAIL(c, SLAG_E_STATE, "debug exports need SLAG_FLAG_KEEP_DEBUG and a lift");
    if (view < c->last_v0 || view >= c->last_v0 + c->last_nb)
        FAIL(c, SLAG_E_STATE, "view not in the last launch");
    HC(c, hipSetDevice(c->device));
    HC(c, hipStreamSynchronize(c->st));
    const uint64_t np = c->last_npairs;
    *len = 0;
    if (!np) return SLAG_OK;
    std::vector<uint32_t> pg(np), wl(np), pb(np);
    std::vector<uint16_t> pv(np);
    HC(c, hipMemcpy(pg.data(), c->pgauss.p, np * 4, hipMemcpyDeviceToHost));
    HC(c, hipMemcpy(wl.data(), c->wlen.p, np * 4, hipMemcpyDeviceToHost));
    HC(c, hipMemcpy(pb.data(), c->psz.p, np * 4, hipMemcpyDeviceToHost));
    HC(c, hipMemcpy(pv.data(), c->pview.p, np * 2, hipMemcpyDeviceToHost));
    const uint16_t vl = (uint16_t)(view - c->last_v0);
    uint64_t seg_off = 0;
    for (int i = 0; i < view; i++) seg_off += (uint64_t)c->nseg[i];
    int64_t m = 0;
    for (uint64_t p = 0; p < np; p++)
        if (pv[p] == vl) m += wl[p];
    *len = m;
    if (m > cap) return SLAG_OK;
    int64_t o = 0;
    std::vector<uint2> row;
    for (uint64_t p = 0; p < np; p++) {
        if (pv[p] != vl || !wl[p]) continue;
        row.resize(wl[p]);
        HC(c, hipMemcpy(row.data(), c->wrow.as<uint2>() + pb[p], wl[p] * 8, hipMemcpyDeviceToHost));
        for (uint32_t i = 0; i < wl[p]; i++) {
            if (gauss) gauss[o] = pg[p];
            if (seg) seg[o] = (uint32_t)(row[i].x - seg_off);
            if (w) { float f; std::memcpy(&f, &row[i].y, 4); w[o] = f; }
            o++;
        }
    }
    return SLAG_OK;
}

}  // extern "C"

extern "C" slag_status slag_get_debug(slag_ctx* c, slag_debug what, int32_t view, void* out,
                                      int64_t cap, int64_t* len)
{
    if (!c || !len || cap < 0 || (cap > 0 && !out)) return SLAG_E_INVALID_ARG;
    c->err.clear();
    *len = 0;
    if (what == SLAG_DEBUG_COUNTERS) {
        HC(c, hipSetDevice(c->device));
        HC(c, hipStreamSynchronize(c->st));
        CK(read_small(c, SM_COUNTERS, 4));
        *len = 32;
        if (cap >= 32) std::memcpy(out, c->host_small + SM_COUNTERS, 32);
        return SLAG_OK;
    }
    if (!(c->opt.flags & SLAG_FLAG_KEEP_DEBUG) || c->last_v0 < 0)
        FAIL(c, SLAG_E_STATE, "debug exports need SLAG_FLAG_KEEP_DEBUG and a lift");
    if (view < c->last_v0 || view >= c->last_v0 + c->last_nb)
        FAIL(c, SLAG_E_STATE, "view not in the last launch");
    HC(c, hipSetDevice(c->device));
    const int W = c->cams[view].width, H = c->cams[view].height;
    switch (what) {
    case SLAG_DEBUG_KEYS:
    case SLAG_DEBUG_TILE_RANGES: {
        int64_t m = 0;
        CK(slag_debug_tile_lists(c, view, nullptr, nullptr, nullptr, 0, &m));
        std::vector<uint32_t> t(m), z(m), g(m);
        if (m) CK(slag_debug_tile_lists(c, view, t.data(), z.data(), g.data(), m, &m));
        if (what == SLAG_DEBUG_KEYS) {
            *len = m * 12;
            if (*len > cap) return SLAG_OK;
            uint32_t* o = static_cast<uint32_t*>(out);
            for (int64_t i = 0; i < m; i++) {
                o[3 * i] = t[i];
                o[3 * i + 1] = z[i];
                o[3 * i + 2] = g[i];
            }
        } else {
            const int64_t nt = (int64_t)((W + c->ts - 1) / c->ts) * ((H + c->ts - 1) / c->ts);
            *len = nt * 8;
            if (*len > cap) return SLAG_OK;
            uint32_t* o = static_cast<uint32_t*>(out);
            int64_t i = 0;
            for (int64_t k = 0; k < nt; k++) {
                o[2 * k] = (uint32_t)i;
                while (i < m && t[i] == (uint32_t)k) i++;
                o[2 * k + 1] = (uint32_t)i;
            }
        }
        return SLAG_OK;
    }
    case SLAG_DEBUG_W_VIEW: {
        int64_t m = 0;
        CK(slag_debug_weights(c, view, nullptr, nullptr, nullptr, 0, &m));
        *len = m * 12;
        if (*len > cap || !m) return SLAG_OK;
        std::vector<uint32_t> g(m), s(m);
        std::vector<float> w(m);
        CK(slag_debug_weights(c, view, g.data(), s.data(), w.data(), m, &m));
        uint32_t* o = static_cast<uint32_t*>(out);
        for (int64_t i = 0; i < m; i++) {
            o[3 * i] = g[i];
            o[3 * i + 1] = s[i];
            std::memcpy(&o[3 * i + 2], &w[i], 4);
        }
        return SLAG_OK;
    }
    case SLAG_DEBUG_PIXEL_T_FINAL:
    case SLAG_DEBUG_PIXEL_WSUM:
    case SLAG_DEBUG_PIXEL_COUNT: {
        if (!c->last_pix)
            FAIL(c, SLAG_E_STATE, "per-pixel exports need a lift with SLAG_FLAG_COUNT");
        const uint64_t P = c->pix_off[c->nviews];
        const uint64_t npx = (uint64_t)W * (uint64_t)H;
        *len = (int64_t)(npx * 4);
        if (*len > cap) return SLAG_OK;
        const int k = what == SLAG_DEBUG_PIXEL_T_FINAL ? 0 : what == SLAG_DEBUG_PIXEL_WSUM ? 1 : 2;
        const uint32_t* src = c->pixdbg.as<uint32_t>() + (uint64_t)k * P + c->pix_off[view];
        HC(c, hipStreamSynchronize(c->st));
        HC(c, hipMemcpy(out, src, npx * 4, hipMemcpyDeviceToHost));
        return SLAG_OK;
    }
    default:
        FAIL(c, SLAG_E_INVALID_ARG, "unknown debug export");
    }
}

// Render-back: one launch of the single view through projection, depth sort,
// binning and tile ranges (no segments), then the attribute walk.
extern "C" slag_status slag_render(slag_ctx* c, int32_t view, const float* attr, int32_t C,
                                   slag_mem attr_where, float* out, float* wsum,
                                   slag_mem out_where)
{
    if (!c) return SLAG_E_INVALID_ARG;
    c->err.clear();
    if (c->n < 0) FAIL(c, SLAG_E_STATE, "Gaussians not set");
    if (c->nviews < 0) FAIL(c, SLAG_E_STATE, "cameras not set");
    if (view < 0 || view >= c->nviews) FAIL(c, SLAG_E_INVALID_ARG, "view out of range");
    if (C < 1 || C > 1024) FAIL(c, SLAG_E_INVALID_ARG, "1 to 1024 attribute channels");
    if ((c->n > 0 && !attr) || !out) FAIL(c, SLAG_E_INVALID_ARG, "null attribute or output pointer");
    if ((attr_where != SLAG_HOST && attr_where != SLAG_DEVICE) ||
        (out_where != SLAG_HOST && out_where != SLAG_DEVICE))
        FAIL(c, SLAG_E_INVALID_ARG, "bad memory kind");
    HC(c, hipSetDevice(c->device));
    hipStream_t st = c->st;
    const slag_camera& cam = c->cams[view];
    const int64_t npix = (int64_t)cam.width * cam.height;
    const int64_t ntiles = (int64_t)((cam.width + c->ts - 1) / c->ts) * ((cam.height + c->ts - 1) / c->ts);
    const int lbits = std::max(1, bit_length((uint64_t)std::max<int64_t>(ntiles - 1, 0)));
    if (lbits > 31) FAIL(c, SLAG_E_CAPACITY, "image too large for 32-bit tile keys");
    float* dout = out;
    float* dws = wsum;
    if (out_where == SLAG_HOST) {
        CK(ensure(c, c->rout, (size_t)npix * (size_t)(C + 1) * 4 + 16));
        dout = c->rout.as<float>();
        dws = dout + (size_t)npix * C;
    }
    const float* dattr = attr;
    if (attr_where == SLAG_HOST && c->n > 0) {
        CK(ensure(c, c->rattr, (size_t)c->n * C * 4));
        HC(c, hipMemcpyAsync(c->rattr.p, attr, (size_t)c->n * C * 4, hipMemcpyHostToDevice, st));
        dattr = c->rattr.as<float>();
    }
    release(c->rbatch.views);
    release(c->rbatch.bucket_view);
    release(c->rbatch.view_cls);
    c->rbatch = Batch();
    const std::vector<uint64_t> seg_off((size_t)c->nviews + 1, 0);   // no segments
    CK(make_batch(c, view, 1, lbits, seg_off, c->rbatch));
    // the shared list buffers are rewritten: the last lift's debug exports go
    const slag_stats keep = c->stats;
    const int32_t flags = c->opt.flags;
    c->opt.flags &= ~SLAG_FLAG_PROFILE;
    c->front_only = true;
    c->front_ival = nullptr;
    c->last_v0 = -1;
    c->lists_valid = false;
    ContractTarget ct{};
    const slag_status s = c->n > 0 ? lift_batch(c, c->rbatch, true, true, ct) : SLAG_OK;
    c->front_only = false;
    c->opt.flags = flags;
    c->stats = keep;
    if (s != SLAG_OK) return s;
    if (c->front_ival) {
        launch_render(c->kernel_w, c->ts, (int)ntiles, c->rbatch.views.as<ViewDev>(), 0,
                      c->bstart.as<uint32_t>(), c->bend.as<uint32_t>(), c->front_ival,
                      c->rec.as<float4>(), c->pgauss.as<uint32_t>(), dattr, C, dout, dws, st);
    } else {
        launch_fill_u32(reinterpret_cast<uint32_t*>(dout), (uint64_t)npix * C, 0u, st);
        if (dws) launch_fill_u32(reinterpret_cast<uint32_t*>(dws), (uint64_t)npix, 0u, st);
    }
    HC(c, hipGetLastError());
    if (out_where == SLAG_HOST) {
        HC(c, hipMemcpyAsync(out, dout, (size_t)npix * C * 4, hipMemcpyDeviceToHost, st));
        if (wsum) HC(c, hipMemcpyAsync(wsum, dws, (size_t)npix * 4, hipMemcpyDeviceToHost, st));
    }
    HC(c, hipStreamSynchronize(st));
    return SLAG_OK;
}
