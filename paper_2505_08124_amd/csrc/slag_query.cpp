// Host side of the cosine-similarity search (include/slag_query.h): argument
// checks, workspace, and the launch sequence qprep -> scores -> per-query
// sort -> top-k rows.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/slag_query.h"
#include "slag_ctx.h"

using namespace slag_host;
using namespace slag;

namespace {

constexpr int QMAX = 64;

// Work arrays of one search, carved by the caller (library workspace).
struct QueryWork {
    const float* emb = nullptr;   // [n][d] on the device
    float* q = nullptr;           // queries staged on the device (host input), or null
    float* qt = nullptr;          // [d][qp]
    unsigned long long* counts = nullptr;   // [qp] + error word
    uint32_t *keys = nullptr, *vals = nullptr, *keys_alt = nullptr, *vals_alt = nullptr;
    uint32_t* hist = nullptr;
    void* scan_ws = nullptr;
};

size_t sort_scan_bytes(int64_t n) { return scan_workspace_bytes(radix_hist_bytes((uint64_t)n) / 4 + 1); }

slag_status check_args(slag_ctx* c, int64_t n, int32_t d, const float* emb, slag_mem ew, int32_t nq,
                       const float* q, slag_mem qw, slag_mem ow)
{
    if (n < 0 || n > 0xFFFFFFF0ll) FAIL(c, SLAG_E_INVALID_ARG, "n out of range");
    if (d <= 0 || d % 16 || d > 4096) FAIL(c, SLAG_E_INVALID_ARG, "d must be a multiple of 16, at most 4096");
    if (nq < 1 || nq > QMAX) FAIL(c, SLAG_E_INVALID_ARG, "1 to 64 query vectors per call");
    if ((n > 0 && !emb) || !q) FAIL(c, SLAG_E_INVALID_ARG, "null embedding or query pointer");
    if ((ew != SLAG_HOST && ew != SLAG_DEVICE) || (qw != SLAG_HOST && qw != SLAG_DEVICE) ||
        (ow != SLAG_HOST && ow != SLAG_DEVICE))
        FAIL(c, SLAG_E_INVALID_ARG, "bad memory kind");
    if (ew == SLAG_DEVICE && (reinterpret_cast<uintptr_t>(emb) & 15))
        FAIL(c, SLAG_E_INVALID_ARG, "device embeddings must be 16-byte aligned");
    if (qw == SLAG_HOST) {
        for (int64_t i = 0; i < (int64_t)nq * d; i++)
            if (!std::isfinite(q[i])) FAIL(c, SLAG_E_INVALID_ARG, "non-finite query value");
    }
    return SLAG_OK;
}

// The search on prepared work arrays: counts (host) and the top-k rows.
slag_status run_query(slag_ctx* c, const QueryWork& w, int64_t n, int d, int nq, const float* qdev,
                      float thr, int k, int64_t* count, uint32_t* top_idx, float* top_cos,
                      slag_mem ow)
{
    hipStream_t st = c->st;
    const int qp = (nq + 15) & ~15;
    uint32_t* err = reinterpret_cast<uint32_t*>(w.counts + QMAX);
    launch_fill_u32(reinterpret_cast<uint32_t*>(w.counts), 2 * QMAX + 2, 0u, st);
    launch_qprep(nq, qp, d, qdev, w.qt, err, st);
    launch_scores(nq, n, d, w.emb, w.qt, thr, k > 0 ? w.keys : nullptr, w.vals, w.counts, st);
    unsigned long long hc[QMAX + 1];
    HC(c, hipMemcpyAsync(hc, w.counts, sizeof(hc), hipMemcpyDeviceToHost, st));
    HC(c, hipStreamSynchronize(st));
    if (reinterpret_cast<uint32_t*>(&hc[QMAX])[0])
        FAIL(c, SLAG_E_INVALID_ARG, "a query vector is zero or not finite");
    if (count)
        for (int i = 0; i < nq; i++) count[i] = (int64_t)hc[i];
    if (k > 0) {
        bool alt = false;
        for (int i = 0; i < nq; i++) {
            const size_t o = (size_t)i * (size_t)n;
            alt = radix_sort_u32(w.keys + o, w.vals + o, w.keys_alt + o, w.vals_alt + o, (uint64_t)n,
                                 32, w.hist, w.scan_ws, nullptr, st);
        }
        const uint32_t* sk = alt ? w.keys_alt : w.keys;
        const uint32_t* sv = alt ? w.vals_alt : w.vals;
        if (ow == SLAG_DEVICE) {
            launch_topk_out(nq, k, n, sk, sv, top_idx, top_cos, st);
        } else {
            // rows are written to the sort's other (now free) pair of
            // arrays, then copied out
            uint32_t* ti = alt ? w.keys : w.keys_alt;
            float* tc = reinterpret_cast<float*>(alt ? w.vals : w.vals_alt);
            launch_topk_out(nq, k, n, sk, sv, ti, tc, st);
            HC(c, hipMemcpyAsync(top_idx, ti, (size_t)nq * k * 4, hipMemcpyDeviceToHost, st));
            HC(c, hipMemcpyAsync(top_cos, tc, (size_t)nq * k * 4, hipMemcpyDeviceToHost, st));
        }
    }
    HC(c, hipStreamSynchronize(st));
    return SLAG_OK;
}

}  // namespace

extern "C" {

slag_status slag_query(slag_ctx* c, int64_t n, int32_t d, const float* emb, slag_mem ew,
                       int32_t nq, const float* q, slag_mem qw, float thr, int32_t k,
                       int64_t* count, uint32_t* top_idx, float* top_cos, slag_mem ow)
{
    if (!c) return SLAG_E_INVALID_ARG;
    c->err.clear();
    CK(check_args(c, n, d, emb, ew, nq, q, qw, ow));
    if (k < 0 || k > n) FAIL(c, SLAG_E_INVALID_ARG, "k must be in [0, n]");
    if (k > 0 && (!top_idx || !top_cos)) FAIL(c, SLAG_E_INVALID_ARG, "null top-k output");
    HC(c, hipSetDevice(c->device));
    QueryState& Q = c->query;
    QueryWork w;
    const int qp = (nq + 15) & ~15;
    if (ew == SLAG_HOST && n > 0) {
        CK(copy_in(c, Q.emb, emb, (size_t)n * d * 4, SLAG_HOST));
        w.emb = Q.emb.as<float>();
    } else {
        w.emb = emb;
    }
    const float* qdev = q;
    if (qw == SLAG_HOST) {
        CK(copy_in(c, Q.q, q, (size_t)nq * d * 4, SLAG_HOST));
        qdev = Q.q.as<float>();
    }
    CK(ensure(c, Q.qt, (size_t)d * qp * 4));
    CK(ensure(c, Q.counts, (2 * QMAX + 2) * 8));
    w.qt = Q.qt.as<float>();
    w.counts = Q.counts.as<unsigned long long>();
    if (k > 0) {
        const size_t m = (size_t)nq * (size_t)n * 4;
        CK(ensure(c, Q.keys, m));
        CK(ensure(c, Q.vals, m));
        CK(ensure(c, Q.keys_alt, m));
        CK(ensure(c, Q.vals_alt, m));
        CK(ensure(c, Q.hist, radix_hist_bytes((uint64_t)n)));
        CK(ensure(c, Q.scan_ws, sort_scan_bytes(n)));
        w.keys = Q.keys.as<uint32_t>();
        w.vals = Q.vals.as<uint32_t>();
        w.keys_alt = Q.keys_alt.as<uint32_t>();
        w.vals_alt = Q.vals_alt.as<uint32_t>();
        w.hist = Q.hist.as<uint32_t>();
        w.scan_ws = Q.scan_ws.p;
    }
    return run_query(c, w, n, d, nq, qdev, thr, k, count, top_idx, top_cos, ow);
}

slag_status slag_query_static(slag_ctx* c, int64_t n, int32_t d, const float* emb, slag_mem ew,
                              int32_t nq, const float* q, slag_mem qw, float thr, int32_t k,
                              int64_t* count, uint32_t* top_idx, float* top_cos, slag_mem ow)
{
    if (!c) return SLAG_E_INVALID_ARG;
    c->err.clear();
    CK(check_args(c, n, d, emb, ew, nq, q, qw, ow));
    if (ew != SLAG_DEVICE && n > 0)
        FAIL(c, SLAG_E_INVALID_ARG, "slag_query_static needs the embeddings in device memory");
    if (k < 0 || k > n) FAIL(c, SLAG_E_INVALID_ARG, "k must be in [0, n]");
    if (k > 0 && (!top_idx || !top_cos)) FAIL(c, SLAG_E_INVALID_ARG, "null top-k output");
    HC(c, hipSetDevice(c->device));
    // the static work area's address on this device (taken at context creation)
    unsigned char* base = static_cast<unsigned char*>(query_scratch(c->device));
    if (!base) FAIL(c, SLAG_E_STATE, "no static work area on this device");
    const int qp = (nq + 15) & ~15;
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    const size_t o_qt = carve((size_t)d * qp * 4);
    const size_t o_cnt = carve((2 * QMAX + 2) * 8);
    const size_t o_q = qw == SLAG_HOST ? carve((size_t)nq * d * 4) : 0;
    size_t o_keys = 0, o_vals = 0, o_ka = 0, o_va = 0, o_hist = 0, o_ws = 0;
    if (k > 0) {
        const size_t m = (size_t)nq * (size_t)n * 4;
        o_keys = carve(m);
        o_vals = carve(m);
        o_ka = carve(m);
        o_va = carve(m);
        o_hist = carve(radix_hist_bytes((uint64_t)n));
        o_ws = carve(sort_scan_bytes(n));
    }
    if (off > (size_t)SLAG_QUERY_SCRATCH_BYTES)
        FAIL(c, SLAG_E_CAPACITY, "slag_query_static: " + std::to_string(off) +
                                     " bytes of work arrays exceed the static area of " +
                                     std::to_string((size_t)SLAG_QUERY_SCRATCH_BYTES) +
                                     " bytes (fewer queries, k = 0, or slag_query)");
    QueryWork w;
    w.emb = emb;
    w.qt = reinterpret_cast<float*>(base + o_qt);
    w.counts = reinterpret_cast<unsigned long long*>(base + o_cnt);
    const float* qdev = q;
    if (qw == SLAG_HOST) {
        float* qs = reinterpret_cast<float*>(base + o_q);
        HC(c, hipMemcpyAsync(qs, q, (size_t)nq * d * 4, hipMemcpyHostToDevice, c->st));
        qdev = qs;
    }
    if (k > 0) {
        w.keys = reinterpret_cast<uint32_t*>(base + o_keys);
        w.vals = reinterpret_cast<uint32_t*>(base + o_vals);
        w.keys_alt = reinterpret_cast<uint32_t*>(base + o_ka);
        w.vals_alt = reinterpret_cast<uint32_t*>(base + o_va);
        w.hist = reinterpret_cast<uint32_t*>(base + o_hist);
        w.scan_ws = base + o_ws;
    }
    return run_query(c, w, n, d, nq, qdev, thr, k, count, top_idx, top_cos, ow);
}

slag_status slag_classify(slag_ctx* c, int64_t n, int32_t d, const float* emb, slag_mem ew,
                          int32_t nc, const float* cls, slag_mem cw, int32_t* label, float* best,
                          slag_mem ow)
{
    if (!c) return SLAG_E_INVALID_ARG;
    c->err.clear();
    CK(check_args(c, n, d, emb, ew, nc, cls, cw, ow));
    if (n > 0 && !label) FAIL(c, SLAG_E_INVALID_ARG, "null label output");
    HC(c, hipSetDevice(c->device));
    QueryState& Q = c->query;
    hipStream_t st = c->st;
    const int qp = (nc + 15) & ~15;
    const float* E = emb;
    if (ew == SLAG_HOST && n > 0) {
        CK(copy_in(c, Q.emb, emb, (size_t)n * d * 4, SLAG_HOST));
        E = Q.emb.as<float>();
    }
    const float* qdev = cls;
    if (cw == SLAG_HOST) {
        CK(copy_in(c, Q.q, cls, (size_t)nc * d * 4, SLAG_HOST));
        qdev = Q.q.as<float>();
    }
    CK(ensure(c, Q.qt, (size_t)d * qp * 4));
    CK(ensure(c, Q.counts, (2 * QMAX + 2) * 8));
    uint32_t* err = reinterpret_cast<uint32_t*>(Q.counts.as<unsigned long long>() + QMAX);
    launch_fill_u32(err, 2, 0u, st);
    launch_qprep(nc, qp, d, qdev, Q.qt.as<float>(), err, st);
    int32_t* lab = label;
    float* bst = best;
    if (ow == SLAG_HOST && n > 0) {
        CK(ensure(c, Q.keys, (size_t)n * 4));
        CK(ensure(c, Q.vals, (size_t)n * 4));
        lab = reinterpret_cast<int32_t*>(Q.keys.p);
        bst = best ? reinterpret_cast<float*>(Q.vals.p) : nullptr;
    }
    launch_classify(nc, n, d, E, Q.qt.as<float>(), lab, bst, st);
    uint32_t herr = 0;
    HC(c, hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, st));
    if (ow == SLAG_HOST && n > 0) {
        HC(c, hipMemcpyAsync(label, lab, (size_t)n * 4, hipMemcpyDeviceToHost, st));
        if (best) HC(c, hipMemcpyAsync(best, bst, (size_t)n * 4, hipMemcpyDeviceToHost, st));
    }
    HC(c, hipStreamSynchronize(st));
    if (herr) FAIL(c, SLAG_E_INVALID_ARG, "a class vector is zero or not finite");
    return SLAG_OK;
}

}  // extern "C"
