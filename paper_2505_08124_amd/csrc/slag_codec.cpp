// Host side of the learned codec (include/slag_codec.h): parameters, the
// training pool, forward and backward passes layer by layer, Adam, and the
// encode/decode steps of the codec lift.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "slag_ctx.h"

using namespace slag;
using namespace slag_host;

namespace {

// Offsets of the packed parameter blocks (floats).
struct Offsets {
    int64_t W1, b1, W2, b2, W3, b3, W4, b4, total;
};

Offsets offsets(int d, int h, int k)
{
    Offsets o;
    int64_t x = 0;
    o.W1 = x; x += (int64_t)h * d;
    o.b1 = x; x += h;
    o.W2 = x; x += (int64_t)k * h;
    o.b2 = x; x += k;
    o.W3 = x; x += (int64_t)h * k;
    o.b3 = x; x += h;
    o.W4 = x; x += (int64_t)d * h;
    o.b4 = x; x += d;
    o.total = x;
    return o;
}

// One product through the matrix-core GEMM, growing the split-K workspace.
slag_status gemm(slag_ctx* c, int M, int N, int K, const void* A, bool a_bf16, int64_t sam,
                 int64_t sak, const float* B, int64_t sbk, int64_t sbn, float* C, int64_t ldc,
                 const GemmEpi& epi)
{
    CodecState& S = c->codec;
    const size_t pf = gemm_part_floats(M, N, K);
    if (pf) CK(ensure(c, S.gpart, pf * 4));
    launch_gemm(S.bf16, a_bf16, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, epi, S.gpart.as<float>(),
                c->st);
    return SLAG_OK;
}

slag_status colsum(slag_ctx* c, int R, int N, const float* X, float* out)
{
    CodecState& S = c->codec;
    CK(ensure(c, S.cpart, colsum_part_floats(R, N) * 4));
    launch_colsum(R, N, X, out, S.cpart.as<float>(), c->st);
    return SLAG_OK;
}

// Encoder over `rows` feature rows: h1 = gelu(F W1^T + b1) (a1 = its
// pre-activation when asked for) and C = h1 W2^T + b2.
slag_status encode(slag_ctx* c, int rows, const void* F, bool f_bf16, float* a1, float* h1,
                   float* C)
{
    CodecState& S = c->codec;
    const Offsets o = offsets(S.d, S.h, S.k);
    const float* P = S.params.as<float>();
    GemmEpi e1;
    e1.bias = P + o.b1;
    e1.act = GEMM_GELU;
    e1.zsave = a1;
    CK(gemm(c, rows, S.h, S.d, F, f_bf16, S.d, 1, P + o.W1, 1, S.d, h1, S.h, e1));
    GemmEpi e2;
    e2.bias = P + o.b2;
    CK(gemm(c, rows, S.k, S.h, h1, false, S.h, 1, P + o.W2, 1, S.h, C, S.k, e2));
    return SLAG_OK;
}

// Decoder over `rows` codes: h2 = gelu(code W3^T + b3) (a3 = pre-activation
// when asked for) and y = h2 W4^T + b4, zero where rowmask <= 0.
slag_status decode(slag_ctx* c, int rows, const float* code, float* a3, float* h2, float* y,
                   const float* rowmask)
{
    CodecState& S = c->codec;
    const Offsets o = offsets(S.d, S.h, S.k);
    const float* P = S.params.as<float>();
    GemmEpi e3;
    e3.bias = P + o.b3;
    e3.act = GEMM_GELU;
    e3.zsave = a3;
    CK(gemm(c, rows, S.h, S.k, code, false, S.k, 1, P + o.W3, 1, S.k, h2, S.h, e3));
    GemmEpi e4;
    e4.bias = P + o.b4;
    e4.rowmask = rowmask;
    CK(gemm(c, rows, S.d, S.h, h2, false, S.h, 1, P + o.W4, 1, S.h, y, S.d, e4));
    return SLAG_OK;
}

// The pool's entries grouped by column: a stable radix sort of (column,
// entry) pairs (entries stay in row order within a column), then each
// column's range and each grouped entry's row.
static slag_status build_csc(slag_ctx* c)
{
    CodecState& S = c->codec;
    if (S.csc_valid) return SLAG_OK;
    const uint64_t nnz = (uint64_t)S.pool_nnz, NS = (uint64_t)std::max<int64_t>(S.pool_seg, 1);
    const size_t m = (size_t)std::max<uint64_t>(nnz, 1) * 4;
    CK(ensure(c, S.csc_key, m));
    CK(ensure(c, S.csc_j, m));
    CK(ensure(c, S.csc_key_alt, m));
    CK(ensure(c, S.csc_j_alt, m));
    CK(ensure(c, S.csc_row, m));
    CK(ensure(c, S.row_of, m));
    CK(ensure(c, S.cbeg, NS * 4));
    CK(ensure(c, S.cend, NS * 4));
    CK(ensure(c, S.csc_hist, radix_hist_bytes(std::max<uint64_t>(nnz, 1))));
    CK(ensure(c, S.csc_ws, scan_workspace_bytes(radix_hist_bytes(std::max<uint64_t>(nnz, 1)) / 4 + 1)));
    hipStream_t st = c->st;
    launch_fill_u32(S.cbeg.as<uint32_t>(), NS, 0u, st);
    launch_fill_u32(S.cend.as<uint32_t>(), NS, 0u, st);
    if (nnz) {
        launch_row_of((uint32_t)S.pool_rows, S.prow.as<uint32_t>(), S.pcol.as<uint32_t>(),
                      S.row_of.as<uint32_t>(), S.csc_key.as<uint32_t>(), S.csc_j.as<uint32_t>(), st);
        const bool alt = radix_sort_u32(S.csc_key.as<uint32_t>(), S.csc_j.as<uint32_t>(),
                                        S.csc_key_alt.as<uint32_t>(), S.csc_j_alt.as<uint32_t>(), nnz,
                                        std::max(1, bit_length(NS - 1)), S.csc_hist.as<uint32_t>(),
                                        S.csc_ws.p, nullptr, st);
        if (alt) {
            std::swap(S.csc_key, S.csc_key_alt);
            std::swap(S.csc_j, S.csc_j_alt);
        }
        launch_csc_ranges((uint32_t)nnz, S.csc_key.as<uint32_t>(), S.csc_j.as<uint32_t>(),
                          S.row_of.as<uint32_t>(), S.cbeg.as<uint32_t>(), S.cend.as<uint32_t>(),
                          S.csc_row.as<uint32_t>(), st);
    }
    S.csc_valid = true;
    return SLAG_OK;
}

// Loss over pool rows [row0, row0 + R) into *loss_dev; with grad, the full
// gradient into codec.grad.
slag_status forward_backward(slag_ctx* c, int64_t row0, int R, bool grad, float* loss_dev)
{
    CodecState& S = c->codec;
    const int d = S.d, h = S.h, k = S.k;
    const int NS = (int)S.pool_seg;
    const Offsets o = offsets(d, h, k);
    const float* P = S.params.as<float>();
    float* G = S.grad.as<float>();
    const size_t ns = (size_t)std::max(NS, 1), nr = (size_t)std::max(R, 1);
    CK(ensure(c, S.a1, ns * h * 4));
    CK(ensure(c, S.h1, ns * h * 4));
    CK(ensure(c, S.C, ns * k * 4));
    CK(ensure(c, S.dC, ns * k * 4));
    CK(ensure(c, S.code, nr * k * 4));
    CK(ensure(c, S.dcode, nr * k * 4));
    CK(ensure(c, S.a3, nr * h * 4));
    CK(ensure(c, S.h2, nr * h * 4));
    CK(ensure(c, S.y, nr * d * 4));
    CK(ensure(c, S.dy, nr * d * 4));
    CK(ensure(c, S.lpart, ((nr + 3) / 4) * 4));
    hipStream_t st = c->st;
    const uint32_t* rp = S.prow.as<uint32_t>() + row0;

    // forward
    CK(encode(c, NS, S.pF.p, false, S.a1.as<float>(), S.h1.as<float>(), S.C.as<float>()));
    launch_mix(R, k, rp, S.pcol.as<uint32_t>(), S.pw.as<float>(), S.C.as<float>(),
               S.code.as<float>(), st);
    CK(decode(c, R, S.code.as<float>(), S.a3.as<float>(), S.h2.as<float>(), S.y.as<float>(),
              nullptr));
    launch_cos_loss(R, d, S.y.as<float>(), S.ptgt.as<float>() + row0 * d, S.dy.as<float>(),
                    S.lpart.as<float>(), loss_dev, st);
    if (!grad) return SLAG_OK;

    // decoder
    GemmEpi none;
    CK(gemm(c, d, h, R, S.dy.p, false, 1, d, S.h2.as<float>(), h, 1, G + o.W4, h, none));
    CK(colsum(c, R, d, S.dy.as<float>(), G + o.b4));
    GemmEpi gb3;                       // da3 = (dy W4) * gelu'(a3), into h2's buffer
    gb3.act = GEMM_GELU_BWD;
    gb3.aux = S.a3.as<float>();
    float* da3 = S.h2.as<float>();
    CK(gemm(c, R, h, d, S.dy.p, false, d, 1, P + o.W4, h, 1, da3, h, gb3));
    CK(gemm(c, h, k, R, da3, false, 1, h, S.code.as<float>(), k, 1, G + o.W3, k, none));
    CK(colsum(c, R, h, da3, G + o.b3));
    CK(gemm(c, R, k, h, da3, false, h, 1, P + o.W3, k, 1, S.dcode.as<float>(), k, none));
    // mixing (transposed through the column grouping: no atomics)
    CK(build_csc(c));
    launch_mix_bwd(NS, k, rp, R, row0, S.cbeg.as<uint32_t>(), S.cend.as<uint32_t>(), S.csc_j.as<uint32_t>(),
                   S.csc_row.as<uint32_t>(), S.pw.as<float>(), S.dcode.as<float>(),
                   S.dC.as<float>(), st);
    // encoder
    CK(gemm(c, k, h, NS, S.dC.p, false, 1, k, S.h1.as<float>(), h, 1, G + o.W2, h, none));
    CK(colsum(c, NS, k, S.dC.as<float>(), G + o.b2));
    GemmEpi gb1;                       // da1 = (dC W2) * gelu'(a1), into h1's buffer
    gb1.act = GEMM_GELU_BWD;
    gb1.aux = S.a1.as<float>();
    float* da1 = S.h1.as<float>();
    CK(gemm(c, NS, h, k, S.dC.p, false, k, 1, P + o.W2, h, 1, da1, h, gb1));
    CK(gemm(c, h, d, NS, da1, false, 1, h, S.pF.as<float>(), d, 1, G + o.W1, d, none));
    CK(colsum(c, NS, h, da1, G + o.b1));
    return SLAG_OK;
}

slag_status need_codec(slag_ctx* c)
{
    if (!c) return SLAG_E_INVALID_ARG;
    c->err.clear();
    if (!c->codec.ready) FAIL(c, SLAG_E_STATE, "codec not initialised");
    HC(c, hipSetDevice(c->device));
    // codec work arrays may be regrown: a captured lift graph would hold stale pointers
    invalidate_graph(c);
    return SLAG_OK;
}

}  // namespace

namespace slag_host {

slag_status codec_encode_table(slag_ctx* c)
{
    CodecState& S = c->codec;
    const size_t rows = std::max<uint64_t>(c->feat_rows, 1);
    CK(ensure(c, S.h1, rows * S.h * 4));
    CK(ensure(c, S.C, rows * S.k * 4));
    return encode(c, (int)c->feat_rows, c->feats.p, c->fdt == SLAG_BF16, nullptr, S.h1.as<float>(),
                  S.C.as<float>());
}

slag_status codec_decode_codes(slag_ctx* c)
{
    CodecState& S = c->codec;
    if (S.bf16 && decode_fused_supported(S.k, S.h, S.d)) {
        const Offsets o = offsets(S.d, S.h, S.k);
        const float* P = S.params.as<float>();
        launch_decode_bf16((int)c->n, S.k, S.h, S.d, S.codes.as<float>(), P + o.W3, P + o.b3,
                           P + o.W4, P + o.b4, c->den.as<float>(), c->num.as<float>(), c->st);
        return SLAG_OK;
    }
    CK(ensure(c, S.hid, (size_t)std::max<int64_t>(c->n, 1) * S.h * 4));
    return decode(c, (int)c->n, S.codes.as<float>(), nullptr, S.hid.as<float>(), c->num.as<float>(),
                  c->den.as<float>());
}

void codec_release(slag_ctx* c)
{
    CodecState& S = c->codec;
    DevBuf* bufs[] = {&S.params, &S.grad, &S.adam_m, &S.adam_v, &S.pF, &S.prow, &S.pcol, &S.pw,
                      &S.ptgt, &S.a1, &S.h1, &S.C, &S.dC, &S.code, &S.dcode, &S.a3, &S.h2,
                      &S.y, &S.dy, &S.gpart, &S.cpart, &S.lpart, &S.loss, &S.rflag, &S.ridx,
                      &S.rlen, &S.roff, &S.rgid, &S.codes, &S.hid, &S.csc_key, &S.csc_j,
                      &S.csc_key_alt, &S.csc_j_alt, &S.csc_row, &S.row_of, &S.cbeg, &S.cend,
                      &S.csc_hist, &S.csc_ws};
    for (DevBuf* b : bufs) release(*b);
    S.csc_valid = false;
}

}  // namespace slag_host

extern "C" {

slag_status slag_codec_init(slag_ctx* c, int32_t d, int32_t hidden, int32_t k,
                            slag_dtype precision, const float* params, slag_mem where)
{
    if (!c) return SLAG_E_INVALID_ARG;
    c->err.clear();
    if (d <= 0 || d > 4096 || hidden <= 0 || hidden > 4096 || hidden % 16 != 0)
        FAIL(c, SLAG_E_INVALID_ARG, "d must be in [1, 4096], hidden a multiple of 16 up to 4096");
    if (k != 16 && k != 32 && k != 48 && k != 64)
        FAIL(c, SLAG_E_NOT_SUPPORTED, "code size k must be 16, 32, 48 or 64");
    if (precision != SLAG_BF16 && precision != SLAG_F32)
        FAIL(c, SLAG_E_INVALID_ARG, "precision must be SLAG_BF16 or SLAG_F32");
    if (!params) FAIL(c, SLAG_E_INVALID_ARG, "null parameters");
    invalidate_graph(c);
    if (where != SLAG_HOST && where != SLAG_DEVICE) FAIL(c, SLAG_E_INVALID_ARG, "bad memory kind");
    HC(c, hipSetDevice(c->device));
    CodecState& S = c->codec;
    const Offsets o = offsets(d, hidden, k);
    const size_t bytes = (size_t)o.total * 4;
    CK(copy_in(c, S.params, params, bytes, where));
    CK(ensure(c, S.grad, bytes));
    CK(ensure(c, S.adam_m, bytes));
    CK(ensure(c, S.adam_v, bytes));
    launch_fill_u32(S.adam_m.as<uint32_t>(), (uint64_t)o.total, 0u, c->st);
    launch_fill_u32(S.adam_v.as<uint32_t>(), (uint64_t)o.total, 0u, c->st);
    if (S.d != d) {                    // the pool's rows have the old dimension
        S.pool_seg = S.pool_rows = S.pool_nnz = 0;
        S.csc_valid = false;
    }
    S.d = d;
    S.h = hidden;
    S.k = k;
    S.bf16 = precision == SLAG_BF16;
    S.nparam = o.total;
    S.step = 0;
    S.ready = true;
    S.have_codes = false;
    if (c->out_is_codec) c->have_out = false;
    HC(c, hipStreamSynchronize(c->st));
    return SLAG_OK;
}

slag_status slag_codec_get_params(slag_ctx* c, float* out, slag_mem where)
{
    CK(need_codec(c));
    if (!out) FAIL(c, SLAG_E_INVALID_ARG, "null output");
    const hipMemcpyKind kd = where == SLAG_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    HC(c, hipMemcpyAsync(out, c->codec.params.p, (size_t)c->codec.nparam * 4, kd, c->st));
    HC(c, hipStreamSynchronize(c->st));
    return SLAG_OK;
}

slag_status slag_codec_clear_pool(slag_ctx* c)
{
    if (!c) return SLAG_E_INVALID_ARG;
    c->err.clear();
    c->codec.pool_seg = c->codec.pool_rows = c->codec.pool_nnz = 0;
    c->codec.csc_valid = false;
    return SLAG_OK;
}

slag_status slag_codec_set_pool(slag_ctx* c, int64_t n_seg, const float* feats, int64_t n_rows,
                                const uint32_t* row_ptr, const uint32_t* col, const float* w,
                                const float* target, slag_mem where)
{
    CK(need_codec(c));
    CodecState& S = c->codec;
    if (n_seg < 0 || n_rows < 0 || n_seg >= ((int64_t)1 << 31) || n_rows >= ((int64_t)1 << 31))
        FAIL(c, SLAG_E_INVALID_ARG, "bad pool size");
    if ((n_seg && !feats) || !row_ptr || (n_rows && !target))
        FAIL(c, SLAG_E_INVALID_ARG, "null pool array");
    if (where != SLAG_HOST && where != SLAG_DEVICE) FAIL(c, SLAG_E_INVALID_ARG, "bad memory kind");
    // validate the row structure on the host
    std::vector<uint32_t> rp(n_rows + 1);
    const hipMemcpyKind kh = where == SLAG_DEVICE ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
    HC(c, hipMemcpy(rp.data(), row_ptr, rp.size() * 4, kh));
    if (rp[0] != 0) FAIL(c, SLAG_E_INVALID_ARG, "row_ptr[0] must be 0");
    for (int64_t r = 0; r < n_rows; r++)
        if (rp[r + 1] < rp[r]) FAIL(c, SLAG_E_INVALID_ARG, "row_ptr must be ascending");
    const uint64_t nnz = rp[n_rows];
    if (nnz && (!col || !w)) FAIL(c, SLAG_E_INVALID_ARG, "null pool array");
    std::vector<uint32_t> cl(nnz);
    if (nnz) HC(c, hipMemcpy(cl.data(), col, nnz * 4, kh));
    for (uint64_t j = 0; j < nnz; j++)
        if (cl[j] >= (uint64_t)n_seg) FAIL(c, SLAG_E_INVALID_ARG, "pool column out of range");
    CK(copy_in(c, S.pF, feats, (size_t)n_seg * S.d * 4, where));
    CK(copy_in(c, S.prow, rp.data(), rp.size() * 4, SLAG_HOST));
    CK(copy_in(c, S.pcol, cl.data(), nnz * 4, SLAG_HOST));
    CK(copy_in(c, S.pw, w, nnz * 4, where));
    CK(copy_in(c, S.ptgt, target, (size_t)n_rows * S.d * 4, where));
    HC(c, hipStreamSynchronize(c->st));
    S.pool_seg = n_seg;
    S.pool_rows = n_rows;
    S.pool_nnz = (int64_t)nnz;
    S.csc_valid = false;
    return SLAG_OK;
}

slag_status slag_codec_add_lift_rows(slag_ctx* c, int64_t max_rows, uint64_t seed, int64_t* added)
{
    CK(need_codec(c));
    CodecState& S = c->codec;
    if (added) *added = 0;
    if (max_rows < 0) FAIL(c, SLAG_E_INVALID_ARG, "negative row count");
    if (!c->have_out || c->out_is_codec || !c->lists_valid)
        FAIL(c, SLAG_E_STATE, "needs a plain lift first (and no render since)");
    if (c->plan.size() != 1) FAIL(c, SLAG_E_STATE, "training rows need all views in one launch");
    if (S.d != c->d) FAIL(c, SLAG_E_STATE, "codec dimension differs from the features'");
    const int64_t n = c->n;
    const uint64_t np = c->last_npairs;
    if (n <= 0 || np == 0 || max_rows == 0) return SLAG_OK;
    hipStream_t st = c->st;
    const Batch& B = c->plan[0];
    uint64_t* small = c->small.as<uint64_t>();
    // merged per-pair weight rows (global segment ids)
    CK(ensure(c, c->wrow, std::max<int64_t>(c->stats.n_part_slots, 1) * 8));
    launch_merge(np, c->pview.as<uint16_t>(), B.views.as<ViewDev>(), c->pinfo.as<uint2>(),
                 c->part.as<uint2>(), c->wrow.as<uint2>(),
                 c->wlen.as<uint32_t>(), reinterpret_cast<unsigned long long*>(small + SM_NNZ), st);
    // sample Gaussians with weight
    const double frac = std::min(1.0, (double)max_rows / (double)n);
    const uint32_t thresh = frac >= 1.0 ? 0xFFFFFFFFu : (uint32_t)(frac * 4294967296.0);
    CK(ensure(c, S.rflag, (size_t)n * 4));
    CK(ensure(c, S.ridx, (size_t)n * 4));
    CK(ensure_scan(c, (uint64_t)n));
    launch_pick_rows(n, c->den.as<float>(), seed, thresh, S.rflag.as<uint32_t>(), st);
    HC(c, hipMemcpyAsync(S.ridx.p, S.rflag.p, (size_t)n * 4, hipMemcpyDeviceToDevice, st));
    scan_u32(S.ridx.as<uint32_t>(), (uint64_t)n, small + SM_TOTALS, c->scan_ws.p, st);
    CK(read_small(c, SM_TOTALS, 1));
    const uint32_t rows = (uint32_t)std::min<uint64_t>(c->host_small[SM_TOTALS], (uint64_t)max_rows);
    if (!rows) return SLAG_OK;
    if ((uint64_t)S.pool_rows + rows >= (1ull << 31)) FAIL(c, SLAG_E_CAPACITY, "pool too large");
    CK(ensure(c, S.rlen, (size_t)rows * 4 + 16));
    CK(ensure(c, S.roff, (size_t)rows * 4 + 16));
    CK(ensure(c, S.rgid, (size_t)rows * 4 + 16));
    launch_row_len(n, B.nb, S.rflag.as<uint32_t>(), S.ridx.as<uint32_t>(), rows,
                   c->rank.as<uint32_t>(), c->pair_of_m.as<uint32_t>(), c->blk_vis.as<uint32_t>(),
                   count_blocks_per_view(n), c->wlen.as<uint32_t>(), S.rlen.as<uint32_t>(),
                   S.rgid.as<uint32_t>(), st);
    HC(c, hipMemcpyAsync(S.roff.p, S.rlen.p, (size_t)rows * 4, hipMemcpyDeviceToDevice, st));
    CK(ensure_scan(c, rows));
    scan_u32(S.roff.as<uint32_t>(), rows, small + SM_TOTALS, c->scan_ws.p, st);
    CK(read_small(c, SM_TOTALS, 1));
    const uint64_t nnz_new = c->host_small[SM_TOTALS];
    if ((uint64_t)S.pool_nnz + nnz_new >= 0xFFFFFFF0ull)
        FAIL(c, SLAG_E_CAPACITY, "pool has too many weight entries");
    const int d = S.d;
    const uint64_t seg_new = c->feat_rows;
    CK(grow_keep(c, S.prow, ((size_t)S.pool_rows + rows + 1) * 4, (size_t)S.pool_rows * 4));
    CK(grow_keep(c, S.pcol, ((size_t)S.pool_nnz + nnz_new) * 4 + 16, (size_t)S.pool_nnz * 4));
    CK(grow_keep(c, S.pw, ((size_t)S.pool_nnz + nnz_new) * 4 + 16, (size_t)S.pool_nnz * 4));
    CK(grow_keep(c, S.ptgt, ((size_t)S.pool_rows + rows) * d * 4, (size_t)S.pool_rows * d * 4));
    CK(grow_keep(c, S.pF, ((size_t)S.pool_seg + seg_new) * d * 4 + 16, (size_t)S.pool_seg * d * 4));
    launch_row_gather(n, B.nb, rows, S.rgid.as<uint32_t>(), S.roff.as<uint32_t>(),
                      (uint32_t)S.pool_nnz, (uint32_t)S.pool_seg, c->rank.as<uint32_t>(),
                      c->pair_of_m.as<uint32_t>(), c->blk_vis.as<uint32_t>(), count_blocks_per_view(n),
                      c->wlen.as<uint32_t>(), c->psz.as<uint32_t>(),
                      c->wrow.as<uint2>(), c->den.as<float>(),
                      S.prow.as<uint32_t>() + S.pool_rows, S.pcol.as<uint32_t>(),
                      S.pw.as<float>(), st);
    launch_fill_u32(S.prow.as<uint32_t>() + S.pool_rows + rows, 1,
                    (uint32_t)(S.pool_nnz + nnz_new), st);
    launch_copy_rows(rows, d, S.rgid.as<uint32_t>(), c->num.as<float>(),
                     S.ptgt.as<float>() + (size_t)S.pool_rows * d, st);
    launch_to_f32((int64_t)(seg_new * d), c->feats.p, c->fdt == SLAG_BF16,
                  S.pF.as<float>() + (size_t)S.pool_seg * d, st);
    HC(c, hipStreamSynchronize(st));
    S.pool_rows += rows;
    S.pool_nnz += (int64_t)nnz_new;
    S.csc_valid = false;
    S.pool_seg += (int64_t)seg_new;
    if (added) *added = rows;
    return SLAG_OK;
}

slag_status slag_codec_pool_size(slag_ctx* c, int64_t* n_seg, int64_t* n_rows, int64_t* nnz)
{
    if (!c) return SLAG_E_INVALID_ARG;
    c->err.clear();
    if (n_seg) *n_seg = c->codec.pool_seg;
    if (n_rows) *n_rows = c->codec.pool_rows;
    if (nnz) *nnz = c->codec.pool_nnz;
    return SLAG_OK;
}

slag_status slag_codec_loss_grad(slag_ctx* c, int64_t row0, int64_t n_rows, float* loss,
                                 float* grad, slag_mem where)
{
    CK(need_codec(c));
    CodecState& S = c->codec;
    if (row0 < 0 || n_rows <= 0 || row0 + n_rows > S.pool_rows)
        FAIL(c, SLAG_E_INVALID_ARG, "row range outside the pool");
    CK(ensure(c, S.loss, 16));
    CK(forward_backward(c, row0, (int)n_rows, grad != nullptr, S.loss.as<float>()));
    float l = 0.0f;
    HC(c, hipMemcpyAsync(&l, S.loss.p, 4, hipMemcpyDeviceToHost, c->st));
    if (grad) {
        const hipMemcpyKind kd = where == SLAG_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        HC(c, hipMemcpyAsync(grad, S.grad.p, (size_t)S.nparam * 4, kd, c->st));
    }
    HC(c, hipStreamSynchronize(c->st));
    if (loss) *loss = l;
    return SLAG_OK;
}

slag_status slag_codec_train(slag_ctx* c, const slag_train_cfg* cfg, float* loss_history)
{
    CK(need_codec(c));
    CodecState& S = c->codec;
    if (!cfg || cfg->steps < 0 || cfg->batch_rows < 0 || !(cfg->lr > 0.0f) ||
        !(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f) || !(cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f) ||
        !(cfg->eps > 0.0f))
        FAIL(c, SLAG_E_INVALID_ARG, "bad training configuration");
    if (S.pool_rows <= 0) FAIL(c, SLAG_E_STATE, "empty training pool");
    const int64_t R = S.pool_rows;
    const int64_t B = cfg->batch_rows > 0 ? std::min<int64_t>(cfg->batch_rows, R) : R;
    CK(ensure(c, S.loss, (size_t)std::max(cfg->steps, 1) * 4 + 16));
    float* lh = S.loss.as<float>();
    for (int s = 0; s < cfg->steps; s++) {
        const int64_t row0 = (int64_t)(((uint64_t)s * (uint64_t)B) % (uint64_t)R);
        const int64_t nr = std::min<int64_t>(B, R - row0);
        CK(forward_backward(c, row0, (int)nr, true, lh + s));
        S.step++;
        launch_adam(S.nparam, S.params.as<float>(), S.grad.as<float>(), S.adam_m.as<float>(),
                    S.adam_v.as<float>(), cfg->lr, cfg->beta1, cfg->beta2, cfg->eps, S.step, c->st);
    }
    if (loss_history && cfg->steps > 0)
        HC(c, hipMemcpyAsync(loss_history, lh, (size_t)cfg->steps * 4, hipMemcpyDeviceToHost, c->st));
    HC(c, hipStreamSynchronize(c->st));
    if (c->out_is_codec) c->have_out = false;
    S.have_codes = false;
    return SLAG_OK;
}

slag_status slag_lift_codec(slag_ctx* c) { return run_lift(c, true); }

slag_status slag_get_codes(slag_ctx* c, float* out, slag_mem where)
{
    if (!c) return SLAG_E_INVALID_ARG;
    c->err.clear();
    if (!c->codec.have_codes) FAIL(c, SLAG_E_STATE, "no codec lift result");
    HC(c, hipSetDevice(c->device));
    if (out && c->n > 0) {
        const hipMemcpyKind kd = where == SLAG_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        HC(c, hipMemcpyAsync(out, c->codec.codes.p, (size_t)c->n * c->codec.k * 4, kd, c->st));
    }
    HC(c, hipStreamSynchronize(c->st));
    return SLAG_OK;
}

}  // extern "C"
