/*
 * slag_query.h -- cosine-similarity search over per-Gaussian embeddings, the
 * inference side of the lift (paper, Method, "Query processing for
 * inference": a query vector, e.g. a CLIP text embedding, is matched against
 * the embedding tensor E_GAUSSIAN by cosine similarity and the matching
 * Gaussians are returned; Experiments: matches above a relevance threshold
 * on the cosine (0.28 in the paper's evaluation), query responses of the
 * best-matching 1k-100k Gaussians, and each Gaussian assigned the class of
 * highest cosine similarity).  The paper runs this in a vector database or
 * as a brute-force search; here it is a brute-force search on the GPU.
 *
 * Scores: cos(g, q) = (E_g . q) / (||E_g|| ||q||) in FP32 (products and sums
 * on the matrix cores, FP32 accumulation); Gaussians with E_g = 0 (no weight
 * in the lift) have no score and never match.  Embeddings and queries must
 * be finite; queries must be non-zero (else SLAG_E_INVALID_ARG).
 *
 * Embedding tables are [n][d] FP32 row-major, d a multiple of 16 (at most
 * 4096), 16-byte aligned; e.g. the output of slag_get_embeddings, or a
 * partition of it.  All calls are ordered on the context's stream and
 * synchronise it before returning (the counts are returned in host memory).
 * A context needs no lift for these calls; any context works.
 */
#ifndef SLAG_QUERY_H
#define SLAG_QUERY_H

#include <stdint.h>

#include "slag.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Search `n_queries` query vectors queries[Q][d] (q_where) in the embeddings
 * emb[n][d] (emb_where; host tables are copied to the library's workspace).
 *   count[Q] (host, may be NULL): number of Gaussians with cos >= threshold;
 *   top_idx[Q][k], top_cos[Q][k] (out_where, may be NULL when k = 0): the k
 *   Gaussians of highest cosine per query, best first, ties by ascending
 *   index; when fewer than k Gaussians have a score the rest of the row is
 *   index 0xFFFFFFFF and cosine -inf.
 * 1 <= Q <= 64, 0 <= k <= n.  Workspace: the library allocates (and keeps)
 * d Q 4 bytes plus, when k > 0, 16 n Q bytes (the per-query sort). */
slag_status slag_query(slag_ctx* ctx, int64_t n, int32_t d, const float* emb, slag_mem emb_where,
                       int32_t n_queries, const float* queries, slag_mem q_where, float threshold,
                       int32_t k, int64_t* count, uint32_t* top_idx, float* top_cos,
                       slag_mem out_where);

/* The same search for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid it): every
 * work array lives in one static device buffer of SLAG_QUERY_SCRATCH_BYTES
 * per GPU (reserved when the library's first context on that GPU is
 * created, held until the process ends) instead of library-allocated
 * workspace; no hipMalloc, hipFree or allocating library call.  emb must be
 * device memory (SLAG_DEVICE); queries and outputs are as for slag_query.
 * Sizes whose work arrays do not fit the buffer (about 16 n Q bytes for
 * k > 0, plus the sort's histograms and 4 d Q + 4 d Q bytes for the queries)
 * are rejected with SLAG_E_CAPACITY.  Results equal slag_query's bit for
 * bit.  All calls on one GPU share the buffer, which keeps the last call's
 * contents: calls that overlap in time on one GPU (two contexts or two host
 * threads) race and must be serialised by the caller. */
#define SLAG_QUERY_SCRATCH_BYTES (128u << 20)
slag_status slag_query_static(slag_ctx* ctx, int64_t n, int32_t d, const float* emb,
                              slag_mem emb_where, int32_t n_queries, const float* queries,
                              slag_mem q_where, float threshold, int32_t k, int64_t* count,
                              uint32_t* top_idx, float* top_cos, slag_mem out_where);

/* Per-Gaussian class (the ScanNet-style semantic labelling of the paper's
 * evaluation): label[g] = the class c of highest cos(g, c) among
 * classes[C][d] (ties to the lower class), -1 where E_g = 0; best[g] (may be
 * NULL) = that cosine (-inf where E_g = 0).  1 <= C <= 64; outputs are
 * out_where-resident [n]. */
slag_status slag_classify(slag_ctx* ctx, int64_t n, int32_t d, const float* emb, slag_mem emb_where,
                          int32_t n_classes, const float* classes, slag_mem c_where, int32_t* label,
                          float* best, slag_mem out_where);

#ifdef __cplusplus
}
#endif
#endif /* SLAG_QUERY_H */
