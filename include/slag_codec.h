/*
 * slag_codec.h -- learned segment-feature codec for the embedding lift.
 *
 * An extension of the lift of slag.h, not part of the paper's method (the
 * paper lifts the full D-dim features and argues against per-scene feature
 * compression).  Segment features are encoded to k-dim codes, the lift
 * accumulates codes with exactly the weights it gives features (the
 * aggregation equation applied to codes: code_g = sum W c_s / sum W), and
 * each Gaussian's code is decoded back to D dimensions.
 *
 * Network (tanh-form GELU, FP32 master parameters):
 *   encoder  c = W2 gelu(W1 f + b1) + b2          D -> H -> k
 *   decoder  y = W4 gelu(W3 c + b3) + b4          k -> H -> D
 * Parameters are one FP32 vector, row-major (out x in), in the order
 *   W1[H][D], b1[H], W2[k][H], b2[k], W3[H][k], b3[H], W4[D][H], b4[D]
 * of length H D + H + k H + k + H k + H + D H + D.
 *
 * Precision: SLAG_BF16 rounds every product operand (weights, features,
 * activations, gradients) to bfloat16 and accumulates in FP32 on the
 * matrix cores; SLAG_F32 keeps FP32 operands (for gradient checks).
 *
 * Training ("through the mixing"): a training row is one Gaussian with
 * normalised weights w_rj over pool segments col_rj and a target embedding
 * t_r (its plain-lift embedding).  Its output is dec(sum_j w_rj enc(F[col_rj]))
 * and the loss is the mean over rows of 1 - cos(output, t_r).  Adam with
 * bias correction updates the FP32 parameters.
 *
 * All functions follow slag.h's conventions: slag_status return, message
 * in slag_last_error, stream-ordered on the context's stream, no aborts.
 */
#ifndef SLAG_CODEC_H
#define SLAG_CODEC_H

#include "slag.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t steps;          /* Adam steps */
    int32_t batch_rows;     /* training rows per step (contiguous slices of the pool,
                               wrapping around); 0 = all rows every step */
    float lr;               /* learning rate (e.g. 1e-3) */
    float beta1, beta2;     /* moment decays (e.g. 0.9, 0.999) */
    float eps;              /* denominator guard (e.g. 1e-8) */
    int64_t reserved[4];    /* zero */
} slag_train_cfg;

/* Set the network shape and parameters.  d = feature dimension (equal to the
 * context's features for lifting), hidden = H (multiple of 16, <= 4096),
 * k in {16, 32, 48, 64}; params = packed vector (host or device, copied);
 * precision SLAG_BF16 or SLAG_F32.  Resets the Adam state. */
slag_status slag_codec_init(slag_ctx* ctx, int32_t d, int32_t hidden, int32_t k,
                            slag_dtype precision, const float* params, slag_mem where);

/* Copy the current FP32 parameters out (packed layout above). */
slag_status slag_codec_get_params(slag_ctx* ctx, float* out, slag_mem where);

/* Empty the training pool. */
slag_status slag_codec_clear_pool(slag_ctx* ctx);

/* Replace the training pool by explicit arrays (host or device, copied):
 * feats [n_seg][d] FP32; row_ptr [n_rows + 1] (row_ptr[0] = 0, ascending,
 * row_ptr[n_rows] = nnz < 2^32); col [nnz] in [0, n_seg); w [nnz] (each
 * row's weights are expected to sum to 1); target [n_rows][d] FP32.
 * Column indices are validated (SLAG_E_INVALID_ARG). */
slag_status slag_codec_set_pool(slag_ctx* ctx, int64_t n_seg, const float* feats, int64_t n_rows,
                                const uint32_t* row_ptr, const uint32_t* col, const float* w,
                                const float* target, slag_mem where);

/* Append training rows from the last plain slag_lift of this context (all
 * views in one launch, features of dimension d): Gaussians with non-zero
 * weight are sampled by SplitMix64(seed + index) < max_rows / N (at most
 * max_rows of them); each row is the Gaussian's weights over all views and
 * segments divided by their sum, its target the lifted embedding; the
 * context's feature table is appended to the pool.  *added (may be NULL)
 * receives the number of rows added. */
slag_status slag_codec_add_lift_rows(slag_ctx* ctx, int64_t max_rows, uint64_t seed,
                                     int64_t* added);

/* Pool sizes (any pointer may be NULL). */
slag_status slag_codec_pool_size(slag_ctx* ctx, int64_t* n_seg, int64_t* n_rows, int64_t* nnz);

/* Loss over pool rows [row0, row0 + n_rows) and its gradient with respect to
 * the packed parameters (grad may be NULL), without updating anything.
 * loss is a host pointer; grad is host or device per `where`. */
slag_status slag_codec_loss_grad(slag_ctx* ctx, int64_t row0, int64_t n_rows, float* loss,
                                 float* grad, slag_mem where);

/* Run cfg->steps Adam steps on the pool.  loss_history (host, may be NULL)
 * receives the loss of each step (before its update).  Synchronises. */
slag_status slag_codec_train(slag_ctx* ctx, const slag_train_cfg* cfg, float* loss_history);

/* Codec lift: encode the context's feature table, run the lift with the
 * codes in place of the features (same weights, same normalisation), and
 * decode every Gaussian's code.  Afterwards slag_get_embeddings returns the
 * decoded [N][d] embeddings (rows without weight are 0) and the same den as
 * the plain lift; slag_get_codes returns the [N][k] codes. */
slag_status slag_lift_codec(slag_ctx* ctx);

/* Codes of the last codec lift, [N][k] FP32, input Gaussian order. */
slag_status slag_get_codes(slag_ctx* ctx, float* out, slag_mem where);

#ifdef __cplusplus
}
#endif

#endif
