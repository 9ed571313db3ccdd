/*
 * mpdp_scorer.h -- learned subgraph scorer for the large-query heuristics.
 *
 * A three-layer MLP, MPDP_SCORER_IN -> 256 -> 256 -> 1 with ReLU, BF16
 * weights and activations, FP32 accumulation (matrix cores for the two wide
 * layers).  It scores a candidate union of two partitions in UnionDP's
 * partition phase (Section 4.2, Alg. 4): the logit of "the union is a node
 * of the optimal plan".  It is trained on plans the exact DP produces for
 * smaller queries (mpdp_optimize_large with MPDP_LARGE_UNIONDP_LEARNED uses
 * it; plain UnionDP is the method without it).  This scorer is not part of
 * the paper: the paper's UnionDP orders the unions by edge weight.
 *
 * Parameters (host arrays, FP32, row-major): w1[IN][256], b1[256],
 * w2[256][256], b2[256], w3[256], b3[1]; layer l computes
 * h_l = relu(h_{l-1} w_l + b_l) and the logit is h_2 . w3 + b3.
 *
 * Device memory is the caller's: a parameter block of
 * mpdp_scorer_param_bytes() bytes (256-byte aligned; FP32 master values,
 * BF16 copies, gradients, Adam moments) and a work buffer of
 * mpdp_scorer_work_bytes(batch) bytes for a batch.  Inputs d_x are batch x
 * MPDP_SCORER_IN BF16 values (bit patterns, row-major); labels d_y are
 * batch FP32 values in {0, 1}.  Every call enqueues on hip_stream; calls
 * that return a host value wait for it.
 */
#ifndef MPDP_SCORER_H
#define MPDP_SCORER_H

#include <stddef.h>
#include <stdint.h>

#include "mpdp.h"

#ifdef __cplusplus
extern "C" {
#endif

#define MPDP_SCORER_IN 32
#define MPDP_SCORER_HIDDEN 256

/* Bytes of the device parameter block. */
size_t mpdp_scorer_param_bytes(void);

/* Bytes of the device work buffer for a batch (0 for batch = 0). */
size_t mpdp_scorer_work_bytes(uint32_t batch);

/* Offsets in the parameter block of the FP32 master values (w1, b1, w2, b2,
 * w3, b3 back to back), the BF16 copies (w1, w2, w3) and the FP32 gradients
 * (same order as the master values). */
mpdp_status mpdp_scorer_layout(size_t *off_master, size_t *off_bf16, size_t *off_grad);

/* Upload FP32 weights from the host, clear gradients and Adam moments,
 * derive the BF16 copies.  MPDP_EINVAL for a null or misaligned pointer or
 * a non-finite value. */
mpdp_status mpdp_scorer_load(void *d_params, const float *w1, const float *b1, const float *w2, const float *b2,
                             const float *w3, const float *b3, void *hip_stream);

/* Logits of a batch into d_logits (device, batch floats). */
mpdp_status mpdp_scorer_forward(const void *d_params, const uint16_t *d_x, uint32_t batch, float *d_logits,
                                void *d_work, size_t work_bytes, void *hip_stream);

/* Mean binary cross-entropy (with logits) of a batch and the gradients of
 * every parameter into the block's gradient region; loss_out (host,
 * nullable) receives the loss. */
mpdp_status mpdp_scorer_grad(void *d_params, const uint16_t *d_x, const float *d_y, uint32_t batch, void *d_work,
                             size_t work_bytes, void *hip_stream, float *loss_out);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected with step
 * >= 1) after mpdp_scorer_grad on the batch; refreshes the BF16 copies. */
mpdp_status mpdp_scorer_train_step(void *d_params, const uint16_t *d_x, const float *d_y, uint32_t batch, float lr,
                                   uint32_t step, void *d_work, size_t work_bytes, void *hip_stream,
                                   float *loss_out);

#ifdef __cplusplus
}
#endif

#endif /* MPDP_SCORER_H */
