/*
 * libtsdf — learned measurement-noise model (gfx950).
 *
 * The paper sets the Kalman measurement variance p_k from a noise model in
 * which the deviation grows quadratically with depth (Section 7.1, Kalman
 * paragraph) and remarks that measurements near edges are poorer
 * (Section 1, Section 7.1).  This model predicts s = log sigma^2 (sigma in
 * metres) per pixel with a 4-32-32-1 perceptron with SiLU activations:
 *   features x = (D, |cos incidence|, min(edge distance, 16 px) / 16, radial px / fx),
 *   a1 = W1 bf16(x) + b1, h1 = bf16(silu(a1)), a2 = W2 h1 + b2, h2 = bf16(silu(a2)),
 *   s = W3 . h2 + b3;
 * bf16 = bfloat16 round to nearest even; products accumulate in float32.
 * In integration (TSDF_NOISE_MLP) p_hat = exp(s) / delta^2, clamped to
 * [p_q e^-4, p_q e^4] around the quadratic p_q = (coeff D^2 / delta)^2, which
 * is also used where the features are undefined.
 *
 * Parameters: 1249 bfloat16 values (device, caller-owned), packed as
 *   W1[32][4] | b1[32] | W2[32][32] | b2[32] | W3[32] | b3
 * (row-major, W[out][in]); the buffer must hold TSDF_MLP_PARAMS_PADDED values.
 * Training keeps float32 master weights and Adam moments (1249 floats each).
 * All calls are stream-ordered and asynchronous; argument errors return
 * TSDF_EINVAL synchronously and enqueue nothing.
 */
#ifndef TSDF_MLP_H
#define TSDF_MLP_H

#include "tsdf.h"

#ifdef __cplusplus
extern "C" {
#endif

#define TSDF_MLP_PARAMS 1249
#define TSDF_MLP_PARAMS_PADDED 1256

/* Per-pixel features of a depth map: feat_dev float [H*W][4], valid_dev
 * uint8 [H*W] (1 where all four features are defined). */
tsdf_status tsdf_mlp_features(const float *depth_dev, const tsdf_intrinsics *K, float *feat_dev,
                              uint8_t *valid_dev, hipStream_t stream);

/* s_dev[k] = network output for feature row x_dev[k] (float [n][4]). */
tsdf_status tsdf_mlp_forward(const void *params_dev, const float *x_dev, int64_t n, float *s_dev,
                             hipStream_t stream);

/* Device workspace bytes for tsdf_mlp_loss_grad with this batch size. */
uint64_t tsdf_mlp_workspace_bytes(int64_t batch);

/* Mean Gaussian negative log-likelihood 1/2 (s + r^2 e^-s) over a batch and
 * its gradient (float [1249], mean over the batch; backward products of
 * layer 2 take bf16(dL/da2) as matrix-core operands).  The batch is positions
 * first .. first+batch-1 of the visiting order k -> (perm_a k + perm_b) mod
 * n_samples over the samples x_dev [n][4], r_dev [n]; perm_a must be coprime
 * to n_samples, 0 < perm_a < n_samples, perm_b < n_samples <= 2^31.
 * loss_dev (may be null) receives the mean loss. */
tsdf_status tsdf_mlp_loss_grad(const void *params_dev, const float *x_dev, const float *r_dev, int64_t n_samples,
                               int64_t first, int64_t batch, uint64_t perm_a, uint64_t perm_b,
                               void *workspace_dev, float *grad_dev, float *loss_dev, hipStream_t stream);

/* One Adam step (bias-corrected, step >= 1) on float master weights; writes
 * the bf16 parameters params_dev = bf16(master). */
tsdf_status tsdf_mlp_adam_step(float *master_dev, float *m_dev, float *v_dev, const float *grad_dev,
                               void *params_dev, int32_t step, float lr, float beta1, float beta2, float eps,
                               hipStream_t stream);

/* Training samples of one frame: every pixel with a measurement, defined
 * features (from tsdf_mlp_features of the same depth) and a raycast hit
 * (vertex_dev from tsdf_raycast at the same pose) gives (x, r = D - z) with z
 * the camera depth of the hit.  Samples are appended in pixel order at
 * *count_dev (device uint64, running total; not reset); rows at or beyond
 * cap are counted but not written.  workspace_dev: at least
 * tsdf_mlp_samples_workspace_bytes(width, height) bytes. */
uint64_t tsdf_mlp_samples_workspace_bytes(int32_t width, int32_t height);
tsdf_status tsdf_mlp_collect_samples(const float *depth_dev, const float *feat_dev, const uint8_t *valid_dev,
                                     const float *vertex_dev, const tsdf_intrinsics *K, const double pose_c2w[12],
                                     void *workspace_dev, uint64_t *count_dev, int64_t cap, float *x_out_dev,
                                     float *r_out_dev, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif
