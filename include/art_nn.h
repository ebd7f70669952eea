/*
 * art_nn.h -- C interface of the layers of the learned surrogate of libart:
 * a 3-D convolution network that maps a coarse sweep (few HEALPix
 * directions) plus the local fields to the mean intensity of a fine sweep.
 * The surrogate is not part of the paper; the sweep it stands in for is the
 * one of art.h (Sect. 2.2-2.3 of Tanaka et al., arXiv:1410.0763).
 *
 * Conventions
 * -----------
 * - Activations are bfloat16 (raw 16-bit words, round-to-nearest-even),
 *   channels-last [D][H][W][C]; V = D*H*W voxels, x fastest.
 * - A layer's weight is w[tap][ci][co] float32 with tap = (dz+1)*9 +
 *   (dy+1)*3 + (dx+1) for offsets dz, dy, dx in {-1, 0, 1}; zero padding, so
 *   out[v][co] = bias[co] + sum_{tap, ci} w[tap][ci][co] x[v + offset(tap)][ci].
 *   The products run on the matrix cores (bf16 inputs, float32 sums).
 * - Every call returns ART_OK or a negative ART_E_* code (art.h) and queues
 *   its work on hip_stream; all pointers are device pointers owned by the
 *   caller, which must keep them valid until the stream has passed the call.
 * - Reductions (weight and bias gradients, the loss) are summed in a fixed
 *   order: results are bitwise reproducible.
 */
#ifndef ART_NN_H
#define ART_NN_H

#ifdef __cplusplus
extern "C" {
#endif

/* Convolution of x (cin = 16 or 32 channels) with 32 output channels.
 * w_k: bf16 [27][32][cin] (made by art_nn_prep_weights); bias: float32 [32]
 * or NULL; relu: apply max(0, .) after the bias.  mask: bf16 [V][32] or
 * NULL: y is set to 0 wherever mask <= 0 (the ReLU gradient of the layer
 * whose output mask is, fused into the input-gradient convolution).
 * Outputs (either may be NULL): y bf16 [V][32], y0 float32 [V] = channel 0
 * of the output (never masked).  W must be a multiple of 32.  ART_E_INVAL on
 * bad sizes or null x/w_k. */
int art_conv3d_fwd(const void *x, int cin, const void *w_k, const float *bias, int D, int H,
                   int W, int relu, const void *mask, void *y, float *y0, void *hip_stream);

/* Weight and bias gradients of one layer:
 * dw[tap][ci][co] = sum_v x[v + offset(tap)][ci] g[v][co] (zero padding) and
 * db[co] = sum_v g[v][co].  x: bf16 [V][cin], the layer input (cin = 16 or
 * 32); g: bf16 [V][32], the gradient at the layer output (art_nn_relu_grad).
 * work: float32 workspace of work_floats >= art_conv3d_bwd_weight_workspace()
 * elements (per-workgroup partial sums, overwritten).  dw: float32
 * [27][cin][32]; db: float32 [32] or NULL.  W must be a multiple of 16.
 * ART_E_INVAL on null pointers, bad sizes or a short workspace. */
int art_conv3d_bwd_weight(const void *x, int cin, const void *g, int D, int H, int W, float *work,
                          long long work_floats, float *dw, float *db, void *hip_stream);

/* Float32 elements of workspace art_conv3d_bwd_weight needs for this shape
 * (-1 for a shape it rejects).  Host only. */
long long art_conv3d_bwd_weight_workspace(int cin, int D, int H, int W);

/* Gradient at a layer output: g = dy where y > 0 (the ReLU of the forward
 * pass; y = NULL for the last layer, which has none), else 0.  dy, y, g:
 * bf16 [V][32]. */
int art_nn_relu_grad(const void *dy, const void *y, int V, void *g, void *hip_stream);

/* Matrix-core copies of one layer's weights w (float32 [27][cin][32]):
 * w_fwd bf16 [27][32][cin] for the forward convolution and w_bwd bf16
 * [27][32][32] for the input gradient (taps mirrored, channels swapped, rows
 * beyond cin zero), used as art_conv3d_fwd(g, 32, w_bwd, NULL, ...). */
int art_nn_prep_weights(const float *w, int cin, void *w_fwd, void *w_bwd, void *hip_stream);

/* Weighted mean squared error of pred against target (float32 [V]):
 * loss[0] = mean(weight (pred - target)^2) (weight float32 [V], or NULL for
 * 1); dy bf16 [V][32] = d loss / d output (channel 0; other channels 0).
 * partial: float32 scratch [256]. */
int art_nn_mse(const float *pred, const float *target, const float *weight, int V, float *partial,
               float *loss, void *dy, void *hip_stream);

/* Loss weights w = (J^2 / mean(J^2) + lambda) / (1 + lambda) (float32 [V];
 * J^2 / mean(J^2) taken as 1 if J is all zero; lambda >= 0): lambda = 0
 * makes the loss on log(J_fine / J_coarse) approximate the squared relative
 * L2 error of J, a large lambda the per-cell squared relative error.
 * partial: float32 scratch [257]. */
int art_nn_sq_weights(const float *J, int V, float lambda, float *partial, float *w,
                      void *hip_stream);

/* One AdamW step on n float32 parameters (decoupled weight decay wd,
 * bias-corrected moments m, v; step >= 1). */
int art_nn_adamw(float *w, const float *g, float *m, float *v, int n, float lr, float beta1,
                 float beta2, float eps, float wd, int step, void *hip_stream);

/* Surrogate input features, bf16 [V][16]: channel k < 3 is
 * (f_k - mu[k]) * inv_sd[k] with f_0 = log(max(J, 1e-30)) (J of the coarse
 * sweep), f_1 = log(max(density, 1e-30)), f_2 = x_hi (neutral fraction), the
 * rest 0.  J, density, x_hi: device float32 [V]; mu, inv_sd: host arrays [3]. */
int art_nn_features(const float *J, const float *density, const float *x_hi, int V, const float *mu,
                    const float *inv_sd, void *x, void *hip_stream);

/* J_out = J_coarse * exp(pred) (elementwise; the surrogate predicts the log
 * ratio of the fine to the coarse incoming mean intensity J_in). */
int art_nn_expand(const float *J_coarse, const float *pred, int V, float *J_out,
                  void *hip_stream);

/* Training target: target = log(J_fine) - log(J_coarse) (both floored at
 * 1e-30), float32 [V]. */
int art_nn_log_ratio(const float *J_fine, const float *J_coarse, int V, float *target,
                     void *hip_stream);

/* count[0] = number of voxels whose features (bf16 [V][16], channels 0-2)
 * leave [lo[k], hi[k]] in any channel k (lo, hi: host arrays [3]): the
 * out-of-distribution measure of the surrogate's acceptance gate.  count is
 * cleared by the call (with a kernel, so the call may be graph-captured). */
int art_nn_ood_count(const void *x, int V, const float *lo, const float *hi, unsigned int *count,
                     void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* ART_NN_H */
