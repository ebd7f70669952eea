/*
 * art_surrogate.h -- the learned surrogate of the fine sweep as a library
 * object: parameters, AdamW state and work buffers of the network, its
 * training step, inference, the acceptance gate with fallback to the fine
 * sweep, and checkpoints.  The surrogate is not part of the paper; the sweep
 * it stands in for is art_sweep (Sect. 2.2-2.3 of Tanaka et al.,
 * arXiv:1410.0763), and its layers are those of art_nn.h.
 *
 * Network
 * -------
 * Input per cell (bf16 [V][16], channels-last, V = nx*ny*nz, x fastest):
 * (log J_coarse, log n, x_HI) of one frequency bin, each shifted by mu and
 * divided by sd (the surrogate's feature statistics), J_coarse and the
 * density n floored at 1e-30 before the logarithm; J_coarse is the mean
 * intensity J (eq mean_intensity) of a sweep at a small Nside, n and x_HI
 * the density and neutral fraction the caller's kappa and S were made from.
 * Six convolution layers (3^3 taps, zero padding, 32 channels, ReLU after
 * the first five) predict p = log(J_in,fine / J_in,coarse), J_in being the
 * incoming part of J (J = J_in + S) of the sweeps at a large and the small
 * Nside; the estimate is J_in = J_in,coarse e^p and J = J_in + S (the local
 * source term is exact at any Nside).  114,209 trainable parameters.
 *
 * Acceptance gate
 * ---------------
 * est_err = val_err + (fraction of cells whose normalised features leave
 * [lo, hi] in any channel).  val_err is the relative L2 error of J the caller
 * measured on held-out fields; lo, hi bound the normalised features seen in
 * training.  A prediction is used only if est_err <= err_bound; otherwise the
 * fine sweep runs instead.
 *
 * Conventions
 * -----------
 * - Every call returns ART_OK or a negative ART_E_* code (art.h) and sets
 *   art_last_error on failure; no call aborts or throws.
 * - Device pointers are caller-owned and must stay valid until hip_stream has
 *   passed the call; work is queued on hip_stream unless a call says it
 *   synchronises.
 * - One surrogate handle must not be used from two threads or two streams at
 *   once (its work buffers are shared by its calls).
 */
#ifndef ART_SURROGATE_H
#define ART_SURROGATE_H

#include "art.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct art_surrogate art_surrogate;

/* Parameter arrays of art_surrogate_param. */
enum {
    ART_SG_W = 0,    /* weights float32 [27][cin][32], cin = 16 for layer 0, else 32 */
    ART_SG_B = 1,    /* bias float32 [32] */
    ART_SG_DW = 2,   /* gradient of the weights (last art_surrogate_gradients) */
    ART_SG_DB = 3    /* gradient of the bias */
};

/* Surrogate for meshes of nx*ny*nz cells (nx a multiple of 32; nx*ny*nz at
 * most 11184810 so that every training buffer stays below 2 GiB).  Weights
 * are normal with standard deviation sqrt(2 / (27 fan_in)) (last layer
 * 1e-3), drawn by a generator seeded with seed; biases and AdamW moments
 * start at 0; the feature statistics start at mu = 0, sd = 1, lo = -inf,
 * hi = +inf, val_err unknown.
 * Allocates about 820 bytes per cell of device memory; synchronises the
 * device.  Ownership: *out belongs to the library until
 * art_surrogate_destroy. */
int art_surrogate_create(int nx, int ny, int nz, unsigned long long seed, art_surrogate **out);

/* Release the surrogate and its device memory (NULL is accepted). */
int art_surrogate_destroy(art_surrogate *s);

/* Number of trainable parameters (114209), or ART_E_INVAL for NULL. */
int art_surrogate_n_params(const art_surrogate *s);

/* Feature statistics and gate data, host arrays [3]: mu, sd (> 0), lo, hi;
 * val_err: held-out relative L2 error of J (negative or NaN: unknown, which
 * makes every art_sweep_surrogate fall back). */
int art_surrogate_set_stats(art_surrogate *s, const float *mu, const float *sd, const float *lo,
                            const float *hi, float val_err);
int art_surrogate_get_stats(const art_surrogate *s, float *mu, float *sd, float *lo, float *hi,
                            float *val_err);

/* Fit mu and sd (mean and population standard deviation) of the three raw
 * features (log J_coarse, log n, x_HI) over n fields (host arrays of n device
 * pointers to float32 [V] J_coarse, density and neutral fraction), and lo, hi
 * = extremes of the normalised features -/+ margin (>= 0).  val_err is left
 * as it is.  Partial sums are double precision, added in a fixed order.
 * Synchronises hip_stream. */
int art_surrogate_fit_stats(art_surrogate *s, int n, const float *const *J_coarse,
                            const float *const *density, const float *const *x_hi, float margin,
                            void *hip_stream);

/* Network input x (bf16 [V][16]) of one field from J_coarse, density and
 * x_HI (device float32 [V]) with the current statistics. */
int art_surrogate_features(const art_surrogate *s, const float *J_coarse, const float *density,
                           const float *x_hi, void *x, void *hip_stream);

/* Training pair of the field loaded in mesh (one bin, shape of the
 * surrogate): the sweeps at nside_coarse and nside_fine (I_bc = 0) write
 * J_coarse (required; the network's input) and J_fine (may be NULL),
 * target = log(J_in,fine / J_in,coarse) and, if weight is not NULL, the loss
 * weights (J_in,coarse^2 / mean J_in,coarse^2 + lambda) / (1 + lambda),
 * lambda >= 0 (art_nn_sq_weights), which make the loss approximate the
 * squared relative L2 error of J_in (lambda = 0) or the per-cell squared
 * log error (large lambda).  All device float32 [V]. */
int art_surrogate_make_pair(art_surrogate *s, art_mesh *mesh, int nside_coarse, int nside_fine,
                            float lambda, float *target, float *weight, float *J_coarse,
                            float *J_fine, void *hip_stream);

/* Gradients of the loss mean(weight (p - target)^2) (weight NULL: 1) with
 * respect to every parameter, kept in the surrogate (ART_SG_DW, ART_SG_DB);
 * loss: device float32 [1] or NULL.  Deterministic. */
int art_surrogate_gradients(art_surrogate *s, const void *x, const float *target,
                            const float *weight, float *loss, void *hip_stream);

/* art_surrogate_gradients followed by one AdamW step (beta1 0.9, beta2
 * 0.999, eps 1e-8; decoupled weight decay wd on the weights only, lr > 0). */
int art_surrogate_train_step(art_surrogate *s, const void *x, const float *target,
                             const float *weight, float lr, float wd, float *loss,
                             void *hip_stream);

/* Prediction p = log(J_in,fine / J_in,coarse) for input x into pred (device
 * float32 [V]). */
int art_surrogate_infer(art_surrogate *s, const void *x, float *pred, void *hip_stream);

/* Copy parameter array `what` (ART_SG_*) of layer 0..5 to buf (write = 0) or
 * from buf into the surrogate (write = 1; ART_SG_W and ART_SG_B only).  buf:
 * device float32 of the array's size. */
int art_surrogate_param(art_surrogate *s, int layer, int what, float *buf, int write,
                        void *hip_stream);

/* Checkpoint: weights, biases, AdamW moments, step count, statistics and
 * shape, with a SHA-256 digest over everything after it.  Both calls
 * synchronise hip_stream.  art_surrogate_load rejects (ART_E_INVAL, the
 * surrogate unchanged) a file that is not a checkpoint, is truncated, fails
 * the digest, or was saved for another mesh shape. */
int art_surrogate_save(art_surrogate *s, const char *path, void *hip_stream);
int art_surrogate_load(art_surrogate *s, const char *path, void *hip_stream);

/* J of a sweep at nside_fine from the sweep at nside_coarse and the network,
 * for the field loaded in mesh (one bin, the surrogate's shape, I_bc = 0)
 * made from density and x_hi (device float32 [V], the network's inputs).
 * If the gate accepts: out->J_in = J_in,coarse e^p, out->J = J_in + S,
 * out->Gamma = gamma_w[0] J (gamma_w host [1] or NULL for 1), out->Heat =
 * heat_in[0] J_in + heat_src[0] S (the mesh's weights, art_set_heating) and
 * out->J_exact = J + (J_exact - J) of the coarse sweep (the network predicts
 * J_in only).  Otherwise out receives art_sweep at nside_fine.
 * out->exit_sum must be NULL.  *used_fallback (0 or 1) and *est_err (NaN
 * while val_err is unknown) may be NULL.  An err_bound <= 0 always falls
 * back.  Synchronises hip_stream once, to read the out-of-range count. */
int art_sweep_surrogate(art_mesh *mesh, art_surrogate *s, const float *density, const float *x_hi,
                        int nside_coarse, int nside_fine, const float *gamma_w, float err_bound,
                        const art_outputs *out, int *used_fallback, float *est_err,
                        void *hip_stream);

/* SHA-256 (FIPS 180-4) of n bytes at data (host) into digest[32]: the
 * checkpoint digest. */
int art_sha256(const void *data, unsigned long long n, unsigned char *digest);

#ifdef __cplusplus
}
#endif

#endif /* ART_SURROGATE_H */
