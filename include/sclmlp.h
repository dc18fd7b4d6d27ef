/*
 * sclmlp — learned droplet-shape surrogate for the sclbm droplet boxes (MI355X,
 * gfx950).
 *
 * The paper follows a droplet's shape through the semi-axes of its ellipsoid and
 * the deformation D = (L - B)/(L + B) (Sec. 2 Eq. 4) while a box is driven by a
 * velocity-gradient history A(t) (Sec. 3 Eq. 14).  This surrogate maps a window
 * of that history — 64 samples of the 9 entries of A, one every 50 lattice
 * steps, oldest first, flattened sample-major to 576 floats — to the 3
 * semi-axes at the window's last sample, in the units the caller trains with
 * (the sclbm workflow uses semi-axes over the droplet's volume-equivalent
 * radius).  The network is a perceptron 576 -> 512 -> 512 -> 512 -> 3 with ReLU
 * on the hidden layers; BF16 weights and activations, FP32 accumulation on the
 * matrix cores, FP32 biases, FP32 master weights, trained with Adam on the mean
 * squared error of the normalised targets.
 *
 * Normalisation (set with sclmlp_set_normalization):
 *   x = (window - in_shift) * in_scale          (576 entries each)
 *   t = (semi_axes - out_shift) * out_scale      (3 entries each)
 *   predicted semi_axes = y / out_scale + out_shift
 *
 * Parameters: one FP32 vector of SCLMLP_NPARAM values, in this order:
 *   W1 [512][576], b1 [512], W2 [512][512], b2 [512], W3 [512][512], b3 [512],
 *   W4 [3][512], b4 [3]   (weights [out][in], row-major).
 *
 * Conventions: dev_* pointers are device memory of the context's GPU, others
 * host memory.  Calls enqueue on the context's stream and return without waiting
 * unless documented to synchronise.  A context is not thread-safe.  Every call
 * returns an sclbm_status (sclbm.h); sclmlp_last_error() gives a thread-local
 * message.  The caller owns the workspace and every buffer; the library
 * allocates no device memory.
 */
#ifndef SCLMLP_H
#define SCLMLP_H

#include "sclbm.h"

#ifdef __cplusplus
extern "C" {
#endif

#define SCLMLP_NIN 576
#define SCLMLP_NHIDDEN 512
#define SCLMLP_NOUT 3
#define SCLMLP_NPARAM 822275

typedef struct sclmlp_ctx sclmlp_ctx;

/* Device workspace for batches of up to max_batch rows (max_batch >= 1). */
sclbm_status sclmlp_workspace_bytes(int64_t max_batch, size_t *bytes);

/* Create a context on the current HIP device over a caller-owned workspace of
 * at least sclmlp_workspace_bytes(max_batch) bytes (256-byte aligned);
 * hip_stream may be NULL (null stream).  Parameters start at zero, the
 * normalisation at shift 0 / scale 1. */
sclbm_status sclmlp_create(int64_t max_batch, void *dev_workspace, size_t bytes, void *hip_stream, sclmlp_ctx **out);
sclbm_status sclmlp_destroy(sclmlp_ctx *ctx);

/* Load all SCLMLP_NPARAM parameters (host FP32, layout above), refresh the BF16
 * copies and reset Adam (moments to zero, step counter to zero).  Synchronises. */
sclbm_status sclmlp_set_params(sclmlp_ctx *ctx, const float *params);
/* Copy the FP32 master parameters / the gradients of the last
 * sclmlp_gradients call to host memory (SCLMLP_NPARAM floats).  Synchronises. */
sclbm_status sclmlp_get_params(sclmlp_ctx *ctx, float *params);
sclbm_status sclmlp_get_grads(sclmlp_ctx *ctx, float *grads);

/* Input and output normalisation (host FP32; scales must be finite and non-zero). */
sclbm_status sclmlp_set_normalization(sclmlp_ctx *ctx, const float in_shift[SCLMLP_NIN],
                                      const float in_scale[SCLMLP_NIN], const float out_shift[SCLMLP_NOUT],
                                      const float out_scale[SCLMLP_NOUT]);

/* Inference: dev_windows [n][576] FP32 -> dev_out [n][3] FP32 semi-axes of the
 * droplet ellipsoid (Sec. 2 Eq. 4) at each window's last sample,
 * 0 <= n <= max_batch. */
sclbm_status sclmlp_predict(sclmlp_ctx *ctx, const float *dev_windows, int64_t n, float *dev_out);

/* Forward and backward pass over a batch of n rows (1 <= n <= max_batch):
 * row m uses dev_windows[idx] and dev_targets[idx] (targets [.][3] FP32, in
 * semi-axis units) with idx = dev_index[m] (int32) or m when dev_index is NULL;
 * ndata is the number of rows of dev_windows / dev_targets.
 *
 * dev_sym (int32 per row, or NULL for none) applies a symmetry of the cubic
 * box to the row's window: id s in [0, 48) names the signed permutation P with
 * P[i][perm(i)] = sign(i), perm the (s / 8)-th permutation of (0, 1, 2) in
 * lexicographic order and sign(i) = -1 where bit i of (s % 8) is set; every
 * sample A of the window becomes P A P^T.  The droplet box (cube, D3Q19
 * lattice, centred droplet, ghost velocity A (x - x_c)) is invariant under these
 * maps, so the semi-axes (the targets) do not change: an exact augmentation.
 *
 * A row whose index lies outside [0, ndata), or whose symmetry id lies outside
 * [0, 48), contributes nothing and is counted (sclmlp_bad_rows).  Leaves the
 * gradient of the mean squared error of the normalised outputs, averaged over
 * the n rows, in the context; dev_loss (may be NULL) receives that loss as one
 * FP64 value. */
sclbm_status sclmlp_gradients(sclmlp_ctx *ctx, const float *dev_windows, const float *dev_targets,
                              const int32_t *dev_index, const int32_t *dev_sym, int64_t n, int64_t ndata,
                              double *dev_loss);

/* One Adam step (bias-corrected) with the gradients in the context, then the
 * BF16 copies.  lr > 0, 0 <= beta1, beta2 < 1, eps > 0. */
sclbm_status sclmlp_adam(sclmlp_ctx *ctx, float lr, float beta1, float beta2, float eps);

/* sclmlp_gradients followed by sclmlp_adam. */
sclbm_status sclmlp_train_step(sclmlp_ctx *ctx, const float *dev_windows, const float *dev_targets,
                               const int32_t *dev_index, const int32_t *dev_sym, int64_t n, int64_t ndata,
                               float lr, float beta1, float beta2, float eps, double *dev_loss);

/* Adam steps taken since sclmlp_set_params. */
sclbm_status sclmlp_get_step(const sclmlp_ctx *ctx, int64_t *step);

/* Rows skipped for an out-of-range index or symmetry id since the context was
 * created.  Synchronises. */
sclbm_status sclmlp_bad_rows(sclmlp_ctx *ctx, int64_t *count);

const char *sclmlp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SCLMLP_H */
