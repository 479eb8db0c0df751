/* Warm-start network of libnld: a small convolutional network that predicts a starting point
 * u0 for the deflated Jacobi PCG (nld.h, pcg_solve with use_u0 = 1) from the noisy image f and
 * the parameters (log alpha, log sigma_l).  Not part of the paper's method: PCG from u0
 * converges to the same solution as from f, the network only shortens the iteration.
 *
 * Architecture: five 3x3 convolutions with zero "same" padding, channels
 * (1 + n_cond) -> 32 -> 32 -> 32 -> 32 -> 1, ReLU after the first four, output u0 = f + y.
 * Input channels: f, then the n_cond conditioning scalars of the image as constant maps.
 * Arithmetic: BF16 activations and weights on the matrix cores with FP32 accumulation; FP32
 * master parameters, gradients and Adam moments; the loss is accumulated in FP64.
 *
 * Parameters are a flat FP32 vector in the order (W_1, b_1, ..., W_5, b_5), W_k of shape
 * [cout][cin][3][3] (cross-correlation: y[co][i][j] = b[co] + sum w[co][ci][a][c]
 * x[ci][i + a - 1][j + c - 1]).
 *
 * Images are batches of n images of h x w pixels, row-major FP32 device arrays [n][h][w];
 * cond is a host array [n][n_cond].  All calls run on the given stream and block until done,
 * except cnn_adam_step.  Errors: NLD_E_INVAL (arguments, checked on the host before any
 * launch), NLD_E_HIP, NLD_E_NOMEM; message in nld_last_error(). */
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nld.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nld_cnn_s* nld_cnn_t;

typedef struct {
  float lr, beta1, beta2, eps;
} nld_adam;

/* New network with n_cond in [0, 31] conditioning channels; He-normal weights from the seed
 * (last layer scaled by 0.1), zero biases, zero Adam state.  Allocates on the current device. */
nld_status cnn_create(nld_cnn_t* out, int32_t n_cond, uint64_t seed);
nld_status cnn_destroy(nld_cnn_t net);
/* Number of parameters, or -1 for a null network. */
int64_t cnn_param_count(nld_cnn_t net);
/* Copy the parameters and/or the last gradient (either may be NULL, not both) to host arrays
 * of cnn_param_count floats. */
nld_status cnn_get_params(nld_cnn_t net, float* theta, float* grad);
/* Replace the parameters (host array of cnn_param_count finite floats). */
nld_status cnn_set_params(nld_cnn_t net, const float* theta);
/* u0 = f + network(f, cond) for n images of h x w (u0: device [n][h][w], caller-owned). */
nld_status cnn_predict(nld_cnn_t net, const float* f, const float* cond, int32_t n, int32_t h,
                       int32_t w, float* u0, hipStream_t s);
/* Forward and backward pass of the mean squared error mean((u0 - target)^2) over all pixels of
 * the batch; stores the gradient in the network (cnn_get_params reads it) and the loss in
 * *loss. */
nld_status cnn_loss_grad(nld_cnn_t net, const float* f, const float* cond, const float* target,
                         int32_t n, int32_t h, int32_t w, double* loss, hipStream_t s);
/* One Adam step (bias-corrected) on the stored gradient; enqueued on s. */
nld_status cnn_adam_step(nld_cnn_t net, const nld_adam* opt, hipStream_t s);

#ifdef __cplusplus
}
#endif
