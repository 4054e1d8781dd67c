/*
 * tomo_unet.h -- C ABI of the learned artefact-correction network in libtomo.so.
 *
 * Not part of the paper's method: a small 3D U-Net that maps a reconstruction made
 * from few views to the reconstruction the dense view set gives, trained on pairs that
 * the library's own reconstruction produces.  Architecture (volumes [C][n][n][n], n a
 * multiple of 4, 8 <= n <= 256; 3x3x3 convolutions with zero padding and bias, ReLU after
 * each but the last):
 *   e1 = relu(conv(relu(conv(x, 1->16)), 16->16))              n^3
 *   e2 = relu(conv(relu(conv(pool(e1), 16->32)), 32->32))      (n/2)^3
 *   b  = relu(conv(relu(conv(pool(e2), 32->64)), 64->64))      (n/4)^3
 *   d2 = relu(conv(relu(conv([up(b), e2], 96->32)), 32->32))   (n/2)^3
 *   d1 = relu(conv(relu(conv([up(d2), e1], 48->16)), 16->16))  n^3
 *   y  = x + conv1x1(d1, 16->1)
 * pool = 2x2x2 average, up = 2x nearest repeat, [a, b] = channel concatenation.
 * Parameters: one float32 vector of tomo_unet_param_count() values: for each layer in
 * the order above, weights [Cout][Cin][k][k][k] then bias [Cout].  The convolutions use
 * the BF16 rounding (nearest even) of the weights; activations, gradients and all sums
 * are FP32 (the loss FP64), in a fixed order: results are bitwise reproducible.  On the
 * matrix cores an FP32 operand is split into two BF16 parts (relative remainder at most
 * 2^-18), so a product carries at most that relative error.
 * Loss: mean squared error.  Optimiser: Adam with bias correction.
 *
 * All device pointers are caller-owned, 256-byte aligned; calls are asynchronous on
 * the stream (hipStream_t as void*, NULL = null stream).  A network object owns the
 * activation and gradient workspace of one volume size and serves one stream at a time.
 */
#ifndef TOMO_UNET_H
#define TOMO_UNET_H

#include "tomo.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tomo_unet_s* tomo_unet_t;

/* Number of float32 parameters (weights and biases of all layers). */
int32_t tomo_unet_param_count(void);

/* Workspace for volumes of edge n.  TOMO_EINVAL for n not a multiple of 4 or outside
 * [8, 256]; TOMO_ENOMEM if the device allocation fails; the message of a failure is
 * tomo_unet_error(NULL). */
tomo_status tomo_unet_create(int32_t n, tomo_unet_t* out);

/* d_y [n^3] = network(d_x [n^3]) with parameters d_params [param_count]. */
tomo_status tomo_unet_forward(tomo_unet_t net, const float* d_params, const float* d_x, float* d_y, void* stream);

/* Forward pass, loss = mean((y - target)^2) into d_loss (device double [1]) and its
 * gradient with respect to the parameters into d_grad [param_count] (overwritten). */
tomo_status tomo_unet_gradient(tomo_unet_t net, const float* d_params, const float* d_x, const float* d_target,
                               float* d_grad, double* d_loss, void* stream);

/* One Adam step (step >= 1; bias correction 1 - beta^step) on d_params with gradient
 * d_grad; d_m and d_v [param_count] are the moment estimates (zero before step 1). */
tomo_status tomo_unet_adam(tomo_unet_t net, float* d_params, const float* d_grad, float* d_m, float* d_v,
                           int32_t step, float lr, float beta1, float beta2, float eps, void* stream);

/* Message of the last failing call on this network (NULL: of the last failed create). */
const char* tomo_unet_error(tomo_unet_t net);

/* Release the workspace (synchronises the device).  NULL is OK. */
tomo_status tomo_unet_destroy(tomo_unet_t net);

#ifdef __cplusplus
}
#endif

#endif /* TOMO_UNET_H */
