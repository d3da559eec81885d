/*
 * sfft_mlp.h -- C ABI of the warm-start network of the SFFT library (gfx950).
 *
 * A small fully connected network predicts the kernel coefficients of the
 * subtraction from the two PSF stamps and the frame position, so that a
 * quick-look difference image needs no normal-matrix solve; the plain solve
 * stays the fallback and judges the prediction through its residual
 * rho = ||beta - Omega theta|| / ||beta|| (sfft_residual in sfft.h).  The
 * paper motivates this with the spatially varying Roman PSF that the kernel
 * must follow ("Statement of need") and the cost of the large linear system
 * ("Future development"); the network itself is this library's addition.
 *
 * Network: h_0 = x, h_l = relu(h_{l-1} W_l + b_l) for l < nl, y = h_{nl-1} W_nl + b_nl.
 * dims[0..nl] are the layer widths (dims[0] inputs, dims[nl] outputs).
 *
 * Parameter vector (FP32, device, caller-owned), layer after layer:
 *   [W_1 (dims[0] x dims[1], row-major: W[i*dims[1] + j]), b_1 (dims[1]), W_2, b_2, ...]
 * Batches are row-major [batch][dims[l]] FP32 device arrays, one sample per row.
 *
 * Conventions: as in sfft.h.  Every call returns an SFFT_* status; pointers
 * are device pointers unless stated; work is enqueued on the handle's HIP
 * stream and nothing synchronises; arguments are checked before anything is
 * enqueued (SFFT_EINVAL); calling out of order gives SFFT_ESTATE.
 */
#ifndef SFFT_MLP_H_
#define SFFT_MLP_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sfft_mlp_s* sfft_mlp;

/* Create a network handle for layer widths dims[0..nlayers] (1 <= nlayers <= 8,
 * 1 <= dims[i] <= 8192) and batches of at most max_batch samples.  The handle
 * allocates its own device scratch: the activations of one batch, two
 * gradient buffers and the BF16 weight copy.  `hip_stream` may be NULL (the
 * null stream).  SFFT_ENOMEM if the scratch cannot be allocated. */
int sfft_mlp_create(const int32_t* dims, int32_t nlayers, int32_t max_batch, void* hip_stream, sfft_mlp* out);

/* Number of FP32 parameters (host output). */
int sfft_mlp_param_count(sfft_mlp m, int64_t* count);

/* Training forward in FP32 (matrix cores, FP32 products and sums):
 * y[batch][dims[nl]] from x[batch][dims[0]].  Keeps the hidden activations
 * in the handle for sfft_mlp_backward. */
int sfft_mlp_forward(sfft_mlp m, const float* params, const float* x, int32_t batch, float* y);

/* Gradient of sum(dy * y) with respect to every parameter, written to
 * grad (same packing as params), for the batch of the last sfft_mlp_forward
 * (same params and x must be passed; SFFT_ESTATE without a forward of that
 * batch size).  FP32 matrix-core products, column sums for the biases. */
int sfft_mlp_backward(sfft_mlp m, const float* params, const float* x, const float* dy, int32_t batch,
                      float* grad);

/* Mean squared error over batch*dims[nl] values: loss = mean((y - t)^2)
 * (device double scalar, summed in FP64) and dy = 2 (y - t) / count. */
int sfft_mlp_mse(sfft_mlp m, const float* y, const float* t, int32_t batch, float* dy, double* loss);

/* One bias-corrected Adam step over all parameters (`step` >= 1 is the
 * 1-based step number): m1 = b1 m1 + (1-b1) g, m2 = b2 m2 + (1-b2) g^2,
 * params -= lr * (m1 / (1 - b1^step)) / (sqrt(m2 / (1 - b2^step)) + eps).
 * params, m1 and m2 are the caller's FP32 master copies, updated in place. */
int sfft_mlp_adam_step(sfft_mlp m, float* params, const float* grad, float* m1, float* m2, int32_t step, float lr,
                       float b1, float b2, float eps);

/* Take a BF16 snapshot of the weights (round to nearest even; biases kept
 * in FP32) for sfft_mlp_infer. */
int sfft_mlp_set_weights_bf16(sfft_mlp m, const float* params);

/* BF16 inference (matrix cores, BF16 operands, FP32 sums): the output layer
 * is de-standardised in FP64, theta[s*ld_theta + j] = y_sj * scale[j] + shift[j]
 * (scale/shift: device double[dims[nl]]; both NULL = identity).
 * SFFT_ESTATE without a prior sfft_mlp_set_weights_bf16. */
int sfft_mlp_infer(sfft_mlp m, const float* x, int32_t batch, const double* scale, const double* shift,
                   double* theta, int64_t ld_theta);

/* Release the handle and its scratch (after its stream has drained). */
void sfft_mlp_destroy(sfft_mlp m);

#ifdef __cplusplus
}
#endif

#endif /* SFFT_MLP_H_ */
