/*
 * recon_cnn.h — C ABI of the learned warm start of the reconstruction library
 * (librecon.so, gfx950).
 *
 * The paper (Ozaki et al., arXiv:1903.10088) speeds up its ordered-subset TV
 * iteration by thinning and an adaptive step (sections 3.C-3.D); this module
 * adds a learned starting point: a small residual CNN maps an early iterate of
 * that iteration to an estimate of the converged image, and the plain
 * iteration then refines it.  The network is trained only on images that the
 * plain iteration itself produced.
 *
 * Network (8 layers, 3x3 kernels, 32 hidden channels, zero "same" padding):
 *   x = mu / mu_scale;  a_0 = bf(x)
 *   z_l = conv(a_{l-1}, bf(W_l)) + b_l,  a_l = bf(relu(z_l))   l = 1..7
 *   z_8 = conv(a_7, bf(W_8)) + b_8;  y = x + z_8;  mu_out = mu + mu_scale * z_8 (= mu_scale * y)
 * conv(a, W)[o][i][j] = sum_c sum_{dy,dx in -1..1} W[o][c][dy+1][dx+1] a[c][i+dy][j+dx]
 * (cross-correlation; a is 0 outside the image), bf() rounds to bfloat16 (round
 * to nearest even): weights and hidden activations are stored in bfloat16, the
 * 32-channel convolutions run on the matrix cores (bfloat16 inputs, float32
 * accumulation), the first and last layers on the vector ALUs in float32.
 *
 * Training minimises L = 1/(B |D|) sum_b sum_{p in D} (y_b[p] - target_b[p] / mu_scale)^2
 * over the reconstruction disc D of each n x n image (pixel centres within n/2
 * pixels of the grid centre), by Adam (Kingma and Ba, ICLR 2015; beta1 0.9,
 * beta2 0.999, eps 1e-8) on float32 master parameters.  The backward signals
 * dL/dz_l of layers 1..7 are stored in bfloat16 (they feed the matrix cores);
 * dL/dz_8 stays float32.  Weight gradients are reduced in a fixed order, so
 * every call is bitwise deterministic.
 *
 * Parameter vector (float32, host or device as stated): for l = 1..8 in turn
 * W_l as [out][in][3][3] then b_l [out]; (in, out) = (1, 32), (32, 32) x 6,
 * (32, 1); recon_cnn_param_count() = 56097 floats.
 *
 * Images: float32 [batch][n][n] row-major, attenuation in 1/mm, device memory
 * owned by the caller.  Calls are asynchronous on `stream` (a hipStream_t)
 * unless stated; a handle is not thread-safe.  Errors: recon_status as in
 * recon.h, message from recon_last_error().
 */
#ifndef RECON_CNN_H
#define RECON_CNN_H

#include <stdint.h>

#include "recon.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct recon_cnn recon_cnn;

/* Number of float32 parameters (56097). */
int64_t recon_cnn_param_count(void);

/* Creates a network on the current device with workspace for training
 * batches of up to max_batch images of up to max_n x max_n (forward passes of
 * larger batches run in chunks of max_batch).  h_params: host float32
 * [param_count] initial parameters, NULL = all zero (the identity map).
 * mu_scale > 0 is the attenuation the network input is divided by (the water
 * value, 0.0049 /mm, in this project).  Adam moments start at zero, step 0.
 * Blocks until done. */
recon_status recon_cnn_create(const float* h_params, int32_t max_batch, int32_t max_n, float mu_scale,
                              recon_cnn** out);
recon_status recon_cnn_destroy(recon_cnn* net);

/* Copies the float32 parameters, Adam moments and step count out of / into
 * the network (host buffers of param_count floats; NULL pointers are skipped).
 * Synchronous. */
recon_status recon_cnn_get_state(recon_cnn* net, float* h_params, float* h_adam_m, float* h_adam_v,
                                 int32_t* h_step);
recon_status recon_cnn_set_state(recon_cnn* net, const float* h_params, const float* h_adam_m,
                                 const float* h_adam_v, int32_t step);

/* Writes / reads the whole network state to / from a file: 8-byte magic
 * "RCNNv001", int64 param_count, int32 step, int32 0, then params, Adam m and
 * Adam v as little-endian float32 arrays.  Synchronous. */
recon_status recon_cnn_save(recon_cnn* net, const char* path);
recon_status recon_cnn_load(recon_cnn* net, const char* path);

/* Inference: d_mu_out = mu + mu_scale * z_8 for each of `batch` n x n images d_mu
 * (d_mu_out may equal d_mu).  project = 1 additionally applies the
 * constraints of the reconstruction (zero outside the disc, max(0, .)
 * inside), so the result can start the iteration.  n <= max_n. */
recon_status recon_cnn_forward(recon_cnn* net, const float* d_mu, float* d_mu_out, int32_t batch, int32_t n,
                               int32_t project, void* stream);

/* Loss and gradient at the current parameters for a batch (batch <=
 * max_batch, n <= max_n) of inputs d_mu and targets d_target.  The gradient
 * is kept for recon_cnn_adam_step and, when d_grad is not NULL, copied to it
 * (device float32 [param_count]); d_loss: NULL or a device double. */
recon_status recon_cnn_loss_grad(recon_cnn* net, const float* d_mu, const float* d_target, int32_t batch,
                                 int32_t n, float* d_grad, double* d_loss, void* stream);

/* One Adam update with learning rate lr from the gradient of the last
 * recon_cnn_loss_grad; increments the step count. */
recon_status recon_cnn_adam_step(recon_cnn* net, float lr, void* stream);

/* recon_cnn_loss_grad followed by recon_cnn_adam_step. */
recon_status recon_cnn_train_step(recon_cnn* net, const float* d_mu, const float* d_target, int32_t batch,
                                  int32_t n, float lr, double* d_loss, void* stream);

/* Copies an internal tensor of the last forward or loss_grad call to d_dst
 * (device memory of at least `bytes` bytes; fails if smaller).
 *   kind 0: activation a_layer, layer 0..7: bfloat16 bits (uint16), layer 0
 *           [batch][n][n], layers 1..7 [batch][n][n][32] (channels last)
 *   kind 1: backward signal dL/dz_layer, layer 1..7: bfloat16 [batch][n][n][32]
 *   kind 2: network output y (normalised), float32 [batch][n][n]
 *   kind 3: dL/dz_8, float32 [batch][n][n]
 * (After a chunked forward pass the tensors hold the last chunk.) */
recon_status recon_cnn_tensor(recon_cnn* net, int32_t kind, int32_t layer, void* d_dst, int64_t bytes,
                              void* stream);

/* Measurement helper: mean duration in ms over `reps` back-to-back launches
 * (after one untimed launch) of each kernel of a training step on the current
 * workspace contents (batch, n as in the last loss_grad call): ms_out[0] a
 * 32-channel forward convolution (conv32 forward), [1] its dgrad form,
 * [2] the 32-channel weight-gradient kernel, [3] the whole forward pass,
 * [4] the whole loss_grad.  Blocks until done. */
recon_status recon_cnn_time_kernels(recon_cnn* net, const float* d_mu, const float* d_target, int32_t batch,
                                    int32_t n, int32_t reps, double* ms_out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RECON_CNN_H */
