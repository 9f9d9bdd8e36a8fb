/*
 * vlbm_nn.h -- C ABI of the learned coarse-grid correction of the VLBM MHD library.
 *
 * This part is an extension of the paper's method (not described there): the
 * method's own runs on a fine 2D lattice, restricted to a coarser one, train a small
 * network that predicts, from the coarse moments at one step, the correction that
 * takes the plain coarse VLBM step to the restricted fine solution.  The coarse run
 * then injects that correction into the populations (f_{k,i} += w_i dQ_k, which
 * shifts the zeroth moments by dQ_k) after each plain coarse step, unless a gate
 * falls back to the plain VLBM.  The training pairs come from a teacher-forced coarse
 * run that takes exactly these steps with the true corrections, so the network is
 * trained against the operator it is applied to.
 * The VLBM pieces it drives are those of include/vlbm.h (Sec. 2.2-2.3 of the paper:
 * moments, equilibrium, BGK update with direct source injection).
 *
 * Network: `layers` convolutions with periodic padding -- 3x3 on nx x ny lattices
 * (dim = 2) or 3x3x3 on nx x ny x nz lattices (dim = 3) -- channels cin -> width ->
 * ... -> width -> cin, exact GELU between layers; operands in bfloat16, accumulation
 * in FP32 on the matrix cores; FP32 master weights, Adam.  Supported shapes: cin = 8
 * (the ideal-MHD moments), width = 32, nx and ny multiples of 16, any nz >= 1.
 *
 * Weight vector layout (FP32, host): for each layer l in order, W_l[o][c][ky][kx]
 * (dim 2) or W_l[o][c][kz][ky][kx] (dim 3) (o output channel, c input channel,
 * kz, ky, kx in 0..2 for offsets -1..1), then b_l[o].  The convolution is
 * z[o,y,x] = b[o] + sum_{c,ky,kx} W[o,c,ky,kx] a[c, y+ky-1, x+kx-1], in 3D
 * z[o,z,y,x] = b[o] + sum_{c,kz,ky,kx} W[o,c,kz,ky,kx] a[c, z+kz-1, y+ky-1, x+kx-1],
 * with periodic indices.
 *
 * Normalisation: inputs are standardised per channel, x = (X - in_mean)/in_std;
 * the network output y is a standardised correction, dQ = out_mean + out_std * y.
 *
 * All device arrays are FP32, channel-major [channel][batch][nz][ny][nx] (x fastest,
 * nz = 1 in 2D) -- the layout of the moments of a context (include/vlbm.h: a batched
 * 2D context, D2Q5 with its nz = batch, or a 3D context, batch 1), which the network
 * reads directly.  Every call is
 * stream-ordered on the network's stream; calls that return host values
 * synchronise it.  Errors as in vlbm.h; vlbm_nn_last_error() gives the message.
 */
#ifndef VLBM_NN_H
#define VLBM_NN_H

#include <stddef.h>
#include <stdint.h>

#include "vlbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vlbm_nn vlbm_nn;

/* Create a network (weights zero, normalisation identity, Adam state zero).
 * dim: 2 (3x3 kernels) or 3 (3x3x3 kernels).  stream: hipStream_t or NULL.
 * *out is NULL on error. */
vlbm_status vlbm_nn_create(int32_t dim, int32_t cin, int32_t width, int32_t layers, void* stream,
                           vlbm_nn** out);
void vlbm_nn_destroy(vlbm_nn* nn);                           /* NULL-safe */
const char* vlbm_nn_last_error(const vlbm_nn* nn);            /* NULL: last create error */

/* Number of FP32 parameters (weights and biases of all layers). */
vlbm_status vlbm_nn_num_params(const vlbm_nn* nn, size_t* n);
/* Host FP32 weight vector in the layout above; n must equal vlbm_nn_num_params.
 * set_weights also resets the Adam state and step count. */
vlbm_status vlbm_nn_set_weights(vlbm_nn* nn, const float* w, size_t n);
vlbm_status vlbm_nn_get_weights(const vlbm_nn* nn, float* w, size_t n);
/* Per-channel normalisation (host arrays of cin doubles; std > 0). */
vlbm_status vlbm_nn_set_norm(vlbm_nn* nn, const double* in_mean, const double* in_std,
                             const double* out_mean, const double* out_std);

/* Inference: X (device, raw moments) -> dQ (device, raw correction, 16-byte aligned).  batch lattices
 * of nz x ny x nx cells; nz must be 1 for a dim-2 network; batch * nz <= 65535 and
 * batch * nz * ny * nx <= 2^28. */
vlbm_status vlbm_nn_forward(vlbm_nn* nn, const float* X, float* dQ, int32_t batch, int32_t nx,
                            int32_t ny, int32_t nz);

/* Mean-squared error between the standardised output and the standardised target
 * (T, device, raw correction) and its gradient.  loss (host) may be NULL; grad
 * (host, vlbm_nn_num_params floats) may be NULL.  The gradient is kept on the
 * device for vlbm_nn_adam_step.  Synchronises when loss or grad is requested. */
vlbm_status vlbm_nn_loss_grad(vlbm_nn* nn, const float* X, const float* T, int32_t batch,
                              int32_t nx, int32_t ny, int32_t nz, double* loss, float* grad);

/* One Adam update of the FP32 master weights with the last gradient
 * (beta1 0.9, beta2 0.999, eps 1e-8 unless changed by vlbm_nn_adam_config). */
vlbm_status vlbm_nn_adam_step(vlbm_nn* nn, float lr);
vlbm_status vlbm_nn_adam_config(vlbm_nn* nn, float beta1, float beta2, float eps);

/* loss_grad followed by adam_step (one training iteration, all on the device). */
vlbm_status vlbm_nn_train_step(vlbm_nn* nn, const float* X, const float* T, int32_t batch,
                               int32_t nx, int32_t ny, int32_t nz, float lr, double* loss);

/* Block mean of a moment field: Qf (device FP32 [K][nz][ny][nx]) -> Qc (device FP32
 * [K][nz/rz][ny/r][nx/r]); rz = r restricts a 3D field, rz = 1 a batch of 2D fields.
 * If minus (device, the shape of Qc) is not NULL it is subtracted (the target of a
 * training pair: restricted fine state minus the plain coarse step).  Accumulated in
 * FP64.  Every extent must be divisible by its factor.  stream: hipStream_t or NULL. */
vlbm_status vlbm_restrict(const float* Qf, int32_t K, int32_t nx, int32_t ny, int32_t nz,
                          int32_t r, int32_t rz, const float* minus, float* Qc, void* stream);

/* f_{k,i} += w_i dQ_k at the context's current step (shifts the zeroth moments by
 * dQ): the teacher-forced coarse run of the training pairs takes each target this
 * way.  dQ: device FP32 [8][N] in the context's moment layout.  Ideal-MHD context with
 * the direct source (2D or 3D, periodic or with static faces, no body or the
 * homogenized one; not the bounce-back body, whose solid cells hold no fluid), any
 * storage form (FP16/BF16 deviations are decoded, incremented in FP32 and encoded
 * again).  Stream-ordered, no synchronisation. */
vlbm_status vlbm_inject(vlbm_ctx* c, const float* dQ);

/* n coarse steps with the learned correction.  Per step: the moments X of the
 * current populations (including the pending correction), dQ = network(X) -- if
 * project_totals is nonzero, minus its mean over each lattice of the batch, channel by
 * channel (the fine run, its restriction and the coarse VLBM all keep the lattice
 * totals of rho, rho u, E and B up to the Powell source, so the true correction has a
 * zero total, and a bias of the network cannot accumulate in the totals) -- the gate
 * (FP64 over the whole lattice or batch: every ||dQ_k||_2 <= bound_corr[k]; the
 * central-difference div B drift ||div(B + dB)||_2 <= (1 + bound_divb_rel) ||div B||_2
 * + bound_divb_abs ||B||_2 with B the in-plane field of X in 2D, all three components
 * in 3D; all finite; without the projection also X + dQ physical in every cell,
 * rho > 0 and p >= 0 -- otherwise
 * dQ := 0, i.e. the plain coarse VLBM step, and the fallback counter is incremented),
 * then the sweep, with the previous step's accepted dQ added as w_i dQ_k to the
 * populations before the collision.  After the last step the pending dQ is added to
 * the populations, so vlbm_moments sees the corrected state.  The context must be an
 * ideal-MHD BGK context (K = cin = 8, any storage form) whose extent the network
 * supports: periodic without a body, 2D (nz = batch of independent lattices, gated
 * together and projected one by one) with a dim-2 network or 3D (one lattice) with a
 * dim-3 network; or 3D with static faces and/or the homogenized body (Sec. 2.4) with a
 * dim-3 network and project_totals = 0 (faces and the body change the totals): there
 * each step evaluates the network on X, runs the plain step (faces, sweep, body), takes
 * the moments X' of its result and gates X' + dQ -- the state the correction would make
 * -- instead of X + dQ; an accepted dQ is added to the populations at once and X' + dQ
 * is the next step's X (eager: the body's box is recomputed on the host each step); the
 * gate's central differences wrap around the lattice as on a periodic one.  bound_corr: host, K doubles.  *n_fallback (host, may be NULL)
 * receives the number of fallbacks in this call.  Synchronises.  The handle keeps the
 * step's buffers (about 128 N + N / 4 bytes for N cells, grown for a larger context), a stream,
 * an event and the graph of a pair of steps from call to call, until vlbm_nn_destroy;
 * the graph is captured again after the context is initialised or restored, for the
 * other starting parity, the other projection setting or another context.  Calls on one
 * network handle must not overlap. */
vlbm_status vlbm_step_corrected(vlbm_ctx* c, vlbm_nn* nn, int32_t n, const double* bound_corr,
                                double bound_divb_rel, double bound_divb_abs, int32_t project_totals,
                                int64_t* n_fallback);

#ifdef __cplusplus
}
#endif
#endif /* VLBM_NN_H */
