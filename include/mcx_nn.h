/* mcx_nn.h -- C ABI of the fluence denoiser in libmcx (gfx950).
 *
 * The paper's method (its per-thread photon loop, Fig. 1) produces noisy
 * Monte Carlo fluence maps whose noise falls as 1/sqrt(photons).  The
 * denoiser is an addition on top of that output: a 3-D residual U-Net that
 * maps a low-photon fluence map (one gate, per launched photon, as returned
 * by mcx_fluence kind MCX_FLUENCE) to an estimate of the high-photon map,
 * trained on pairs of maps the simulator itself produces.  It works in log
 * space, u = (ln max(phi, 1e-12) - (-16)) / 4, and adds its output to u
 * (a global residual), so an untrained network (zero output layer) returns
 * its input.
 *
 * Network with channels c[0..L-1] on an nz x ny x nx grid (each side a
 * multiple of 2^(L-1)); every convolution has a bias per output channel:
 *   level 0:  relu(conv3 1 -> c0), relu(conv3 c0 -> c0)            = skip 0
 *   level l:  relu(down c[l-1] -> c[l]), relu(conv3 c[l] -> c[l])   = skip l
 *   bottom:   relu(conv3 c[L-1] -> c[L-1])
 *   up to l:  relu(up c[l+1] -> c[l] + skip l), relu(conv3 c[l] -> c[l])
 *   output:   u + conv3 c0 -> 1
 * conv3 = 3x3x3 convolution, stride 1, zero padding; down = 2x2x2
 * convolution, stride 2; up = 2x2x2 transposed convolution, stride 2.
 * Weights are BF16 on the matrix cores with FP32 accumulation; activations
 * and back-propagated activation gradients are stored as BF16; master
 * weights, weight gradients, the loss and Adam state are FP32.
 *
 * Parameters, as one FP32 array in layer order (the order above): for each
 * layer its weights w[taps][cin][cout] (taps 27 for conv3 with tap
 * t = (dz+1)*9 + (dy+1)*3 + (dx+1) reading x[z+dz][y+dy][x+dx]; taps 8 for
 * down / up with t = 4a + 2b + c for the offset (a, b, c) in {0,1}^3) and
 * then its biases b[cout].
 *
 * Loss: mean squared error between the output and the target's u over the
 * voxels whose target fluence is at least 1e-8 of the target's maximum.
 * Optimiser: Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected).
 *
 * All volume arguments are device pointers of nx*ny*nz floats, x fastest,
 * read (or written) on `hip_stream` (a hipStream_t; NULL = the null
 * stream, as for HIP calls).  Parameter and gradient copies wait for the
 * whole device.  Calls on one network must not overlap in time (they share
 * its activation buffers): keep them on one stream.  Errors as in mcx.h
 * (mcx_last_error has the message).
 */
#ifndef MCX_NN_H
#define MCX_NN_H

#include <stdint.h>

#include "mcx.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mcx_nn mcx_nn;

/* Layer kinds of the single-layer calls. */
enum { MCX_NN_CONV3 = 0, MCX_NN_DOWN = 1, MCX_NN_UP = 2 };

/* Network with nlevels (1..6) levels of channels[i] (1..1024, increasing
 * not required) for volumes of nx x ny x nz voxels (each a multiple of
 * 2^(nlevels-1)); parameters start at zero (set them with
 * mcx_nn_set_params).  Allocates all activation, gradient and optimiser
 * buffers on `device`.  MCX_EINVAL / MCX_ENODEV / MCX_ENOMEM. */
mcx_status mcx_nn_create(const int32_t *channels, int32_t nlevels, int32_t nx, int32_t ny,
                         int32_t nz, int32_t device, mcx_nn **out);
void mcx_nn_destroy(mcx_nn *nn);

/* Number of FP32 parameters (weights and biases of every layer). */
uint64_t mcx_nn_param_count(const mcx_nn *nn);

/* Copy all parameters in (host array of mcx_nn_param_count floats; also
 * clears the Adam moments and step count) or out; copy out the gradients
 * of the last mcx_nn_loss_grad / mcx_nn_train_step.  MCX_ERANGE when n
 * differs from mcx_nn_param_count.  Blocking (waits for the device). */
mcx_status mcx_nn_set_params(mcx_nn *nn, const float *host, uint64_t n);
mcx_status mcx_nn_get_params(mcx_nn *nn, float *host, uint64_t n);
mcx_status mcx_nn_get_grads(mcx_nn *nn, float *host, uint64_t n);

/* Adam's state, for checkpoints: first and second moments (host arrays of
 * mcx_nn_param_count floats each, in parameter order) and the step count
 * (the next step uses step + 1 in its bias corrections).  Set it after
 * mcx_nn_set_params, which clears it.  MCX_ERANGE when n differs from
 * mcx_nn_param_count, MCX_EINVAL for a NULL array or a negative step.
 * Blocking. */
mcx_status mcx_nn_get_adam(mcx_nn *nn, float *m, float *v, uint64_t n, int32_t *step);
mcx_status mcx_nn_set_adam(mcx_nn *nn, const float *m, const float *v, uint64_t n, int32_t step);

/* Denoise phi_in into phi_out (fluence, may be NULL) and/or u_out (the
 * network output in u space, may be NULL).  Async. */
mcx_status mcx_nn_forward(mcx_nn *nn, const float *phi_in, float *phi_out, float *u_out,
                          void *hip_stream);

/* Denoise phi_in averaged over symmetries of the square x-y cross-section
 * (those of mcx_nn_mirror_xy, ops 0 .. nsym-1): for each op the input is
 * transformed, denoised, and the output in u space transformed back; the
 * outputs are averaged in u space (u_out) and turned into fluence
 * (phi_out).  For a source on the cross-section's centre line each
 * transformed input is the map of the mirrored volume, so every pass
 * estimates the same map (the training pairs are augmented with the same
 * symmetries).  nsym = 1 is mcx_nn_forward.  Costs nsym forward passes;
 * uses the network's loss buffers as scratch (do not overlap with
 * mcx_nn_loss_grad / mcx_nn_train_step on the same network).  MCX_EINVAL
 * for nsym not in {1, 2, 4, 8}, or 8 with nx != ny.  Async. */
mcx_status mcx_nn_forward_sym(mcx_nn *nn, const float *phi_in, float *phi_out, float *u_out,
                              int32_t nsym, void *hip_stream);

/* Forward pass on phi_in, loss against phi_target and backward pass: the
 * gradients of every parameter (mcx_nn_get_grads), replacing the current
 * gradients, or added to them when accumulate != 0 (for steps over several
 * volumes).  *loss (may be NULL) receives this volume's loss, which makes
 * the call wait for the stream; with loss == NULL it is async. */
mcx_status mcx_nn_loss_grad(mcx_nn *nn, const float *phi_in, const float *phi_target,
                            int32_t accumulate, double *loss, void *hip_stream);

/* Fused backward pass (on by default): where a 3x3x3 layer on a grid of
 * at least 1024 4x4x8 tiles maps 32 channels to 32 (the full-resolution
 * layers) and the layer below takes no skip gradient, the layer's
 * input-gradient product also applies the ReLU mask of the layer below,
 * rounds to BF16 and sums that layer's bias gradient per workgroup, so
 * that the layer below's gradient is not written as FP32 and read again
 * (the chain rule through a ReLU; the denoiser is an addition to the
 * paper's method).  Gradients equal those of the unfused pass except for
 * the bias gradients of the folded layers, whose FP32 sums are added in
 * another order.  on != 0 enables it; *nfolded (may be NULL) receives the
 * number of layers whose gradient the fold produces (0 when off).
 * MCX_EINVAL for NULL nn.  Takes effect at the next mcx_nn_loss_grad; do
 * not call while one runs. */
mcx_status mcx_nn_set_fused_backward(mcx_nn *nn, int32_t on, int32_t *nfolded);

/* One Adam step with learning rate lr on g = grad_scale * (current
 * gradients), with g scaled down to global L2 norm max_norm when its norm
 * is larger (max_norm <= 0: no clipping).  Async. */
mcx_status mcx_nn_adam(mcx_nn *nn, float lr, float grad_scale, float max_norm, void *hip_stream);

/* mcx_nn_loss_grad (replacing the gradients) followed by mcx_nn_adam with
 * grad_scale 1 and no clipping. */
mcx_status mcx_nn_train_step(mcx_nn *nn, const float *phi_in, const float *phi_target, float lr,
                             double *loss, void *hip_stream);

/* Training-data augmentation: out[z][y][x] = in[z][y'][x'] for one of the
 * eight symmetries of the square x-y cross-section, op in 0..7:
 * (x', y') = (y, x) when op & 4, else (x, y); then x' -> nx-1-x' when op & 1
 * and y' -> ny-1-y' when op & 2.  For a problem whose source sits on the
 * cross-section's centre line and points along z, a symmetry maps an
 * (input, target) pair of fluence maps to the pair of the mirrored volume
 * (with the source moved to the mirrored voxel).  in, out: FP32 device
 * buffers [nz][ny][nx], distinct.  MCX_EINVAL for NULL or equal buffers,
 * non-positive sizes, op outside 0..7, or a swap with nx != ny (checked
 * before any HIP call).  Async on hip_stream (NULL = the null stream). */
mcx_status mcx_nn_mirror_xy(const float *in, float *out, int32_t nx, int32_t ny, int32_t nz,
                            int32_t op, void *hip_stream);

/* Single layers on device buffers (the network's kernels, for tests and
 * for callers building other graphs).  (nx, ny, nz) is the layer's input
 * grid; the output grid is the same (conv3), half (down) or twice (up) per
 * axis.  x: BF16 bits [input voxel][cin]; w: FP32 [taps][cin][cout];
 * b: FP32 [cout] (may be NULL in forward); skip: BF16 bits [output
 * voxel][cout] added before the ReLU (may be NULL); y: [output
 * voxel][cout], FP32 when y_f32 else BF16 bits.  Backward takes the BF16
 * gradient gy of the layer output (after any ReLU mask) and overwrites gx
 * (FP32 [input voxel][cin], may be NULL), gw and gb (may be NULL).
 * Temporary weight packs (and, for 3x3x3 layers whose reductions are
 * split over workgroups, FP32 workspaces of partial sums) are allocated
 * per call; both wait for the stream before returning. */
mcx_status mcx_nn_layer_forward(int32_t kind, int32_t nx, int32_t ny, int32_t nz, int32_t cin,
                                int32_t cout, const uint16_t *x, const float *w, const float *b,
                                const uint16_t *skip, int32_t relu, int32_t y_f32, void *y,
                                void *hip_stream);
mcx_status mcx_nn_layer_backward(int32_t kind, int32_t nx, int32_t ny, int32_t nz, int32_t cin,
                                 int32_t cout, const uint16_t *x, const float *w,
                                 const uint16_t *gy, float *gx, float *gw, float *gb,
                                 void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* MCX_NN_H */
