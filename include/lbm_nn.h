/*
 * lbm_nn.h - C ABI of the kernels of the warm-start network (liblbm.so).
 *
 * The network maps a solid mask to an initial velocity field that starts the
 * lattice Boltzmann iteration closer to its steady state; the plain iteration
 * run to the residual tolerance still decides the result.  These entry
 * points are its layers, each a HIP kernel on gfx950: 3x3x3 convolutions as
 * implicit GEMMs on BF16 matrix cores (v_mfma_f32_16x16x32_bf16) with FP32
 * accumulation, and the pooling, upsampling, activation, loss and optimiser
 * steps around them.
 *
 * Conventions.  All tensor pointers are device pointers owned by the caller;
 * nothing is allocated.  Tensors are channels-last, t[((n*D + z)*H + y)*W + x]
 * [c]; shapes (n, d, h, w, c).  Convolutions wrap periodically in z, y and x
 * (the simulated cells are periodic).  Weights are w[co][tap][ci] with
 * tap = (dz+1)*9 + (dy+1)*3 + (dx+1).  "bf16" tensors hold raw BF16 values
 * (16 bits each, 16-byte aligned); "float" tensors FP32.  Work is enqueued on
 * the given hipStream_t (NULL: null stream).  Errors: LBM_ERR_INVALID_ARG for
 * bad shapes or pointers, LBM_ERR_WORKSPACE for a short workspace,
 * LBM_ERR_DEVICE if the launch failed.
 */
#ifndef LBM_NN_H
#define LBM_NN_H

#include <stddef.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* y[m][co] = bias[co] + sum_{tap,ci} x[m + off(tap)][ci] w[co][tap][ci].
 * x bf16 (n,d,h,w,ci), ci a multiple of 8; w bf16 [co][27][ci]; bias float[co]
 * or NULL; y float (n,d,h,w,co). */
lbm_status nn_conv3d_forward(const void* x, const void* w, const float* bias, float* y, int n,
                             int d, int h, int w_, int ci, int co, void* stream);

/* The forward convolution followed by nn_activation_forward, in one kernel:
 * a = bf16(relu ? max(y, 0) : y) (bf16, n,d,h,w,co; relu 0 or 1) with y as
 * above, never stored in FP32.  Bit-identical to the two calls. */
lbm_status nn_conv3d_forward_act(const void* x, const void* w, const float* bias, void* a, int n,
                                 int d, int h, int w_, int ci, int co, int relu, void* stream);

/* wt[ci][tap][co] = w[co][26 - tap][ci] (bf16), the weights of the
 * backward-data convolution. */
lbm_status nn_conv3d_flip_weights(const void* w, void* wt, int ci, int co, void* stream);

/* dx = gradient of the forward convolution with respect to x, given dy (bf16,
 * co channels, co a multiple of 8) and the flipped weights wt; dx float with
 * ci channels. */
lbm_status nn_conv3d_backward_data(const void* dy, const void* wt, float* dx, int n, int d, int h,
                                   int w_, int ci, int co, void* stream);

/* Workspace bytes (and voxel splits) nn_conv3d_backward_weight needs; ci and
 * co multiples of 8. */
lbm_status nn_conv3d_backward_weight_workspace(int n, int d, int h, int w_, int ci, int co,
                                               size_t* bytes, int* splits);

/* dw[co][tap][ci] = sum_m dy[m][co] x[m + off(tap)][ci] (float), from x and
 * dy in bf16; the voxel sum is split over workgroups and folded in a fixed
 * order (deterministic). */
lbm_status nn_conv3d_backward_weight(const void* x, const void* dy, float* dw, void* workspace,
                                     size_t workspace_bytes, int n, int d, int h, int w_, int ci,
                                     int co, void* stream);

/* Workspace bytes of nn_bias_grad for m voxels of c channels. */
lbm_status nn_bias_grad_workspace(long long m, int c, size_t* bytes);

/* db[c] = sum over m voxels of dy[m][c] (float), summed per voxel range into
 * the workspace and folded in a fixed order (deterministic). */
lbm_status nn_bias_grad(const float* dy, float* db, void* workspace, size_t workspace_bytes,
                        long long m, int c, void* stream);

/* The backward of an activation fused with what the convolution's backward
 * needs: dz = relu ? (a > 0 ? da : 0) : da for m voxels of c channels, stored
 * as bf16 (dz), and db[ch] = sum over voxels of the FP32 dz (float[c]), with
 * the workspace of nn_bias_grad_workspace(m, c).  Bit-identical to
 * nn_relu_backward, nn_cast_bf16 and nn_bias_grad.  a (bf16) may be NULL
 * when relu is 0. */
lbm_status nn_relu_backward_bias(const float* da, const void* a, void* dz, float* db, void* ws,
                                 size_t ws_bytes, long long m, int c, int relu, void* stream);

/* a = bf16(relu ? max(z, 0) : z) for n values. */
lbm_status nn_activation_forward(const float* z, void* a, long long n, int relu, void* stream);

/* dz = da where the stored activation a (bf16) is positive, else 0. */
lbm_status nn_relu_backward(const float* da, const void* a, float* dz, long long n, void* stream);

/* y = bf16(x) for n values (round to nearest even). */
lbm_status nn_cast_bf16(const float* x, void* y, long long n, void* stream);

/* 2x2x2 average pooling of x (bf16, n,d,h,w,c; even d, h, w) into y (bf16,
 * halved), and its gradient (float dy coarse -> float dx fine). */
lbm_status nn_pool2_forward(const void* x, void* y, int n, int d, int h, int w_, int c,
                            void* stream);
lbm_status nn_pool2_backward(const float* dy, float* dx, int n, int d, int h, int w_, int c,
                             void* stream);

/* Periodic trilinear prolongation by 2 (the two-grid warm start): y (float,
 * n,2d,2h,2w,c) from the first c of the cx channels of x (float, coarse
 * n,d,h,w,cx; c <= cx).  Fine node i of an axis lies between coarse nodes,
 * 3/4 from the nearer m = i/2 and 1/4 from the farther (m-1 for even i, m+1
 * for odd i) and takes 0.75 x[m] + 0.25 x[far], axes z, y, x in turn; then
 * y *= scale[ch] (device float[c], or NULL for 1). */
lbm_status nn_prolongate2(const float* x, float* y, int n, int d, int h, int w_, int cx, int c,
                          const float* scale, void* stream);

/* Start fields of a warm start for lbm_init_equilibrium_device, from the
 * predicted targets t (float, n,d,h,w,cx; velocity targets in channels 0-2,
 * cx >= 3) and the fluid mask (uint8, n,d,h,w; nonzero = fluid).  fields
 * (device double[4*n*d*h*w], [drho | u_x | u_y | u_z] in cell order, the
 * boxes stacked along z as in a batch): drho = -(delta_rho/w)(x - (w-1)/2)
 * on fluid cells (the linear profile of the pressure drop across x); u =
 * factor * t on fluid cells none of whose 18 lattice neighbours (periodic
 * within the box) is solid, else 0 (a velocity imposed on the wall layer
 * excites slowly decaying oscillations of the bounce-back links). */
lbm_status nn_warm_start_fields(const float* t, int cx, const void* fluid, double* fields, int n,
                                int d, int h, int w_, double factor, double delta_rho,
                                void* stream);

/* Nearest-neighbour upsampling by 2 of x (bf16, coarse n,d,h,w,c) into y, and
 * its gradient (sum over the 8 children; dims are the coarse ones). */
lbm_status nn_upsample2_forward(const void* x, void* y, int n, int d, int h, int w_, int c,
                                void* stream);
lbm_status nn_upsample2_backward(const float* dy, float* dx, int n, int d, int h, int w_, int c,
                                 void* stream);

/* y = [a | b] along channels (bf16, m voxels); split of a float gradient
 * (either output may be NULL). */
lbm_status nn_concat_channels(const void* a, const void* b, void* y, long long m, int ca, int cb,
                              void* stream);
lbm_status nn_split_channels(const float* dy, float* da, float* db, long long m, int ca, int cb,
                             void* stream);

/* y += x (float, n values). */
lbm_status nn_add(float* y, const float* x, long long n, void* stream);

/* Weighted mean-squared error over the first `used` of c channels:
 * loss = sum_m weight[m] sum_{ch<used} (pred - target)^2 / norm, written as
 * n_partial per-block partial sums (double) whose sum is the loss; grad
 * (float, m x c) = d loss / d pred.  target is m x used, weight m values. */
lbm_status nn_masked_mse(const float* pred, const float* target, const float* weight, float* grad,
                         double* partial, int n_partial, long long m, int c, int used,
                         double norm, void* stream);

/* Adam step on FP32 master weights w (n values) with gradient g and moments
 * m1, m2 (step >= 1 counts updates); w_bf16 (or NULL) receives bf16(w). */
lbm_status nn_adam(float* w, const float* g, float* m1, float* m2, void* w_bf16, long long n,
                   float lr, float beta1, float beta2, float eps, int step, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* LBM_NN_H */
