/*
 * lbm_cnn.h -- kernels of the learned refinement-flag predictor: a small 3D
 * convolutional network over per-block averaged (rho, u) that predicts the
 * kinetic sensor's block maximum some steps ahead, so that regridding can
 * refine ahead of moving features.  The network is not part of the paper;
 * the sensor it predicts is (Sec. 3.2, block maxima of Sec. 3.4).
 *
 * Layouts and conventions:
 *   - Activations are float32, channels last: x[n][z][y][x][c], with the
 *     channel stride C4 = the channel count rounded up to a multiple of 4
 *     (padding channels hold zeros).  Grids are D x H x W voxels.
 *   - A 3x3x3 convolution with zero padding ("same" size) maps Ci to Co
 *     channels.  Float32 master weights are w[co][tap][ci], tap = (kz*3 +
 *     ky)*3 + kx; the kernels read them packed to bfloat16 as a matrix
 *     [Co16][K16] (K = 27 * Ci4, both sides padded to multiples of 16) made
 *     by lbm_cnn_pack_weights.
 *   - Products run on the matrix cores (bfloat16 inputs, float32
 *     accumulation: v_mfma_f32_16x16x16_bf16); everything else is float32.
 *   - All device pointers are caller-owned; every call is asynchronous on
 *     `stream` (hipStream_t, NULL: null stream) and returns 0 on success or
 *     a negative code (-1: bad argument, -3: HIP launch error).
 */
#ifndef LBM_CNN_H
#define LBM_CNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Number of uint16 (bfloat16) values of a packed weight matrix. */
int64_t lbm_cnn_packed_size(int32_t co, int32_t ci);

/* Packs w[co][27][ci] (float32) into bfloat16 [Co16][K16].  flip != 0 packs
 * instead the weights of the data-gradient convolution: out channel ci, in
 * channel co, tap mirrored (26 - tap), i.e. the matrix [Ci16][27 * Co4]. */
int32_t lbm_cnn_pack_weights(const float *w, int32_t co, int32_t ci, int32_t flip, uint16_t *packed,
                             void *stream);

/* y[n][v][co] = act(sum_{tap, ci} w[co][tap][ci] x[n][v + tap - 13][ci] + bias[co]),
 * act = relu if relu != 0, identity otherwise; bias may be NULL.  mask (NULL:
 * none, else laid out like y) then zeroes every output whose mask value is
 * not > 0: the data-gradient convolution followed by the ReLU backward of
 * the layer below (mask = that layer's activation), the same bits as
 * lbm_cnn_relu_backward on the unmasked output.  Writes all Co4 channels of
 * y (padding channels get 0 + bias 0).  packed comes from
 * lbm_cnn_pack_weights(co, ci). */
int32_t lbm_cnn_conv3d_forward(const float *x, int32_t n, int32_t d, int32_t h, int32_t wd, int32_t ci,
                               const uint16_t *packed, int32_t co, const float *bias, int32_t relu,
                               const float *mask, float *y, void *stream);

/* Bytes of the float32 workspace lbm_cnn_conv3d_wgrad needs (the partial
 * sums; its contents between calls do not matter).  Calls that overlap in
 * time must not share a workspace. */
int64_t lbm_cnn_wgrad_workspace(int32_t n, int32_t d, int32_t h, int32_t wd, int32_t ci, int32_t co);

/* Weight and bias gradients of the convolution:
 *   gw[co][tap][ci] = sum_{n, v} gz[n][v][co] x[n][v + tap - 13][ci],
 *   gb[co] = sum_{n, v} gz[n][v][co]  (gb may be NULL; summed in float32
 *   from the unrounded gz).
 * Deterministic: per-workgroup partial sums (chunks of 512 voxels) in
 * `work`, folded in a fixed order. */
int32_t lbm_cnn_conv3d_wgrad(const float *x, const float *gz, int32_t n, int32_t d, int32_t h, int32_t wd,
                             int32_t ci, int32_t co, float *work, float *gw, float *gb, void *stream);

/* The first half of lbm_cnn_conv3d_wgrad: only the per-chunk partial sums,
 * in `work` (lbm_cnn_wgrad_workspace bytes), for a later
 * lbm_cnn_adam_layer_fold, which folds them; the workspace must then stay
 * untouched until that call. */
int32_t lbm_cnn_conv3d_wgrad_partials(const float *x, const float *gz, int32_t n, int32_t d, int32_t h, int32_t wd,
                                      int32_t ci, int32_t co, float *work, void *stream);

/* One layer's backward pass in a single launch: the weight-gradient partial
 * sums of lbm_cnn_conv3d_wgrad_partials (input x with ci channels, output
 * gradient gz with co channels, into `work`) and the data gradient of
 * lbm_cnn_conv3d_forward(gz, ..., co, packed_flip, ci, NULL, 0, mask, gin)
 * (packed_flip from lbm_cnn_pack_weights with flip 1).  The same results as
 * those two calls, which it makes itself for shapes outside its fused forms
 * (4 or 16 padded channels each way, rows of a multiple of 4 voxels).  gz 16-
 * and packed_flip 8-byte aligned; -1 on a NULL pointer (mask may be NULL)
 * or a size < 1. */
int32_t lbm_cnn_backward_layer(const float *x, const float *gz, int32_t n, int32_t d, int32_t h, int32_t wd,
                               int32_t ci, int32_t co, float *work, const uint16_t *packed_flip, const float *mask,
                               float *gin, void *stream);

/* g[i] = (a[i] > 0) ? g[i] : 0 for i < count (ReLU backward, in place). */
int32_t lbm_cnn_relu_backward(const float *a, float *g, int64_t count, void *stream);

/* Mean squared error of channel 0 of y (channel stride ystride) against
 * target[v], v < count: loss[0] = mean (y - t)^2 (float32, written on the
 * device), g[v][0] = 2 (y - t) / count and g's other channels 0.  loss
 * must hold LBM_CNN_LOSS_FLOATS floats: loss[1..] receive per-workgroup
 * partial sums, folded in a fixed order (deterministic). */
#define LBM_CNN_LOSS_FLOATS 257
int32_t lbm_cnn_mse(const float *y, int32_t ystride, const float *target, int64_t count, float *g,
                    float *loss, void *stream);

/* One Adam update (Kingma & Ba) of count parameters at step t >= 1. */
int32_t lbm_cnn_adam(float *w, const float *g, float *m, float *v, int64_t count, float lr, float beta1,
                     float beta2, float eps, int32_t t, void *stream);

/* The same update with its hyperparameters in device memory, so that a
 * training step can be captured once into a HIP graph and replayed: hyper
 * holds LBM_CNN_HYPER_FLOATS floats, [0] lr, [1] beta1, [2] beta2, [3] eps,
 * [4] the step t (a whole number stored as a float; start from 0).
 * lbm_cnn_adam_begin opens a step: it writes lr, beta1, beta2, eps (taken
 * by value, so a captured graph replays them unchanged) and adds 1 to t, in
 * one single-thread kernel; lbm_cnn_adam_dev then updates count parameters,
 * forming the bias corrections 1 - beta^t on the device.  Both return -1 on
 * a NULL pointer or a hyperparameter out of range (lr >= 0, 0 <= beta < 1,
 * eps > 0), -3 if the launch fails; asynchronous on `stream`. */
#define LBM_CNN_HYPER_FLOATS 8
int32_t lbm_cnn_adam_begin(float *hyper, float lr, float beta1, float beta2, float eps, void *stream);
int32_t lbm_cnn_adam_dev(float *w, const float *g, float *m, float *v, int64_t count, const float *hyper,
                         void *stream);

/* lbm_cnn_adam_dev over one convolution layer in a single launch: weights
 * w [co][27][ci] with gradient gw and moments mw, vw, and bias b [co] with
 * gb, mb, vb; each updated weight is also written to packed and packed_flip
 * in the layouts lbm_cnn_pack_weights gives with flip 0 and 1 (their
 * padding entries, written by an earlier lbm_cnn_pack_weights, are left
 * alone).  Sizes as for lbm_cnn_pack_weights; -1 on a NULL pointer or
 * co, ci < 1, -3 if the launch fails. */
int32_t lbm_cnn_adam_layer(float *w, float *b, const float *gw, const float *gb, float *mw, float *vw, float *mb,
                           float *vb, int32_t co, int32_t ci, uint16_t *packed, uint16_t *packed_flip,
                           const float *hyper, void *stream);

/* lbm_cnn_adam_layer taking the gradient as the partial sums that
 * lbm_cnn_conv3d_wgrad_partials left in `work` for the batch shape
 * (n, d, h, wd): the fold of lbm_cnn_conv3d_wgrad and the update in one
 * launch, the same bits as lbm_cnn_conv3d_wgrad followed by
 * lbm_cnn_adam_layer.  gw [co][27][ci] and gb [co] receive the folded
 * gradient when not NULL.  -1 on a NULL pointer or a size < 1. */
int32_t lbm_cnn_adam_layer_fold(float *w, float *b, const float *work, int32_t n, int32_t d, int32_t h, int32_t wd,
                                float *mw, float *vw, float *mb, float *vb, int32_t co, int32_t ci, uint16_t *packed,
                                uint16_t *packed_flip, const float *hyper, float *gw, float *gb, void *stream);

/* One layer's state for lbm_cnn_adam_layers_fold: the arguments of
 * lbm_cnn_adam_layer_fold (work: that layer's partial sums from
 * lbm_cnn_conv3d_wgrad_partials or lbm_cnn_backward_layer; gw, gb may be
 * NULL). */
typedef struct lbm_cnn_layer {
    float *w, *b;
    const float *work;
    float *mw, *vw, *mb, *vb;
    uint16_t *packed, *packed_flip;
    float *gw, *gb;
    int32_t co, ci;
} lbm_cnn_layer;
#define LBM_CNN_MAX_LAYERS 8

/* lbm_cnn_adam_layer_fold for nlayers <= LBM_CNN_MAX_LAYERS layers (a host
 * array; their partials all for the batch shape (n, d, h, wd)) in a single
 * launch: the same bits as one call per layer.  -1 on a NULL pointer, a
 * size < 1 or too many layers. */
int32_t lbm_cnn_adam_layers_fold(int32_t nlayers, const lbm_cnn_layer *layers, int32_t n, int32_t d, int32_t h,
                                 int32_t wd, const float *hyper, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_CNN_H */
