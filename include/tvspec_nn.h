/*
 * tvspec_nn -- the learned surrogate of the spectral TV decomposition on one
 * AMD MI355X (gfx950): a convolutional network that maps an image directly
 * to its spectral bands and residual, trained on decompositions computed by
 * the model-driven path of tvspec.h.
 *
 * The paper (Grossmann, Korolev, Gilboa, Schoenlieb, arXiv 2006.10004)
 * replaces the decomposition pipeline by a network Psi(f) ~ (b^1..b^K)
 * (Sec. 3) built from 3x3 convolutions with biases and ReLU activations,
 * trained with the normalised mean squared error of Sec. 3 and Adam
 * (Sec. 4.1).  This library builds its encoder-decoder variant (Sec. 4.5:
 * max-pooling down, upsampling and skip connections up):
 *
 *   level widths w0..w3 = 48, 96, 192, 384 at 1, 1/2, 1/4, 1/8 resolution;
 *   per level two 3x3 conv + ReLU; 2x2 max-pooling between encoder levels;
 *   decoder: nearest 2x upsampling, concatenation [upsampled, skip] along
 *   channels, two 3x3 conv + ReLU; a final 3x3 conv (no activation) to
 *   out_channels = 4 bands x 3 colour channels + 3 residual channels = 15.
 *   The first layer sees the image as 2 f - 1 (centred; images lie in
 *   [0, 1]); this fixed map is part of the network.  The residual outputs
 *   are f plus the last layer's residual channels (a skip from the input, as
 *   in the residual learning of DnCNN, the network the paper builds on): the
 *   residual is most of the image and the layer only learns its difference
 *   from f, which is minus the sum of the bands.
 *
 * Arithmetic: bfloat16 weights and activations, float32 accumulation in
 * the matrix cores (v_mfma_f32_16x16x32_bf16), float32 biases, outputs,
 * loss, gradients of the parameters and Adam state (float32 master
 * weights).  Activation gradients are stored in bfloat16.
 *
 * Layouts: images are channels-last inside the library; the entry points
 * take the decomposition's own layouts (noted per call).  Every device
 * pointer is the caller's unless stated; calls are ordered on `stream`.
 * Return codes are those of tvspec.h; tvspec_last_error() has the text.
 */
#ifndef TVSPEC_NN_H
#define TVSPEC_NN_H

#include <stddef.h>

#include "tvspec.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * 3x3 "same" convolution, channels last, as the network uses it:
 *   y[p][o] = act(bias[o] + sum_{dy,dx,c} x[p + (dy-1, dx-1)][c] w[o][dy][dx][c])
 * with zero padding, p = (b, i, j) over B x H x W pixels.
 *   x     device bfloat16 [B][H][W][Cin], Cin a multiple of 8
 *   w     device bfloat16 [Cout][3][3][Cin], Cout a multiple of 16
 *   bias  device float32 [Cout] or NULL
 *   relu  0 or 1 (max(., 0) after the bias)
 *   y     device [B][H][W][Cout], bfloat16 (y_f32 = 0) or float32 (y_f32 = 1)
 * Errors: TVSPEC_EINVAL for sizes or null pointers.
 */
TVSPEC_API int tvspec_nn_conv3x3(const void *x, int B, int H, int W, int Cin, const void *w,
                                 const float *bias, int Cout, int relu, void *y, int y_f32,
                                 void *stream);

/*
 * Gradient of the convolution in its input: dx = conv3x3^T(dy) with the
 * same weights (no bias); an optional mask (bfloat16 [B][H][W][Cin]) zeroes
 * dx wherever mask <= 0 (the ReLU of the producing layer).  dy bfloat16
 * [B][H][W][Cout] (Cout a multiple of 8), w as tvspec_nn_conv3x3 (Cin a
 * multiple of 16), dx bfloat16 [B][H][W][Cin].  The weights are transposed
 * and flipped into workspace the library owns.
 */
TVSPEC_API int tvspec_nn_conv3x3_dgrad(const void *dy, int B, int H, int W, int Cout, const void *w,
                                       int Cin, const void *mask, void *dx, void *stream);

/*
 * Gradient of the convolution in its weights and bias:
 *   dw[o][dy][dx][c] = sum_p dy[p][o] x[p + (dy-1, dx-1)][c],  db[o] = sum_p dy[p][o]
 * x bfloat16 [B][H][W][Cin] (Cin a multiple of 8), dy bfloat16
 * [B][H][W][Cout] (Cout a multiple of 8), dw float32 [Cout][3][3][Cin],
 * db float32 [Cout] or NULL.  Deterministic (fixed-order reductions).
 */
TVSPEC_API int tvspec_nn_conv3x3_wgrad(const void *x, const void *dy, int B, int H, int W, int Cin,
                                       int Cout, float *dw, float *db, void *stream);

/* The network. */
typedef struct tvspec_net tvspec_net;

/* Number of output channels: 4 bands x 3 channels + 3 residual channels. */
#define TVSPEC_NET_IN_CHANNELS 3
#define TVSPEC_NET_BANDS 4
#define TVSPEC_NET_OUT_CHANNELS 15

/*
 * Create the network for images of H x W (multiples of 8) and batches of up
 * to max_batch, on the current device, with He-normal weights drawn from a
 * counter-based generator seeded by `seed`, zero biases and a zero output
 * layer (so training starts from zero bands and residual f, loss 1 per
 * group), and output
 * scales of 1.  Activations, gradients and Adam state for max_batch are
 * allocated here.
 */
TVSPEC_API int tvspec_net_create(int H, int W, int max_batch, unsigned long long seed, tvspec_net **out);

/*
 * Parameters as one float32 vector: for each layer in the order e1a, e1b,
 * e2a, e2b, e3a, e3b, e4a, e4b, d3a, d3b, d2a, d2b, d1a, d1b, out, the
 * weights [Cout][3][3][Cin] followed by the bias [Cout] (Cin of e1a is 3,
 * Cout of out is 15).  get/set copy through host memory.
 */
TVSPEC_API int tvspec_net_num_params(tvspec_net *net, long long *n);
TVSPEC_API int tvspec_net_get_params(tvspec_net *net, float *host, long long n);
TVSPEC_API int tvspec_net_set_params(tvspec_net *net, const float *host, long long n);

/*
 * Fixed (not trained) scale of each output channel: output c =
 * scale[c] * (the last convolution's channel c).  The bands of a
 * decomposition are small next to the image (their RMS can be 1e-3 of it);
 * scaling each output by its band's typical size lets the last layer work
 * in units of order 1.  scale: host float32 [15], each > 0.
 */
TVSPEC_API int tvspec_net_set_output_scale(tvspec_net *net, const float *scale);

/*
 * Floor of the loss's denominators: each group's ||t_bj||^2 is raised by
 * kappa 3 H W scale_j^2, kappa times the energy of a group whose RMS equals
 * its output scale (the dataset's typical band size when the scales are set
 * that way).  An image with a nearly empty band (a crop inside a large flat
 * shape has almost no coarse-scale content) then cannot dominate a batch's
 * gradient.  kappa = 0 (the default) is the paper's loss; kappa finite, >= 0.
 */
TVSPEC_API int tvspec_net_set_loss_floor(tvspec_net *net, float kappa);

/*
 * Gradient-norm clipping for tvspec_net_train_step.  Each step computes the
 * L2 norm of the whole parameter gradient (fixed-order sum, deterministic)
 * and compares it with a running average of past norms (seeded by the first
 * step, then avg <- 0.99 avg + 0.01 min(norm, clip avg)).  If it exceeds
 * clip x avg, the gradient is scaled down to clip x avg before the Adam
 * update, so a single outlier batch cannot throw the moments off.  clip = 0
 * (the default) turns clipping off; otherwise clip must be >= 1.
 * tvspec_net_set_params resets the running average.
 */
TVSPEC_API int tvspec_net_set_grad_clip(tvspec_net *net, float clip);

/*
 * The last training step's gradient norm, the running average after it and
 * the factor the gradient was scaled by (host floats; waits for the device).
 */
TVSPEC_API int tvspec_net_grad_stats(tvspec_net *net, float *norm, float *avg, float *scale);

/*
 * Forward pass.  f device float32 [B][3][H][W]; out device float32
 * [B][15][H][W] (channel 3j + c = band j of colour c for j < 4, 12 + c =
 * residual of colour c, which is f + scale * the last layer's channel).
 * B <= max_batch.
 */
TVSPEC_API int tvspec_net_forward(tvspec_net *net, const float *f, int B, float *out, void *stream);

/*
 * Forward pass that also checks its result: as tvspec_net_forward, and
 * err (device float32 [B], or NULL) receives each image's
 * reconstruction-identity error as tvspec_net_identity_error defines it,
 * computed on the stored outputs while they are written (no second pass
 * over out; the sum runs in a fixed order, so the value is deterministic,
 * and equals tvspec_net_identity_error's up to the order of summation).
 */
TVSPEC_API int tvspec_net_forward_checked(tvspec_net *net, const float *f, int B, float *out, float *err,
                                          void *stream);

/*
 * One training step on a batch: forward, normalised MSE loss against the
 * decomposition (bands device float64 [B][4][3][H][W], residual device
 * float64 [B][3][H][W], the layouts of tvspec_decompose_batch_dev with four
 * bands), backward, gradient-norm clipping if set (tvspec_net_set_grad_clip),
 * one Adam step (lr, beta1 0.9, beta2 0.999, eps 1e-8).
 * The loss groups the output into 5 bands of 3 channels (the 4 bands and
 * the residual):  (1/(5B)) sum_b sum_j ||o_bj - t_bj||^2 / (||t_bj||^2 + floor_j) with
 * t_bj the band for j < 4; for the residual group the numerator is
 * ||o - residual||^2 and the denominator ||residual - f||^2, the size of what
 * the residual's learned part has to carry; floor_j is set by
 * tvspec_net_set_loss_floor (0 by default).  A group with a zero
 * denominator contributes 0.
 * *loss (host) receives the batch loss; the call then waits for the
 * stream.  With loss = NULL the step is only enqueued on the stream (the
 * caller may prepare the next batch meanwhile); tvspec_net_last_loss reads
 * the latest step's loss later.
 */
TVSPEC_API int tvspec_net_train_step(tvspec_net *net, const float *f, const double *bands,
                                     const double *residual, int B, float lr, float *loss, void *stream);

/*
 * The loss of the latest training step or loss evaluation on this network:
 * waits for `stream` (where that step was enqueued), then copies it to
 * *loss (host).
 */
TVSPEC_API int tvspec_net_last_loss(tvspec_net *net, float *loss, void *stream);

/*
 * The loss and the parameter gradients of a batch without an update
 * (grads: host float32 in the layout of tvspec_net_get_params, or NULL).
 */
TVSPEC_API int tvspec_net_loss_grad(tvspec_net *net, const float *f, const double *bands,
                                    const double *residual, int B, float *loss, float *grads,
                                    void *stream);

/*
 * Reconstruction-identity error of decompositions in the network's output
 * layout (Eq. (7): f = sum of bands + residual):
 *   err[b] = mean over the 3 channels and H x W pixels of
 *            |f - sum_j band_j - residual|
 * f device float32 [B][3][H][W], out device float32 [B][15][H][W], err
 * device float32 [B].  Serving uses it to decide when a surrogate result
 * falls back to the model-driven path.
 */
TVSPEC_API int tvspec_net_identity_error(const float *f, const float *out, int B, int H, int W, float *err,
                                         void *stream);

TVSPEC_API int tvspec_net_destroy(tvspec_net *net);

#ifdef __cplusplus
}
#endif

#endif /* TVSPEC_NN_H */
