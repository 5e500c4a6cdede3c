/*
 * lalm_unet.h -- C ABI of the learned warm start (gfx950, BF16 MFMA).
 *
 * Not part of the paper's method: a small 2D U-Net maps an image after a
 * few OS-LALM iterations to an estimate of the image after many iterations;
 * plain OS-LALM remains the fallback and the arbiter (its cost value decides
 * whether the estimate is kept, and the RMS difference to x* is the figure
 * of merit).  Architecture (3 levels, 3x3 convolutions + ReLU, 2x2 max
 * pooling, 2x2 stride-2 transposed convolutions, skip concatenations, 1x1
 * head, residual output):
 *   e1a 1->32, e1b 32->32 | pool | e2a 32->64, e2b 64->64 | pool |
 *   e3a 64->128, e3b 128->128 | up2 128->64, cat e2b | d2a 128->64,
 *   d2b 64->64 | up1 64->32, cat e1b | d1a 64->32, d1b 32->32 | head 32->1;
 *   the network sees u = in_scale * x and out = x + head(.) / in_scale
 *   (in_scale brings images of attenuation values to order one).
 * Parameters: one FP32 vector of lalm_unet_param_count() values; for each
 * layer in the order above its weights then its biases; 3x3 weights
 * [Cout][3][3][Cin], transposed-conv weights [2][2][Cout][Cin] (output pixel
 * (2y+a, 2x+b) = W[a][b] . in[y][x] + b), head [Cin] + 1 bias.
 * Numerics: weights, the input and every stored activation and gradient
 * tensor in bfloat16 (round to nearest even), MFMA products accumulated in
 * FP32, loss and parameter gradients in FP32 with FP64 loss sums.
 * Images are FP32 [batch][H][W] device arrays; H and W multiples of 4.
 */
#ifndef LALM_UNET_H
#define LALM_UNET_H

#include "lalm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lalm_unet lalm_unet;

/* Number of FP32 parameters (465953). */
LALM_API int64_t lalm_unet_param_count(void);

/* Workspace for batches up to batch_max of height x width images (allocated
 * here, once).  LALM_E_INVALID for sizes that are not positive multiples of
 * 4; LALM_E_NOMEM when allocation fails. */
LALM_API lalm_status lalm_unet_create(int32_t batch_max, int32_t height, int32_t width, lalm_unet **out);
LALM_API lalm_status lalm_unet_destroy(lalm_unet *net);

/* out = net(x) for batch images (FP32 device arrays [batch][H][W]);
 * nonneg = 1 clamps the output at zero (the constraint set of the method). */
LALM_API lalm_status lalm_unet_forward(lalm_unet *net, const float *params, const float *x, float *out,
                                       int32_t batch, double in_scale, int32_t nonneg, hipStream_t stream);

/* Loss = mean over the mask's pixels (mask: device uint8 [H][W], the same
 * for every image) of (hu_scale * (net(x) - target))^2; writes the FP32
 * gradient of the loss w.r.t. params into grad (device, param_count values)
 * and the loss to loss_dev[0] (device double).  Deterministic. */
LALM_API lalm_status lalm_unet_loss_grad(lalm_unet *net, const float *params, const float *x,
                                         const float *target, const uint8_t *mask, double in_scale,
                                         double hu_scale, int32_t batch, float *grad, double *loss_dev,
                                         hipStream_t stream);

/* Layer-by-layer inspection (a measurement aid, not part of the method):
 * lalm_unet_loss_grad, and a copy of every tensor the kernels store in
 * bfloat16, converted to FP32 (exact), into the device array capture of at
 * least lalm_unet_capture_elems(batch, H, W) floats.  Tensors are NHWC
 * [batch][h][w][C] and follow each other in this order (level 1: H x W,
 * level 2: H/2 x W/2, level 3: H/4 x W/4; channels in brackets):
 *   activations  e1a[32] e1b[32] (1), p1[32] e2a[64] e2b[64] (2), p2[64]
 *                e3a[128] e3b[128] (3), up2[64] d2a[64] d2b[64] (2),
 *                up1[32] d1a[32] d1b[32] (1);
 *   output gradients of the layers, after the ReLU mask, as the backward
 *   pass stores them: dz_d1b dz_d1a dz_up1 [32] (1), dz_d2b dz_d2a dz_up2
 *                [64] (2), dz_e3b dz_e3a [128] (3), dz_e2b dz_e2a [64] (2),
 *                dz_e1b dz_e1a [32] (1).
 * The input of every layer is one of these tensors (or x), so each layer's
 * kernels can be checked on their own inputs.  Errors as
 * lalm_unet_loss_grad, and LALM_E_INVALID when capture is null or too
 * small.  lalm_unet_capture_elems returns 0 for invalid sizes. */
LALM_API int64_t lalm_unet_capture_elems(int32_t batch, int32_t height, int32_t width);
LALM_API lalm_status lalm_unet_capture(lalm_unet *net, const float *params, const float *x, const float *target,
                                       const uint8_t *mask, double in_scale, double hu_scale, int32_t batch,
                                       float *grad, double *loss_dev, float *capture, int64_t capture_elems,
                                       hipStream_t stream);

/* Adam step t (1-based, bias-corrected; beta1 0.9, beta2 0.999, eps 1e-8)
 * on FP32 master parameters with moment buffers m, v (device arrays). */
LALM_API lalm_status lalm_unet_adam(lalm_unet *net, float *params, const float *grad, float *m, float *v,
                                    int64_t t, double lr, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* LALM_UNET_H */
