/*
 * sg_upsampler.h -- C ABI of the learned upsampler (gfx950, MFMA).
 *
 * Fewer rays per frame (Sec 5.3 renders in a space that needs fewer rays and
 * resamples): the volume is ray cast at half the resolution one pyramid
 * level coarser, and a small convolutional network predicts the
 * full-resolution frame from that render's premultiplied RGBA and depth.
 * The network (BF16 weights and activations, FP32 accumulation on MFMA):
 *   x0  [N][H][W][8]   r, g, b, a, depth code 1/(1 + t/depth_scale) (0 where
 *                      the ray never reached the depth threshold), 0, 0, 0
 *   h1 = relu(conv3x3(x0)), h2 = relu(conv3x3(h1)), h3 = relu(conv3x3(h2)),
 *   o  = conv3x3(h3)                 (32 channels each; zero padding)
 *   full-resolution pixel (2y + sy, 2x + sx), s = 2 sy + sx:
 *     rgba = bilinear x2 of x0's rgba (half-pixel centres, clamped edges)
 *            + o[y][x][5s .. 5s+3],
 *     err  = o[y][x][5s+4]^2, a prediction of that pixel's mean squared RGB
 *            error; its frame mean predicts the frame's PSNR, which decides
 *            whether the caller falls back to a full-resolution render.
 *   At inference, a low-resolution pixel whose 9 x 9 neighbourhood of x0
 *   (the receptive field of the four layers; outside the image counts as
 *   zero) holds no nonzero value yields rgba 0 and err 0 at its four
 *   full-resolution pixels (background: its bilinear base is 0; the
 *   network's constant response to an empty input is dropped). Tiles whose
 *   whole input region is empty skip the network. Training (sg_up_gradients,
 *   sg_up_train_step) evaluates the network everywhere.
 * Weights are packed layer by layer as w[9][c_in][32] (tap = 3 (dy+1) +
 * (dx+1)) followed by b[32], with c_in = 8, 32, 32, 32.
 *
 * Conventions as in sg.h: every call returns an sg_status; device pointers
 * are read or written in hip_stream order; the upsampler owns its weights,
 * optimiser state and scratch; it is not thread-safe, and calls on one
 * upsampler that overlap on different streams race on its scratch.
 */
#ifndef SG_UPSAMPLER_H
#define SG_UPSAMPLER_H
#include <stdint.h>

#include "sg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sg_upsampler sg_upsampler; /* opaque */

/* Number of floats in the packed weights (all four layers). */
int64_t sg_up_param_count(void);

/* Create an upsampler on a device with scratch for batches of up to
 * max_pixels low-resolution pixels (N * H * W) and zero weights.
 * Errors: SG_ERR_INVALID_ARG, SG_ERR_OUT_OF_MEMORY, SG_ERR_DEVICE. */
sg_status sg_up_create(int32_t device, int64_t max_pixels, sg_upsampler **out);
sg_status sg_up_destroy(sg_upsampler *up);

/* Copy packed weights in (host floats, sg_up_param_count of them; also
 * resets the optimiser state) or out. Synchronous. */
sg_status sg_up_set_weights(sg_upsampler *up, const float *params, int64_t n);
sg_status sg_up_get_weights(sg_upsampler *up, float *params, int64_t n);

/* Inference on n low-resolution images of h x w:
 *   rgba  device float [n][h][w][4] (a render's premultiplied output)
 *   depth device float [n][h][w]    (its first-hit depth, +inf = none)
 *   content NULL, or device uint8 [n][(h + 7) / 8][(w + 7) / 8]: the
 *         input's content mask as sg_render_views fills sg_view.tile_any
 *         (one byte per 8 x 8-pixel block, nonzero if a pixel of the block
 *         has a nonzero rgba component or a finite depth); the images'
 *         masks back to back. With NULL the call builds the same mask from
 *         rgba and depth. A mask byte of 0 where the block has content
 *         gives wrong output there; extra nonzero bytes only cost time.
 *   out_rgba device float [n][2h][2w][4]
 *   out_err  NULL or device float [n][2h][2w] (predicted squared error)
 *   mse_pred NULL or host double [n]: mean predicted squared error per
 *            image (synchronises hip_stream when given)
 * n * h * w <= max_pixels. The fused network (the default) runs only on the
 * 16 x 16 tiles whose input region (the tile and the 4-pixel reach of the
 * four layers) meets a nonzero block of the mask; every other tile is
 * background, written without a look at the input. */
sg_status sg_up_forward(sg_upsampler *up, int32_t n, int32_t h, int32_t w,
                        const float *rgba, const float *depth, const uint8_t *content,
                        double depth_scale, float *out_rgba, float *out_err,
                        double *mse_pred, void *hip_stream);

/* Inference as sg_up_forward, and the fallback decision taken on the device
 * without a host round trip: *fallback (device int32) = 1 when the frame's
 * predicted PSNR, 10 log10(1 / m) with m the mean over the n images of
 * their mean predicted squared error, is below threshold_db, else 0. Pass
 * the flag to sg_render_views_if to render the frame at full resolution
 * only when the prediction fails. Asynchronous. */
sg_status sg_up_forward_flag(sg_upsampler *up, int32_t n, int32_t h, int32_t w,
                             const float *rgba, const float *depth, const uint8_t *content,
                             double depth_scale, float *out_rgba, float *out_err,
                             double threshold_db, int32_t *fallback, void *hip_stream);

/* Gradients of the training loss (mean squared RGBA error against target,
 * plus err_weight times the mean squared error of the error head against
 * each pixel's actual RMS RGB error, held constant) for one batch:
 *   target device float [n][2h][2w][4]
 *   grads  NULL or host float [sg_up_param_count()] (packed like the
 *          weights; synchronises)
 *   loss   NULL or host double (synchronises) */
sg_status sg_up_gradients(sg_upsampler *up, int32_t n, int32_t h, int32_t w,
                          const float *rgba, const float *depth, double depth_scale,
                          const float *target, double err_weight, float *grads,
                          double *loss, void *hip_stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) with
 * learning rate lr on the gradients of the batch (as sg_up_gradients). */
sg_status sg_up_train_step(sg_upsampler *up, int32_t n, int32_t h, int32_t w,
                           const float *rgba, const float *depth, double depth_scale,
                           const float *target, double err_weight, double lr,
                           double *loss, void *hip_stream);

/* How sg_up_forward runs the network: fused != 0 (the default) in one
 * kernel per 16 x 16 tile of low-resolution pixels with every activation in
 * LDS; fused == 0 layer by layer through device buffers (the path training
 * uses; it leaves the activations sg_up_read_buffer returns). Both give the
 * same output bit for bit (same products, same accumulation order); the
 * predicted mean squared errors may differ in the last bits (per-image sums
 * taken in another order). */
sg_status sg_up_set_fused(sg_upsampler *up, int32_t fused);

/* Test hook: copy the first `bytes` of an activation of the last gradient
 * call, or of the last forward call made layer by layer, to host memory
 * (synchronises the device): which = 0 x0 (bf16 [P][8]), 1..3 h1..h3 (bf16
 * [P][32]), 4 o (float [P][32]). */
sg_status sg_up_read_buffer(sg_upsampler *up, int32_t which, void *host, int64_t bytes);

#ifdef __cplusplus
}
#endif
#endif /* SG_UPSAMPLER_H */
