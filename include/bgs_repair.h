/* Learned gap/edge repair of the affiliated eye: a small convolutional
 * network that fills the holes the forward reprojection leaves (the
 * disocclusions and cracks of Sec. 3.4-3.5), as an alternative to gap
 * interpolation plus ROI re-rendering.  Inference and training run on the
 * GPU: 3x3 convolutions as implicit GEMMs on bf16 MFMA with fp32
 * accumulation, Adam in fp32.
 *
 * Network (three-level U-Net, every 3x3 convolution zero-padded, ReLU
 * after all but the last):
 *   level 1 (H x W):      e1a 5->16, e1b 16->16
 *   level 2 (H/2 x W/2):  e2a 16->32, e2b 32->32   input: 2x2 mean pool of e1b
 *   level 3 (H/4 x W/4):  e3a 32->64, e3b 64->64   input: 2x2 mean pool of e2b
 *   level 2:              d2 96->32                 input: [nearest 2x upsample of e3b, e2b]
 *   level 1:              d1 48->16                 input: [upsample of d2, e1b]
 *   level 1:              out 16->4, no activation
 * Inputs per pixel: warped RGB (zeroed at holes), hole mask, 1/z (0 at
 * holes and for infinite depth).  Output channels 0-2 are a residual r:
 * rgb_out = rgb + hole * r, so only holes change; channel 3, e, predicts
 * the pixel's squared error s = mean over channels of (rgb_out - target)^2.
 * Training loss over hole pixels: sum_c (rgb_out_c - target_c)^2 / (3 N) +
 * sum (e - s)^2 / N, N = max(1, holes), s held constant in the gradient.
 *
 * Parameters: one flat fp32 device array, per layer in the order above
 * W[cout][cin][3][3] then b[cout] (bgs_repair_num_params elements).
 * Activations and weights are held in bfloat16 (round to nearest even),
 * accumulations in fp32.
 *
 * Images: rgb and target [B][3][H][W] fp32, z [B][H][W] fp32, hole
 * [B][H][W] u8 (nonzero = hole), all device pointers, planar and dense.
 * H and W must be multiples of 4 in [4, 8192], the batch in [1, 1000].
 * All calls are asynchronous on the given HIP stream (null: the default
 * stream); device buffers belong to the caller.  Errors: BGS_ERR_INVALID_ARG for a bad size or a null
 * pointer, BGS_ERR_WORKSPACE for a workspace smaller than
 * bgs_repair_workspace_size, BGS_ERR_HIP for a failed launch; nothing is
 * launched on an argument error. */
#ifndef BGS_REPAIR_H
#define BGS_REPAIR_H

#include "bgs.h"

#ifdef __cplusplus
extern "C" {
#endif

BGS_API int32_t bgs_repair_num_params(int64_t* n);

/* Workspace bytes for a batch of B images of H x W; train = 1 adds the
 * gradient buffers that bgs_repair_grad needs.  Allocate 256-byte aligned. */
BGS_API int32_t bgs_repair_workspace_size(int32_t batch, int32_t height, int32_t width, int32_t train,
                                          size_t* bytes);

/* Inference: rgb_out [B][3][H][W] = rgb + hole * r; err_out [B][H][W]
 * (may be null) = e at holes, 0 elsewhere. */
BGS_API int32_t bgs_repair_forward(const float* params, int32_t batch, int32_t height, int32_t width,
                                   const float* rgb, const float* z, const uint8_t* hole, float* rgb_out,
                                   float* err_out, void* ws, size_t ws_bytes, void* hip_stream);

/* Mean predicted squared error over the holes of each image, the fallback
 * policy's measure: out[b] (device, batch floats) = sum of err_out[b] over
 * hole pixels / max(1, holes), with err_out as bgs_repair_forward writes it.
 * scratch: device, BGS_REPAIR_HOLE_ERROR_SCRATCH(batch) floats.  Summation
 * order is fixed (deterministic).  batch in [1, 1000], sides in [1, 16384]. */
#define BGS_REPAIR_HOLE_ERROR_SCRATCH(batch) (512 * (size_t)(batch))
BGS_API int32_t bgs_repair_hole_error(const float* err, const uint8_t* hole, int32_t batch, int32_t height,
                                      int32_t width, float* out, float* scratch, void* hip_stream);

/* Forward and backward pass: loss (one device float) and the gradient of
 * the loss in the parameter layout (grad, device, overwritten).  rgb_out
 * may be null. */
BGS_API int32_t bgs_repair_grad(const float* params, int32_t batch, int32_t height, int32_t width,
                                const float* rgb, const float* z, const uint8_t* hole, const float* target,
                                float* grad, float* loss, float* rgb_out, void* ws, size_t ws_bytes,
                                void* hip_stream);

/* Block shape of the convolution launches, for every later call in the
 * process: rows = output rows per block (2, 4 or 8; inputs wider than 64
 * channels take at most 4, and 8 rows, or 4 rows of such inputs, take at
 * most two output tiles, else fewer rows), tiles = 16-channel output tiles
 * per block (1-4, capped at the layer's).  0 leaves the choice to the library, which picks
 * from the grid size (the default).  Results do not depend on the shape: a
 * pixel's sums run in the same order under every shape.  Not synchronised
 * with calls in flight on other host threads.  BGS_ERR_INVALID_ARG for
 * other values. */
BGS_API int32_t bgs_repair_set_block_shape(int32_t rows, int32_t tiles);

/* One Adam step (Kingma and Ba, 2015) over n parameters, step >= 1 the
 * 1-based step count used for the bias correction; params, m and v are
 * updated in place (fp32). */
BGS_API int32_t bgs_repair_adam(float* params, const float* grad, float* m, float* v, int64_t n, int32_t step,
                                float lr, float beta1, float beta2, float eps, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif
