/*
 * msr_unet.h -- C ABI of the learned warm start of libmsr.
 *
 * The minor cycle of step 2 (Eq. 5, solved by Algorithm 1) starts from an
 * initial image; the paper starts from zero.  This part predicts a better
 * start with a small U-Net from the two images step 2 already has -- the
 * long-baseline dirty image i_H and the low-resolution image l = i_L of step 1
 * (Sect. 3.2) -- and FISTA still runs to the same tolerance from it, so the
 * plain cold start stays both the fallback and the reference.  The network is not
 * part of the paper.
 *
 * Network (base width w, L levels; w = 32, L = 4 by default):
 *   input      (i_H / s, l / s), s = max |l| of the image (1 if l = 0), stored
 *              as 8 channels (2 used)
 *   encoder    level j = 0 .. L-1 at resolution (H / 2^j, W / 2^j): two 3x3
 *              convolutions with ReLU, width w 2^j; a 2x2 average pool between
 *              levels
 *   decoder    level j = L-2 .. 0: nearest 2x upsampling of the level below,
 *              concatenated with the encoder output of level j, two 3x3
 *              convolutions with ReLU, width w 2^j
 *   head       1x1 convolution to one channel, no activation
 *   warm start x0 = s * max(head, 0)
 * All convolutions are zero padded ("same").  Activations and weights are
 * bfloat16, products run on the matrix cores with float32 accumulation;
 * gradients, the master weights and the Adam moments are float32.
 *
 * Parameters are one float32 vector (msr_unet_param_count entries): for each
 * 3x3 convolution in the order encoder level 0 (first, second), ..., encoder
 * level L-1, decoder level L-2, ..., decoder level 0, the weights
 * W[cout][kpad] with k = (3 ky + kx) cin + ci (ky, kx in 0..2 for the offsets
 * -1..1, ci the input channel; cin = 8 for the first convolution, the
 * concatenation puts the upsampled channels first), kpad = 9 cin rounded up
 * to a multiple of 32, entries k >= 9 cin unused; then its bias b[cout].
 * Last the head: w[w], b[1].
 *
 * Images are float32, row-major, device arrays of batch x H x W; H and W
 * must be multiples of 2^(L-1).  Status codes and stream conventions are
 * those of msr.h; all device memory is the caller's workspace.
 */
#ifndef MSR_UNET_H
#define MSR_UNET_H

#include "msr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct msr_unet msr_unet;

typedef struct msr_unet_config {
    int32_t in_channels; /* 2: (i_H, l) */
    int32_t base_width;  /* w, a multiple of 8, at most 128 */
    int32_t levels;      /* L, 2 .. 6 */
    int32_t device;
} msr_unet_config;

typedef struct msr_adam {
    double lr, beta1, beta2, eps;
} msr_adam;

/* Number of float32 parameters (0 for an invalid configuration). */
size_t msr_unet_param_count(const msr_unet_config* cfg);

/* Bytes of device workspace for batches of up to `batch` images of
 * height x width (0 if invalid). */
size_t msr_unet_workspace_bytes(const msr_unet_config* cfg, int batch, int height, int width);

msr_status msr_unet_init(const msr_unet_config* cfg, msr_unet** out);
void msr_unet_destroy(msr_unet* net);
const char* msr_unet_last_error(const msr_unet* net);

/* Hands over the workspace (256-byte aligned) sized for (batch, height,
 * width); parameters and optimiser state live in it, so set them after. */
msr_status msr_unet_set_workspace(msr_unet* net, void* dev, size_t bytes, int batch, int height, int width);

/* Copies a parameter vector (device, float32) in and resets the Adam moments
 * and step count. */
msr_status msr_unet_set_params(msr_unet* net, const float* params, void* stream);

/* Copies the float32 master parameters out (device). */
msr_status msr_unet_get_params(msr_unet* net, float* params_out, void* stream);

/* Training checkpoints.  msr_unet_save writes the configuration, the FP32
 * master parameters, Adam's two moment arrays and its step count to the file
 * `path` (8-byte magic "MSRUNET1", int32 in_channels, base_width, levels, 0,
 * int64 parameter count, int64 step, then the three float32 arrays, host byte
 * order); msr_unet_load reads one into a network of the same configuration
 * (MSR_ERR_INVALID for another configuration or a damaged file) and rebuilds
 * the bfloat16 weights, so that training continues as if uninterrupted.
 * save needs parameters (msr_unet_set_params or a load); both need the
 * workspace and synchronise the stream. */
msr_status msr_unet_save(msr_unet* net, const char* path, void* stream);
msr_status msr_unet_load(msr_unet* net, const char* path, void* stream);

/* Warm starts x0 (batch x H x W) from the long-baseline dirty images and the
 * low-resolution images. */
msr_status msr_unet_forward(msr_unet* net, const float* dirty_h, const float* low_res, float* x0_out, int batch,
                            void* stream);

/* Mean squared error between the head output and target / s over the batch,
 * and its gradient with respect to every parameter (grad_out: device,
 * msr_unet_param_count floats, may be NULL).  Synchronises the stream. */
msr_status msr_unet_loss_grad(msr_unet* net, const float* dirty_h, const float* low_res, const float* target,
                              int batch, double* loss, float* grad_out, void* stream);

/* One Adam step on that loss (bias-corrected moments, float32 master
 * weights; the bfloat16 copies are refreshed).  *loss (may be NULL) receives
 * the loss before the step.  Synchronises the stream. */
msr_status msr_unet_train_step(msr_unet* net, const float* dirty_h, const float* low_res, const float* target,
                               int batch, const msr_adam* opt, double* loss, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MSR_UNET_H */
