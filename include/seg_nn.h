/*
 * seg_nn.h - C ABI of the learned surrogate detector in libseg.so.
 *
 * The paper identifies spiking pixels per time segment with a U-Net on the
 * segment's two summary images (Sec. III-C, trained with binary
 * cross-entropy and RMSProp on synthetic data). The surrogate here takes the
 * segment's frames themselves: per pixel the 50 frames are normalised as
 * (V - mean) / sqrt(mean + 25), three temporal convolutions (32 channels,
 * kernel 5; strides 5, 2 and 1 with padding 0, 2, 0: 50 -> 10 -> 5 -> 1
 * samples) feed a 2-D U-Net of depth 3 (32 / 64 / 128 channels, two 3x3
 * convolutions with ReLU per level, 2x2 max pooling, 2x2 stride-2 transposed
 * convolutions, skip concatenation), and a 1x1 convolution gives one logit
 * per pixel; the probability is its sigmoid. Weights are FP32 masters with a
 * BF16 copy; every convolution is a BF16 MFMA product with FP32 accumulation.
 *
 * Layouts: frames uint16 [batch][50][height][width]; probabilities, labels and
 * logits float [batch][height][width]; parameters float [n] in the order and
 * shapes reported by seg_nn_param_layout (weight [rows][cols] row-major, then
 * its bias). height and width must be multiples of 4.
 *
 * Ownership: the caller owns the parameter array and the workspace (device
 * memory); the library allocates nothing. Errors as in seg.h.
 */
#ifndef SEG_NN_H
#define SEG_NN_H

#include <stddef.h>
#include <stdint.h>

#include "seg.h"

#ifdef __cplusplus
extern "C" {
#endif

#define SEG_NN_LAYERS 16   /* t1 t2 t3 e1a e1b e2a e2b e3a e3b u2 d2a d2b u1 d1a d1b out */

typedef struct seg_nn seg_nn;   /* opaque */

/* Number of FP32 parameters. */
int seg_nn_param_count(size_t* n);

/* Shape and offsets of layer `index` (< SEG_NN_LAYERS): weight [rows][cols]
 * at w_offset, bias at b_offset (rows entries, rows / 4 for the transposed
 * convolutions u2 and u1, whose weight rows are (out_channel * 4 + 2a + b)). */
int seg_nn_param_layout(uint32_t index, uint32_t* rows, uint32_t* cols,
                        size_t* w_offset, size_t* b_offset);

/* Workspace bytes for batches of up to `batch` segments of height x width. */
int seg_nn_workspace_bytes(uint32_t batch, uint32_t height, uint32_t width,
                           size_t* bytes);

/* Bind the caller's parameters (dev, FP32 [n]) and workspace. */
int seg_nn_create(uint32_t batch, uint32_t height, uint32_t width,
                  float* dev_params, void* dev_workspace, size_t bytes,
                  seg_nn** out);

/* After the caller wrote the parameters: refresh the BF16 copy and reset the
 * optimizer state. */
int seg_nn_sync_weights(seg_nn* n, void* stream);

/* Probabilities for `batch` segments (dev_prob may be NULL: kept inside). */
int seg_nn_forward(seg_nn* n, const uint16_t* dev_frames, uint32_t batch,
                   float* dev_prob, void* stream);

/* Forward, mean binary cross-entropy against dev_labels (0/1 per pixel) and
 * backward; gradients stay in the workspace for seg_nn_step and are also
 * copied to dev_grad (FP32 [n]) when it is not NULL; *host_loss (if not NULL)
 * receives the loss after a stream synchronisation. */
int seg_nn_backward(seg_nn* n, const uint16_t* dev_frames, const float* dev_labels,
                    uint32_t batch, float* dev_grad, float* host_loss, void* stream);

/* RMSProp with the last gradients: v = rho v + (1 - rho) g^2,
 * w -= lr g / (sqrt(v) + eps); refreshes the BF16 copy. */
int seg_nn_step(seg_nn* n, float lr, float rho, float eps, void* stream);

/* Copy the logits of the last forward ([batch][height][width]) to dev_out. */
int seg_nn_logits(seg_nn* n, float* dev_out, void* stream);

/* The MFMA product on its own, for checking: C [M][N] = op(A) op(B) with
 * operands rounded to BF16, A stored [M][K] ([K][M] when a_trans), B stored
 * [K][N] ([N][K] when b_trans); splits > 1 splits K and needs scratch of
 * splits * M * N floats. */
int seg_nn_gemm_test(const float* A, int a_trans, const float* B, int b_trans,
                     float* C, int M, int N, int K, int splits, float* scratch,
                     void* stream);

/* Batch capacity and frame size the network was created for. */
int seg_nn_shape(const seg_nn* n, uint32_t* batch, uint32_t* height, uint32_t* width);

int seg_nn_destroy(seg_nn* n);

/* ---- the paper's input: summary-image patches (Sec. III-C) -----------------
 *
 * The same U-Net without the temporal layers: its first convolution reads a
 * 2-channel patch (S_i, T_i) of a segment's summary images, normalised inside
 * as channel 0 = (S - mean over the patch) / max(sd over the patch, 1e-3)
 * and channel 1 = T / sqrt(S + 25). Over a frame it runs on 64 x 64 patches
 * at origins every 32 pixels (the last one flush with the far edge, frames
 * of at least 64 x 64), and a frame pixel's probability is the mean of the
 * patches' probabilities weighted by w(u) w(v), w(u) = 1 - |u - 31.5| / 32
 * (u, v: the pixel's position in the patch). A network made by
 * seg_nn_st_create takes these calls in place of the frame calls (which
 * return SEG_E_STATE on it, and the other way round); seg_nn_sync_weights,
 * seg_nn_step, seg_nn_logits, seg_nn_shape and seg_nn_destroy are shared.
 * The parameter table is that of seg_nn_param_layout with layers t1, t2, t3
 * empty (0 x 0) and e1a of 32 x 18.
 *   dev_st  device float [batch][2][height][width]: raw S then raw T. */
#define SEG_NN_INPUT_FRAMES    0
#define SEG_NN_INPUT_SUMMARIES 1
int seg_nn_st_param_count(size_t* n);
int seg_nn_st_param_layout(uint32_t index, uint32_t* rows, uint32_t* cols,
                           size_t* w_offset, size_t* b_offset);
int seg_nn_st_workspace_bytes(uint32_t batch, uint32_t height, uint32_t width,
                              size_t* bytes);
int seg_nn_st_create(uint32_t batch, uint32_t height, uint32_t width,
                     float* dev_params, void* dev_workspace, size_t bytes,
                     seg_nn** out);
int seg_nn_st_forward(seg_nn* n, const float* dev_st, uint32_t batch,
                      float* dev_prob, void* stream);
int seg_nn_st_backward(seg_nn* n, const float* dev_st, const float* dev_labels,
                       uint32_t batch, float* dev_grad, float* host_loss,
                       void* stream);
/* SEG_NN_INPUT_FRAMES or SEG_NN_INPUT_SUMMARIES. Errors: SEG_E_INVAL. */
int seg_nn_input(const seg_nn* n, uint32_t* input);
/* Patches of a height x width frame (both >= 64). Errors: SEG_E_INVAL. */
int seg_nn_st_patch_count(uint32_t height, uint32_t width, uint32_t* n);
/* dev_out [n_patch][2][64][64] from device S and T ([height][width] float). */
int seg_nn_st_patches(const float* dev_S, const float* dev_T, uint32_t height,
                      uint32_t width, float* dev_out, void* stream);
/* dev_out [height][width] from patch probabilities [n_patch][64][64]. */
int seg_nn_st_merge(const float* dev_prob, uint32_t height, uint32_t width,
                    float* dev_out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SEG_NN_H */
