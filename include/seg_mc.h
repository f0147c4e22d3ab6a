/*
 * seg_mc.h - C ABI of the motion correction in libseg.so.
 *
 * The paper's first stage (Sec. II) cancels motion before segmentation. It
 * measures image similarity by the zero-mean normalised cross-correlation
 * (ZNCC): 21 x 21-pixel patches tile the image, ZNCC is evaluated for every
 * patch and every candidate motion vector (with table-based area sums), and
 * the patch values are aggregated into the most likely motion vector of the
 * frame. This library fixes what the paper leaves open:
 *   - the template is the integer mean (rounded half up) of given frames,
 *     normally the first 50 of the recording;
 *   - the candidates are all integer vectors d = (dy, dx), |dy|, |dx| <= R,
 *     ordered by dy, then dx (index (dy + R)(2R + 1) + dx + R);
 *   - the tiles form a grid of (H - 2R) / 21 rows and (W - 2R) / 21 columns,
 *     centred in the frame minus an R-pixel margin;
 *   - ZNCC compares the frame's tile at p with the template's window at
 *     p + d (0 where either has zero variance);
 *   - a vector's score is the sum of its ZNCC over the tiles; the largest
 *     score wins, ties going to the lowest index;
 *   - the motion of the frame is m = -d (the displacement of its content
 *     relative to the template), and the corrected frame is
 *     C(y, x) = F(y + my, x + mx) where that pixel lies in the frame and the
 *     template's T(y, x) where it does not.
 *
 * Conventions are those of seg.h: int status (SEG_OK or SEG_E_*), frames
 * uint16 [n][height][width], "dev" pointers are HIP device memory, the
 * caller owns the workspace and all buffers, a HIP error makes the object
 * fail permanently (SEG_E_DEVICE), one thread at a time per object.
 */
#ifndef SEG_MC_H
#define SEG_MC_H

#include <stddef.h>
#include <stdint.h>

#include "seg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct seg_mc seg_mc;   /* opaque */

typedef struct seg_mc_config {
  uint32_t height, width;   /* frame size; at least 21 + 2 radius each         */
  uint32_t radius;          /* R, 1..10 (8): candidate vectors |dy|, |dx| <= R  */
} seg_mc_config;

/* Default configuration (radius 8). Errors: SEG_E_INVAL (NULL, zero size). */
int seg_mc_default_config(uint32_t height, uint32_t width, seg_mc_config* out);

/* Device workspace bytes for this configuration (template, its integral
 * images and window tables, per-slice score sums for 2,048 frames).
 * Errors: SEG_E_INVAL (NULL; radius outside 1..10; frame smaller than one
 * tile plus the margin; larger than 2048 x 2048). */
int seg_mc_workspace_bytes(const seg_mc_config* cfg, size_t* bytes);

/* Create a corrector on the current HIP device over the caller's workspace
 * (device, 256-byte aligned, at least seg_mc_workspace_bytes, kept until
 * seg_mc_destroy). Errors: SEG_E_INVAL, SEG_E_CAPACITY (workspace too small). */
int seg_mc_create(const seg_mc_config* cfg, void* dev_workspace, size_t bytes, seg_mc** out);

/* Number of tiles P and candidate vectors V. Errors: SEG_E_INVAL. */
int seg_mc_layout(const seg_mc* mc, uint32_t* n_patches, uint32_t* n_vectors);

/* Build the template from n_frames device frames (1..65536): per pixel
 * floor((sum + n/2) / n), then its integral images and the window sums of
 * every tile and vector. Ordered on `stream`; the frames must stay valid
 * until the stream passes the call. Errors: SEG_E_INVAL, SEG_E_DEVICE. */
int seg_mc_set_template(seg_mc* mc, const uint16_t* dev_frames, uint32_t n_frames, void* stream);

/* Copy the template ([height][width] uint16) to host memory (synchronises
 * the device). Errors: SEG_E_INVAL, SEG_E_STATE (no template). */
int seg_mc_get_template(seg_mc* mc, uint16_t* host_out);

/* Motion of each of n_frames device frames.
 *   dev_motion  device int32 [n_frames][2]: (my, mx) per frame
 *   dev_scores  device double [n_frames][V] vector scores, or NULL
 * Ordered on `stream`, no synchronisation. Frames are scored in launches of
 * up to 2,048; results do not depend on how a recording is split into calls.
 * The score buffer lives in the workspace: calls of one corrector on
 * different streams must not overlap.
 * Errors: SEG_E_INVAL (NULL with n_frames > 0), SEG_E_STATE (no template),
 * SEG_E_DEVICE. */
int seg_mc_estimate(seg_mc* mc, const uint16_t* dev_frames, uint64_t n_frames,
                    int32_t* dev_motion, double* dev_scores, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * motion of up to SEG_MC_STATIC_MAX_FRAMES frames, exactly as
 * seg_mc_estimate computes it (same kernels, same order of sums, same
 * results), but the per-slice partial ZNCC sums go to a fixed device array
 * inside the library instead of the corrector's workspace. That array holds
 * 7 MiB on every GPU the library runs on, from the first corrector created
 * there until the process ends; nothing is allocated or freed by this call.
 * Every call on one GPU shares that GPU's array (each call writes every
 * entry it reads, so nothing carries over between calls): calls that overlap
 * in time on one GPU, from any corrector or stream, race, and the caller
 * must order them (one stream, or events). Ordered on `stream`, no
 * synchronisation.
 * Errors: SEG_E_INVAL (NULL with n_frames > 0), SEG_E_STATE (no template),
 * SEG_E_CAPACITY (n_frames > SEG_MC_STATIC_MAX_FRAMES), SEG_E_DEVICE (the
 * array's device address could not be resolved, or a launch failed). */
#define SEG_MC_STATIC_MAX_FRAMES 256
int seg_mc_estimate_static(seg_mc* mc, const uint16_t* dev_frames, uint64_t n_frames,
                           int32_t* dev_motion, double* dev_scores, void* stream);

/* Corrected frames: dev_out[t](y, x) = dev_frames[t](y + my, x + mx) with
 * (my, mx) = dev_motion[t] where that pixel lies in the frame, else the
 * template's value at (y, x). dev_out must not overlap dev_frames.
 * Errors: SEG_E_INVAL, SEG_E_STATE (no template), SEG_E_DEVICE. */
int seg_mc_apply(seg_mc* mc, const uint16_t* dev_frames, uint64_t n_frames,
                 const int32_t* dev_motion, uint16_t* dev_out, void* stream);

/* Release the corrector (not the workspace). NULL is a no-op. */
int seg_mc_destroy(seg_mc* mc);

#ifdef __cplusplus
}
#endif

#endif /* SEG_MC_H */
