/*
 * seg.h - C ABI of the MI355X neuron-segmentation library (libseg.so).
 *
 * The library implements the segmentation stage of Bando et al., "Real-time
 * Neuron Segmentation for Voltage Imaging" (BIBM 2023), Sec. III:
 *   - the motion-corrected video V(x, t) (Sec. III-B) is cut into
 *     non-overlapping segments of L = 50 frames;
 *   - each segment is summarised by the temporal mean S_i (Eq. 1) and the
 *     max-minus-median image T_i of the Gaussian-smoothed video (Eq. 2);
 *   - the plain detector normalises T_i by a per-pixel noise scale, detects
 *     spike events, filters event regions by area, solidity and eccentricity
 *     and aggregates them over segments (Sec. III-D);
 *   - each connected component of the aggregate mask is factorised as
 *     P ~ F A (Eq. 3) into possibly overlapping footprints f_j with
 *     per-segment activities a_j, whose binarised footprints are the ROI
 *     masks (Sec. III-D).
 *
 * Conventions
 *   - Every function returns an int status: SEG_OK (0) or a negative SEG_E_*.
 *     No function throws, aborts or exits.
 *   - Frames are uint16, row-major [n][height][width], width fastest.
 *   - "dev" pointers are HIP device pointers; "host" pointers are ordinary
 *     host memory. `stream` is a hipStream_t (NULL = the default stream).
 *   - The caller owns the workspace (device memory of seg_workspace_bytes()
 *     bytes) and every frame buffer. The library never allocates device
 *     memory for a session, and sessions share no state, with two
 *     process-wide exceptions: one lock serialises the cooperative NMF
 *     launches of concurrent finalizes (so their grids cannot each hold part
 *     of the device waiting for the rest), and seg_mc_estimate_static
 *     (seg_mc.h) keeps its partial sums in a fixed device array per GPU.
 *   - A session is used by one thread at a time.
 *   - A HIP error inside a session makes it fail permanently (sticky):
 *     every later call on it returns SEG_E_DEVICE; other sessions are
 *     unaffected.
 */
#ifndef SEG_H
#define SEG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define SEG_OK          0
#define SEG_E_INVAL    -1  /* NULL pointer, bad configuration or argument     */
#define SEG_E_SHAPE    -2  /* frame size or buffer size mismatch               */
#define SEG_E_STATE    -3  /* call not allowed in the session's current state */
#define SEG_E_CAPACITY -4  /* more frames than max_frames, workspace too small */
#define SEG_E_DEVICE   -5  /* a HIP call failed (sticky for the session)       */
#define SEG_E_NOMODEL  -6  /* surrogate detector selected but no model loaded */

/* detectors */
#define SEG_DET_PLAIN     0  /* noise-normalised max - median events (Eq. 2)        */
#define SEG_DET_SURROGATE 1  /* learned spiking-pixel maps (seg_nn.h, Sec. III-C);
                                events where the probability >= event_z, NMF on the
                                probabilities; height and width multiples of 4     */
#define SEG_DET_UNET      2  /* the paper's U-Net on 64 x 64 patches of each
                                segment's (S_i, T_i), merged by weighted averaging
                                (seg_nn_st_*, Sec. III-C); events and NMF as for the
                                surrogate; height and width at least 64           */

/* execution of the per-component NMF (Eq. 3); every path computes the same
 * factorisation, they differ in the order of sums over pixels only */
#define SEG_NMF_AUTO   0  /* split when it applies, else one workgroup per component */
#define SEG_NMF_SINGLE 1  /* one workgroup per component                            */
#define SEG_NMF_SPLIT  2  /* each component over several co-resident workgroups;
                             seg_finalize fails with SEG_E_CAPACITY where the split
                             does not apply (no cooperative launch, too many
                             segments for LDS, more slices than compute units)     */

/* image kinds for seg_get_image (all [height][width]) */
#define SEG_IMG_MEAN        0  /* float: mean of S_i over segments (Eq. 1)         */
#define SEG_IMG_CORR        1  /* float: 8-neighbour correlation image             */
#define SEG_IMG_NOISE       2  /* float: per-pixel noise scale sigma(x)            */
#define SEG_IMG_EVENT_COUNT 3  /* int32: number of segments with an event          */
#define SEG_IMG_MASK_COUNT  4  /* int32: number of segments whose kept regions
                                  cover the pixel (n_b)                             */
#define SEG_IMG_LABELS      5  /* int32: components of the aggregate mask, 0 = none,
                                  numbered 1..n by minimum raster index            */

/* per-segment map kinds for seg_get_segment_maps (each [K][height][width] float) */
#define SEG_MAP_S 0            /* spatial summary, Eq. 1                            */
#define SEG_MAP_T 1            /* temporal summary, Eq. 2                           */
#define SEG_MAP_P 2            /* detection map p_i = max(0, T_i / sigma - theta)   */
#define SEG_MAP_B 3            /* kept-region mask b_i as 0.0 / 1.0                 */
#define SEG_MAP_D 4            /* noise-scale term D_i = mean over the segment of
                                  max(0, median - smoothed value)                   */

typedef struct seg_config {
  uint32_t height, width;   /* frame size in pixels, >= 1                          */
  uint32_t seg_len;         /* L; this build supports 50 (Sec. III-B)              */
  uint32_t max_frames;      /* capacity of one session; sizes the workspace        */
  float    gauss_sigma;     /* sd of the smoothing Gaussian, 3 px (Sec. III-B)     */
  uint32_t gauss_radius;    /* taps |k| <= radius, 1..12 (12 = 4 sigma)            */
  float    event_z;         /* theta: event when T_i / sigma >= theta (5.0); for the
                               surrogate, when the probability >= theta (0.5)     */
  uint32_t min_event_segs;  /* c_min: b = [sum_i b_i >= c_min] (2; 1 = the OR)     */
  uint32_t area_min, area_max;  /* region area bounds in pixels (16, 1600)         */
  float    solidity_min;    /* area / convex-hull area of pixel squares (0.75)     */
  float    ecc_max;         /* eccentricity of the pixel-centre covariance (0.95)  */
  uint32_t nmf_max_rank;    /* SPA rank cap per component, 1..8 (6)                */
  uint32_t nmf_sweeps;      /* HALS sweeps after the initial A update (200)        */
  float    spa_delta;       /* SPA stops below delta x the first pick's norm (0.3) */
  float    footprint_level; /* mask = footprint >= level x its peak (0.25)         */
  float    sigma_floor;     /* no event where sigma < floor (1e-3)                 */
  uint32_t detector;        /* SEG_DET_PLAIN or SEG_DET_SURROGATE                 */
  uint32_t nmf_path;        /* SEG_NMF_AUTO, SEG_NMF_SINGLE or SEG_NMF_SPLIT       */
} seg_config;

typedef struct seg_session seg_session;   /* opaque */
struct seg_nn;                            /* the surrogate network, seg_nn.h */

/* Fill *out with the default configuration for height x width frames and a
 * capacity of max_frames. Errors: SEG_E_INVAL (NULL out or zero size). */
int seg_default_config(uint32_t height, uint32_t width, uint32_t max_frames,
                       seg_config* out);

/* Bytes of device workspace a session with this configuration needs.
 * Errors: SEG_E_INVAL (NULL or invalid configuration). */
int seg_workspace_bytes(const seg_config* cfg, size_t* bytes);

/* Create a session on the current HIP device using the caller's workspace
 * (dev, at least seg_workspace_bytes bytes, 256-byte aligned). The workspace
 * must stay allocated until seg_destroy. Errors: SEG_E_INVAL,
 * SEG_E_CAPACITY (workspace too small). */
int seg_create(const seg_config* cfg, void* dev_workspace, size_t bytes,
               seg_session** out);

/* Append n_frames frames (dev, [n_frames][height][width] uint16) to the
 * session, stream-ordered and asynchronous: the caller must not overwrite
 * the frames until `stream` has passed this call. Frames that do not yet
 * complete a segment are copied into the workspace and carried to the next
 * push, so any blocking of the video gives the same result. A trailing
 * partial segment at finalize is ignored.
 * Errors: SEG_E_INVAL, SEG_E_STATE (after finalize), SEG_E_CAPACITY
 * (total frames > max_frames), SEG_E_DEVICE. */
int seg_push_frames(seg_session* s, const uint16_t* dev_frames,
                    uint32_t n_frames, void* stream);

/* Run the footprint reconstruction (events, region filter, aggregation,
 * components, per-component NMF) on everything pushed so far. Blocks until
 * the results are on the host. Needs at least one complete segment.
 * Errors: SEG_E_STATE (already finalized or no segment), SEG_E_DEVICE. */
int seg_finalize(seg_session* s, void* stream);

/* Number of complete segments K pushed so far. */
int seg_num_segments(const seg_session* s, uint32_t* k);

/* Footprints after seg_finalize, ordered by component then by the raster
 * index of the footprint peak. *n_out receives the count N; at most
 * `capacity` footprints are copied. Any output pointer may be NULL.
 *   weights  host float [capacity][height][width]: f_j scaled to peak 1
 *   masks    host uint8 [capacity][height][width]: f_j >= footprint_level
 *   activity host float [capacity][K]: a_j, one value per segment
 *   component host int32 [capacity]: the component label of each footprint
 * Errors: SEG_E_STATE (not finalized). */
int seg_get_footprints(seg_session* s, uint32_t capacity, uint32_t* n_out,
                       float* weights, uint8_t* masks, float* activity,
                       int32_t* component);

/* Voltage traces (Sec. II, the stage after segmentation): for every
 * footprint j of a finalized session and every frame t of dev_frames, the
 * mean intensity over the footprint's mask (the pixels seg_get_footprints
 * reports in `masks`):
 *     trace_j(t) = sum_{x in mask_j} V_t(x) / |mask_j|
 * The sum is exact (integers); the mean is one FP64 division rounded to FP32.
 *   dev_frames device uint16 [n_frames][height][width]; any frames of the
 *              session's size (the segmented recording or later ones)
 *   dev_out    device float, footprint j's trace at dev_out[j * ld + t],
 *              t < n_frames; ld >= n_frames. A recording pushed in blocks
 *              fills one [N][T] array by offsetting dev_out by the block's
 *              first frame and keeping ld = T.
 * Work is ordered on `stream`; the call does not synchronise, except for the
 * first call on a session, which uploads the mask tables (a few bytes per
 * masked pixel) into the workspace. Nothing is written when N = 0 or
 * n_frames = 0. The caller owns both buffers.
 * Errors: SEG_E_INVAL (NULL pointer with n_frames > 0, ld < n_frames),
 * SEG_E_STATE (not finalized), SEG_E_CAPACITY (the mask tables do not fit
 * the workspace's NMF factor region; only for frames of a few pixels),
 * SEG_E_DEVICE. */
int seg_extract_traces(seg_session* s, const uint16_t* dev_frames, uint64_t n_frames,
                       float* dev_out, uint64_t ld, void* stream);

/* Copy one SEG_IMG_* image ([height][width], float or int32) to host_out.
 * Every kind needs a finalized session. Errors: SEG_E_INVAL, SEG_E_STATE. */
int seg_get_image(seg_session* s, int kind, void* host_out);

/* Copy `count` per-segment maps starting at segment `first` of kind SEG_MAP_*
 * into dev_out ([count][height][width] float, device memory), ordered on
 * `stream`. S, T and D are available after the push that completes a
 * segment; P and B need a finalized session.
 * Errors: SEG_E_INVAL (range), SEG_E_STATE, SEG_E_DEVICE. */
int seg_get_segment_maps(seg_session* s, int kind, uint32_t first,
                         uint32_t count, float* dev_out, void* stream);

/* Load precomputed per-segment summaries instead of pushing frames, then
 * finalize as usual. This is the entry point for stage isolation: the
 * footprint reconstruction (events, region filter, aggregation, components,
 * NMF) runs on summaries computed elsewhere, e.g. by a reference
 * implementation, so it can be checked on its own; it also resumes a
 * recording whose summaries were kept. All pointers are host memory:
 *   T, S, D  float [k][height][width]   Eq. 2, Eq. 1, noise-scale term D_i
 *   U        float [k][height][width]   sum over the segment of V - R_i
 *   P        float [5][k][height][width] sums over the segment of
 *            (V(x) - R_i(x)) (V(y) - R_i(y)) for y = x, x + (0,1), x + (1,0),
 *            x + (1,1), x + (1,-1), with R_i any per-pixel integer reference
 * U and P may be NULL (the correlation image is then 0). The session must be
 * fresh (nothing pushed). A SEG_DET_UNET session runs its network on the
 * loaded S and T here (its model must be set: SEG_E_NOMODEL); a
 * SEG_DET_SURROGATE session cannot load summaries (SEG_E_STATE), since its
 * maps come from the frames. Errors: SEG_E_INVAL, SEG_E_STATE,
 * SEG_E_CAPACITY, SEG_E_NOMODEL, SEG_E_DEVICE. */
int seg_load_summaries(seg_session* s, uint32_t k, const float* T,
                       const float* S, const float* D, const float* U,
                       const float* P);

/* ---- serving: several recordings in one launch (continuous batching) ----
 *
 * A batch object owns a slot table that describes, for every session of a
 * push, where its frames and per-segment outputs are. The streaming kernel
 * is captured once in a HIP graph whose launch reads that table from device
 * memory, so each push rewrites the table (one host-to-device copy) and
 * replays the graph. Every session's result is the same as when it is
 * pushed alone: each (segment, tile) item runs the same code on the same data.
 * Pushes of one batch object may use different streams: each push orders its
 * table upload after the previous push's replay.
 */
typedef struct seg_batch seg_batch;   /* opaque */

/* Device bytes of a batch table for up to max_slots sessions (<= 64). */
int seg_batch_bytes(uint32_t max_slots, size_t* bytes);

/* Create a batch object using the caller's device memory dev_table (at least
 * seg_batch_bytes bytes, 256-byte aligned); it also allocates a pinned host
 * copy of the table. Errors: SEG_E_INVAL, SEG_E_CAPACITY, SEG_E_DEVICE. */
int seg_batch_create(uint32_t max_slots, void* dev_table, size_t bytes, seg_batch** out);

/* Append n_frames[k] frames (dev_frames[k], device memory) to sessions[k] for
 * k < count, as seg_push_frames would, with one graph launch on `stream` for
 * all complete segments. Sessions must be distinct, open, on the batch's
 * device and use the plain detector. All checks happen before anything is launched: on error nothing is
 * pushed. Errors: SEG_E_INVAL, SEG_E_STATE, SEG_E_CAPACITY, SEG_E_DEVICE. */
int seg_push_batch(seg_batch* b, seg_session* const* sessions,
                   const uint16_t* const* dev_frames, const uint32_t* n_frames,
                   uint32_t count, void* stream);

/* Release the batch object (not the caller's device table). */
int seg_batch_destroy(seg_batch* b);

/* Attach the network of a learned detector (before the first push). For
 * SEG_DET_SURROGATE a frame network (seg_nn_create) of the session's height
 * and width; for SEG_DET_UNET a summary network (seg_nn_st_create) of
 * 64 x 64 patches, run on each segment's patches as the push completes it
 * (and on every segment given to seg_load_summaries). The network is used on
 * the push stream and must outlive the session's pushes.
 * Errors: SEG_E_INVAL, SEG_E_STATE, SEG_E_SHAPE (wrong network shape or
 * input). */
int seg_set_model(seg_session* s, struct seg_nn* net);

/* Release the session (not the caller's workspace). NULL is a no-op. */
int seg_destroy(seg_session* s);

/* Checkpoint and resume of an open session (a long recording, or moving it
 * to another device). The state is what later pushes and the finalize need:
 * the frames carried toward the next segment and every completed segment's
 * summaries (T, S, D, U and the five co-moment sums; for the surrogate
 * detector also its probability maps), behind a header with the
 * configuration. Copies are ordered on `stream` and complete on return.
 *
 * seg_state_bytes: host bytes seg_export_state writes for this session now.
 * seg_export_state: write the state to `host` (at least seg_state_bytes).
 *   Errors: SEG_E_INVAL, SEG_E_STATE (finalized), SEG_E_CAPACITY (buffer too
 *   small), SEG_E_DEVICE.
 * seg_import_state: restore a state into a fresh session (nothing pushed)
 *   created with the same configuration; pushes then continue where the
 *   exported session stopped, with bit-identical results. Errors: SEG_E_INVAL
 *   (NULL, not a state, or another configuration), SEG_E_STATE (session not
 *   fresh), SEG_E_CAPACITY (buffer shorter than the state), SEG_E_DEVICE. */
int seg_state_bytes(const seg_session* s, size_t* bytes);
int seg_export_state(seg_session* s, void* host, size_t bytes, void* stream);
int seg_import_state(seg_session* s, const void* host, size_t bytes, void* stream);

/* Device timing and work of the last seg_finalize (from HIP events recorded
 * on the caller's stream around the launches; no extra synchronisation). */
typedef struct seg_profile {
  float    maps_ms;          /* events, regions, aggregation, components (a7-a9) */
  float    nmf_ms;           /* the per-component NMF launch (a10)               */
  double   nmf_flops;        /* its algorithmic FP64 operations: SPA steps plus
                                HALS products F^T P, P A^T (2 M_c K N each), the
                                Gram matrices and the row/column updates         */
  uint32_t nmf_path;         /* SEG_NMF_SINGLE or SEG_NMF_SPLIT as taken         */
  uint32_t nmf_workgroups;   /* workgroups of that launch                        */
  uint32_t components;       /* components of the aggregate mask                 */
  uint32_t max_rank;         /* largest SPA rank among them                      */
} seg_profile;

/* Fill *out for the last seg_finalize. Errors: SEG_E_INVAL (NULL),
 * SEG_E_STATE (not finalized). */
int seg_get_profile(const seg_session* s, seg_profile* out);

/* Static description of a status code. */
const char* seg_strerror(int code);

/* The sticky error of a session (SEG_OK if none). */
int seg_last_error(const seg_session* s);

#ifdef __cplusplus
}
#endif

#endif /* SEG_H */
