/*
 * sgm.h -- C ABI of the MI355X (gfx950) library for reduced-space semi-global
 * matching fused by a per-pixel Kalman filter.
 *
 * Method: Popovic, Hadviger, Markovic, Petrovic, "Computationally efficient
 * dense moving object detection based on reduced space disparity
 * estimation".  Section 2 defines the matcher (census cost, Eq. 1
 * aggregation, winner-takes-all) and the per-pixel filter (Eq. 2-6);
 * Section 4 defines moving objects as the places where the predicted and the
 * measured disparity disagree.
 *
 * Conventions shared by every entry point:
 *  - Image, state and output pointers are DEVICE pointers (HIP global
 *    memory).  The 4x4 ego-motion matrix is a HOST pointer and is copied into
 *    the launch arguments before the call returns.
 *  - `stream` is a hipStream_t (NULL = the default stream).  All work is
 *    enqueued on it and the call returns without waiting, except where a
 *    function says it synchronises.  Inputs must stay alive and unmodified,
 *    and outputs must not be read, until the stream has passed the call.
 *  - The context owns every scratch buffer and the filter state; it never
 *    allocates after sgm_create.  A context must not be used from two host
 *    threads at once; different contexts are independent.
 *  - Images are 8-bit, row-major, `pitch` bytes between rows (pitch >= width).
 *    Dense per-pixel arrays are row-major with width elements per row.
 *  - Return value: SGM_OK or a negative error code; on error nothing was
 *    enqueued and sgm_last_error() describes the failure.
 *  - Camera: rectified pair, x right, y down, z forward, right camera at
 *    +baseline along x, disparity d = x_left - x_right in [0, max_disp-1].
 */
#ifndef SGM_H
#define SGM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SGM_OK 0
#define SGM_EINVAL (-1)   /* bad dimensions, parameters or pointers */
#define SGM_ENOMEM (-2)   /* device allocation failed in sgm_create */
#define SGM_EHIP (-3)     /* a HIP runtime call or kernel launch failed */
#define SGM_ESTATE (-4)   /* sgm_reduced_frame before any full frame / set_state */

/* per-pixel flags of a frame (sgm_get_stage SGM_STAGE_FLAGS) */
#define SGM_FLAG_PRED 1u     /* a prediction exists (splat winner or filled hole) */
#define SGM_FLAG_RESET 2u    /* previous frame forced a full-range search here */
#define SGM_FLAG_FULLWIN 4u  /* this frame searched [0, max_disp-1] */

typedef struct sgm_context sgm_context;

typedef struct {
    int32_t width, height;      /* 16 <= width <= 4096, 16 <= height, width*height <= 2^24 */
    int32_t max_disp;           /* disparities 0..max_disp-1, 2 <= max_disp <= 256 */
    int32_t census_w, census_h; /* odd census window, census_w*census_h-1 <= 64 bits */
    uint32_t path_mask;         /* bit k enables path k: 0 (+1,0) 1 (-1,0) 2 (0,+1) 3 (0,-1)
                                   4 (+1,+1) 5 (-1,-1) 6 (-1,+1) 7 (+1,-1); 0x0F nondiagonal */
    int32_t p1, p2;             /* Eq. 1 penalties, 0 <= p1 <= p2, census bits + p2 + p1 <= 255 */
    double k_sigma;             /* search window half-width in standard deviations */
    double q, r;                /* process / measurement noise variance (px^2), Eq. 4 / Eq. 6 */
    double chi2_gate;           /* innovation test threshold on nu^2 / (p^- + r) */
    double disc_thresh;         /* discontinuity rejection threshold (px) */
    double f, cx, cy, baseline; /* focal length (px), principal point (px), baseline (m) */
} sgm_params;

/* Fill `out` with the defaults for a width x height x max_disp problem:
 * census 9x7, 8 paths, P1=7, P2=86, k_sigma=3, q=0.5, r=1, chi2 99% (1 dof),
 * disc_thresh=2, f=0.58*width, principal point at the image centre, B=0.54. */
int sgm_default_params(sgm_params *out, int32_t width, int32_t height, int32_t max_disp);

/* Validate `prm` and allocate a context with every device buffer it will
 * need (worst case: all windows full range).  Synchronous. */
int sgm_create(const sgm_params *prm, sgm_context **out);

/* Wait for the context's outstanding work on the device and free it. */
void sgm_destroy(sgm_context *ctx);

/* Full-range frame (Section 2.4: the limits initially cover the whole search
 * space, which is conventional SGM).  Every pixel searches [0, max_disp-1];
 * the filter restarts from the measurement: d = d_z, p = r, no motion. */
int sgm_full_frame(sgm_context *ctx, const uint8_t *left, const uint8_t *right, int32_t pitch,
                   void *stream);

/* Steady-state frame (Section 2.4, Eq. 2-6): predict the disparity and its
 * variance by splatting the previous state through the ego-motion
 * T_k_km1 (host, row-major 4x4, X_k = R X_{k-1} + t in metres), fill zoom
 * holes, reject predictions near discontinuities, match only inside
 * [d^ - k sigma, d^ + k sigma] (full range where there is no prediction or
 * a reset is pending), then run the Kalman correction and the innovation
 * test.  SGM_ESTATE if no full frame (or set_state) came first. */
int sgm_reduced_frame(sgm_context *ctx, const uint8_t *left, const uint8_t *right, int32_t pitch,
                      const double T_k_km1[16], void *stream);

/* Copy the current filter output into caller memory (out_pitch elements per
 * row): disparity d^k (Eq. 5) and variance p^k (Eq. 6) as float32, moving
 * mask (1 = the innovation failed the test, Section 4) as uint8. */
int sgm_get_disparity(sgm_context *ctx, float *out, int32_t out_pitch, void *stream);
int sgm_get_variance(sgm_context *ctx, float *out, int32_t out_pitch, void *stream);
int sgm_get_motion_mask(sgm_context *ctx, uint8_t *out, int32_t out_pitch, void *stream);

/* Filter state (checkpoint / restore): d, p as float64 and the per-pixel
 * RESET flags, dense width*height arrays. */
int sgm_get_state(sgm_context *ctx, double *d, double *p, uint8_t *sflags, void *stream);
int sgm_set_state(sgm_context *ctx, const double *d, const double *p, const uint8_t *sflags,
                  void *stream);

/* The matcher alone on caller-given windows (Section 2: "SGM also inputs
 * two values for each pixel that define the range for disparity search"):
 * lo, hi int32 per pixel, 0 <= lo <= hi < max_disp (checked on the device;
 * violations are clamped and reported by sgm_get_stage SGM_STAGE_STATUS).
 * Writes the integer winner d* (int32) and the sub-pixel measurement d_z
 * (float64).  Leaves the filter state untouched. */
int sgm_match_windows(sgm_context *ctx, const uint8_t *left, const uint8_t *right, int32_t pitch,
                      const int32_t *lo, const int32_t *hi, int32_t *dstar, double *dz, void *stream);

/* Intermediate results of the last frame, for tests and inspection.
 * Per-pixel stages are dense width*height arrays; cost-volume stages are
 * ragged: pixel p's cells d = lo[p]..hi[p] sit at [offset[p], offset[p+1])
 * in raster order of p.  `bytes` must equal the stage size:
 *   SGM_STAGE_CENSUS_L / _R  uint64 per pixel
 *   SGM_STAGE_LO / _HI       int32 per pixel (window of the last frame)
 *   SGM_STAGE_OFFSETS        uint32, width*height+1 entries
 *   SGM_STAGE_COST           uint8 per cell (Hamming cost; recorded only while
 *                            sgm_set_debug(ctx, 1) is on)
 *   SGM_STAGE_SUM            uint16 per cell (S = sum of L_r; recorded only
 *                            while sgm_set_debug(ctx, 1) is on)
 *   SGM_STAGE_PATH0 + k      uint8 per cell (L_r of path k, enabled paths)
 *   SGM_STAGE_DHAT / _PM     float64 per pixel (prediction, 0 if none)
 *   SGM_STAGE_FLAGS          uint8 per pixel (SGM_FLAG_*)
 *   SGM_STAGE_DSTAR          int32 per pixel;  SGM_STAGE_DZ float64 per pixel
 *   SGM_STAGE_STATUS         uint32: number of windows clamped by match_windows
 * sgm_cost_cells() synchronises the stream and returns the cell count M. */
enum {
    SGM_STAGE_CENSUS_L = 0, SGM_STAGE_CENSUS_R, SGM_STAGE_LO, SGM_STAGE_HI, SGM_STAGE_OFFSETS,
    SGM_STAGE_COST, SGM_STAGE_SUM, SGM_STAGE_DHAT, SGM_STAGE_PM, SGM_STAGE_FLAGS,
    SGM_STAGE_DSTAR, SGM_STAGE_DZ, SGM_STAGE_STATUS,
    SGM_STAGE_PATH0 = 16
};
int sgm_get_stage(sgm_context *ctx, int32_t stage, void *out, size_t bytes, void *stream);
int sgm_cost_cells(sgm_context *ctx, int64_t *cells, void *stream);
int sgm_set_debug(sgm_context *ctx, int32_t on);

/* Per-stage GPU time, for benchmarks.  While profiling is on, every frame
 * records a HIP event before and after each stage's launches on the frame's
 * own stream (events come from a pool made by sgm_set_profiling, so the
 * frame path still allocates nothing).  sgm_set_profiling(ctx, 1) starts a
 * new accumulation, 0 stops it.  sgm_read_profile synchronises `stream`,
 * then writes the accumulated milliseconds of each stage (SGM_PROF_COUNT
 * doubles, in the order of the enum) and the number of frames measured. */
enum { SGM_PROF_CENSUS = 0, SGM_PROF_PREDICT, SGM_PROF_COST, SGM_PROF_AGG_H, SGM_PROF_AGG_V, SGM_PROF_WTA,
       SGM_PROF_COUNT };   /* AGG_H: horizontal paths (timed on an internal stream); AGG_V: the others */
int sgm_set_profiling(sgm_context *ctx, int32_t on);
int sgm_read_profile(sgm_context *ctx, double *ms, int64_t *frames, void *stream);

/* ---- batches of independent stereo streams --------------------------------
 * A batch owns one context per stream (uneven sizes and disparity ranges are
 * allowed) and runs a frame step of every stream with the streams' kernels
 * spread over internal lanes (HIP streams, default priority) forked from and
 * joined back into the caller's stream.  Input images are the caller's
 * device buffers given at creation (pointers and pitches fixed for the
 * batch's lifetime; write each new frame into them, stream-ordered, before
 * the step).  Per-step ego-motions go through device memory.
 *
 * sgm_batch_create: n streams, params[i], left[i], right[i] device buffers,
 *   pitch[i] bytes.  Allocates everything (contexts, lanes, save area).
 * sgm_batch_context: stream i's context (outputs, state, stages); owned by
 *   the batch.
 * sgm_batch_full: full-range frame of every stream (Section 2.4 start).
 * sgm_batch_step: steady-state frame of every stream; T is a HOST array of
 *   n row-major 4x4 matrices.  SGM_ESTATE before sgm_batch_full.
 * sgm_batch_step_graph: stepping as a captured HIP graph.  Disabled: always
 *   returns SGM_EINVAL (its first run crashed the host process during stream
 *   capture; the cause has not been shown).
 * sgm_batch_set_schedule: lanes (1..16) and order (0: streams as given,
 *   round-robin; 1: largest full-range work first onto the least-loaded lane).
 * sgm_batch_autotune: times every (lanes, order) candidate over `reps` steps
 *   with ego-motions T, keeps the fastest (written to chosen[0], chosen[1]
 *   when not NULL) and restores every stream's filter state and motion mask
 *   (the per-frame stages of sgm_get_stage show the last trial step);
 *   synchronises the stream. */
typedef struct sgm_batch sgm_batch;
int sgm_batch_create(int32_t n, const sgm_params *params, const uint8_t *const *left,
                     const uint8_t *const *right, const int32_t *pitch, sgm_batch **out);
void sgm_batch_destroy(sgm_batch *b);
sgm_context *sgm_batch_context(sgm_batch *b, int32_t i);
int sgm_batch_full(sgm_batch *b, void *stream);
int sgm_batch_step(sgm_batch *b, const double *T, void *stream);
int sgm_batch_step_graph(sgm_batch *b, const double *T, void *stream);
int sgm_batch_set_schedule(sgm_batch *b, int32_t lanes, int32_t order);
int sgm_batch_autotune(sgm_batch *b, const double *T, int32_t reps, int32_t *chosen, void *stream);

/* Thread-local message describing the last nonzero return on this thread. */
const char *sgm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
