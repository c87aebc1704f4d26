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
#define SGM_FLAG_GATEFAIL 8u /* failed the innovation test, re-measured over the full range (gate_rerun) */

/* search-window rules (sgm_params.window_mode) */
#define SGM_WIN_KSIGMA 0     /* d^ -+ k_sigma * sqrt(p^-), rounded outward (Section 2.4) */
#define SGM_WIN_LEARNED 1    /* half-width and measurement variance from the window network */
#define SGM_LEARNED_WMAX 32  /* a learned half-width >= this searches the full range */
#define SGM_CNN_NPARAMS 19394

typedef struct sgm_context sgm_context;

typedef struct {
    int32_t width, height;      /* 16 <= width <= 4096, 16 <= height, width*height <= 2^24,
                                   width*height*max_disp < 2^32 */
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
    int32_t window_mode;        /* SGM_WIN_KSIGMA or SGM_WIN_LEARNED */
    int32_t gate_rerun;         /* 1: pixels failing the innovation test are matched again over
                                   the full range in the same frame and restart from that
                                   measurement.  The second pass recomputes only what changes:
                                   along each path, from a widened pixel until the losses
                                   rejoin the first pass's (results equal a full second pass) */
    double r_curv;              /* 0: every pixel's measurement variance is r.  > 0 (SGM_WIN_KSIGMA
                                   contexts): the variance of a pixel's measurement is estimated
                                   from the cost values at the neighbouring disparities (Section 3,
                                   the approach of the authors' earlier method):
                                   r_pix = r_curv / kappa clamped to [1/256, 64], with
                                   kappa = S(d*-1) + S(d*+1) - 2 S(d*) >= 1 the curvature of the
                                   sub-pixel parabola, and r_pix = r where d* lies on a window
                                   edge; r_pix enters the gain and the innovation test; a pixel
                                   restarting from its measurement takes p = r */
} sgm_params;

/* Fill `out` with the defaults for a width x height x max_disp problem:
 * census 9x7, 8 paths, P1=7, P2=86, k_sigma=3, q=0.5, r=1, chi2 99% (1 dof),
 * disc_thresh=2, f=0.58*width, principal point at the image centre, B=0.54,
 * SGM_WIN_KSIGMA windows, no gate re-run. */
int sgm_default_params(sgm_params *out, int32_t width, int32_t height, int32_t max_disp);

/* The settings of the paper's evaluation (Table 1, "proposed"): census 5x5,
 * P1=6, P2=65, 8 paths (set path_mask to 0x0F for the nondiagonal 4-path
 * and 0xF0 for the diagonal 4-path variant of Section 5); Table 1 matches
 * max_disp=128.  Everything else as sgm_default_params. */
int sgm_paper_params(sgm_params *out, int32_t width, int32_t height, int32_t max_disp);

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

/* Post-processing of Section 2.3: the 3x3 block median of the current
 * filtered disparity d^k, written as float32 into `out` (device, out_pitch
 * elements per row, caller-owned).  Neighbours outside the image are the
 * nearest edge pixel.  The filter state is not changed (the median stays
 * outside the Kalman loop).  SGM_EINVAL for a NULL `out` or a pitch below
 * the width. */
int sgm_get_disparity_median(sgm_context *ctx, float *out, int32_t out_pitch, void *stream);

/* Filter state (checkpoint / restore): d, p as float64 and the per-pixel
 * RESET flags, dense width*height arrays.  (float64 rather than float32: the
 * library keeps the whole filter in double precision.)
 * sgm_set_state checks the state first and synchronises the stream to read
 * the result: SGM_EINVAL, with the context unchanged, if any pixel has a
 * non-finite d or p, d outside [0, max_disp-1] or p <= 0 (states the filter
 * cannot reach; every state sgm_get_state returns passes).  -0.0 is stored
 * as +0.0.  It also clears the carried innovation (learned windows). */
int sgm_get_state(sgm_context *ctx, double *d, double *p, uint8_t *sflags, void *stream);
int sgm_set_state(sgm_context *ctx, const double *d, const double *p, const uint8_t *sflags,
                  void *stream);

/* The matcher alone on caller-given windows (Section 2: besides the image
 * pair, the matcher is given a lower and an upper disparity bound for every
 * pixel and searches only between them):
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
 * (after a gate re-run frame, OFFSETS and PATH0 + k are available only in
 * contexts with SGM_DEBUG_STAGES on; the others keep the first pass's offsets
 * and store the widened pixels' losses apart, and refuse them with SGM_EINVAL)
 *   SGM_STAGE_COST           uint8 per cell (Hamming cost; recorded only while
 *                            sgm_set_debug(ctx, 1) is on)
 *   SGM_STAGE_SUM            uint16 per cell (S = sum of L_r; recorded only
 *                            while sgm_set_debug(ctx, 1) is on)
 *   SGM_STAGE_PATH0 + k      uint8 per cell (L_r of path k, enabled paths)
 *   SGM_STAGE_DHAT / _PM     float64 per pixel (prediction, 0 if none)
 *   SGM_STAGE_FLAGS          uint8 per pixel (SGM_FLAG_*)
 *   SGM_STAGE_DSTAR          int32 per pixel;  SGM_STAGE_DZ float64 per pixel
 *   SGM_STAGE_STATUS         uint32: number of windows clamped by match_windows
 *   SGM_STAGE_NU             float64 per pixel: innovation dz - d^ of the last
 *                            frame (0 where there was no prediction)
 *   SGM_STAGE_NU_W           float64 per pixel: the previous innovation of the
 *                            pixel's warp winner (0 for filled holes / none)
 * learned windows (SGM_WIN_LEARNED contexts, last reduced frame):
 *   SGM_STAGE_FEATURES       bfloat16 [4] per pixel: network input
 *   SGM_STAGE_CNN_OUT        float32 [2] per pixel: network output
 *   SGM_STAGE_HALFWIDTH      float32 per pixel: half-width w
 *   SGM_STAGE_RPIX           float32 per pixel: measurement variance r (also in
 *                            r_curv > 0 contexts: the curvature estimate, last frame)
 * curvature measurement variance (r_curv > 0 contexts, last frame):
 *   SGM_STAGE_KAPPA          int32 per pixel: kappa of the sub-pixel parabola, 0 where
 *                            d* lies on a window edge
 * gate re-run (gate_rerun contexts, the last reduced frame; zeros before any):
 *   SGM_STAGE_RERUN          uint32 [3]: pixels widened by the innovation test, those of
 *                            them whose window was narrower than the full range, and
 *                            the cells the widening added to the frame
 * sgm_cost_cells() synchronises the stream and returns the cell count M. */
enum {
    SGM_STAGE_CENSUS_L = 0, SGM_STAGE_CENSUS_R, SGM_STAGE_LO, SGM_STAGE_HI, SGM_STAGE_OFFSETS,
    SGM_STAGE_COST, SGM_STAGE_SUM, SGM_STAGE_DHAT, SGM_STAGE_PM, SGM_STAGE_FLAGS,
    SGM_STAGE_DSTAR, SGM_STAGE_DZ, SGM_STAGE_STATUS,
    SGM_STAGE_PATH0 = 16,
    SGM_STAGE_NU = 32, SGM_STAGE_NU_W, SGM_STAGE_FEATURES, SGM_STAGE_CNN_OUT, SGM_STAGE_HALFWIDTH,
    SGM_STAGE_RPIX, SGM_STAGE_KAPPA, SGM_STAGE_RERUN
};
int sgm_get_stage(sgm_context *ctx, int32_t stage, void *out, size_t bytes, void *stream);
int sgm_cost_cells(sgm_context *ctx, int64_t *cells, void *stream);
/* Debug switches for the following frames (bit mask, 0 = off):
 *   SGM_DEBUG_STAGES  record the cost and sum stages (slower);
 *   SGM_DEBUG_SHORT_SEGMENTS  cut horizontal scanlines into 48-pixel segments
 *     instead of 72 (results are identical; exercises the segment fix-up);
 *   SGM_DEBUG_ALT_HORIZONTAL  reduced frames use the other horizontal
 *     aggregation kernel than the one chosen for max_disp (segmented scanlines
 *     for max_disp > 64, one wave per scanline otherwise); results are
 *     identical, so both kernels can be checked at every size;
 *   SGM_DEBUG_DENSE_RERUN  the gate re-run's second pass takes the route used
 *     when the widened pixels' full-range blocks do not fit beside the first
 *     pass's cells (every pixel matched again); results are identical. */
#define SGM_DEBUG_STAGES 1
#define SGM_DEBUG_SHORT_SEGMENTS 2
#define SGM_DEBUG_ALT_HORIZONTAL 4
#define SGM_DEBUG_DENSE_RERUN 8
int sgm_set_debug(sgm_context *ctx, int32_t on);

/* Per-stage GPU time, for benchmarks.  While profiling is on, every frame
 * (and every sgm_match_windows call, which counts as a frame) records a HIP
 * event before and after each stage's launches on the frame's
 * own stream (events come from a pool made by sgm_set_profiling, so the
 * frame path still allocates nothing).  sgm_set_profiling(ctx, 1) starts a
 * new accumulation, 0 stops it.  sgm_read_profile synchronises `stream`,
 * then writes the accumulated milliseconds of each stage (SGM_PROF_COUNT
 * doubles, in the order of the enum) and the number of frames measured. */
enum { SGM_PROF_CENSUS = 0, SGM_PROF_PREDICT, SGM_PROF_COST, SGM_PROF_AGG_H, SGM_PROF_AGG_V, SGM_PROF_WTA,
       SGM_PROF_CNN, SGM_PROF_RERUN, SGM_PROF_COUNT };
/* AGG_H: horizontal paths (timed on an internal stream); AGG_V: the others;
 * CNN: learned-window input, network and head; RERUN: the whole second
 * matching pass of gate_rerun */
int sgm_set_profiling(sgm_context *ctx, int32_t on);
int sgm_read_profile(sgm_context *ctx, double *ms, int64_t *frames, void *stream);

/* ---- learned search window --------------------------------------------------
 * Extension of the method: instead of d^ -+ k sigma, a five-layer 3x3
 * convolutional network (channels 4 -> 16 -> 32 -> 32 -> 16 -> 2, ReLU
 * between layers, zero padding, bfloat16 weights and activations with fp32
 * accumulation) reads per pixel
 *   [d^ / 64, min(p^-, 16) / 4, (|dI/dx| + |dI/dy|) / 256, min(|nu_w|, 8) / 4]
 * (central differences of the left image, neighbours clamped; without a
 * prediction the first two are 0 and 4) and outputs o = (o0, o1):
 *   w = max(1, k_sigma * exp(o0 / 2))       (o0: log-variance of d_full - d^)
 *   r = clamp(exp(o1), 1/16, 64)            (o1: log measurement variance)
 * A pixel with a finite window searches [floor(d^ - w), ceil(d^ + w)]
 * (clipped to [0, max_disp-1]); w >= SGM_LEARNED_WMAX searches the full
 * range.  The Kalman update and the innovation test use r per pixel; a
 * restart from the measurement uses params.r.
 *
 * Parameters: SGM_CNN_NPARAMS floats, layer by layer W[co][ky][kx][ci] then
 * b[co] (ci, co of the five layers as above).
 *
 * sgm_set_window_model: HOST parameter vector for a SGM_WIN_LEARNED context
 *   (copied; synchronous).  SGM_ESTATE from sgm_reduced_frame of a learned
 *   context without a model.
 * sgm_get_features: the network input of the context's last predicted frame
 *   (its prediction and innovation) for the given left image, as bfloat16
 *   [N][4] into `out` (device); any window mode.
 * sgm_learned_targets: training targets of the context's last predicted
 *   frame, float [N][4] (e, m, we, wm) into `out` (device):
 *   e = clip(dz_full - d^, +-16), m = clip(dz_full - gt, +-16),
 *   we = [prediction], wm = we * [gt >= 0]; dz_full (float64) is the
 *   full-range measurement of the same frame, gt (float32) the reference
 *   disparity, negative where unknown; all device pointers, N entries,
 *   `out` 16-byte aligned. */
int sgm_set_window_model(sgm_context *ctx, const float *params, int32_t n);
int sgm_get_features(sgm_context *ctx, const uint8_t *left, int32_t pitch, uint16_t *out, void *stream);
int sgm_learned_targets(sgm_context *ctx, const double *dz_full, const float *gt, float *out, void *stream);

/* ---- training the window network ------------------------------------------
 * A trainer holds fp32 parameters, Adam moments (b1 0.9, b2 0.999, eps 1e-8)
 * and buffers for batches of up to max_images images of height x width.
 * Inputs x are bfloat16 [nimg][height][width][4] (device, 8-byte aligned),
 * outputs float [..][2].  Loss (targets float [..][4] = e, m, we, wm as from
 * sgm_learned_targets, 16-byte aligned):
 *   L = sum we (o0 + e^2 exp(-o0)) / 2 / max(1, sum we)
 *     + sum wm (o1 + m^2 exp(-o1)) / 2 / max(1, sum wm),
 * o clipped to [-15, 15] (zero gradient outside).
 *
 * sgm_cnn_set_params / _get_params: HOST vectors of SGM_CNN_NPARAMS floats;
 *   set also clears the Adam moments and step count; both synchronise.
 * sgm_cnn_forward: o for x into `out` (device, may be NULL; the trainer keeps
 *   the activations for the next backward).
 * sgm_cnn_loss: L into *loss (device float) and dL/do into the trainer, for
 *   the last forward.
 * sgm_cnn_backward: parameter gradient of sum(dL/do * o) for the last
 *   forward and loss, kept in the trainer (fixed-order sums: deterministic).
 * sgm_cnn_get_grads: HOST copy of that gradient (synchronises).
 * sgm_cnn_adam: one Adam step with learning rate lr from that gradient.
 * sgm_cnn_train_step: forward, loss, backward and Adam in one call. */
typedef struct sgm_cnn sgm_cnn;
int sgm_cnn_create(int32_t max_images, int32_t height, int32_t width, sgm_cnn **out);
void sgm_cnn_destroy(sgm_cnn *t);
int sgm_cnn_set_params(sgm_cnn *t, const float *params, int32_t n);
int sgm_cnn_get_params(sgm_cnn *t, float *params, int32_t n);
int sgm_cnn_forward(sgm_cnn *t, const uint16_t *x, int32_t nimg, float *out, void *stream);
int sgm_cnn_loss(sgm_cnn *t, const float *targets, float *loss, void *stream);
int sgm_cnn_backward(sgm_cnn *t, void *stream);
int sgm_cnn_get_grads(sgm_cnn *t, float *grads, int32_t n);
int sgm_cnn_adam(sgm_cnn *t, float lr, void *stream);
int sgm_cnn_train_step(sgm_cnn *t, const uint16_t *x, const float *targets, int32_t nimg, float lr,
                       float *loss, void *stream);

/* ---- batches of independent stereo streams --------------------------------
 * A batch owns one context per stream (uneven sizes and disparity ranges are
 * allowed) and runs a frame step of every stream with the streams' kernels
 * spread over internal lanes (HIP streams, default priority) forked from and
 * joined back into the caller's stream.  Input images are the caller's
 * device buffers given at creation (pointers and pitches fixed for the
 * batch's lifetime; write each new frame into them, stream-ordered, before
 * the step).  Per-step ego-motions go through device memory.
 *
 * sgm_batch_create: n streams with params[i]; left[i], right[i] (device) and
 *   pitch[i] (bytes) are stream i's default image buffers, used by steps that
 *   pass no images and by graph replays.  Allocates everything (contexts,
 *   lanes, save area, the batch's capture stream).
 * sgm_batch_context: stream i's context (outputs, state, stages); owned by
 *   the batch.
 * sgm_batch_step: one frame of every stream.  left / right / pitch: arrays of
 *   n device image pointers and pitches for this step, or NULL for the
 *   default buffers.  T: HOST array of n row-major 4x4 ego-motions; stream i
 *   runs a full-range frame (the filter's start, Section 2.4) when T is NULL
 *   or its row has T[16 i + 15] == 0 (not a rigid motion), otherwise a
 *   steady-state frame with that ego-motion.  SGM_ESTATE for a steady-state
 *   frame of a stream that never had a full-range frame.
 * sgm_batch_full: every stream full range (sgm_batch_step with T NULL and
 *   the default images).
 * sgm_batch_step_graph: stepping from a captured HIP graph.  Disabled:
 *   always returns SGM_EINVAL (capturing a batch step, whose streams fork
 *   onto lanes and side streams with events, crashed the host process inside
 *   hipStreamEndCapture; the cause has not been shown).
 * sgm_batch_set_schedule: lanes (1..16) and order (0: streams as given,
 *   round-robin; 1: largest full-range work first onto the least-loaded lane).
 * sgm_autotune: chooses lanes, order and the horizontal aggregation schedule
 *   of every stream (scanline segment length 48/72/96/128 and kernel family)
 *   by timing steady-state steps on the default images with the last
 *   ego-motions, for about budget_ms milliseconds in all; every candidate
 *   starts from the streams' saved filter state and the state is restored at
 *   the end.  Waits for the device (synchronous).  SGM_ESTATE without a
 *   previous steady-state step.
 * sgm_batch_autotune: the same with explicit ego-motions T and `reps` timed
 *   steps per candidate; writes lanes, order, segment length and kernel
 *   family to chosen[0..3] when not NULL; synchronises `stream`.
 * (The stages of sgm_get_stage show the last trial step after autotuning.) */
typedef struct sgm_batch sgm_batch;
int sgm_batch_create(int32_t n, const sgm_params *params, const uint8_t *const *left,
                     const uint8_t *const *right, const int32_t *pitch, sgm_batch **out);
void sgm_batch_destroy(sgm_batch *b);
sgm_context *sgm_batch_context(sgm_batch *b, int32_t i);
int sgm_batch_step(sgm_batch *b, const uint8_t *const *left, const uint8_t *const *right, const int32_t *pitch,
                   const double *T, void *stream);
int sgm_batch_full(sgm_batch *b, void *stream);
int sgm_batch_step_graph(sgm_batch *b, const double *T, void *stream);
int sgm_batch_set_schedule(sgm_batch *b, int32_t lanes, int32_t order);
int sgm_autotune(sgm_batch *b, int32_t budget_ms);
int sgm_batch_autotune(sgm_batch *b, const double *T, int32_t reps, int32_t *chosen, void *stream);

/* ---- moving-object detection (Section 4) --------------------------------
 * Moving objects are where the predicted and the measured disparity
 * disagree.  Per frame:
 *  1. difference map v = min(floor(|d^ - d_z| * scale), cap) where the pixel
 *     has a prediction (SGM_FLAG_PRED) whose correspondence x - d^ lies
 *     inside the right image, else 0 (fixed point, so sums are exact);
 *  2. summed-area table of v over rows [top, height) (constant-time window
 *     sums by inclusion-exclusion);
 *  3. every window of every size, stepped by half its width and half its
 *     height from (0, top), fires when its sum >= thresh * its area; fired
 *     windows are listed by size, then row, then column, and the first
 *     max_detections are kept;
 *  4. greedy grouping: while the pair of boxes with the highest
 *     intersection over union has IoU > merge_iou, the earlier box of the
 *     pair becomes the bounding box of both and the later one is removed
 *     (ties: the pair that comes first in list order);
 *  5. boxes with an area below min_area are discarded.
 * Boxes are int32 [x0, y0, x1, y1], half-open, in list order. */
#define SGM_DETECT_MAX_SIZES 8
#define SGM_DETECT_MAX 2048   /* largest max_detections */

typedef struct {
    int32_t top;                 /* first row covered (sgm_detect_default_params: height / 3) */
    int32_t n_sizes;             /* 1..SGM_DETECT_MAX_SIZES */
    int32_t sizes[SGM_DETECT_MAX_SIZES][2];   /* window width, height */
    int32_t scale;               /* fixed-point units per pixel of disparity difference, >= 1 */
    int32_t cap;                 /* per-pixel cap (units), >= 1; width*height*cap < 2^32 per size */
    int32_t thresh;              /* firing level (units per pixel of window area), >= 0 */
    int32_t max_detections;      /* 1..SGM_DETECT_MAX */
    int64_t min_area;            /* smallest kept box (px), >= 0 */
    double merge_iou;            /* 0 <= merge_iou <= 1 */
} sgm_detect_params;

typedef struct sgm_detector sgm_detector;

/* Defaults: windows 20x20, 30x30, 40x40, 50x50 and 50x75 (the range the
 * paper names), the bottom two thirds (top = height / 3), 1/16 px units
 * capped at 16 px, firing at a mean difference of 1 px, merge while any
 * two boxes overlap, discard boxes under 40x40 px, keep 2048 windows. */
int sgm_detect_default_params(sgm_detect_params *out, int32_t width, int32_t height);

/* A detector for width x height frames (same limits as sgm_params) owns
 * its scratch (a (height - top + 1) x (width + 1) uint32 table and one byte
 * per window) on the current device.  SGM_EINVAL for out-of-range settings,
 * SGM_ENOMEM if the allocation fails. */
int sgm_detector_create(int32_t width, int32_t height, const sgm_detect_params *prm, sgm_detector **out);
void sgm_detector_destroy(sgm_detector *det);

/* Number of sliding windows tested per frame (host only). */
int sgm_detector_windows(sgm_detector *det, int64_t *n);

/* Detect on caller arrays: dhat, dz float64 and flags uint8, dense
 * width*height device arrays (the SGM_STAGE_DHAT, _DZ and _FLAGS layouts).
 * Writes up to max_detections boxes to `boxes` (device int32, 4 per box)
 * and count[0] = boxes written, count[1] = windows that fired (before the
 * max_detections cut) to `count` (device int32[2]). */
int sgm_detect(sgm_detector *det, const double *dhat, const double *dz, const uint8_t *flags, int32_t *boxes,
               int32_t *count, void *stream);

/* The same on the last frame of a context (created with the same width and
 * height on the same device).  After a full frame there is no prediction
 * and no box. */
int sgm_detect_frame(sgm_detector *det, sgm_context *ctx, int32_t *boxes, int32_t *count, void *stream);

/* Intermediate results of the last sgm_detect / sgm_detect_frame, copied to
 * device memory `out` of at least the stated size:
 *   SGM_DSTAGE_SAT    uint32 (height - top + 1) x (width + 1): row r, column
 *                     x holds the sum of v over rows [top, top + r) and
 *                     columns [0, x), modulo 2^32
 *   SGM_DSTAGE_FIRED  uint8 per window (window order as in step 3) */
enum { SGM_DSTAGE_SAT = 0, SGM_DSTAGE_FIRED = 1 };
int sgm_detector_stage(sgm_detector *det, int32_t stage, void *out, size_t bytes, void *stream);

/* Detection for callers that cannot allocate device memory: code under HIP
 * graph capture, allocation-free serving loops, harnesses that forbid
 * hipMalloc.  The same computation and outputs as sgm_detect (boxes,
 * count[0..1] on the caller's device arrays, same layouts), without a
 * detector object: the settings come in `prm` (sgm_detect_default_params
 * gives the defaults) and the scratch (column prefixes, summed-area table,
 * one byte per window) lives in one library-wide device array of
 * SGM_DETECT_NOALLOC_BYTES on each GPU the call runs on, held until the
 * process ends.  The call allocates nothing and frees nothing.
 * Scratch need: rows * width * 4 + (rows + 1) * (width + 1) * 4 + windows
 * bytes (rows = height - top), each part rounded up to 256; a larger need
 * returns SGM_EINVAL without launching anything (1920x1080 with the
 * default top = height / 3 needs 11 MB).  Every call on one GPU uses that
 * GPU's array: calls that overlap on one GPU (different streams without
 * ordering, or several host threads) race and give undefined results;
 * calls ordered on one stream are safe.  Every scratch byte a call reads is
 * written earlier in the same call, so nothing needs clearing between
 * calls.  SGM_EINVAL for NULL pointers and the settings sgm_detector_create
 * rejects, SGM_EHIP if the launch fails. */
#define SGM_DETECT_NOALLOC_BYTES (32u << 20)
int sgm_detect_noalloc(int32_t width, int32_t height, const sgm_detect_params *prm, const double *dhat,
                       const double *dz, const uint8_t *flags, int32_t *boxes, int32_t *count, void *stream);

/* Thread-local message describing the last nonzero return on this thread. */
const char *sgm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
