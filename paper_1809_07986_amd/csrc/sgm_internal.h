// Internal declarations shared by the kernels and the C ABI of the gfx950
// library (reduced-space SGM + per-pixel Kalman filter).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sgm.h"

namespace sgmk {

constexpr int kMaxDisp = 256;          // windows are packed as (lo, width-1) bytes
constexpr int kMaxPaths = 8;
constexpr int kCnnLayers = 5;          // learned window network
constexpr int kHMaxSeg = 86;           // horizontal aggregation: segments per scanline (>= 4096 / 48)
constexpr int kDetMaxSizes = 8;         // moving-object detection: window sizes
constexpr int kDetMaxBoxes = 2048;      // moving-object detection: windows kept for grouping (LDS-resident)

// Device-side layout of one context.  Per-pixel arrays have N = W*H
// entries in raster order; cost-volume arrays have N*D entries (the worst
// case: every window full range), of which the first M = off[N] are used.
struct DevBuffers {
    uint64_t *cen_l, *cen_r;   // census strings
    uint16_t *win;             // window: lo | (width-1) << 8
    uint32_t *off;             // ragged offsets, N+1
    uint32_t *scan_part;       // scan partial sums
    uint8_t *cost;             // Hamming cost per cell
    uint8_t *lr;               // L_r per enabled path, stride N*D
    uint16_t *sum;             // S per cell (debug only)
    double *d, *p;             // filter state
    uint8_t *sflags, *mask;    // RESET for the next frame, moving mask
    double *dhat, *pm;         // prediction
    uint8_t *flags;            // SGM_FLAG_* of the frame
    int32_t *dstar;            // integer winner
    double *dz;                // sub-pixel measurement
    // splatting scratch
    unsigned long long *zkey;  // max d' bits per target
    uint32_t *zidx;            // min source index among the max-d' sources
    int32_t *tgt;              // target per source (-1 dropped)
    double *dprime, *pprime;   // splatted disparity / variance per source
    uint8_t *has, *rw;
    double *dw, *pw;
    uint32_t *status;
    uint32_t *rerun;           // gate re-run counters and switches of this frame [RR_WORDS]
    uint8_t *moved;            // gate re-run: widened pixel whose window was not the full range
    uint8_t *touched;          // gate re-run: pixel whose second-pass result may differ from the first
    uint32_t *woff;            // gate re-run: offset of a moved pixel's full-range block
    uint8_t *hflag;            // horizontal aggregation: flagged segments [2][H][kHMaxSeg]
    // learned window (allocated in learned mode only, except nu / nu_w)
    double *nu;                // innovation of the last frame (0 without prediction)
    double *nu_w;              // previous innovation of each pixel's warp winner
    uint16_t *feat;            // network input, bfloat16 [N][4]
    uint16_t *act_a, *act_b;   // activations, bfloat16 [N][32] each
    float *cnn_out;            // network output [N][2]
    float *hw, *rpix;          // half-width and measurement variance per pixel
    int32_t *kappa;            // curvature of the sub-pixel parabola (r_curv > 0 contexts)
    float *theta;              // network parameters (fp32)
    uint64_t *frag;            // bfloat16 MFMA operands of the parameters
};

// gate re-run counter block (DevBuffers::rerun), zeroed before each second pass
enum {
    RR_NW = 0,        // pixels widened by the innovation test
    RR_NMOVED,        // ... of them, pixels whose window was narrower than the full range
    RR_EXTRA,         // cells the widening adds (sum of D - width over the widened pixels)
    RR_M1,            // cells of the first pass
    RR_RANK,          // full-range blocks handed out so far
    RR_SKIP_DENSE,    // skip word of the dense second pass: 0 unless the blocks did not fit
    RR_SKIP_SPARSE,   // skip word of the sparse second pass: 0 when it does not run
    RR_WORDS = 8
};

struct Geometry {
    int W, H, D, N;
    size_t lr_stride;          // bytes between the path-loss buffers: N*D rounded up to 256
    int hseg;                  // horizontal aggregation: pixels per scanline segment (72, or 48 in debug)
    bool halt;                 // reduced frames: the other horizontal kernel than the size-based choice
    bool rr_dense;             // gate re-run: always take the dense second pass's fallback route (debug)
    bool rr_room;              // gate re-run: the path buffers hold N*D cells more, so the sparse pass always fits
    int cw, ch, nbits;
    int p1, p2;
    int npaths;
    int8_t rx[kMaxPaths], ry[kMaxPaths];
};

struct WarpConst {
    double T[12];          // rows of [R | t]
    double f, cx, cy, B, fB, zmin, q;
};

struct CorrectConst {
    double r, gate, k_sigma, disc;
    double curv;           // > 0: per-pixel r = curv / kappa of the sub-pixel parabola (clamped)
};

// kernel launchers (all asynchronous on `s`); return hipError_t of the launch
hipError_t launch_census(const Geometry &g, const uint8_t *left, const uint8_t *right, int pitch,
                         uint64_t *cl, uint64_t *cr, hipStream_t s);
hipError_t launch_full_windows(const Geometry &g, DevBuffers &b, hipStream_t s);
hipError_t launch_given_windows(const Geometry &g, DevBuffers &b, const int32_t *lo, const int32_t *hi,
                                hipStream_t s);
// Tdev: ego-motion in device memory (row-major 4x4), or NULL to use wc.T
hipError_t launch_predict(const Geometry &g, DevBuffers &b, const WarpConst &wc, const double *Tdev,
                          const CorrectConst &cc, hipStream_t s);
hipError_t launch_cost(const Geometry &g, DevBuffers &b, hipStream_t s);
// Eq. 1 aggregation: horizontal paths (one scanline per wave) and the
// vertical + diagonal paths (16 scanlines per block); the two launches are
// independent and may run on different streams.
int count_horizontal_paths(const Geometry &g);
// dense: every window is the full range (the full-frame kernels)
// skip: when not NULL, the launches of a second (gate re-run) pass read *skip on
// the device and do nothing when it is 0 (no pixel was widened)
hipError_t launch_agg_h(const Geometry &g, DevBuffers &b, bool dense, hipStream_t s, const uint32_t *skip = nullptr);
hipError_t launch_agg_v(const Geometry &g, DevBuffers &b, bool dense, hipStream_t s, const uint32_t *skip = nullptr);
// mode 0: full frame (restart filter), 1: reduced frame (Kalman), 2: matcher only;
// rpix: per-pixel measurement variance (NULL: cc.r); sparse: only the pixels the
// gate re-run's sparse second pass marked, the moved ones read from their
// full-range blocks
hipError_t launch_wta_correct(const Geometry &g, DevBuffers &b, const CorrectConst &cc, int mode,
                              bool debug_sum, const float *rpix, hipStream_t s, const uint32_t *skip = nullptr,
                              bool sparse = false);
// prediction without the offset scan (launch_predict = this + launch_scan)
hipError_t launch_predict_core(const Geometry &g, DevBuffers &b, const WarpConst &wc, const double *Tdev,
                               const CorrectConst &cc, hipStream_t s);
hipError_t launch_scan(const Geometry &g, DevBuffers &b, hipStream_t s, const uint32_t *skip = nullptr);

// learned window (sgm_cnn.hip)
size_t cnn_frag_count();
size_t cnn_part_floats();
size_t cnn_loss_part_floats();
hipError_t cnn_pack(const float *theta, uint64_t *frag, hipStream_t s);
hipError_t cnn_forward(const float *theta, const uint64_t *frag, const uint16_t *x, int nimg, int H, int W,
                       uint16_t *a1, uint16_t *a2, uint16_t *a3, uint16_t *a4, float *out, hipStream_t s);
hipError_t cnn_backward(const float *theta, const uint64_t *frag, const uint16_t *x, const uint16_t *a1,
                        const uint16_t *a2, const uint16_t *a3, const uint16_t *a4, const uint16_t *dz5, int nimg,
                        int H, int W, uint16_t *g0, uint16_t *g1, float *part, float *grad, hipStream_t s);
hipError_t cnn_loss(const float *out, const float *tgt, size_t P, float *cnt, float *part, uint16_t *dz,
                    float *loss, hipStream_t s);
hipError_t cnn_adam(float *theta, float *m, float *v, const float *g, int step, float lr, hipStream_t s);
hipError_t launch_features(const Geometry &g, const DevBuffers &b, const uint8_t *left, int pitch, uint16_t *feat,
                           hipStream_t s);
// a frame's window network: input, five layers and head (five launches)
hipError_t cnn_forward_frame(const Geometry &g, DevBuffers &b, const uint8_t *left, int pitch, float k_sigma,
                             hipStream_t s);
// gate re-run: widen the windows of the pixels that failed the innovation test
// (counts into b.rerun).  sparse: also mark them for the sparse second pass,
// place the full-range blocks and set the two skip words
hipError_t launch_gate_widen(const Geometry &g, DevBuffers &b, bool sparse, hipStream_t s);
// blocks of the widening kernels (3 counters each follow the RR_WORDS of DevBuffers::rerun)
int gate_parts(const Geometry &g);
// the sparse second pass's scanline walks (all enabled paths, one launch)
hipError_t launch_rerun_walk(const Geometry &g, DevBuffers &b, hipStream_t s);
hipError_t launch_targets(const Geometry &g, const DevBuffers &b, const double *dz_full, const float *gt, float *tgt,
                          hipStream_t s);
hipError_t launch_windows_to_lohi(const Geometry &g, const DevBuffers &b, int32_t *out, int which,
                                  hipStream_t s);
hipError_t launch_state_to_f32(const Geometry &g, const double *src, float *dst, int pitch, hipStream_t s);
hipError_t launch_copy_u8(const Geometry &g, const uint8_t *src, uint8_t *dst, int pitch, hipStream_t s);
// injected state: count invalid entries into *bad (zeroed first); copy into the context
hipError_t launch_check_state(const Geometry &g, const double *d, const double *p, uint32_t *bad, hipStream_t s);
hipError_t launch_load_state(const Geometry &g, DevBuffers &b, const double *d, const double *p, const uint8_t *sf,
                             hipStream_t s);
hipError_t launch_median3x3(const Geometry &g, const double *src, float *dst, int pitch, hipStream_t s);

// moving-object detection: window grid and grouping settings (kernel argument)
struct DetectGeom {
    int W, H, top, rows;                // rows = H - top scanned rows
    int nsizes;
    int w[kDetMaxSizes], h[kDetMaxSizes];
    int sx[kDetMaxSizes], sy[kDetMaxSizes];   // window steps
    int nx[kDetMaxSizes];                     // windows per row of windows
    int base[kDetMaxSizes + 1];               // first window index of each size; base[nsizes] = total
    int scale, cap, thresh, maxdet;
    long long min_area;
    double merge_iou;
};
hipError_t launch_detect(const DetectGeom &dg, const double *dhat, const double *dz, const uint8_t *flags,
                         uint32_t *colp, uint32_t *sat, uint8_t *fire, int32_t *boxes, int32_t *count, hipStream_t s);

}  // namespace sgmk
