/*
 * Plain CPU oracle (test infrastructure only): reduced-space SGM fused by a
 * per-pixel Kalman filter.  Host pointers, dense arrays, double precision for
 * all floating-point state.  Used by the tests, the smoke check and the
 * benchmark's CPU baseline; never by the GPU library.
 */
#ifndef SGM_ORACLE_H
#define SGM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* per-pixel flags of a predicted frame */
#define ORC_PRED 1u     /* a prediction (warp winner or filled hole) survived */
#define ORC_RESET 2u    /* full-range search forced by the previous frame */
#define ORC_FULLWIN 4u  /* this frame searched [0, D-1] */
#define ORC_GATEFAIL 8u /* re-measured over [0, D-1] after failing the innovation test */
#define ORC_LEARNED_WMAX 32.0   /* a learned half-width at or above this means "full range" */

typedef struct {
    int32_t width, height, max_disp;
    int32_t census_w, census_h;
    uint32_t path_mask;
    int32_t p1, p2;
    double k_sigma, q, r, chi2_gate, disc_thresh;
    double f, cx, cy, baseline;
} orc_params;

int orc_census(const uint8_t *img, int W, int H, int cw, int ch, uint64_t *out);
int orc_cost(const uint64_t *cl, const uint64_t *cr, int W, int H, int D, int nbits,
             const int32_t *lo, const int32_t *hi, int32_t *C);
int orc_aggregate(const int32_t *C, int W, int H, int D, const int32_t *lo, const int32_t *hi,
                  int p1, int p2, unsigned path_mask, int32_t *S, int32_t *Lr_out);
int orc_wta(const int32_t *S, int W, int H, int D, const int32_t *lo, const int32_t *hi,
            int32_t *dstar, double *dz);
int orc_match(const orc_params *prm, const uint8_t *left, const uint8_t *right,
              const int32_t *lo, const int32_t *hi, int32_t *dstar, double *dz,
              int32_t *C_out, int32_t *S_out);
int orc_predict(const orc_params *prm, const double *d, const double *p, const uint8_t *sflags,
                const double T[16], double *dhat, double *pm, uint8_t *flags, int32_t *lo, int32_t *hi);
int orc_predict_aux(const orc_params *prm, const double *d, const double *p, const uint8_t *sflags,
                    const double *aux_src, const double T[16], double *dhat, double *pm, uint8_t *flags,
                    int32_t *lo, int32_t *hi, double *aux_out);
int orc_curvature_r(const int32_t *S, int W, int H, int D, const int32_t *lo, const int32_t *hi,
                    const int32_t *dstar, double r_curv, double r_const, double *rpix, int32_t *kappa);
int orc_learned_windows(const orc_params *prm, const double *dhat, const double *hw, uint8_t *flags,
                        int32_t *lo, int32_t *hi);
int orc_correct_ex(const orc_params *prm, const double *dhat, const double *pm, const uint8_t *flags,
                   const int32_t *lo, const int32_t *hi, const int32_t *dstar, const double *dz,
                   const double *rpix, double *d, double *p, uint8_t *mask, uint8_t *sflags, double *nu_out);
int orc_median3x3(const double *d, int W, int H, double *out);

/* moving-object detection (Section 4) */
typedef struct {
    int32_t top;                 /* first row the windows cover */
    int32_t n_sizes;             /* window sizes in use (<= 8) */
    int32_t sizes[8][2];         /* width, height */
    int32_t scale, cap, thresh;  /* fixed point of |d^ - d_z|, per-pixel cap, firing level */
    int32_t max_detections;      /* windows kept for grouping */
    int64_t min_area;            /* smaller final boxes are discarded */
    double merge_iou;            /* merge while the best IoU exceeds this */
} orc_detect_params;

int orc_motion_values(const double *dhat, const double *dz, const uint8_t *flags, int W, int H, int scale,
                      int cap, int32_t *v);
int orc_integral(const int32_t *v, int W, int H, int64_t *S);
int orc_detect_windows(const orc_detect_params *dp, const int64_t *S, int W, int H, int32_t *boxes,
                       int32_t *n_fired);
int orc_merge_boxes(int32_t *boxes, int n, double merge_iou, int64_t min_area);
int orc_detect(const orc_detect_params *dp, const double *dhat, const double *dz, const uint8_t *flags, int W,
               int H, int32_t *boxes, int32_t *n_fired);
int orc_correct(const orc_params *prm, const double *dhat, const double *pm, const uint8_t *flags,
                const int32_t *lo, const int32_t *hi, const int32_t *dstar, const double *dz,
                double *d, double *p, uint8_t *mask, uint8_t *sflags);
int orc_full_frame(const orc_params *prm, const uint8_t *left, const uint8_t *right,
                   double *d, double *p, uint8_t *sflags, uint8_t *mask,
                   int32_t *lo, int32_t *hi, int32_t *dstar, double *dz);
int orc_reduced_frame(const orc_params *prm, const uint8_t *left, const uint8_t *right,
                      const double T[16], double *d, double *p, uint8_t *sflags, uint8_t *mask,
                      double *dhat, double *pm, uint8_t *flags, int32_t *lo, int32_t *hi,
                      int32_t *dstar, double *dz);

#ifdef __cplusplus
}
#endif
#endif
