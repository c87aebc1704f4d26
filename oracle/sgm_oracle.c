/*
 * Plain CPU oracle for reduced-space SGM fused by a per-pixel Kalman filter
 * (Popovic, Hadviger, Markovic, Petrovic, "Computationally efficient dense
 * moving object detection based on reduced space disparity estimation").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * statement of what the GPU path computes.  It shares no code, header, table
 * or helper with the GPU library and is used only by the tests, the smoke
 * check and the benchmark's CPU baseline.
 *
 * Dense storage, scalar loops, double precision for every floating-point
 * quantity.  Each function names the passage of the paper it follows.  Where
 * the paper is silent the reading used is stated at the function (the design
 * notes list all of them).
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -shared -fPIC (no FMA
 * contraction, so every floating-point operation is one IEEE-754 rounding in
 * the order written).  That build runs on one thread and is the parity
 * reference.  The same source built with -fopenmp (the CPU baseline) runs the
 * loops marked "omp" on several threads: each such loop's iterations write
 * disjoint outputs and read only values finished before the loop, so both
 * builds give identical results.
 */
#include "sgm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_INF 1000000000

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* ------------------------------------------------------------------------
 * Census transform (Section 2.1, "Matching cost calculation").
 * Each pixel is described by comparing its neighbours inside a cw x ch
 * window with the centre.  Reading of the unspecified details: bit = 1 when
 * the neighbour is strictly darker than the centre; neighbours are visited in
 * raster order (rows top to bottom, columns left to right) skipping the
 * centre, and each new bit is shifted in at the least significant end, so the
 * first neighbour ends in the most significant used bit; outside the image
 * the nearest edge pixel is used.
 * ---------------------------------------------------------------------- */
int orc_census(const uint8_t *img, int W, int H, int cw, int ch, uint64_t *out)
{
    if (cw < 1 || ch < 1 || (cw % 2) == 0 || (ch % 2) == 0 || cw * ch - 1 > 64)
        return -1;
    int rx = cw / 2, ry = ch / 2;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; y++) {
        for (int x = 0; x < W; x++) {
            uint8_t c = img[y * W + x];
            uint64_t bits = 0;
            for (int dy = -ry; dy <= ry; dy++) {
                for (int dx = -rx; dx <= rx; dx++) {
                    if (dx == 0 && dy == 0)
                        continue;
                    int yy = clampi(y + dy, 0, H - 1);
                    int xx = clampi(x + dx, 0, W - 1);
                    bits = (bits << 1) | (uint64_t)(img[yy * W + xx] < c ? 1 : 0);
                }
            }
            out[y * W + x] = bits;
        }
    }
    return 0;
}

static int popcount64(uint64_t v)
{
    int n = 0;
    while (v) {
        n += (int)(v & 1u);
        v >>= 1;
    }
    return n;
}

/* ------------------------------------------------------------------------
 * Matching cost (Section 2.1): Hamming distance between the left census at
 * (x, y) and the right census at (x - d, y).  Reading: when x - d < 0 the
 * match is outside the right image and gets the largest possible cost, the
 * number of census bits.  Only cells inside the pixel's window [lo, hi] are
 * computed (the reduced search space of Section 2); C is dense [H][W][D] and
 * cells outside the window are left untouched.
 * ---------------------------------------------------------------------- */
int orc_cost(const uint64_t *cl, const uint64_t *cr, int W, int H, int D, int nbits,
             const int32_t *lo, const int32_t *hi, int32_t *C)
{
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; y++) {
        for (int x = 0; x < W; x++) {
            int p = y * W + x;
            for (int d = lo[p]; d <= hi[p]; d++) {
                int32_t c;
                if (x - d < 0)
                    c = nbits;
                else
                    c = popcount64(cl[p] ^ cr[y * W + (x - d)]);
                C[(size_t)p * D + d] = c;
            }
        }
    }
    return 0;
}

/* Path directions r; the predecessor of p along r is p - r.  Reading of which
 * four are "nondiagonal" (Table 2): the horizontal and vertical ones, bits
 * 0..3 of the path mask; the diagonal ones are bits 4..7. */
static const int PATH_DX[8] = {+1, -1, 0, 0, +1, -1, -1, +1};
static const int PATH_DY[8] = {0, 0, +1, -1, +1, -1, +1, -1};

/* ------------------------------------------------------------------------
 * Cost aggregation, Eq. (1) (Section 2.2), on per-pixel disparity windows.
 *
 *   L_r(p,d) = C(p,d) + min( L_r(p-r,d), L_r(p-r,d-1)+P1, L_r(p-r,d+1)+P1,
 *                            min_i L_r(p-r,i)+P2 ) - min_i L_r(p-r,i)
 *
 * Readings: (a) the trailing subtraction of the predecessor's minimum is the
 * usual normalisation that keeps the accumulated loss small enough for 16-bit
 * integers (the paper stores it in 16 bits); it shifts every L_r(p,.) by the
 * same amount and so changes no minimiser.  (b) With reduced search spaces
 * the predecessor only has values inside its own window W_{p-r}; every term
 * that refers to a disparity outside it is absent (+infinity), and the P2
 * term's minimum runs over W_{p-r}.  (c) A pixel whose predecessor lies
 * outside the image starts the path: L_r(p,d) = C(p,d).
 * The sum over the selected paths is S(p,d) = sum_r L_r(p,d), for d in W_p.
 * If Lr_out is not NULL, path k's L_r is stored at Lr_out[k][p][d].
 *
 * Visit order: the predecessor p - r is always finished before p.  A
 * horizontal path's scanlines are the image rows, independent of each other
 * (omp: rows in parallel); for the other paths p - r lies in the previous row
 * of the sweep, so the pixels of one row are independent (omp: the pixels of
 * a row in parallel, rows in sweep order).
 * ---------------------------------------------------------------------- */

/* Eq. (1) at pixel (x, y) of path (rx, ry), from its finished predecessor */
static void agg_pixel(const int32_t *C, int32_t *Lr, int W, int H, int D, const int32_t *lo, const int32_t *hi,
                      int p1, int p2, int rx, int ry, int x, int y)
{
    int p = y * W + x;
    int qx = x - rx, qy = y - ry;
    if (qx < 0 || qx >= W || qy < 0 || qy >= H) {
        for (int d = lo[p]; d <= hi[p]; d++)
            Lr[(size_t)p * D + d] = C[(size_t)p * D + d];
        return;
    }
    int q = qy * W + qx;
    int mq = ORC_INF;
    for (int i = lo[q]; i <= hi[q]; i++)
        if (Lr[(size_t)q * D + i] < mq)
            mq = Lr[(size_t)q * D + i];
    for (int d = lo[p]; d <= hi[p]; d++) {
        int best = mq + p2;
        if (d >= lo[q] && d <= hi[q] && Lr[(size_t)q * D + d] < best)
            best = Lr[(size_t)q * D + d];
        if (d - 1 >= lo[q] && d - 1 <= hi[q] && Lr[(size_t)q * D + d - 1] + p1 < best)
            best = Lr[(size_t)q * D + d - 1] + p1;
        if (d + 1 >= lo[q] && d + 1 <= hi[q] && Lr[(size_t)q * D + d + 1] + p1 < best)
            best = Lr[(size_t)q * D + d + 1] + p1;
        Lr[(size_t)p * D + d] = C[(size_t)p * D + d] + best - mq;
    }
}

int orc_aggregate(const int32_t *C, int W, int H, int D, const int32_t *lo, const int32_t *hi,
                  int p1, int p2, unsigned path_mask, int32_t *S, int32_t *Lr_out)
{
    size_t cells = (size_t)W * H * D;
    int32_t *Lr = (int32_t *)malloc(cells * sizeof(int32_t));
    if (!Lr)
        return -2;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            int p = y * W + x;
            for (int d = lo[p]; d <= hi[p]; d++)
                S[(size_t)p * D + d] = 0;
        }
    for (int k = 0; k < 8; k++) {
        if (!(path_mask & (1u << k)))
            continue;
        int rx = PATH_DX[k], ry = PATH_DY[k];
        if (ry == 0) {
#pragma omp parallel for schedule(static)
            for (int y = 0; y < H; y++)
                for (int ix = 0; ix < W; ix++)
                    agg_pixel(C, Lr, W, H, D, lo, hi, p1, p2, rx, ry, (rx >= 0) ? ix : W - 1 - ix, y);
        } else {
            for (int iy = 0; iy < H; iy++) {
                int y = (ry >= 0) ? iy : H - 1 - iy;
#pragma omp parallel for schedule(static)
                for (int x = 0; x < W; x++)
                    agg_pixel(C, Lr, W, H, D, lo, hi, p1, p2, rx, ry, x, y);
            }
        }
#pragma omp parallel for schedule(static)
        for (int y = 0; y < H; y++)
            for (int x = 0; x < W; x++) {
                int p = y * W + x;
                for (int d = lo[p]; d <= hi[p]; d++) {
                    S[(size_t)p * D + d] += Lr[(size_t)p * D + d];
                    if (Lr_out)
                        Lr_out[(size_t)k * cells + (size_t)p * D + d] = Lr[(size_t)p * D + d];
                }
            }
    }
    free(Lr);
    return 0;
}

/* ------------------------------------------------------------------------
 * Winner-takes-all (Section 2.3) with a parabolic sub-pixel fit.
 * d* is the smallest disparity of the window attaining min_d S(p,d) (reading:
 * ties go to the lower disparity).  When both d*-1 and d*+1 lie in the
 * window, a parabola through the three sums gives the offset
 * (a - b) / (2 (a + b)), a = S(d*-1)-S(d*) >= 1, b = S(d*+1)-S(d*) >= 0;
 * otherwise the measurement is d* itself.
 * ---------------------------------------------------------------------- */
int orc_wta(const int32_t *S, int W, int H, int D, const int32_t *lo, const int32_t *hi,
            int32_t *dstar, double *dz)
{
#pragma omp parallel for schedule(static)
    for (int p = 0; p < W * H; p++) {
        const int32_t *s = S + (size_t)p * D;
        int best = lo[p];
        for (int d = lo[p] + 1; d <= hi[p]; d++)
            if (s[d] < s[best])
                best = d;
        dstar[p] = best;
        if (best - 1 >= lo[p] && best + 1 <= hi[p]) {
            int a = s[best - 1] - s[best];
            int b = s[best + 1] - s[best];
            dz[p] = (double)best + (double)(a - b) / (double)(2 * (a + b));
        } else {
            dz[p] = (double)best;
        }
    }
    return 0;
}

/* Full pipeline of the matcher on given windows: census, cost, aggregation,
 * WTA.  C and S are dense [H][W][D] scratch owned by the caller (or NULL to
 * let the oracle allocate them). */
int orc_match(const orc_params *prm, const uint8_t *left, const uint8_t *right,
              const int32_t *lo, const int32_t *hi, int32_t *dstar, double *dz,
              int32_t *C_out, int32_t *S_out)
{
    int W = prm->width, H = prm->height, D = prm->max_disp;
    size_t n = (size_t)W * H, cells = n * D;
    uint64_t *cl = (uint64_t *)malloc(n * sizeof(uint64_t));
    uint64_t *cr = (uint64_t *)malloc(n * sizeof(uint64_t));
    int32_t *C = C_out ? C_out : (int32_t *)malloc(cells * sizeof(int32_t));
    int32_t *S = S_out ? S_out : (int32_t *)malloc(cells * sizeof(int32_t));
    int rc = 0;
    if (!cl || !cr || !C || !S) {
        rc = -2;
        goto done;
    }
    if (orc_census(left, W, H, prm->census_w, prm->census_h, cl) ||
        orc_census(right, W, H, prm->census_w, prm->census_h, cr)) {
        rc = -1;
        goto done;
    }
    orc_cost(cl, cr, W, H, D, prm->census_w * prm->census_h - 1, lo, hi, C);
    rc = orc_aggregate(C, W, H, D, lo, hi, prm->p1, prm->p2, prm->path_mask, S, NULL);
    if (rc)
        goto done;
    orc_wta(S, W, H, D, lo, hi, dstar, dz);
done:
    free(cl);
    free(cr);
    if (!C_out)
        free(C);
    if (!S_out)
        free(S);
    return rc;
}

/* ------------------------------------------------------------------------
 * Prediction (Section 2.4, Eq. 2-4) and the rules that follow it.
 *
 * Eq. (2) maps disparity-space points omega = (x, y, d) of frame k-1 into
 * frame k with a 4x4 matrix.  Reading: the matrix is the ego-motion T
 * (X_k = R X_{k-1} + t, metric camera coordinates) conjugated by the stereo
 * projection, followed by the homogeneous division.  Written out with
 * h = ((x-cx) B, (y-cy) B, f B) (= d * X):
 *     h' = R h + t d,   x' = f h'_x / h'_z + cx,   y' = f h'_y / h'_z + cy,
 *     d' = f B d / h'_z,   Phi = d' / d = f B / h'_z  (Eq. 3, defined at d=0),
 *     p' = Phi^2 p + q   (Eq. 4).
 * Readings: a source is dropped when h'_z <= 1e-9 f B (behind the camera),
 * when its nearest target pixel floor(x'+0.5), floor(y'+0.5) is outside the
 * image, or when d' > D-1.  Several sources landing on one target: the
 * largest d' (nearest surface) wins, then the smallest source index y*W+x.
 * The winner's RESET bit travels with it.
 *
 * Zooming holes (Section 2.4): a target without a winner that has known
 * left and right neighbours, or known upper and lower neighbours, takes the
 * mean disparity and the mean variance of those neighbours (all valid pairs:
 * 2 or 4 values, summed in the order left, right, up, down).  Reading: one
 * pass over the winners only; the RESET bits of the contributors are OR-ed.
 *
 * Discontinuities (Section 2.4): "reject the predicted disparities near
 * disparity discontinuities".  Reading: on the filled map, a predicted pixel
 * is rejected when a predicted pixel of its 8-neighbourhood differs by more
 * than disc_thresh.  (Under forward motion the nearer surface spreads apart
 * and occluded background lands in the one-pixel gaps of its splat; where a
 * gap row crosses a gap column only the diagonal neighbours still show the
 * nearer surface.)
 *
 * Search limits (Section 2.4): the paper writes d^{k|k-1} +- p^{k|k-1}.
 * Reading: +- k_sigma standard deviations, rounded outward:
 * lo = max(0, floor(dh - k sqrt(p))), hi = min(D-1, ceil(dh + k sqrt(p))).
 * A pixel without a prediction, or with RESET, searches the whole range
 * [0, D-1] (the initialisation of Section 2.4).
 *
 * Inputs: previous state d, p (double), sflags (ORC_RESET bit).
 * Outputs: dhat, pm (double), flags (ORC_PRED | ORC_RESET | ORC_FULLWIN), lo, hi.
 * ---------------------------------------------------------------------- */
int orc_predict(const orc_params *prm, const double *d, const double *p, const uint8_t *sflags,
                const double T[16], double *dhat, double *pm, uint8_t *flags, int32_t *lo, int32_t *hi)
{
    return orc_predict_aux(prm, d, p, sflags, NULL, T, dhat, pm, flags, lo, hi, NULL);
}

/* As orc_predict; in addition, when aux_src and aux_out are given, a target
 * whose warp winner is source s receives aux_out = aux_src[s] (the learned
 * window's "previous innovation" input travels with the winner); filled
 * holes and targets without a prediction receive 0. */
int orc_predict_aux(const orc_params *prm, const double *d, const double *p, const uint8_t *sflags,
                    const double *aux_src, const double T[16], double *dhat, double *pm, uint8_t *flags,
                    int32_t *lo, int32_t *hi, double *aux_out)
{
    int W = prm->width, H = prm->height, D = prm->max_disp;
    size_t n = (size_t)W * H;
    double f = prm->f, B = prm->baseline, cx = prm->cx, cy = prm->cy;
    double fB = f * B;
    int64_t *win = (int64_t *)malloc(n * sizeof(int64_t));   /* winning source per target */
    double *dw = (double *)malloc(n * sizeof(double));
    double *pw = (double *)malloc(n * sizeof(double));
    uint8_t *rw = (uint8_t *)malloc(n);
    uint8_t *has = (uint8_t *)malloc(n);
    uint8_t *pred = (uint8_t *)malloc(n);
    uint8_t *rst = (uint8_t *)malloc(n);
    if (!win || !dw || !pw || !rw || !has || !pred || !rst) {
        free(win); free(dw); free(pw); free(rw); free(has); free(pred); free(rst);
        return -2;
    }
    for (size_t t = 0; t < n; t++) {
        win[t] = -1;
        dw[t] = 0.0;
        pw[t] = 0.0;
        rw[t] = 0;
        has[t] = 0;
    }
    /* warp and z-buffer */
    for (int y = 0; y < H; y++) {
        for (int x = 0; x < W; x++) {
            int s = y * W + x;
            double X = ((double)x - cx) * B;
            double Y = ((double)y - cy) * B;
            double ds = d[s];
            double hx = ((T[0] * X + T[1] * Y) + T[2] * fB) + T[3] * ds;
            double hy = ((T[4] * X + T[5] * Y) + T[6] * fB) + T[7] * ds;
            double hz = ((T[8] * X + T[9] * Y) + T[10] * fB) + T[11] * ds;
            if (!(hz > 1e-9 * fB))
                continue;
            double xp = (f * hx) / hz + cx;
            double yp = (f * hy) / hz + cy;
            double dp = (fB * ds) / hz;
            double phi = fB / hz;
            double pp = (phi * phi) * p[s] + prm->q;
            double ux = xp + 0.5, uy = yp + 0.5;
            if (!(ux >= 0.0 && ux < (double)W && uy >= 0.0 && uy < (double)H))
                continue;
            if (!(dp <= (double)(D - 1)))
                continue;
            int tx = (int)floor(ux), ty = (int)floor(uy);
            int t = ty * W + tx;
            /* sources are visited in increasing index, so a strictly larger d'
             * is needed to replace the current winner */
            if (win[t] < 0 || dp > dw[t]) {
                win[t] = s;
                dw[t] = dp;
                pw[t] = pp;
                rw[t] = (uint8_t)(sflags[s] & ORC_RESET);
            }
        }
    }
    for (size_t t = 0; t < n; t++)
        has[t] = win[t] >= 0;
    if (aux_src && aux_out) {
        for (size_t t = 0; t < n; t++)
            aux_out[t] = win[t] >= 0 ? aux_src[win[t]] : 0.0;
    }
    /* zooming-hole fill from the winners */
    for (int y = 0; y < H; y++) {
        for (int x = 0; x < W; x++) {
            int t = y * W + x;
            pred[t] = has[t];
            dhat[t] = dw[t];
            pm[t] = pw[t];
            rst[t] = rw[t];
            if (has[t])
                continue;
            int hpair = x - 1 >= 0 && x + 1 < W && has[t - 1] && has[t + 1];
            int vpair = y - 1 >= 0 && y + 1 < H && has[t - W] && has[t + W];
            if (hpair && vpair) {
                dhat[t] = (((dw[t - 1] + dw[t + 1]) + dw[t - W]) + dw[t + W]) / 4.0;
                pm[t] = (((pw[t - 1] + pw[t + 1]) + pw[t - W]) + pw[t + W]) / 4.0;
                rst[t] = rw[t - 1] | rw[t + 1] | rw[t - W] | rw[t + W];
                pred[t] = 1;
            } else if (hpair) {
                dhat[t] = (dw[t - 1] + dw[t + 1]) / 2.0;
                pm[t] = (pw[t - 1] + pw[t + 1]) / 2.0;
                rst[t] = rw[t - 1] | rw[t + 1];
                pred[t] = 1;
            } else if (vpair) {
                dhat[t] = (dw[t - W] + dw[t + W]) / 2.0;
                pm[t] = (pw[t - W] + pw[t + W]) / 2.0;
                rst[t] = rw[t - W] | rw[t + W];
                pred[t] = 1;
            }
        }
    }
    /* discontinuity rejection, decided on the filled map before any pixel is
     * rejected (has[] is reused to hold the decision) */
    for (int y = 0; y < H; y++) {
        for (int x = 0; x < W; x++) {
            int t = y * W + x;
            int ok = pred[t];
            if (ok) {
                for (int yy = y - 1; yy <= y + 1; yy++) {
                    for (int xx = x - 1; xx <= x + 1; xx++) {
                        if (xx < 0 || xx >= W || yy < 0 || yy >= H || (xx == x && yy == y))
                            continue;
                        int u = yy * W + xx;
                        if (pred[u] && fabs(dhat[t] - dhat[u]) > prm->disc_thresh)
                            ok = 0;
                    }
                }
            }
            has[t] = (uint8_t)ok;
        }
    }
    /* search limits */
    for (size_t t = 0; t < n; t++) {
        int ok = has[t];
        uint8_t fl = 0;
        if (ok)
            fl |= ORC_PRED;
        if (rst[t])
            fl |= ORC_RESET;
        int full = !ok || rst[t] || !(dhat[t] >= 0.0 && dhat[t] <= (double)(D - 1));
        if (full) {
            fl |= ORC_FULLWIN;
            lo[t] = 0;
            hi[t] = D - 1;
        } else {
            double s = sqrt(pm[t]);
            double a = dhat[t] - prm->k_sigma * s;
            double b = dhat[t] + prm->k_sigma * s;
            int l = (int)floor(a), h = (int)ceil(b);
            lo[t] = l < 0 ? 0 : l;
            hi[t] = h > D - 1 ? D - 1 : h;
        }
        if (!ok) {
            dhat[t] = 0.0;
            pm[t] = 0.0;
            if (aux_src && aux_out)
                aux_out[t] = 0.0;
        }
        flags[t] = fl;
    }
    free(win); free(dw); free(pw); free(rw); free(has); free(pred); free(rst);
    return 0;
}

/* ------------------------------------------------------------------------
 * Correction (Section 2.4, Eq. 5-6) and the innovation test.
 * K = p^- / (p^- + r) (reading: the gain the paper leaves unprinted is the
 * optimal one); d = dh + K (dz - dh); p = (1-K)^2 p^- + K^2 r (Eq. 6).
 * A pixel whose window was the full range (no prediction, or RESET) starts
 * over from the measurement: d = dz, p = r (the initialisation of Section
 * 2.4).
 * Moving objects (Section 4) are where prediction and measurement disagree.
 * Reading: a pixel with a prediction is marked moving when the normalised
 * innovation nu^2 / (p^- + r) exceeds chi2_gate.  RESET for the next frame is
 * set for moving pixels and for pixels whose minimum sat on an inner window
 * edge (d* = lo > 0 or d* = hi < D-1).
 * ---------------------------------------------------------------------- */
int orc_correct(const orc_params *prm, const double *dhat, const double *pm, const uint8_t *flags,
                const int32_t *lo, const int32_t *hi, const int32_t *dstar, const double *dz,
                double *d, double *p, uint8_t *mask, uint8_t *sflags)
{
    return orc_correct_ex(prm, dhat, pm, flags, lo, hi, dstar, dz, NULL, d, p, mask, sflags, NULL);
}

/* As orc_correct, with
 *  - rpix: per-pixel measurement variance r of the learned window (NULL:
 *    prm->r everywhere); a restart from the measurement always takes prm->r;
 *  - nu_out: the innovation dz - dhat of pixels with a prediction, 0
 *    elsewhere (NULL: not written);
 *  - ORC_GATEFAIL pixels (re-measured over the full range after failing the
 *    innovation test of a first pass, FULLWIN also set): restart from the
 *    measurement, stay marked moving, RESET for the next frame. */
int orc_correct_ex(const orc_params *prm, const double *dhat, const double *pm, const uint8_t *flags,
                   const int32_t *lo, const int32_t *hi, const int32_t *dstar, const double *dz,
                   const double *rpix, double *d, double *p, uint8_t *mask, uint8_t *sflags, double *nu_out)
{
    int n = prm->width * prm->height, D = prm->max_disp;
#pragma omp parallel for schedule(static)
    for (int t = 0; t < n; t++) {
        double r = rpix ? rpix[t] : prm->r;
        int moving = 0;
        double nu = 0.0, S = 0.0;
        if (flags[t] & ORC_PRED) {
            nu = dz[t] - dhat[t];
            S = pm[t] + r;
            moving = (nu * nu) / S > prm->chi2_gate;
        }
        if (nu_out)
            nu_out[t] = nu;
        if (flags[t] & ORC_GATEFAIL) {
            d[t] = dz[t];
            p[t] = prm->r;
            mask[t] = 1;
            sflags[t] = ORC_RESET;
            continue;
        }
        if (flags[t] & ORC_FULLWIN) {
            d[t] = dz[t];
            p[t] = prm->r;
        } else {
            double K = pm[t] / S;
            double a = 1.0 - K;
            d[t] = dhat[t] + K * nu;
            p[t] = (a * a) * pm[t] + (K * K) * r;
        }
        int sat = (dstar[t] == lo[t] && lo[t] > 0) || (dstar[t] == hi[t] && hi[t] < D - 1);
        mask[t] = (uint8_t)moving;
        sflags[t] = (uint8_t)((moving || sat) ? ORC_RESET : 0);
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Per-pixel measurement variance from the cost curvature.  Section 3 says the
 * authors' earlier method estimated the measurement noise from the cost
 * values at the neighbouring disparities, without a formula.  Reading: near
 * its minimum the aggregated cost is a negative log-likelihood up to a scale,
 *     S(d) ~ S(d*) + kappa (d - d_z)^2 / 2,
 * with kappa = a + b = S(d*-1) + S(d*+1) - 2 S(d*), the second difference
 * through the three sums of the sub-pixel parabola (kappa >= 1, since a >= 1
 * by the lowest-disparity tie rule); the measurement variance is then
 *     r = r_curv / kappa,   clamped to [1/256, 64],
 * with r_curv (cost units x px^2) a parameter fitted to ground truth.  Where
 * the parabola is not defined (d* on a window edge) kappa = 0 and
 * r = r_const.  S is dense [H][W][D] (only window cells are read).
 * ---------------------------------------------------------------------- */
int orc_curvature_r(const int32_t *S, int W, int H, int D, const int32_t *lo, const int32_t *hi,
                    const int32_t *dstar, double r_curv, double r_const, double *rpix, int32_t *kappa)
{
    for (int p = 0; p < W * H; p++) {
        const int32_t *s = S + (size_t)p * D;
        const int ds = dstar[p];
        int k = 0;
        double r = r_const;
        if (ds - 1 >= lo[p] && ds + 1 <= hi[p]) {
            k = (s[ds - 1] - s[ds]) + (s[ds + 1] - s[ds]);
            r = r_curv / (double)k;
            if (r < 1.0 / 256.0)
                r = 1.0 / 256.0;
            if (r > 64.0)
                r = 64.0;
        }
        rpix[p] = r;
        kappa[p] = k;
    }
    return 0;
}

/* Learned search windows: a pixel that still has a finite window after the
 * prediction gets [floor(dhat - w), ceil(dhat + w)] clipped to [0, D-1],
 * with w its predicted half-width; w >= ORC_LEARNED_WMAX (or NaN) sends it to
 * the full range (FULLWIN). */
int orc_learned_windows(const orc_params *prm, const double *dhat, const double *hw, uint8_t *flags,
                        int32_t *lo, int32_t *hi)
{
    int n = prm->width * prm->height, D = prm->max_disp;
    for (int t = 0; t < n; t++) {
        if (flags[t] & ORC_FULLWIN)
            continue;
        if (!(hw[t] < ORC_LEARNED_WMAX)) {
            flags[t] |= ORC_FULLWIN;
            lo[t] = 0;
            hi[t] = D - 1;
            continue;
        }
        int l = (int)floor(dhat[t] - hw[t]), h = (int)ceil(dhat[t] + hw[t]);
        lo[t] = l < 0 ? 0 : l;
        hi[t] = h > D - 1 ? D - 1 : h;
    }
    return 0;
}

/* Frame 0 (Section 2.4: limits initially cover the whole search space, which
 * is conventional SGM): full windows, then d = dz, p = r, no motion. */
int orc_full_frame(const orc_params *prm, const uint8_t *left, const uint8_t *right,
                   double *d, double *p, uint8_t *sflags, uint8_t *mask,
                   int32_t *lo, int32_t *hi, int32_t *dstar, double *dz)
{
    int n = prm->width * prm->height;
    for (int t = 0; t < n; t++) {
        lo[t] = 0;
        hi[t] = prm->max_disp - 1;
    }
    int rc = orc_match(prm, left, right, lo, hi, dstar, dz, NULL, NULL);
    if (rc)
        return rc;
    for (int t = 0; t < n; t++) {
        d[t] = dz[t];
        p[t] = prm->r;
        sflags[t] = 0;
        mask[t] = 0;
    }
    return 0;
}

/* One steady-state frame: predict, match inside the windows, correct. */
int orc_reduced_frame(const orc_params *prm, const uint8_t *left, const uint8_t *right,
                      const double T[16], double *d, double *p, uint8_t *sflags, uint8_t *mask,
                      double *dhat, double *pm, uint8_t *flags, int32_t *lo, int32_t *hi,
                      int32_t *dstar, double *dz)
{
    int rc = orc_predict(prm, d, p, sflags, T, dhat, pm, flags, lo, hi);
    if (rc)
        return rc;
    rc = orc_match(prm, left, right, lo, hi, dstar, dz, NULL, NULL);
    if (rc)
        return rc;
    return orc_correct(prm, dhat, pm, flags, lo, hi, dstar, dz, d, p, mask, sflags);
}

/* ------------------------------------------------------------------------
 * Post-processing (Section 2.3): 3x3 block median of the filtered disparity,
 * outside the Kalman loop (the state is not changed).  Reading: neighbours
 * outside the image are clamped to the edge, so every pixel takes the median
 * (5th smallest) of 9 values.
 * ---------------------------------------------------------------------- */
int orc_median3x3(const double *d, int W, int H, double *out)
{
    for (int y = 0; y < H; y++) {
        for (int x = 0; x < W; x++) {
            double v[9];
            int n = 0;
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++)
                    v[n++] = d[clampi(y + dy, 0, H - 1) * W + clampi(x + dx, 0, W - 1)];
            /* insertion sort of 9 values */
            for (int i = 1; i < 9; i++) {
                double t = v[i];
                int j = i - 1;
                while (j >= 0 && v[j] > t) {
                    v[j + 1] = v[j];
                    j--;
                }
                v[j + 1] = t;
            }
            out[y * W + x] = v[4];
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Moving-object detection (Section 4).
 *
 * Readings (the paper gives the structure, not every constant):
 *  - the difference map is |d^ - d_z| where the frame has a prediction
 *    (ORC_PRED) whose correspondence x - d^ lies inside the right image, and
 *    0 elsewhere (no measurement is possible left of that), in fixed point:
 *    floor(|d^ - d_z| * scale) capped at `cap`, so window sums are exact
 *    integers;
 *  - a window "is high relative to its area" when its sum is at least
 *    thresh * area (thresh in the same fixed-point units per pixel);
 *  - windows of every listed size slide with a step of half their width and
 *    half their height, from row `top` (the bottom two thirds: top = H/3) to
 *    the bottom edge; detections are listed by size, then row, then column,
 *    and at most max_detections are kept;
 *  - the greedy grouping merges the pair with the highest intersection over
 *    union (exact rational comparison; ties: the pair that comes first in
 *    list order) into its bounding box, in the place of the earlier box,
 *    while that IoU exceeds merge_iou;
 *  - boxes with an area below min_area are then discarded.
 * Boxes are half-open [x0, x1) x [y0, y1).
 * ---------------------------------------------------------------------- */
int orc_motion_values(const double *dhat, const double *dz, const uint8_t *flags, int W, int H, int scale,
                      int cap, int32_t *v)
{
    for (int y = 0; y < H; y++) {
        for (int x = 0; x < W; x++) {
            const int i = y * W + x;
            if ((flags[i] & ORC_PRED) && (double)x - dhat[i] >= 0.0)
                v[i] = (int32_t)fmin(floor(fabs(dhat[i] - dz[i]) * (double)scale), (double)cap);
            else
                v[i] = 0;
        }
    }
    return 0;
}

/* Summed-area table: S[y][x] = sum of v over rows < y and columns < x
 * ((H+1) x (W+1) entries), so any box sum takes four lookups
 * (inclusion-exclusion). */
int orc_integral(const int32_t *v, int W, int H, int64_t *S)
{
    for (int x = 0; x <= W; x++)
        S[x] = 0;
    for (int y = 1; y <= H; y++) {
        int64_t row = 0;
        S[(size_t)y * (W + 1)] = 0;
        for (int x = 1; x <= W; x++) {
            row += v[(size_t)(y - 1) * W + (x - 1)];
            S[(size_t)y * (W + 1) + x] = S[(size_t)(y - 1) * (W + 1) + x] + row;
        }
    }
    return 0;
}

static int64_t box_sum(const int64_t *S, int W, int x0, int y0, int x1, int y1)
{
    const size_t s = (size_t)W + 1;
    return S[(size_t)y1 * s + x1] - S[(size_t)y0 * s + x1] - S[(size_t)y1 * s + x0] + S[(size_t)y0 * s + x0];
}

int orc_detect_windows(const orc_detect_params *dp, const int64_t *S, int W, int H, int32_t *boxes,
                       int32_t *n_fired)
{
    int kept = 0, fired = 0;
    for (int s = 0; s < dp->n_sizes; s++) {
        const int w = dp->sizes[s][0], h = dp->sizes[s][1];
        const int sx = w / 2 > 0 ? w / 2 : 1, sy = h / 2 > 0 ? h / 2 : 1;
        for (int y0 = dp->top; y0 + h <= H; y0 += sy) {
            for (int x0 = 0; x0 + w <= W; x0 += sx) {
                int64_t sum = box_sum(S, W, x0, y0, x0 + w, y0 + h);
                if (sum >= (int64_t)dp->thresh * w * h) {
                    fired++;
                    if (kept < dp->max_detections) {
                        boxes[4 * kept + 0] = x0;
                        boxes[4 * kept + 1] = y0;
                        boxes[4 * kept + 2] = x0 + w;
                        boxes[4 * kept + 3] = y0 + h;
                        kept++;
                    }
                }
            }
        }
    }
    *n_fired = fired;
    return kept;
}

static int64_t box_area(const int32_t *b) { return (int64_t)(b[2] - b[0]) * (b[3] - b[1]); }

static int64_t box_inter(const int32_t *a, const int32_t *b)
{
    int64_t w = (int64_t)(a[2] < b[2] ? a[2] : b[2]) - (a[0] > b[0] ? a[0] : b[0]);
    int64_t h = (int64_t)(a[3] < b[3] ? a[3] : b[3]) - (a[1] > b[1] ? a[1] : b[1]);
    return w > 0 && h > 0 ? w * h : 0;
}

/* Greedy grouping on a list of n boxes (in place); returns the number left. */
int orc_merge_boxes(int32_t *boxes, int n, double merge_iou, int64_t min_area)
{
    while (n >= 2) {
        int bi = -1, bj = -1;
        int64_t bI = 0, bU = 1;
        for (int i = 0; i < n; i++) {
            for (int j = i + 1; j < n; j++) {
                int64_t I = box_inter(boxes + 4 * i, boxes + 4 * j);
                int64_t U = box_area(boxes + 4 * i) + box_area(boxes + 4 * j) - I;
                /* I / U > bI / bU, exactly */
                if (bi < 0 || I * bU > bI * U) {
                    bi = i;
                    bj = j;
                    bI = I;
                    bU = U;
                }
            }
        }
        if (!((double)bI > merge_iou * (double)bU))
            break;
        int32_t *a = boxes + 4 * bi, *b = boxes + 4 * bj;
        if (b[0] < a[0]) a[0] = b[0];
        if (b[1] < a[1]) a[1] = b[1];
        if (b[2] > a[2]) a[2] = b[2];
        if (b[3] > a[3]) a[3] = b[3];
        memmove(boxes + 4 * bj, boxes + 4 * (bj + 1), sizeof(int32_t) * 4 * (size_t)(n - bj - 1));
        n--;
    }
    int m = 0;
    for (int i = 0; i < n; i++) {
        if (box_area(boxes + 4 * i) >= min_area) {
            memmove(boxes + 4 * m, boxes + 4 * i, sizeof(int32_t) * 4);
            m++;
        }
    }
    return m;
}

int orc_detect(const orc_detect_params *dp, const double *dhat, const double *dz, const uint8_t *flags, int W,
               int H, int32_t *boxes, int32_t *n_fired)
{
    int32_t *v = (int32_t *)malloc(sizeof(int32_t) * (size_t)W * H);
    int64_t *S = (int64_t *)malloc(sizeof(int64_t) * (size_t)(W + 1) * (H + 1));
    if (!v || !S) {
        free(v);
        free(S);
        return -1;
    }
    orc_motion_values(dhat, dz, flags, W, H, dp->scale, dp->cap, v);
    orc_integral(v, W, H, S);
    int n = orc_detect_windows(dp, S, W, H, boxes, n_fired);
    n = orc_merge_boxes(boxes, n, dp->merge_iou, dp->min_area);
    free(v);
    free(S);
    return n;
}

/* Threads the parallel loops use: omp_get_max_threads() in the -fopenmp
 * build, 1 in the parity build. */
#ifdef _OPENMP
#include <omp.h>
int orc_threads(void) { return omp_get_max_threads(); }
#else
int orc_threads(void) { return 1; }
#endif
