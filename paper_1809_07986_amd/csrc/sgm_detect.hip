// Moving-object detection of Section 4 on gfx950.
//
// The difference map |d^ - d_z| (fixed point, where a prediction exists and
// its correspondence x - d^ lies inside the right image) is turned into a
// summed-area table over the scanned rows, every sliding window is tested
// against "sum high relative to the area" with four lookups
// (inclusion-exclusion), and one workgroup groups the windows that fired:
// repeatedly the pair with the highest intersection over union is replaced
// by its bounding box, then boxes below the minimum area are dropped.
//
// Kernels (one launch each, in stream order):
//   k_det_rows    one workgroup per scanned row: difference values and the
//                 inclusive prefix along the row (row r+1 of the table).
//   k_det_cols    one thread per table column: prefix down the rows.
//   k_det_windows one thread per window: fired / not fired.
//   k_det_group   one workgroup of 1024 threads: ordered compaction of the
//                 fired windows, greedy grouping with a cached best partner
//                 per box, minimum-area filter, output.
//
// The table holds uint32 sums that may wrap: a window sum is the
// inclusion-exclusion of four entries modulo 2^32, exact because the host
// rejects windows whose largest possible sum reaches 2^32.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "sgm_internal.h"

namespace sgmk {

namespace {

__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(v, o, 64);
        if (lane >= o)
            v += t;
    }
    return v;
}

// Exclusive prefix of v over the whole workgroup (blockDim.x a multiple of
// 64, at most 1024); *total receives the sum.  Contains two barriers.
__device__ int block_excl_scan(int v, int *lds16, int *total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int inc = wave_incl_scan(v);
    if (lane == 63)
        lds16[wave] = inc;
    __syncthreads();
    int before = 0, all = 0;
    for (int w = 0; w < nw; w++) {
        int t = lds16[w];
        before += w < wave ? t : 0;
        all += t;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

__device__ __forceinline__ void window_box(const DetectGeom &dg, int t, int &x0, int &r0, int &w, int &h)
{
    int s = 0;
    while (s + 1 < dg.nsizes && t >= dg.base[s + 1])
        s++;
    const int local = t - dg.base[s];
    const int iy = local / dg.nx[s], ix = local - iy * dg.nx[s];
    x0 = ix * dg.sx[s];
    r0 = iy * dg.sy[s];
    w = dg.w[s];
    h = dg.h[s];
}

struct Box {
    int x0, y0, x1, y1;
};

__device__ __forceinline__ Box get_box(const short4 *bx, int i)
{
    short4 b = bx[i];
    return Box{b.x, b.y, b.z, b.w};
}

__device__ __forceinline__ int area(const Box &b) { return (b.x1 - b.x0) * (b.y1 - b.y0); }

__device__ __forceinline__ int inter(const Box &a, const Box &b)
{
    int w = min(a.x1, b.x1) - max(a.x0, b.x0);
    int h = min(a.y1, b.y1) - max(a.y0, b.y0);
    return w > 0 && h > 0 ? w * h : 0;
}

// (I1 / U1, idx1) ranks before (I2 / U2, idx2): larger ratio, then the lower
// index.  I = -1 marks "no candidate" (ranks after every real ratio).
__device__ __forceinline__ bool ranks_before(int I1, int U1, int i1, int I2, int U2, int i2)
{
    long long a = (long long)I1 * U2, b = (long long)I2 * U1;
    return a > b || (a == b && i1 < i2);
}

__device__ __forceinline__ void wave_best(int &I, int &U, int &idx)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        int I2 = __shfl_xor(I, o, 64), U2 = __shfl_xor(U, o, 64), i2 = __shfl_xor(idx, o, 64);
        if (ranks_before(I2, U2, i2, I, U, idx)) {
            I = I2;
            U = U2;
            idx = i2;
        }
    }
}

}  // namespace

__global__ void __launch_bounds__(256) k_det_rows(DetectGeom dg, const double *__restrict__ dhat,
                                                  const double *__restrict__ dz, const uint8_t *__restrict__ flags,
                                                  uint32_t *__restrict__ sat)
{
    __shared__ int lds[16];
    const int r = blockIdx.x, y = dg.top + r;
    const size_t stride = (size_t)dg.W + 1;
    uint32_t *row = sat + (size_t)(r + 1) * stride;
    if (threadIdx.x == 0)
        row[0] = 0;
    int carry = 0;
    for (int x0 = 0; x0 < dg.W; x0 += 256) {
        const int x = x0 + threadIdx.x;
        int v = 0;
        if (x < dg.W) {
            const size_t i = (size_t)y * dg.W + x;
            const double dh = dhat[i];
            if ((flags[i] & SGM_FLAG_PRED) && (double)x - dh >= 0.0)
                v = (int)fmin(floor(fabs(dh - dz[i]) * (double)dg.scale), (double)dg.cap);
        }
        int total;
        int ex = block_excl_scan(v, lds, &total);
        if (x < dg.W)
            row[x + 1] = (uint32_t)(carry + ex + v);
        carry += total;
    }
}

__global__ void __launch_bounds__(256) k_det_cols(DetectGeom dg, uint32_t *__restrict__ sat)
{
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x > dg.W)
        return;
    const size_t stride = (size_t)dg.W + 1;
    sat[x] = 0;
    uint32_t acc = 0;
    for (int r = 1; r <= dg.rows; r++) {
        acc += sat[(size_t)r * stride + x];
        sat[(size_t)r * stride + x] = acc;
    }
}

__global__ void __launch_bounds__(256) k_det_windows(DetectGeom dg, const uint32_t *__restrict__ sat,
                                                     uint8_t *__restrict__ fire)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= dg.base[dg.nsizes])
        return;
    int x0, r0, w, h;
    window_box(dg, t, x0, r0, w, h);
    const size_t stride = (size_t)dg.W + 1;
    const uint32_t *a = sat + (size_t)r0 * stride, *b = sat + (size_t)(r0 + h) * stride;
    const uint32_t sum = b[x0 + w] - a[x0 + w] - b[x0] + a[x0];
    fire[t] = (uint64_t)sum >= (uint64_t)dg.thresh * (uint64_t)(w * h) ? 1 : 0;
}

__global__ void __launch_bounds__(1024) k_det_group(DetectGeom dg, const uint8_t *__restrict__ fire,
                                                    int32_t *__restrict__ out, int32_t *__restrict__ count)
{
    __shared__ short4 bx[kDetMaxBoxes];
    __shared__ int bI[kDetMaxBoxes], bU[kDetMaxBoxes];
    __shared__ short bj[kDetMaxBoxes];
    __shared__ uint8_t alive[kDetMaxBoxes];
    __shared__ short flagged[kDetMaxBoxes];
    __shared__ int lds[16];
    __shared__ int redI[16], redU[16], redX[16];
    __shared__ int sel[3];
    __shared__ int nflag;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nwin = dg.base[dg.nsizes];

    // ordered compaction of the fired windows (window order = size, row, column)
    const int chunk = (nwin + 1023) / 1024;
    const int c0 = min(tid * chunk, nwin), c1 = min(c0 + chunk, nwin);
    int mine = 0;
    for (int t = c0; t < c1; t++)
        mine += fire[t];
    int fired;
    int pos = block_excl_scan(mine, lds, &fired);
    for (int t = c0; t < c1; t++) {
        if (fire[t]) {
            if (pos < dg.maxdet) {
                int x0, r0, w, h;
                window_box(dg, t, x0, r0, w, h);
                const int y0 = dg.top + r0;
                bx[pos] = make_short4((short)x0, (short)y0, (short)(x0 + w), (short)(y0 + h));
            }
            pos++;
        }
    }
    const int n = min(fired, dg.maxdet);
    for (int i = tid; i < n; i += 1024)
        alive[i] = 1;
    __syncthreads();

    // best partner of every box: highest IoU, then the lowest index
    for (int i = tid; i < n; i += 1024) {
        const Box a = get_box(bx, i);
        const int aa = area(a);
        int BI = -1, BU = 1, BJ = INT_MAX;
        for (int j = 0; j < n; j++) {
            if (j == i)
                continue;
            const Box b = get_box(bx, j);
            const int I = inter(a, b), U = aa + area(b) - I;
            if (ranks_before(I, U, j, BI, BU, BJ)) {
                BI = I;
                BU = U;
                BJ = j;
            }
        }
        bI[i] = BI;
        bU[i] = BU;
        bj[i] = BJ == INT_MAX ? (short)-1 : (short)BJ;
    }
    __syncthreads();

    for (;;) {
        // the pair with the highest IoU: the best box, then its partner
        int I = -1, U = 1, X = INT_MAX;
        for (int i = tid; i < n; i += 1024) {
            if (alive[i] && bj[i] >= 0 && ranks_before(bI[i], bU[i], i, I, U, X)) {
                I = bI[i];
                U = bU[i];
                X = i;
            }
        }
        wave_best(I, U, X);
        if (lane == 0) {
            redI[wave] = I;
            redU[wave] = U;
            redX[wave] = X;
        }
        __syncthreads();
        if (wave == 0) {
            I = lane < 16 ? redI[lane] : -1;
            U = lane < 16 ? redU[lane] : 1;
            X = lane < 16 ? redX[lane] : INT_MAX;
            wave_best(I, U, X);
            if (lane == 0) {
                sel[0] = I;
                sel[1] = U;
                sel[2] = X;
                nflag = 0;
            }
        }
        __syncthreads();
        const int si = sel[2];
        if (si == INT_MAX || !((double)sel[0] > dg.merge_iou * (double)sel[1]))
            break;
        const int sj = bj[si];
        const Box A = get_box(bx, si), B = get_box(bx, sj);
        const Box m{min(A.x0, B.x0), min(A.y0, B.y0), max(A.x1, B.x1), max(A.y1, B.y1)};
        const int am = area(m);
        // boxes whose partner was one of the pair search again; the others
        // only compare the merged box with their current partner
        for (int k = tid; k < n; k += 1024) {
            if (!alive[k] || k == sj)
                continue;
            if (k == si || bj[k] == si || bj[k] == sj) {
                flagged[atomicAdd(&nflag, 1)] = (short)k;
                continue;
            }
            const Box b = get_box(bx, k);
            const int Ik = inter(b, m), Uk = area(b) + am - Ik;
            if (ranks_before(Ik, Uk, si, bI[k], bU[k], bj[k])) {
                bI[k] = Ik;
                bU[k] = Uk;
                bj[k] = (short)si;
            }
        }
        __syncthreads();
        if (tid == 0) {
            bx[si] = make_short4((short)m.x0, (short)m.y0, (short)m.x1, (short)m.y1);
            alive[sj] = 0;
        }
        __syncthreads();
        const int nf = nflag;
        for (int f = wave; f < nf; f += 16) {
            const int k = flagged[f];
            const Box a = get_box(bx, k);
            const int aa = area(a);
            int BI = -1, BU = 1, BJ = INT_MAX;
            for (int j = lane; j < n; j += 64) {
                if (j == k || !alive[j])
                    continue;
                const Box b = get_box(bx, j);
                const int Ij = inter(a, b), Uj = aa + area(b) - Ij;
                if (ranks_before(Ij, Uj, j, BI, BU, BJ)) {
                    BI = Ij;
                    BU = Uj;
                    BJ = j;
                }
            }
            wave_best(BI, BU, BJ);
            if (lane == 0) {
                bI[k] = BI;
                bU[k] = BU;
                bj[k] = BJ == INT_MAX ? (short)-1 : (short)BJ;
            }
        }
        __syncthreads();
    }

    // drop boxes below the minimum area, keep list order
    const int ch2 = (n + 1023) / 1024;
    const int d0 = min(tid * ch2, n), d1 = min(d0 + ch2, n);
    int keep = 0;
    for (int i = d0; i < d1; i++)
        keep += alive[i] && (long long)area(get_box(bx, i)) >= dg.min_area;
    int kept;
    int o = block_excl_scan(keep, lds, &kept);
    for (int i = d0; i < d1; i++) {
        if (alive[i]) {
            const Box b = get_box(bx, i);
            if ((long long)area(b) >= dg.min_area) {
                out[4 * o + 0] = b.x0;
                out[4 * o + 1] = b.y0;
                out[4 * o + 2] = b.x1;
                out[4 * o + 3] = b.y1;
                o++;
            }
        }
    }
    if (tid == 0) {
        count[0] = kept;
        count[1] = fired;
    }
}

hipError_t launch_detect(const DetectGeom &dg, const double *dhat, const double *dz, const uint8_t *flags,
                         uint32_t *sat, uint8_t *fire, int32_t *boxes, int32_t *count, hipStream_t s)
{
    if (dg.rows > 0)
        hipLaunchKernelGGL(k_det_rows, dim3(dg.rows), dim3(256), 0, s, dg, dhat, dz, flags, sat);
    hipLaunchKernelGGL(k_det_cols, dim3((dg.W + 1 + 255) / 256), dim3(256), 0, s, dg, sat);
    const int nwin = dg.base[dg.nsizes];
    if (nwin > 0)
        hipLaunchKernelGGL(k_det_windows, dim3((nwin + 255) / 256), dim3(256), 0, s, dg, sat, fire);
    hipLaunchKernelGGL(k_det_group, dim3(1), dim3(1024), 0, s, dg, fire, boxes, count);
    return hipGetLastError();
}

}  // namespace sgmk
