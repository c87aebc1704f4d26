// gfx950 kernels for reduced-space SGM fused by a per-pixel Kalman filter.
//
// Stages of one frame (Section 2 of the paper):
//   census (2.1) -> [prediction: splat, zoom-hole fill, discontinuity
//   rejection, windows (2.4, Eq. 2-4)] -> ragged offsets -> Hamming cost
//   (2.1) -> Eq. 1 aggregation along 8 paths (2.2) -> winner-takes-all with
//   parabolic sub-pixel fit (2.3) -> Kalman correction (Eq. 5-6) and the
//   innovation test (Section 4).
//
// Build with -ffp-contract=off: every double-precision expression below is
// evaluated one IEEE-754 operation at a time in the order written, so the
// filter state is reproducible bit for bit.

#include "sgm_internal.h"

namespace sgmk {

// ---------------------------------------------------------------------------
// wave helpers
// ---------------------------------------------------------------------------

// DPP row rotate (within each row of 16 lanes): lane i reads lane (i+n)&15.
template <int N>
__device__ __forceinline__ int row_ror(int v)
{
    // every lane has a source, so the "old" operand is never used and the
    // move can fold into the instruction that consumes it
    return __builtin_amdgcn_mov_dpp(v, 0x120 + N, 0xF, 0xF, true);
}

// min over the 16 lanes of a DPP row; every lane receives the result
__device__ __forceinline__ int row_min16(int v)
{
    v = min(v, row_ror<8>(v));
    v = min(v, row_ror<4>(v));
    v = min(v, row_ror<2>(v));
    v = min(v, row_ror<1>(v));
    return v;
}

// a launch of a gate re-run pass with no widened pixel does nothing: that pass
// would reproduce the first one
__device__ __forceinline__ bool pass_skipped(const uint32_t *skip) { return skip && *skip == 0u; }

// order LDS traffic of the lanes of one wave (no instruction beyond waits)
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// census transform (Section 2.1)
// bit = neighbour < centre, raster order of the window skipping the centre,
// first neighbour in the most significant used bit, clamp-to-edge borders.
// One thread per pixel; a (32+2rx) x (8+2ry) tile of the image sits in LDS.
// blockIdx.z selects the left (0) or right (1) image.
// ---------------------------------------------------------------------------

constexpr int CEN_BX = 32, CEN_BY = 8, CEN_MAXR = 7;

__global__ __launch_bounds__(CEN_BX *CEN_BY) void k_census(const uint8_t *__restrict__ left,
                                                           const uint8_t *__restrict__ right, int pitch,
                                                           int W, int H, int rx, int ry,
                                                           uint64_t *__restrict__ cl, uint64_t *__restrict__ cr)
{
    __shared__ uint8_t tile[CEN_BY + 2 * CEN_MAXR][CEN_BX + 2 * CEN_MAXR];
    const uint8_t *img = blockIdx.z ? right : left;
    uint64_t *out = blockIdx.z ? cr : cl;
    const int bx0 = blockIdx.x * CEN_BX, by0 = blockIdx.y * CEN_BY;
    const int tw = CEN_BX + 2 * rx, th = CEN_BY + 2 * ry;
    for (int i = threadIdx.y * CEN_BX + threadIdx.x; i < tw * th; i += CEN_BX * CEN_BY) {
        int ty = i / tw, tx = i - ty * tw;
        int gy = min(max(by0 + ty - ry, 0), H - 1);
        int gx = min(max(bx0 + tx - rx, 0), W - 1);
        tile[ty][tx] = img[(size_t)gy * pitch + gx];
    }
    __syncthreads();
    const int x = bx0 + threadIdx.x, y = by0 + threadIdx.y;
    if (x >= W || y >= H)
        return;
    const int cyl = threadIdx.y + ry, cxl = threadIdx.x + rx;
    const int c = tile[cyl][cxl];
    uint64_t bits = 0;
    for (int dy = -ry; dy <= ry; dy++) {
        for (int dx = -rx; dx <= rx; dx++) {
            if (dx == 0 && dy == 0)
                continue;
            bits = (bits << 1) | (uint64_t)(tile[cyl + dy][cxl + dx] < c);
        }
    }
    out[(size_t)y * W + x] = bits;
}

// 9x7 specialisation (the configured window): fully unrolled, the two halves
// of the 62-bit string are built in 32-bit registers.
__global__ __launch_bounds__(CEN_BX *CEN_BY) void k_census97(const uint8_t *__restrict__ left,
                                                             const uint8_t *__restrict__ right, int pitch,
                                                             int W, int H, uint64_t *__restrict__ cl,
                                                             uint64_t *__restrict__ cr)
{
    constexpr int RX = 4, RY = 3, TW = CEN_BX + 2 * RX, TH = CEN_BY + 2 * RY;
    __shared__ uint8_t tile[TH][TW + 4];
    const uint8_t *img = blockIdx.z ? right : left;
    uint64_t *out = blockIdx.z ? cr : cl;
    const int bx0 = blockIdx.x * CEN_BX, by0 = blockIdx.y * CEN_BY;
    for (int i = threadIdx.y * CEN_BX + threadIdx.x; i < TW * TH; i += CEN_BX * CEN_BY) {
        int ty = i / TW, tx = i - ty * TW;
        int gy = min(max(by0 + ty - RY, 0), H - 1);
        int gx = min(max(bx0 + tx - RX, 0), W - 1);
        tile[ty][tx] = img[(size_t)gy * pitch + gx];
    }
    __syncthreads();
    const int x = bx0 + threadIdx.x, y = by0 + threadIdx.y;
    if (x >= W || y >= H)
        return;
    const int c = tile[threadIdx.y + RY][threadIdx.x + RX];
    uint32_t hi = 0, lo = 0;
    int n = 0;
#pragma unroll
    for (int dy = -RY; dy <= RY; dy++) {
#pragma unroll
        for (int dx = -RX; dx <= RX; dx++) {
            if (dx == 0 && dy == 0)
                continue;
            uint32_t bit = tile[threadIdx.y + RY + dy][threadIdx.x + RX + dx] < c;
            if (n < 30)
                hi = (hi << 1) | bit;
            else
                lo = (lo << 1) | bit;
            n++;
        }
    }
    out[(size_t)y * W + x] = ((uint64_t)hi << 32) | lo;
}

hipError_t launch_census(const Geometry &g, const uint8_t *left, const uint8_t *right, int pitch,
                         uint64_t *cl, uint64_t *cr, hipStream_t s)
{
    dim3 blk(CEN_BX, CEN_BY), grd((g.W + CEN_BX - 1) / CEN_BX, (g.H + CEN_BY - 1) / CEN_BY, 2);
    if (g.cw == 9 && g.ch == 7)
        hipLaunchKernelGGL(k_census97, grd, blk, 0, s, left, right, pitch, g.W, g.H, cl, cr);
    else
        hipLaunchKernelGGL(k_census, grd, blk, 0, s, left, right, pitch, g.W, g.H, g.cw / 2, g.ch / 2, cl, cr);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// windows
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint16_t pack_win(int lo, int hi) { return (uint16_t)(lo | ((hi - lo) << 8)); }

// full range everywhere (Section 2.4 initialisation); offsets are p*D
__global__ void k_full_windows(int N, int D, uint16_t *win, uint32_t *off, uint8_t *flags, double *dhat,
                               double *pm)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > N)
        return;
    off[p] = (uint32_t)p * (uint32_t)D;
    if (p == N)
        return;
    win[p] = pack_win(0, D - 1);
    flags[p] = SGM_FLAG_FULLWIN;
    dhat[p] = 0.0;
    pm[p] = 0.0;
}

hipError_t launch_full_windows(const Geometry &g, DevBuffers &b, hipStream_t s)
{
    int n = g.N + 1;
    hipLaunchKernelGGL(k_full_windows, dim3((n + 255) / 256), dim3(256), 0, s, g.N, g.D, b.win, b.off, b.flags,
                       b.dhat, b.pm);
    return hipGetLastError();
}

// caller-given windows; out-of-range windows are clamped and counted
__global__ void k_given_windows(int N, int D, const int32_t *lo, const int32_t *hi, uint16_t *win,
                                uint8_t *flags, uint32_t *status)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N)
        return;
    int l = lo[p], h = hi[p];
    int lc = min(max(l, 0), D - 1);
    int hc = min(max(h, lc), D - 1);
    if (lc != l || hc != h)
        atomicAdd(status, 1u);
    win[p] = pack_win(lc, hc);
    flags[p] = (lc == 0 && hc == D - 1) ? SGM_FLAG_FULLWIN : 0;
}

hipError_t launch_scan(const Geometry &g, DevBuffers &b, hipStream_t s, const uint32_t *skip);

__global__ void k_zero_u32(uint32_t *p) { *p = 0u; }

hipError_t launch_given_windows(const Geometry &g, DevBuffers &b, const int32_t *lo, const int32_t *hi,
                                hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, b.status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_given_windows, dim3((g.N + 255) / 256), dim3(256), 0, s, g.N, g.D, lo, hi, b.win,
                       b.flags, b.status);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    return launch_scan(g, b, s, nullptr);
}

// ---------------------------------------------------------------------------
// prediction (Section 2.4, Eq. 2-4)
// Eq. 2 as the ego-motion conjugated by the stereo projection, with the
// homogeneous division: h = ((x-cx)B, (y-cy)B, fB), h' = R h + t d,
// x' = f h'_x/h'_z + cx, y' = f h'_y/h'_z + cy, d' = fB d / h'_z,
// Phi = fB / h'_z (Eq. 3), p' = Phi^2 p + q (Eq. 4).
// Splat to the nearest pixel; z-buffer: largest d' wins, ties to the
// smallest source index.  Two atomic passes make the choice exact and
// independent of scheduling: max over the bit patterns of d' (non-negative
// doubles order like their bits), then min source index among the sources
// holding that maximum.
// ---------------------------------------------------------------------------

__global__ void k_splat(int W, int H, int D, WarpConst wc, const double *__restrict__ Tdev,
                        const double *__restrict__ d, const double *__restrict__ p, int32_t *__restrict__ tgt,
                        double *__restrict__ dprime, double *__restrict__ pprime,
                        unsigned long long *__restrict__ zkey)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= W * H)
        return;
    if (Tdev) {
        // ego-motion from device memory (row-major 4x4; graph replays update it)
#pragma unroll
        for (int i = 0; i < 12; i++)
            wc.T[i] = Tdev[i];
    }
    int y = s / W, x = s - y * W;
    double X = ((double)x - wc.cx) * wc.B;
    double Y = ((double)y - wc.cy) * wc.B;
    double ds = d[s];
    double hx = ((wc.T[0] * X + wc.T[1] * Y) + wc.T[2] * wc.fB) + wc.T[3] * ds;
    double hy = ((wc.T[4] * X + wc.T[5] * Y) + wc.T[6] * wc.fB) + wc.T[7] * ds;
    double hz = ((wc.T[8] * X + wc.T[9] * Y) + wc.T[10] * wc.fB) + wc.T[11] * ds;
    int t = -1;
    double dp = 0.0, pp = 0.0;
    if (hz > wc.zmin) {
        double xp = (wc.f * hx) / hz + wc.cx;
        double yp = (wc.f * hy) / hz + wc.cy;
        dp = (wc.fB * ds) / hz;
        double phi = wc.fB / hz;
        pp = (phi * phi) * p[s] + wc.q;
        double ux = xp + 0.5, uy = yp + 0.5;
        if (ux >= 0.0 && ux < (double)W && uy >= 0.0 && uy < (double)H && dp <= (double)(D - 1)) {
            int tx = (int)floor(ux), ty = (int)floor(uy);
            t = ty * W + tx;
            atomicMax(&zkey[t], (unsigned long long)__double_as_longlong(dp));
        }
    }
    tgt[s] = t;
    dprime[s] = dp;
    pprime[s] = pp;
}

__global__ void k_splat_ties(int N, const int32_t *__restrict__ tgt, const double *__restrict__ dprime,
                             const unsigned long long *__restrict__ zkey, uint32_t *__restrict__ zidx)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N)
        return;
    int t = tgt[s];
    if (t >= 0 && (unsigned long long)__double_as_longlong(dprime[s]) == zkey[t])
        atomicMin(&zidx[t], (uint32_t)s);
}

// gather the winner; re-arm the z-buffer for the next frame
__global__ void k_splat_resolve(int N, unsigned long long *__restrict__ zkey, uint32_t *__restrict__ zidx,
                                const double *__restrict__ dprime, const double *__restrict__ pprime,
                                const uint8_t *__restrict__ sflags, const double *__restrict__ nu,
                                uint8_t *__restrict__ has, double *__restrict__ dw, double *__restrict__ pw,
                                uint8_t *__restrict__ rw, double *__restrict__ nu_w)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N)
        return;
    uint32_t w = zidx[t];
    if (w != 0xFFFFFFFFu) {
        has[t] = 1;
        dw[t] = dprime[w];
        pw[t] = pprime[w];
        rw[t] = sflags[w] & SGM_FLAG_RESET;
        nu_w[t] = nu[w];
    } else {
        has[t] = 0;
        dw[t] = 0.0;
        pw[t] = 0.0;
        rw[t] = 0;
        nu_w[t] = 0.0;
    }
    zkey[t] = 0ull;
    zidx[t] = 0xFFFFFFFFu;
}

// zooming holes: a target without a winner whose left & right (or upper &
// lower) neighbours both have winners takes their mean disparity and mean
// variance; with both pairs, the mean of four (summed left, right, up, down).
// The splat results are read from a tile staged in LDS: entry s is pixel
// (x, y), its row neighbours are s -/+ 1 and its column neighbours s -/+ ls.
__device__ __forceinline__ void fill_hole(int W, int H, int s, int ls, int x, int y, const uint8_t *has,
                                          const double *dw, const double *pw, const uint8_t *rw, uint8_t &pr,
                                          double &dv, double &pv, uint8_t &rv)
{
    pr = has[s];
    dv = dw[s];
    pv = pw[s];
    rv = rw[s];
    if (pr)
        return;
    const bool hp = x - 1 >= 0 && x + 1 < W && has[s - 1] && has[s + 1];
    const bool vp = y - 1 >= 0 && y + 1 < H && has[s - ls] && has[s + ls];
    if (hp && vp) {
        dv = (((dw[s - 1] + dw[s + 1]) + dw[s - ls]) + dw[s + ls]) / 4.0;
        pv = (((pw[s - 1] + pw[s + 1]) + pw[s - ls]) + pw[s + ls]) / 4.0;
        rv = rw[s - 1] | rw[s + 1] | rw[s - ls] | rw[s + ls];
        pr = 1;
    } else if (hp) {
        dv = (dw[s - 1] + dw[s + 1]) / 2.0;
        pv = (pw[s - 1] + pw[s + 1]) / 2.0;
        rv = rw[s - 1] | rw[s + 1];
        pr = 1;
    } else if (vp) {
        dv = (dw[s - ls] + dw[s + ls]) / 2.0;
        pv = (pw[s - ls] + pw[s + ls]) / 2.0;
        rv = rw[s - ls] | rw[s + ls];
        pr = 1;
    }
}

// Hole fill, then discontinuity rejection (8-neighbourhood of the filled
// map, decided before any rejection) and the search limits d^ +- k sigma,
// rounded outward.  A block fills a 64 x 4 tile plus a one-pixel halo in
// LDS, so the filled map never goes to memory; the splat results it reads
// (the tile plus a two-pixel margin) are staged in LDS first, all loads at once.
constexpr int FD_TW = 64, FD_TH = 4, FD_LW = FD_TW + 2, FD_LN = FD_LW * (FD_TH + 2);
constexpr int FD_SW = FD_TW + 4, FD_SN = FD_SW * (FD_TH + 4);
constexpr int FD_SPER = (FD_SN + FD_TW * FD_TH - 1) / (FD_TW * FD_TH);   // staged entries per thread

__global__ __launch_bounds__(FD_TW *FD_TH) void k_fill_disc(int W, int H, int D, CorrectConst cc,
                                                            const uint8_t *__restrict__ has,
                                                            const double *__restrict__ dw,
                                                            const double *__restrict__ pw,
                                                            const uint8_t *__restrict__ rw, uint8_t *__restrict__ flags,
                                                            uint16_t *__restrict__ win, double *__restrict__ dhat,
                                                            double *__restrict__ pm, double *__restrict__ nu_w)
{
    __shared__ double sd[FD_LN], sp[FD_LN];
    __shared__ uint8_t spr[FD_LN], srs[FD_LN];
    __shared__ double gdw[FD_SN], gpw[FD_SN];
    __shared__ uint8_t ghas[FD_SN], grw[FD_SN];
    const int x0 = blockIdx.x * FD_TW - 1, y0 = blockIdx.y * FD_TH - 1;
    {
        // stage the splat results of pixels (x0 - 1 .., y0 - 1 ..); outside the image: none
        double vd[FD_SPER], vp[FD_SPER];
        uint8_t vh[FD_SPER], vr[FD_SPER];
#pragma unroll
        for (int k = 0; k < FD_SPER; k++) {
            const int i = threadIdx.x + k * FD_TW * FD_TH;
            const int sy = i / FD_SW, sx = i - sy * FD_SW;
            const int x = x0 - 1 + sx, y = y0 - 1 + sy;
            const bool in = i < FD_SN && x >= 0 && x < W && y >= 0 && y < H;
            const int t = in ? y * W + x : 0;
            vh[k] = has[t];
            vr[k] = rw[t];
            vd[k] = dw[t];
            vp[k] = pw[t];
            if (!in)
                vh[k] = vr[k] = 0;
        }
#pragma unroll
        for (int k = 0; k < FD_SPER; k++) {
            const int i = threadIdx.x + k * FD_TW * FD_TH;
            if (i < FD_SN) {
                ghas[i] = vh[k];
                grw[i] = vr[k];
                gdw[i] = vd[k];
                gpw[i] = vp[k];
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < FD_LN; i += FD_TW * FD_TH) {
        const int ly = i / FD_LW, lx = i - ly * FD_LW;
        const int x = x0 + lx, y = y0 + ly;
        uint8_t pr = 0, rv = 0;
        double dv = 0.0, pv = 0.0;
        if (x >= 0 && x < W && y >= 0 && y < H)
            fill_hole(W, H, (ly + 1) * FD_SW + lx + 1, FD_SW, x, y, ghas, gdw, gpw, grw, pr, dv, pv, rv);
        spr[i] = pr;   // outside the image: no prediction (no neighbour)
        sd[i] = dv;
        sp[i] = pv;
        srs[i] = rv;
    }
    __syncthreads();
    const int lx = threadIdx.x % FD_TW + 1, ly = threadIdx.x / FD_TW + 1;
    const int x = x0 + lx, y = y0 + ly;
    if (x >= W || y >= H)
        return;
    const int c = ly * FD_LW + lx, t = y * W + x;
    bool ok = spr[c];
    const double dv = sd[c];
    if (ok) {
        for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++) {
                const int u = c + dy * FD_LW + dx;
                if ((dx || dy) && spr[u] && fabs(dv - sd[u]) > cc.disc)
                    ok = false;
            }
    }
    const uint8_t rs = srs[c];
    uint8_t fl = 0;
    if (ok)
        fl |= SGM_FLAG_PRED;
    if (rs)
        fl |= SGM_FLAG_RESET;
    const bool full = !ok || rs || !(dv >= 0.0 && dv <= (double)(D - 1));
    const double pv = sp[c];
    if (full) {
        fl |= SGM_FLAG_FULLWIN;
        win[t] = pack_win(0, D - 1);
    } else {
        const double sdv = sqrt(pv);
        const double a = dv - cc.k_sigma * sdv;
        const double b = dv + cc.k_sigma * sdv;
        int l = (int)floor(a), h = (int)ceil(b);
        l = l < 0 ? 0 : l;
        h = h > D - 1 ? D - 1 : h;
        win[t] = pack_win(l, h);
    }
    flags[t] = fl;
    dhat[t] = ok ? dv : 0.0;
    pm[t] = ok ? pv : 0.0;
    if (!ok)
        nu_w[t] = 0.0;
}

hipError_t launch_predict(const Geometry &g, DevBuffers &b, const WarpConst &wc, const double *Tdev,
                          const CorrectConst &cc, hipStream_t s)
{
    hipError_t e = launch_predict_core(g, b, wc, Tdev, cc, s);
    if (e != hipSuccess)
        return e;
    return launch_scan(g, b, s, nullptr);
}

hipError_t launch_predict_core(const Geometry &g, DevBuffers &b, const WarpConst &wc, const double *Tdev,
                               const CorrectConst &cc, hipStream_t s)
{
    dim3 blk(256), grd((g.N + 255) / 256);
    hipLaunchKernelGGL(k_splat, grd, blk, 0, s, g.W, g.H, g.D, wc, Tdev, b.d, b.p, b.tgt, b.dprime, b.pprime,
                       b.zkey);
    hipLaunchKernelGGL(k_splat_ties, grd, blk, 0, s, g.N, b.tgt, b.dprime, b.zkey, b.zidx);
    hipLaunchKernelGGL(k_splat_resolve, grd, blk, 0, s, g.N, b.zkey, b.zidx, b.dprime, b.pprime, b.sflags, b.nu,
                       b.has, b.dw, b.pw, b.rw, b.nu_w);
    hipLaunchKernelGGL(k_fill_disc, dim3((g.W + FD_TW - 1) / FD_TW, (g.H + FD_TH - 1) / FD_TH), dim3(FD_TW * FD_TH), 0,
                       s, g.W, g.H, g.D, cc, b.has, b.dw, b.pw, b.rw, b.flags, b.win, b.dhat, b.pm, b.nu_w);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// ragged offsets: exclusive prefix sum of the window widths (4096 pixels
// per block, see k_scan_sums / k_scan_apply).  off[N] is the total cell
// count M.
// ---------------------------------------------------------------------------

constexpr int SCAN_T = 1024, SCAN_PER = 4, SCAN_BLOCK = SCAN_T * SCAN_PER;

__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *total)
{
    __shared__ uint32_t wsum[SCAN_T / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t u = __shfl_up(incl, o, 64);
        if (lane >= o)
            incl += u;
    }
    if (lane == 63)
        wsum[wv] = incl;
    __syncthreads();
    if (wv == 0) {
        uint32_t w = lane < SCAN_T / 64 ? wsum[lane] : 0u;
        uint32_t wi = w;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            uint32_t u = __shfl_up(wi, o, 64);
            if (lane >= o)
                wi += u;
        }
        if (lane < SCAN_T / 64)
            wsum[lane] = wi - w;
        if (lane == SCAN_T / 64 - 1)
            *total = wi;
    }
    __syncthreads();
    return incl - v + wsum[wv];
}

// Two passes: the window widths summed per block of SCAN_BLOCK pixels, then
// each block adds the sums of the blocks before it to its own exclusive scan
// (the block sums are few, so every block reads them all).
__global__ __launch_bounds__(SCAN_T) void k_scan_sums(int N, const uint16_t *__restrict__ win,
                                                      uint32_t *__restrict__ part, const uint32_t *skip)
{
    if (pass_skipped(skip))
        return;
    __shared__ uint32_t tot;
    const int base = blockIdx.x * SCAN_BLOCK + threadIdx.x * SCAN_PER;
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < SCAN_PER; i++) {
        const int p = base + i;
        sum += p < N ? (uint32_t)(win[p] >> 8) + 1u : 0u;
    }
    (void)block_excl_scan(sum, &tot);
    if (threadIdx.x == 0)
        part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_apply(int N, const uint16_t *__restrict__ win,
                                                       uint32_t *__restrict__ off,
                                                       const uint32_t *__restrict__ part, const uint32_t *skip)
{
    if (pass_skipped(skip))
        return;
    __shared__ uint32_t tot, before_tot;
    // sum of the block sums before this block
    uint32_t pre = 0;
    for (int i = threadIdx.x; i < (int)blockIdx.x; i += SCAN_T)
        pre += part[i];
    (void)block_excl_scan(pre, &before_tot);
    const uint32_t before = before_tot;
    const int base = blockIdx.x * SCAN_BLOCK + threadIdx.x * SCAN_PER;
    uint32_t w[SCAN_PER];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < SCAN_PER; i++) {
        const int p = base + i;
        w[i] = p < N ? (uint32_t)(win[p] >> 8) + 1u : 0u;
        sum += w[i];
    }
    uint32_t ex = before + block_excl_scan(sum, &tot);
#pragma unroll
    for (int i = 0; i < SCAN_PER; i++) {
        const int p = base + i;
        if (p < N)
            off[p] = ex;
        ex += w[i];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0)
        off[N] = before + tot;
}

hipError_t launch_scan(const Geometry &g, DevBuffers &b, hipStream_t s, const uint32_t *skip)
{
    int nparts = (g.N + SCAN_BLOCK - 1) / SCAN_BLOCK;   // <= SCAN_BLOCK, checked at create
    hipLaunchKernelGGL(k_scan_sums, dim3(nparts), dim3(SCAN_T), 0, s, g.N, b.win, b.scan_part, skip);
    hipLaunchKernelGGL(k_scan_apply, dim3(nparts), dim3(SCAN_T), 0, s, g.N, b.win, b.off, b.scan_part, skip);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Hamming cost (Section 2.1) on the ragged volume.
// A block owns PIX consecutive pixels; their cells are the contiguous range
// [off[p0], off[p0+PIX]).  Threads stride over that range (coalesced
// stores) and find their pixel by binary search over the block's offsets.
// ---------------------------------------------------------------------------

constexpr int COST_PIX = 256;

__device__ __forceinline__ int find_pixel(const uint32_t *offs, int n, uint32_t c)
{
    // largest i in [0, n) with offs[i] <= c
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (offs[mid] <= c)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(COST_PIX) void k_cost(int W, int N, int nbits, const uint64_t *__restrict__ cl,
                                                   const uint64_t *__restrict__ cr, const uint16_t *__restrict__ win,
                                                   const uint32_t *__restrict__ off, uint8_t *__restrict__ cost)
{
    __shared__ uint32_t soff[COST_PIX];
    __shared__ uint16_t swin[COST_PIX];
    __shared__ uint64_t scl[COST_PIX];
    const int p0 = blockIdx.x * COST_PIX;
    const int np = min(COST_PIX, N - p0);
    if ((int)threadIdx.x < np) {
        soff[threadIdx.x] = off[p0 + threadIdx.x];
        swin[threadIdx.x] = win[p0 + threadIdx.x];
        scl[threadIdx.x] = cl[p0 + threadIdx.x];
    }
    __syncthreads();
    const uint32_t c0 = soff[0], c1 = off[p0 + np];
    for (uint32_t c = c0 + threadIdx.x; c < c1; c += COST_PIX) {
        int i = find_pixel(soff, np, c);
        int p = p0 + i;
        int d = (swin[i] & 255) + (int)(c - soff[i]);
        int x = p % W;
        uint8_t v;
        if (x - d < 0)
            v = (uint8_t)nbits;
        else
            v = (uint8_t)__popcll(scl[i] ^ cr[p - d]);
        cost[c] = v;
    }
}

hipError_t launch_cost(const Geometry &g, DevBuffers &b, hipStream_t s)
{
    hipLaunchKernelGGL(k_cost, dim3((g.N + COST_PIX - 1) / COST_PIX), dim3(COST_PIX), 0, s, g.W, g.N, g.nbits,
                       b.cen_l, b.cen_r, b.win, b.off, b.cost);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Eq. 1 aggregation on ragged windows (Section 2.2).
//
// A group of G lanes walks one scanline of one path direction.  Lanes map to
// ABSOLUTE disparities: lane l of chunk j holds d = j*G + l, for the chunks
// that intersect the current pixel's window.  The predecessor's L_r(q, d)
// therefore stays in the same lane and register from one pixel to the next,
// its neighbours d-1 and d+1 come from the adjacent lanes through DPP, and
// the recurrence never touches memory:
//   L_r(p,d) = C(p,d) + min(L(q,d), L(q,d-1)+P1, L(q,d+1)+P1, m_q+P2) - m_q
// with q = p - r and m_q the minimum over q's window; any term whose
// disparity lies outside q's window is absent, and the first pixel of a
// scanline takes L_r = C.  Register values outside the window they were
// computed for are never read unmasked, so chunks a pixel does not touch
// can keep stale values.  The matching cost C(p,d) = popcount(cL(p) xor
// cR(x-d)) (the number of census bits when x-d < 0) is computed in place
// from census strings staged in LDS; the cost volume never goes through
// HBM.  Results are stored per path as bytes in the ragged layout
// (L_r <= Nc + P2 <= 255, checked at create).
//
// Global loads are issued one batch ahead into registers that are read only
// at the batch boundary, where they are written to LDS; the next pixel's
// metadata and right census are read from LDS while the current pixel is
// processed.
//   k_agg_h: horizontal paths, one scanline (image row) per wave (G = 64);
//            the row's right census is staged once, windows/offsets/left
//            census stream through an LDS ring one batch ahead.
//   k_agg_v: vertical and diagonal paths, G = 16 (a DPP row): 16 adjacent
//            scanlines per block of four waves (adjacent columns, or adjacent
//            diagonals, which cover a contiguous run of pixels at every row);
//            each batch of rows stages the run's census strings, windows,
//            offsets and the right-census span it can match against.
// ---------------------------------------------------------------------------

struct AggArgs {
    const uint64_t *cl, *cr;
    const uint16_t *win;
    const uint32_t *off;
    uint8_t *lr;
    size_t lr_stride;
    int W, H, D, nbits, p1, p2;
    int8_t rx[kMaxPaths], ry[kMaxPaths];
    int8_t slot[kMaxPaths];   // output buffer index of each listed path
    int kmin[kMaxPaths];      // first chain index of each listed path (k_agg_v)
    uint8_t *hflag;           // horizontal segments whose two trajectories never met [path][H][AH2_MAXSEG]
    const uint32_t *skip;     // when not NULL and *skip == 0 the launch does nothing (gate re-run pass)
};


constexpr int LBIG = 0x3FFF;   // "absent" predecessor term (> any L_r + P1)

// DPP move: row_shr:1 (0x111) / wave_shr:1 (0x138) give lane i the value of
// lane i-1, row_shl:1 (0x101) / wave_shl:1 (0x130) that of lane i+1,
// row_ror:n (0x120+n) that of lane (i-n) mod 16 of the same row; lanes
// without a source receive LBIG.
template <int CTRL>
__device__ __forceinline__ int dpp(int v)
{
    return __builtin_amdgcn_update_dpp(LBIG, v, CTRL, 0xF, 0xF, false);
}

// lane i <- lane i-1 / i+1 of the same group (the group's first / last lane
// receives LBIG and is patched by the caller)
template <int G>
__device__ __forceinline__ int from_prev_lane(int v) { return G == 64 ? dpp<0x138>(v) : dpp<0x111>(v); }
template <int G>
__device__ __forceinline__ int from_next_lane(int v) { return G == 64 ? dpp<0x130>(v) : dpp<0x101>(v); }

// min over a group of G lanes, result in every lane of the group
template <int G>
__device__ __forceinline__ int group_min(int v)
{
    v = row_min16(v);
    if (G == 32) {
        // two groups per wave: combine the row minima with scalar reads
        // (a cross-lane shuffle would take an LDS round trip)
        const int a = min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16));
        const int b = min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48));
        v = (threadIdx.x & 32) ? b : a;
    }
    if (G == 64) {
        int a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 16);
        int c = __builtin_amdgcn_readlane(v, 32), d = __builtin_amdgcn_readlane(v, 48);
        v = min(min(a, b), min(c, d));
    }
    return v;
}

// min / max of a group-uniform value over the four 16-lane groups of a wave
__device__ __forceinline__ int wave_min4(int v)
{
    int a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 16);
    int c = __builtin_amdgcn_readlane(v, 32), d = __builtin_amdgcn_readlane(v, 48);
    return min(min(a, b), min(c, d));
}
__device__ __forceinline__ int wave_max4(int v)
{
    int a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 16);
    int c = __builtin_amdgcn_readlane(v, 32), d = __builtin_amdgcn_readlane(v, 48);
    return max(max(a, b), max(c, d));
}

// Per-group recurrence state: L_r of the previous pixel by absolute
// disparity, LBIG outside its window (so absent terms need no test), and
// its minimum.
template <int MAXCH>
struct Chain {
    int Lp[MAXCH];
    int mq;
};

// right census needed by chunk j at column x (crow[i] holds column crow_x0+i;
// x-d < 0 reads entry 0 and is replaced by the fixed cost)
template <int G, int MAXCH>
__device__ __forceinline__ void read_crow(uint64_t (&crv)[MAXCH], const uint64_t *crow, int crow_x0, int x, int lane,
                                          int jlo, int jhi)
{
#pragma unroll
    for (int j = 0; j < MAXCH; j++) {
        if (j < jlo || j > jhi)
            continue;
        const int d = j * G + lane;
        crv[j] = crow[max(x - d - crow_x0, 0)];
    }
}

// every chunk, unconditionally: a fixed number of LDS reads per step keeps
// the wait counters exact, so a read issued for the next step is not waited
// for in this one
template <int G, int MAXCH>
__device__ __forceinline__ void read_crow_all(uint64_t (&crv)[MAXCH], const uint64_t *crow, int x, int lane)
{
#pragma unroll
    for (int j = 0; j < MAXCH; j++)
        crv[j] = crow[max(x - (j * G + lane), 0)];
}

// min over the G lanes of a group with DPP, result in every lane of the group
template <int G>
__device__ __forceinline__ int group_min_dpp(int v)
{
    v = min(v, __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, false));   // row_ror:8
    v = min(v, __builtin_amdgcn_mov_dpp(v, 0x124, 0xF, 0xF, false));   // row_ror:4
    v = min(v, __builtin_amdgcn_mov_dpp(v, 0x122, 0xF, 0xF, false));   // row_ror:2
    v = min(v, __builtin_amdgcn_mov_dpp(v, 0x121, 0xF, 0xF, false));   // row_ror:1
    if (G == 64) {
        // every lane holds its row's minimum: combine the four rows
        v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x142, 0xA, 0xF, false));   // row_bcast:15 -> rows 1, 3
        v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x143, 0xC, 0xF, false));   // row_bcast:31 -> rows 2, 3
        v = __builtin_amdgcn_readlane(v, 63);
    }
    return v;
}

// One step of Eq. 1 for this group's pixel (column x, window [lo, hi],
// ragged offset oc).  Chunks jlo..jhi (uniform over the wave) are computed,
// the others are reset to LBIG; `active`: this group has a pixel at this
// step (uniform per group).
template <int G, int MAXCH>
__device__ __forceinline__ void agg_step(Chain<MAXCH> &st, int lane, bool active, bool first, uint64_t clp, int x,
                                         int lo, int hi, uint32_t oc, const uint64_t (&crv)[MAXCH], int jlo, int jhi,
                                         int p1, int p2, int nbits, uint8_t *lrk)
{
    int Ln[MAXCH];
    int rmin = LBIG;
    const int mq = st.mq;
    const int cap = first ? LBIG : mq + p2;    // the P2 term (none on the first pixel)
    const int base = first ? 0 : -mq;
#pragma unroll
    for (int j = 0; j < MAXCH; j++) {
        Ln[j] = LBIG;
        if (j < jlo || j > jhi)
            continue;
        const int d = j * G + lane;
        // neighbours at d-1 and d+1 in the previous pixel's registers
        int pm = from_prev_lane<G>(st.Lp[j]);
        int pp = from_next_lane<G>(st.Lp[j]);
        if (j > 0) {
            const int edge = G == 64 ? __builtin_amdgcn_readlane(st.Lp[j - 1], 63) : dpp<0x121>(st.Lp[j - 1]);
            pm = lane == 0 ? edge : pm;
        }
        if (j < MAXCH - 1) {
            const int edge = G == 64 ? __builtin_amdgcn_readlane(st.Lp[j + 1], 0) : dpp<0x12F>(st.Lp[j + 1]);
            pp = lane == G - 1 ? edge : pp;
        }
        const int best = first ? 0 : min(min(st.Lp[j], cap), min(pm, pp) + p1);
        const int c = d > x ? nbits : __popcll(clp ^ crv[j]);
        const int L = c + best + base;
        const bool in = active && (unsigned)(d - lo) <= (unsigned)(hi - lo);
        Ln[j] = in ? L : LBIG;
        rmin = min(rmin, Ln[j]);
    }
#pragma unroll
    for (int j = 0; j < MAXCH; j++) {
        if (j < jlo || j > jhi)
            continue;
        const int d = j * G + lane;
        if (Ln[j] != LBIG)
            lrk[oc + (uint32_t)(d - lo)] = (uint8_t)Ln[j];
    }
    const int m = group_min_dpp<G>(rmin);
    if (active) {
#pragma unroll
        for (int j = 0; j < MAXCH; j++)
            st.Lp[j] = Ln[j];
        st.mq = m;
    }
}

struct MetaEntry {
    uint64_t cl;
    uint32_t off, win;
};

// ---- horizontal paths: one scanline per wave ------------------------------

constexpr int AH_B = 64;   // batch of pixels per metadata load (one per lane)

__host__ __device__ constexpr size_t agg_h_lds(int W) { return (size_t)W * 8; }

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

template <int MAXCH>
__global__ __launch_bounds__(64) void k_agg_h(AggArgs a, int raise_prio)
{
    if (pass_skipped(a.skip))
        return;
    // with ragged windows (D <= 64, or the other kernel chosen) its waves
    // issue at the vertical kernel's priority; dense windows keep the default
    if (raise_prio)
        __builtin_amdgcn_s_setprio(1);
    constexpr int G = 64;
    extern __shared__ __align__(16) uint8_t smem[];
    const int W = a.W;
    uint64_t *crow = (uint64_t *)smem;   // [W]
    const int pi = blockIdx.y;
    const int k = a.slot[pi];
    const int rx = a.rx[pi];
    const int lane = threadIdx.x;
    const int row = blockIdx.x;
    const int rowp = row * W;
    // stage the row's right census
    {
        const uint64_t *src = a.cr + (size_t)rowp;
        if ((rowp & 1) == 0) {
            const uint4 *s4 = (const uint4 *)src;
            uint4 *d4 = (uint4 *)crow;
#pragma unroll 8
            for (int i = lane; i < W / 2; i += 64)
                d4[i] = s4[i];
            if ((W & 1) && lane == 0)
                crow[W - 1] = src[W - 1];
        } else {
#pragma unroll 8
            for (int i = lane; i < W; i += 64)
                crow[i] = src[i];
        }
    }
    // metadata batches live in registers, one pixel per lane
    auto px = [&](int t) { return rowp + (rx > 0 ? t : W - 1 - t); };
    uint64_t bcl;
    uint32_t boff, bwin;
    {
        const int p = px(min(lane, W - 1));
        bcl = a.cl[p];
        boff = a.off[p];
        bwin = a.win[p];
    }
    __syncthreads();
    uint8_t *lrk = a.lr + (size_t)k * a.lr_stride;
    const int p1 = a.p1, p2 = a.p2, nbits = a.nbits;
    Chain<MAXCH> st;
#pragma unroll
    for (int j = 0; j < MAXCH; j++)
        st.Lp[j] = LBIG;
    st.mq = 0;
    uint64_t crvA[MAXCH], crvB[MAXCH];
    read_crow_all<G, MAXCH>(crvA, crow, rx > 0 ? 0 : W - 1, lane);   // pixel 0's right census
    // one step: pixel t (metadata from lane s of the batch registers) with
    // census `cur`; the census of pixel t+1 is read into `nxt`
    auto step = [&](int t, int s, uint64_t nb_cl, uint32_t nb_off, uint32_t nb_win, uint64_t(&cur)[MAXCH],
                    uint64_t(&nxt)[MAXCH]) {
        const uint64_t cl = readlane64(bcl, s);
        const uint32_t off = (uint32_t)__builtin_amdgcn_readlane((int)boff, s);
        const uint32_t win = (uint32_t)__builtin_amdgcn_readlane((int)bwin, s);
        read_crow_all<G, MAXCH>(nxt, crow, rx > 0 ? min(t + 1, W - 1) : max(W - 2 - t, 0), lane);
        const int lo = (int)(win & 255), hi = lo + (int)(win >> 8);
        agg_step<G, MAXCH>(st, lane, true, t == 0, cl, rx > 0 ? t : W - 1 - t, lo, hi, off, cur, lo / G, hi / G,
                           p1, p2, nbits, lrk);
        (void)nb_cl;
        (void)nb_off;
    };
    const int nb = (W + AH_B - 1) / AH_B;
    for (int b = 0; b < nb; b++) {
        // next batch, requested a batch ahead
        const int p = px(min((b + 1) * AH_B + lane, W - 1));
        const uint64_t ncl = a.cl[p];
        const uint32_t noff = a.off[p], nwin = a.win[p];
        const int steps = min(AH_B, W - b * AH_B);
        int s = 0;
        for (; s + 1 < steps; s += 2) {
            step(b * AH_B + s, s, ncl, noff, nwin, crvA, crvB);
            step(b * AH_B + s + 1, s + 1, ncl, noff, nwin, crvB, crvA);
        }
        if (s < steps) {
            // odd tail (last batch only): one step, then the census is in B
            step(b * AH_B + s, s, ncl, noff, nwin, crvA, crvB);
#pragma unroll
            for (int j = 0; j < MAXCH; j++)
                crvA[j] = crvB[j];
        }
        bcl = ncl;
        boff = noff;
        bwin = nwin;
    }
}

// ---- vertical and diagonal paths ------------------------------------------

constexpr int AV_G = 16, AV_NG = 16, AV_T = AV_G * AV_NG, AV_B = 8;

__host__ __device__ constexpr int agg_v_span(int D) { return AV_NG + D - 1; }

__host__ __device__ constexpr size_t agg_v_lds(int D)
{
    return (size_t)2 * AV_B * agg_v_span(D) * 8 + (size_t)2 * AV_B * AV_NG * sizeof(MetaEntry);
}

// loads of one batch of rows held in registers between issue and LDS write
constexpr int AV_MAXCR = (AV_B * (AV_NG + kMaxDisp - 1) + AV_T - 1) / AV_T;   // per thread

template <int MAXCH>
__global__ __launch_bounds__(AV_T) void k_agg_v(AggArgs a)
{
    extern __shared__ __align__(16) uint8_t smem[];
    const int W = a.W, H = a.H, D = a.D;
    const int span = AV_NG + D - 1;
    uint64_t *cbuf = (uint64_t *)smem;                                            // [2][B][span]
    MetaEntry *mbuf = (MetaEntry *)(smem + (size_t)2 * AV_B * span * 8);          // [2][B][NG]
    const int pi = blockIdx.y;
    const int k = a.slot[pi];
    const int rx = a.rx[pi], ry = a.ry[pi];
    const int kmin = a.kmin[pi];
    const int nchains = rx == 0 ? W : W + H - 1;
    if (blockIdx.x * AV_NG >= nchains)
        return;                                        // uniform over the block
    const int kb = kmin + blockIdx.x * AV_NG;          // chain index of group 0
    const int grp = threadIdx.x / AV_G, lane = threadIdx.x % AV_G;
    const int kc = kb + grp;
    const bool chain_ok = blockIdx.x * AV_NG + grp < nchains;
    const int ys = ry > 0 ? 0 : H - 1;
    uint8_t *lrk = a.lr + (size_t)k * a.lr_stride;
    const int p1 = a.p1, p2 = a.p2, nbits = a.nbits;

    // sweep row t: y = ys + ry*t, chain kc sits at x = kc + rx*t.  The block's
    // run is x in [kb + rx*t, kb + NG-1 + rx*t]; its matching span starts
    // D-1 columns left of the run.
    auto span_x0 = [&](int t) { return kb + rx * t - (D - 1); };

    uint64_t rc[AV_MAXCR];
    uint64_t rmcl;
    uint32_t rmoff, rmwin;
    auto issue = [&](int bt) {
#pragma unroll
        for (int i = 0; i < AV_MAXCR; i++) {
            const int e = threadIdx.x + i * AV_T;
            const int r = e / span, c = e - r * span;
            const int t = bt * AV_B + r;
            const int xx = span_x0(t) + c;
            const bool ok = r < AV_B && t < H && xx >= 0 && xx < W;
            const size_t idx = ok ? (size_t)(ys + ry * t) * W + xx : 0;
            const uint64_t v = a.cr[idx];
            rc[i] = ok ? v : 0ull;
        }
        {
            const int e = threadIdx.x;   // AV_B * AV_NG = 128 entries
            const int r = e / AV_NG, g = e - r * AV_NG;
            const int t = bt * AV_B + r;
            const int xx = kb + g + rx * t;
            const bool ok = e < AV_B * AV_NG && t < H && xx >= 0 && xx < W;
            const int pix = ok ? (ys + ry * t) * W + xx : 0;
            const uint64_t vcl = a.cl[pix];
            const uint32_t voff = a.off[pix], vwin = a.win[pix];
            rmcl = ok ? vcl : 0ull;
            rmoff = ok ? voff : 0u;
            rmwin = ok ? vwin : 0u;
        }
    };
    auto commit = [&](int buf) {
        uint64_t *cb = cbuf + (size_t)buf * AV_B * span;
#pragma unroll
        for (int i = 0; i < AV_MAXCR; i++) {
            const int e = threadIdx.x + i * AV_T;
            if (e < AV_B * span)
                cb[e] = rc[i];
        }
        if (threadIdx.x < AV_B * AV_NG) {
            MetaEntry m;
            m.cl = rmcl;
            m.off = rmoff;
            m.win = rmwin;
            mbuf[buf * AV_B * AV_NG + threadIdx.x] = m;
        }
    };
    issue(0);
    commit(0);
    __syncthreads();
    Chain<MAXCH> st;
#pragma unroll
    for (int j = 0; j < MAXCH; j++)
        st.Lp[j] = LBIG;
    st.mq = 0;
    bool started = false;
    const int nbt = (H + AV_B - 1) / AV_B;
    for (int bt = 0; bt < nbt; bt++) {
        issue(bt + 1);
        const uint64_t *cb = cbuf + (size_t)(bt & 1) * AV_B * span;
        const MetaEntry *mb = mbuf + (bt & 1) * AV_B * AV_NG;
        const int rows = min(AV_B, H - bt * AV_B);
        for (int r = 0; r < rows; r++) {
            const int t = bt * AV_B + r;
            const int x = kc + rx * t;
            const bool act = chain_ok && x >= 0 && x < W;   // uniform per group
            const MetaEntry e = mb[r * AV_NG + grp];
            const int lo = (int)(e.win & 255), hi = lo + (int)(e.win >> 8);
            // chunks touched by any active group of the wave
            const int jlo = wave_min4(act ? lo / AV_G : MAXCH);
            const int jhi = wave_max4(act ? hi / AV_G : -1);
            if (jlo <= jhi) {
                uint64_t crv[MAXCH];
                read_crow<AV_G, MAXCH>(crv, cb + (size_t)r * span, span_x0(t), x, lane, jlo, jhi);
                agg_step<AV_G, MAXCH>(st, lane, act, !started, e.cl, x, lo, hi, e.off, crv, jlo, jhi, p1, p2, nbits,
                                      lrk);
                started = started || act;
            }
        }
        // buffer (bt+1)&1 was last read in batch bt-1, which the previous
        // barrier closed; this barrier publishes it for batch bt+1
        commit((bt + 1) & 1);
        __syncthreads();
    }
}

// ---- vertical and diagonal paths, LDS-resident recurrence state ----------
//
// Staging as in k_agg_v (NG chains per block, 8-row batches of right census
// and pixel metadata in LDS, here in one buffer), but each chain (a group of
// G lanes) keeps the previous pixel's L_r in LDS, indexed by absolute
// disparity (slot d + 4, two buffers by step parity), and reads its d-1, d,
// d+1 terms back masked by that pixel's window.  A step first covers the
// disparities lo .. lo + G - 1 of its window, one per lane, which is the whole
// of a narrow window.  The rest of a wider window (full range, wide learned
// windows) is covered in quads: lane i of a group computes the four
// disparities 4m .. 4m + 3 of quad m, G quads per round from the quad holding
// lo + G, so a full-range step at D = 128 takes one narrow pass and two
// rounds (16 lanes) or one (32 lanes) instead of eight or four passes.  A
// quad's six predecessor terms and its four results are then aligned LDS
// words.  The rounds run to the largest count among the wave's chains.

// max of a group-uniform value over the groups of G lanes of a wave
template <int G>
__device__ __forceinline__ int group_max(int v)
{
    if (G == 16)
        return wave_max4(v);
    return max(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 32));
}
constexpr int AV2_OFF = 4;   // state slot of disparity d is d + 4 (quads start on 8-byte words)

// slots per chain: idle lanes clamp to disparity (D + 3) & ~3 and read up to
// five past it; a multiple of four, so that every chain's buffer is 8-byte aligned
__host__ __device__ constexpr int agg_v2_spad(int D) { return (D + 3 + 6 + AV2_OFF + 3) & ~3; }

// staged census entries kept in front of the first row: a quad's dead cells
// past the window read up to 7 entries below a row's start
constexpr int AV2_CPAD = 8;

__host__ __device__ constexpr size_t agg_v2_lds(int D, int NG, int B)
{
    return (size_t)(AV2_CPAD + B * (NG + D - 1)) * 8 + (size_t)B * NG * sizeof(MetaEntry) +
           (size_t)2 * NG * agg_v2_spad(D) * sizeof(uint16_t);
}

// NG chains of G lanes per block (NG * G threads), B rows per staged batch, D <= MAXD
template <int NG, int B, int G, int MAXD>
__device__ __forceinline__ void agg_v2_chains(const AggArgs &a, const int pi)
{
    constexpr int AV_NG = NG, AV_B = B, AV_T = NG * G;
    // staged census loads per thread, sized for the largest D of the instance
    constexpr int AV_MAXCR = (AV_B * (AV_NG + MAXD - 1) + AV_T - 1) / AV_T;
    extern __shared__ __align__(16) uint8_t smem[];
    const int W = a.W, H = a.H, D = a.D;
    const int span = AV_NG + D - 1;
    const int spad = agg_v2_spad(D);
    // one staging buffer: a batch's loads wait in registers until every wave has left the previous batch
    uint64_t *cbuf = (uint64_t *)smem + AV2_CPAD;                                 // [B][span]
    MetaEntry *mbuf = (MetaEntry *)(cbuf + (size_t)AV_B * span);                  // [B][NG]
    uint16_t *sbuf = (uint16_t *)(mbuf + (size_t)AV_B * AV_NG);                   // [2][NG][spad]
    const int k = a.slot[pi];
    const int rx = a.rx[pi], ry = a.ry[pi];
    const int kmin = a.kmin[pi];
    const int nchains = rx == 0 ? W : W + H - 1;
    if (blockIdx.x * AV_NG >= nchains)
        return;                                        // uniform over the block
    const int kb = kmin + blockIdx.x * AV_NG;          // chain index of group 0
    const int grp = threadIdx.x / G, lane = threadIdx.x % G;
    const int kc = kb + grp;
    const bool chain_ok = blockIdx.x * AV_NG + grp < nchains;
    const int ys = ry > 0 ? 0 : H - 1;
    uint8_t *lrk = a.lr + (size_t)k * a.lr_stride;
    const int p1 = a.p1, p2 = a.p2, nbits = a.nbits;
    auto span_x0 = [&](int t) { return kb + rx * t - (D - 1); };

    uint64_t rc[AV_MAXCR];
    uint64_t rmcl;
    uint32_t rmoff, rmwin;
    auto issue = [&](int bt) {
#pragma unroll
        for (int i = 0; i < AV_MAXCR; i++) {
            const int e = threadIdx.x + i * AV_T;
            const int r = e / span, c = e - r * span;
            const int t = bt * AV_B + r;
            const int xx = span_x0(t) + c;
            const bool ok = r < AV_B && t < H && xx >= 0 && xx < W;
            const size_t idx = ok ? (size_t)(ys + ry * t) * W + xx : 0;
            const uint64_t v = a.cr[idx];
            rc[i] = ok ? v : 0ull;
        }
        {
            const int e = threadIdx.x;   // AV_B * AV_NG <= AV_T entries
            const int r = e / AV_NG, g = e - r * AV_NG;
            const int t = bt * AV_B + r;
            const int xx = kb + g + rx * t;
            const bool ok = e < AV_B * AV_NG && t < H && xx >= 0 && xx < W;
            const int pix = ok ? (ys + ry * t) * W + xx : 0;
            const uint64_t vcl = a.cl[pix];
            const uint32_t voff = a.off[pix], vwin = a.win[pix];
            rmcl = ok ? vcl : 0ull;
            rmoff = ok ? voff : 0u;
            rmwin = ok ? vwin : 0u;
        }
    };
    auto commit = [&]() {
#pragma unroll
        for (int i = 0; i < AV_MAXCR; i++) {
            const int e = threadIdx.x + i * AV_T;
            if (e < AV_B * span)
                cbuf[e] = rc[i];
        }
        if (threadIdx.x < AV_B * AV_NG) {
            MetaEntry m;
            m.cl = rmcl;
            m.off = rmoff;
            m.win = rmwin;
            mbuf[threadIdx.x] = m;
        }
    };
    issue(0);
    commit();
    __syncthreads();
    // state buffers: this chain's slots in buffer 0 and the distance to buffer 1
    const int sb0 = grp * spad, sdel = AV_NG * spad;
    int cur = 0;                    // state buffer holding L_r of the previous pixel
    int mq = 0, loq = 0, hiq = -1;  // its minimum and window (empty before the first pixel)
    int started = 0;                // all ones once the chain has had a pixel
    int x = kc;                     // column of the chain's pixel on sweep row t: kc + rx*t
    const int nbt = (H + AV_B - 1) / AV_B;
    for (int bt = 0; bt < nbt; bt++) {
        issue(bt + 1);
        const uint64_t *cb = cbuf;
        const MetaEntry *mb = mbuf;
        const int rows = min(AV_B, H - bt * AV_B);
        MetaEntry en = mb[grp];                        // metadata of the batch's first row
        for (int r = 0; r < rows; r++, x += rx) {
            const bool act = chain_ok && (unsigned)x < (unsigned)W;   // uniform per group
            const MetaEntry e = en;
            // the next row's metadata is read a step ahead: its LDS latency overlaps this step
            en = mb[min(r + 1, rows - 1) * AV_NG + grp];
            const int lo = (int)(e.win & 255), hi = lo + (int)(e.win >> 8);
            if (__ballot(act) == 0)
                continue;                                  // no chain of the wave is on the image
            const bool wide = act && hi - lo >= G;          // cells beyond the one-per-lane pass
            const int qb = sb0 + (cur ? sdel : 0);         // previous pixel's L_r (slot d + 4)
            const int pb = sb0 + (cur ? 0 : sdel);
            // before the first pixel every term is masked off and mq is 0
            const int cap = mq + p2;                       // the P2 term
            const uint32_t spanq = (uint32_t)(hiq - loq);   // previous window (used once started)
            const uint64_t *crow = cb + (size_t)r * span;
            const int cbase = grp + D - 1;                 // the chain's column in the staged span
            int rmin = LBIG;
            // the one-per-lane pass over lo .. lo + G - 1: reads, then results
            const int dn = min(lo + lane, D);              // keeps idle lanes inside the chain's slots
            const bool nlive = act && lo + lane <= hi;
            // unconditional reads; out-of-window terms become LBIG (absent)
            const int nv0 = sbuf[qb + dn + AV2_OFF], nvm = sbuf[qb + dn + AV2_OFF - 1],
                      nvp = sbuf[qb + dn + AV2_OFF + 1];
            const uint64_t ncr = crow[max(cbase - dn, 0)];
            auto narrow = [&]() {
                const uint32_t tq = (uint32_t)(dn - loq);
                const int a0 = tq <= spanq ? nv0 : LBIG;
                const int am = tq - 1u <= spanq ? nvm : LBIG;
                const int ap = tq + 1u <= spanq ? nvp : LBIG;
                const int best = min(min(a0, cap), min(am, ap) + p1) & started;
                const int pc = __popcll(e.cl ^ ncr);
                const int c = dn > x ? nbits : pc;
                const int L = nlive ? c + best - mq : LBIG;
                // idle lanes write LBIG into slots outside the window (masked when read)
                sbuf[pb + dn + AV2_OFF] = (uint16_t)L;
                if (nlive)
                    lrk[e.off + (uint32_t)(dn - lo)] = (uint8_t)L;
                rmin = min(rmin, L);
            };
            // a quad: four disparities dq .. dq + 3 (dq a multiple of 4) of a wide window
            struct QuadIn {
                int dq;
                uint32_t wlo, whi;
                uint2 wmid;
                uint64_t cr[4];
            };
            auto quad_load = [&](int d0) {
                QuadIn qi;
                qi.dq = min(d0, (D + 3) & ~3);             // idle lanes stay inside the chain's slots
                // predecessor terms of dq - 1 .. dq + 4 from three aligned words
                const uint16_t *qs = sbuf + qb + qi.dq + AV2_OFF;
                qi.wlo = *(const uint32_t *)(qs - 2);
                qi.wmid = *(const uint2 *)qs;
                qi.whi = *(const uint32_t *)(qs + 4);
                // right census of columns x - dq - 3 .. x - dq (the index is >= -7,
                // inside the front entries, and below 0 for dead cells only)
                const uint64_t *cp = crow + (cbase - qi.dq - 3);
#pragma unroll
                for (int j = 0; j < 4; j++)
                    qi.cr[j] = cp[3 - j];
                return qi;
            };
            auto quad = [&](const QuadIn &qi) {
                const int dq = qi.dq;
                int pv[6] = {(int)(qi.wlo >> 16), (int)(qi.wmid.x & 0xFFFFu), (int)(qi.wmid.x >> 16),
                             (int)(qi.wmid.y & 0xFFFFu), (int)(qi.wmid.y >> 16), (int)(qi.whi & 0xFFFFu)};
                const uint32_t tq0 = (uint32_t)(dq - 1 - loq);
#pragma unroll
                for (int i = 0; i < 6; i++)
                    pv[i] = tq0 + (uint32_t)i <= spanq ? pv[i] : LBIG;
                int L4[4];
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    const int d = dq + j;
                    const int best = min(min(pv[j + 1], cap), min(pv[j], pv[j + 2]) + p1) & started;
                    const int c = d > x ? nbits : (int)__popcll(e.cl ^ qi.cr[j]);
                    L4[j] = wide && d <= hi ? c + best - mq : LBIG;
                    rmin = min(rmin, L4[j]);
                }
                if (wide) {
                    // slots above hi lie outside the window (masked when read)
                    uint2 wv;
                    wv.x = (uint32_t)L4[0] | ((uint32_t)L4[1] << 16);
                    wv.y = (uint32_t)L4[2] | ((uint32_t)L4[3] << 16);
                    *(uint2 *)(sbuf + pb + dq + AV2_OFF) = wv;
#pragma unroll
                    for (int j = 0; j < 4; j++)
                        if (dq + j <= hi)
                            lrk[e.off + (uint32_t)(dq + j - lo)] = (uint8_t)L4[j];
                }
            };
            if (__ballot(wide)) {
                // quads from the one holding lo + G (cells below lo + G are recomputed
                // alike); the first round's reads go out beside the narrow pass's
                const int q0 = (lo + G) & ~3;
                const int nq = wide ? (hi - q0) / (4 * G) + 1 : 0;
                const int nqw = group_max<G>(nq);
                const QuadIn q1 = quad_load(q0 + 4 * lane);
                narrow();
                quad(q1);
                for (int j = 1; j < nqw; j++)
                    quad(quad_load(q0 + 4 * (G * j + lane)));
            } else {
                narrow();
            }
            const int m = group_min<G>(rmin);
            if (act) {
                mq = m;
                loq = lo;
                hiq = hi;
                started = -1;
            }
            cur ^= 1;
            wave_lds_sync();   // this step's state writes precede the next step's reads
        }
        __syncthreads();   // every wave has left this batch's staging
        commit();
        __syncthreads();
    }
}

// Vertical chains get VG = 32 lanes each (8 per block): full-range pixels line
// up along some columns (the left border, vertical edges) and would otherwise
// make a few blocks take twice as long as the rest; diagonal chains cross
// such columns and keep 16 lanes (16 per block).  At D <= 64 the windows are
// short enough for 16 lanes on vertical chains too (VG = 16).
// (MAXD bounds D: the staging registers of D <= 128 are half those of 256).
template <int MAXD, int VG>
__global__ __launch_bounds__(256) void k_agg_v2(AggArgs a)
{
    if (pass_skipped(a.skip))
        return;
    const int pi = blockIdx.y;
    // this kernel runs beside the horizontal passes on a second stream: at
    // D <= 128 it is the longer of the two and its waves win issue
    // arbitration; at larger D the two run at equal priority (raising either
    // one only moves time between them)
    if (MAXD <= 128)
        __builtin_amdgcn_s_setprio(1);
    if (a.rx[pi] == 0)
        agg_v2_chains<256 / VG, 8, VG, MAXD>(a, pi);
    else
        agg_v2_chains<16, 8, 16, MAXD>(a, pi);
}

// ---- horizontal paths: 256 / G scanlines per block, LDS state, segments ----
//
// Scanline y of a horizontal direction is cut into segments of `seg` steps
// (step t is column rx > 0 ? t : W-1-t).  Three kernels:
//  HS_SPEC  every segment at once, each started as if the scanline began there
//           (segment 0 is then exact);
//  HS_FIX   every segment s >= 1 at once, two 16-lane trajectories per
//           scanline: A from the losses stored at the end of segment s-1, B
//           restarted like HS_SPEC, so B reproduces the stored values.  Where A
//           equals B at a pixel, the recurrence is deterministic and every
//           later stored value of the segment is A's continuation; until then A
//           writes its losses.  A scanline whose A and B never meet in the
//           segment is flagged;
//  HS_SEQ   for flagged scanlines only, walks the later segments in order,
//           restarting each from the exact end of the previous one and
//           comparing with the stored losses until they agree.
// When no segment s-1 is flagged, the end of s-1 stored after HS_SPEC is
// exact (by induction from segment 0), so HS_FIX made segment s exact.
// Each block keeps its scanlines' right census in LDS rings indexed by
// absolute column (column c in slot c mod R): a segment starts by staging the
// D+7 columns its first 8-step batch can reach, and each later batch adds the
// 8 columns it reaches beyond the previous one.  The pixels' metadata is
// staged per batch.

enum { HS_SPEC = 0, HS_FIX = 1, HS_SEQ = 2 };
constexpr int AH2_NG = 16, AH2_T = AH2_NG * AV_G, AH2_B = 8;
constexpr int AH2_MAXSEG = kHMaxSeg;
static_assert(AH2_MAXSEG * 48 >= 4096, "segments of the widest image");

// census ring length per scanline: a power of two >= D + 2B - 1 (a batch's
// reach plus the next batch's new columns); 16-lane groups serve D <= 128
__host__ __device__ constexpr int agg_h2_ring(int G) { return G == 16 ? 256 : 512; }

__host__ __device__ constexpr size_t agg_h2_lds(int D, int G)
{
    return (size_t)(AH2_T / G) * agg_h2_ring(G) * 8 + (size_t)2 * AH2_B * (AH2_T / G) * sizeof(MetaEntry) +
           (size_t)2 * (AH2_T / G) * agg_v2_spad(D) * sizeof(uint16_t);
}

template <int MODE, int G>
__global__ __launch_bounds__(AH2_T) void k_agg_h2(AggArgs a, int seg, int nseg)
{
    if (pass_skipped(a.skip))
        return;
    constexpr int NGG = AH2_T / G;                          // groups of G lanes per block
    constexpr int NC = MODE == HS_FIX ? NGG / 2 : NGG;       // scanlines per block
    // staged census loads per thread: 16-lane groups serve D <= 128, 32-lane groups D <= 256
    constexpr int MAXD = G == 16 ? 128 : kMaxDisp;
    constexpr int MAXCR = (NGG * (MAXD + AH2_B - 1) + AH2_T - 1) / AH2_T;
    extern __shared__ __align__(16) uint8_t smem[];
    const int W = a.W, H = a.H, D = a.D;
    const int spad = agg_v2_spad(D);
    constexpr int R = agg_h2_ring(G);
    static_assert(R >= MAXD + 2 * AH2_B - 1, "ring holds a batch's reach and the next batch's columns");
    uint64_t *ring = (uint64_t *)smem;                                               // [NC][R]
    MetaEntry *mbuf = (MetaEntry *)(smem + (size_t)NGG * R * 8);                     // [2][B][NC]
    uint16_t *sbuf = (uint16_t *)((uint8_t *)mbuf + (size_t)2 * AH2_B * NGG * sizeof(MetaEntry));
    const int pi = blockIdx.z;
    const int k = a.slot[pi];
    const int rx = a.rx[pi];
    const int y0 = blockIdx.x * NC;
    const int grp = threadIdx.x / G, lane = threadIdx.x % G;
    const int cg = MODE == HS_FIX ? grp >> 1 : grp;   // scanline of this group
    const bool traj_a = MODE != HS_FIX || (grp & 1) == 0;
    const int y = y0 + cg;
    const bool row_ok = y < H;
    uint8_t *lrk = a.lr + (size_t)k * a.lr_stride;
    uint8_t *flag = a.hflag + ((size_t)pi * H + (row_ok ? y : 0)) * AH2_MAXSEG;
    const int p1 = a.p1, p2 = a.p2, nbits = a.nbits;
    auto colx = [&](int t) { return rx > 0 ? t : W - 1 - t; };
    // first census column a batch starting at step tb can need
    auto span_x0 = [&](int tb) { return rx > 0 ? tb - (D - 1) : W - tb - AH2_B - (D - 1); };

    if (MODE == HS_SEQ) {
        // nothing to do unless a scanline of the block was flagged
        int any = 0;
        for (int i = threadIdx.x; i < NC * AH2_MAXSEG; i += AH2_T) {
            const int c = i / AH2_MAXSEG, sg = i % AH2_MAXSEG;
            if (y0 + c < H && sg >= 1 && sg < nseg - 1)
                any |= a.hflag[((size_t)pi * H + y0 + c) * AH2_MAXSEG + sg];
        }
        if (!__syncthreads_or(any))
            return;
    }

    // segment start: every census column the first batch (steps from tb) reaches
    auto fill = [&](int tb) {
        const int n = D + AH2_B - 1, c0 = span_x0(tb);
        uint64_t rc[MAXCR];
#pragma unroll
        for (int i = 0; i < MAXCR; i++) {
            const int e = threadIdx.x + i * AH2_T;
            const int c = e / n, col = c0 + (e - c * n);
            const bool ok = c < NC && y0 + c < H && col >= 0 && col < W;
            const size_t idx = ok ? (size_t)(y0 + c) * W + col : 0;
            const uint64_t v = a.cr[idx];
            rc[i] = ok ? v : 0ull;
        }
#pragma unroll
        for (int i = 0; i < MAXCR; i++) {
            const int e = threadIdx.x + i * AH2_T;
            const int c = e / n, col = c0 + (e - c * n);
            if (c < NC)
                ring[c * R + (col & (R - 1))] = rc[i];
        }
    };
    // later batches: the B columns the batch from tn reaches beyond the
    // previous one (rx > 0: tn.., rx < 0: its lowest B), one per thread, and
    // the batch's metadata; loaded a batch ahead and written at its end
    const int nc = threadIdx.x / AH2_B, nk = threadIdx.x % AH2_B;
    auto new_col = [&](int tn) { return (rx > 0 ? tn : span_x0(tn)) + nk; };
    uint64_t rn;
    uint64_t rmcl;
    uint32_t rmoff, rmwin;
    auto issue_cols = [&](int tn) {
        const int col = new_col(tn);
        const bool ok = nc < NC && y0 + nc < H && col >= 0 && col < W;
        const size_t idx = ok ? (size_t)(y0 + nc) * W + col : 0;
        const uint64_t v = a.cr[idx];
        rn = ok ? v : 0ull;
    };
    auto issue_meta = [&](int tb, int tend) {
        const int e = threadIdx.x;
        const int r = e / NC, c = e - r * NC;
        const int t = tb + r, yy = y0 + c;
        const bool ok = e < AH2_B * NC && t < tend && yy < H;
        const int pix = ok ? yy * W + colx(t) : 0;
        const uint64_t vcl = a.cl[pix];
        const uint32_t voff = a.off[pix], vwin = a.win[pix];
        rmcl = ok ? vcl : 0ull;
        rmoff = ok ? voff : 0u;
        rmwin = ok ? vwin : 0u;
    };
    auto commit_cols = [&](int tn) {
        if (nc < NC)
            ring[nc * R + (new_col(tn) & (R - 1))] = rn;
    };
    auto commit_meta = [&](int buf) {
        if (threadIdx.x < AH2_B * NC) {
            MetaEntry m;
            m.cl = rmcl;
            m.off = rmoff;
            m.win = rmwin;
            mbuf[buf * AH2_B * NGG + threadIdx.x] = m;
        }
    };

    // state buffers: this group's slots in buffer 0 and the distance to buffer 1
    const int sb0 = grp * spad, sdel = NGG * spad;
    int cur = 0;                    // state buffer holding L_r of the previous pixel
    int mq = 0, loq = 0, hiq = -1;  // its minimum and window
    int started = 0;                // all ones once the trajectory has a state (mq is 0 before)
    bool done = false;              // the trajectory has met the stored losses
    bool ran = false;               // HS_SEQ: the previous segment was recomputed to its end
    const int s_first = MODE == HS_SPEC ? (int)blockIdx.y : MODE == HS_FIX ? (int)blockIdx.y + 1 : 2;
    const int s_last = MODE == HS_SEQ ? nseg - 1 : s_first;
    for (int sg = s_first; sg <= s_last; sg++) {
        const int t0 = sg * seg, t1 = min(W, t0 + seg);
        bool active = row_ok;       // this group works on segment sg
        if (MODE == HS_SEQ) {
            const bool need = row_ok && (ran || flag[sg - 1] != 0);
            if (!__syncthreads_or(need ? 1 : 0))
                continue;           // no scanline of the block needs this segment
            active = need;
        }
        if (MODE != HS_SPEC) {
            // exact state at the end of segment sg-1 (trajectory A): kept in
            // LDS when HS_SEQ recomputed that segment to its end, else the
            // stored losses.  The whole wave runs this block (cross-lane
            // reductions inside); groups that keep their state load nothing.
            const bool load = active && traj_a && !(MODE == HS_SEQ && ran);
            const int p = (row_ok ? y : 0) * W + colx(t0 - 1);
            const uint32_t wv = a.win[p];
            const uint32_t off = a.off[p];
            const int lo = (int)(wv & 255), hi = lo + (int)(wv >> 8);
            const int nt = load ? hi / G - lo / G + 1 : 0;
            const int ntw = group_max<G>(nt);
            const int qb = sb0 + (cur ? sdel : 0);
            int rmin = LBIG;
            for (int j = 0; j < ntw; j++) {
                const int d = (lo / G) * G + G * j + lane;
                if (j < nt && d >= lo && d <= hi) {
                    const int v = lrk[off + (uint32_t)(d - lo)];
                    sbuf[qb + d + AV2_OFF] = (uint16_t)v;
                    rmin = min(rmin, v);
                }
            }
            const int m = group_min<G>(rmin);
            if (load) {
                mq = m;
                loq = lo;
                hiq = hi;
                started = -1;
            }
            if (MODE == HS_FIX && !traj_a)
                started = 0;        // trajectory B restarts like HS_SPEC (it never loads: mq is 0)
            wave_lds_sync();
        }
        done = !active;
        issue_meta(t0, t1);
        fill(t0);
        commit_meta(0);
        __syncthreads();
        const int nbt = (t1 - t0 + AH2_B - 1) / AH2_B;
        for (int bt = 0; bt < nbt; bt++) {
            const int tb = t0 + bt * AH2_B;
            if (bt + 1 < nbt) {
                issue_cols(tb + AH2_B);
                issue_meta(tb + AH2_B, t1);
            }
            const uint64_t *crow = ring + (size_t)cg * R;
            const MetaEntry *mb = mbuf + (bt & 1) * AH2_B * NGG;
            const int rows = min(AH2_B, t1 - tb);
            MetaEntry en = mb[cg];                          // metadata of the batch's first step
            for (int r = 0; r < rows; r++) {
                const int x = colx(tb + r);
                const bool act = row_ok && !done;            // uniform per group (and per scanline in HS_FIX)
                const MetaEntry e = en;
                // the next step's metadata is read a step ahead: its LDS latency overlaps this step
                en = mb[min(r + 1, rows - 1) * NC + cg];
                const int lo = (int)(e.win & 255), hi = lo + (int)(e.win >> 8);
                if (__ballot(act) == 0)
                    continue;                                  // no group of the wave is working
                const bool wide = act && hi - lo >= G;          // cells beyond the one-per-lane pass
                const int qb = sb0 + (cur ? sdel : 0);
                const int pb = sb0 + (cur ? 0 : sdel);
                // before the first pixel every term is masked off and mq is 0
                const int cap = mq + p2;
                const uint32_t spanq = (uint32_t)(hiq - loq);   // previous window (used once started)
                int rmin = LBIG;
                bool diff = false;
                // one result: compare (HS_FIX: with the other trajectory; HS_SEQ:
                // with the stored loss) and store (trajectory A)
                auto emit = [&](int d, int L, bool live) {
                    if (MODE == HS_FIX) {
                        // lane i of trajectory A sits G lanes below lane i of B
                        const int other = __shfl_xor(L, G, 64);
                        diff = diff || (live && other != L);
                    }
                    if (live) {
                        uint8_t *dst = lrk + e.off + (uint32_t)(d - lo);
                        if (MODE == HS_SEQ)
                            diff = diff || (*dst != (uint8_t)L);
                        if (traj_a)
                            *dst = (uint8_t)L;
                    }
                    rmin = min(rmin, L);
                };
                // the one-per-lane pass over lo .. lo + G - 1: reads, then results
                const int dn = min(lo + lane, D);              // keeps idle lanes inside the group's slots
                const bool nlive = act && lo + lane <= hi;
                // unconditional reads; out-of-window terms become LBIG (absent)
                const int nv0 = sbuf[qb + dn + AV2_OFF], nvm = sbuf[qb + dn + AV2_OFF - 1],
                          nvp = sbuf[qb + dn + AV2_OFF + 1];
                const uint64_t ncr = crow[(x - dn) & (R - 1)];  // right census at column x - d
                auto narrow = [&]() {
                    const uint32_t tq = (uint32_t)(dn - loq);
                    const int a0 = tq <= spanq ? nv0 : LBIG;
                    const int am = tq - 1u <= spanq ? nvm : LBIG;
                    const int ap = tq + 1u <= spanq ? nvp : LBIG;
                    const int best = min(min(a0, cap), min(am, ap) + p1) & started;
                    const int pc = __popcll(e.cl ^ ncr);
                    const int c = dn > x ? nbits : pc;
                    const int L = nlive ? c + best - mq : LBIG;
                    // idle lanes write LBIG into slots outside the window (masked when read)
                    sbuf[pb + dn + AV2_OFF] = (uint16_t)L;
                    emit(dn, L, nlive);
                };
                // a quad: four disparities dq .. dq + 3 (dq a multiple of 4) of a wide window
                struct QuadIn {
                    int dq;
                    uint32_t wlo, whi;
                    uint2 wmid;
                    uint64_t cr[4];
                };
                auto quad_load = [&](int d0) {
                    QuadIn qi;
                    qi.dq = min(d0, (D + 3) & ~3);             // idle lanes stay inside the group's slots
                    // predecessor terms of dq - 1 .. dq + 4 from three aligned words
                    const uint16_t *qs = sbuf + qb + qi.dq + AV2_OFF;
                    qi.wlo = *(const uint32_t *)(qs - 2);
                    qi.wmid = *(const uint2 *)qs;
                    qi.whi = *(const uint32_t *)(qs + 4);
#pragma unroll
                    for (int j = 0; j < 4; j++)
                        qi.cr[j] = crow[(x - qi.dq - j) & (R - 1)];
                    return qi;
                };
                auto quad = [&](const QuadIn &qi) {
                    const int dq = qi.dq;
                    int pv[6] = {(int)(qi.wlo >> 16), (int)(qi.wmid.x & 0xFFFFu), (int)(qi.wmid.x >> 16),
                                 (int)(qi.wmid.y & 0xFFFFu), (int)(qi.wmid.y >> 16), (int)(qi.whi & 0xFFFFu)};
                    const uint32_t tq0 = (uint32_t)(dq - 1 - loq);
#pragma unroll
                    for (int i = 0; i < 6; i++)
                        pv[i] = tq0 + (uint32_t)i <= spanq ? pv[i] : LBIG;
                    int L4[4];
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        const int d = dq + j;
                        const int best = min(min(pv[j + 1], cap), min(pv[j], pv[j + 2]) + p1) & started;
                        const int c = d > x ? nbits : (int)__popcll(e.cl ^ qi.cr[j]);
                        L4[j] = wide && d <= hi ? c + best - mq : LBIG;
                    }
                    if (wide) {
                        // slots above hi lie outside the window (masked when read)
                        uint2 wv;
                        wv.x = (uint32_t)L4[0] | ((uint32_t)L4[1] << 16);
                        wv.y = (uint32_t)L4[2] | ((uint32_t)L4[3] << 16);
                        *(uint2 *)(sbuf + pb + dq + AV2_OFF) = wv;
                    }
#pragma unroll
                    for (int j = 0; j < 4; j++)
                        emit(dq + j, L4[j], wide && dq + j <= hi);
                };
                if (__ballot(wide)) {
                    // quads from the one holding lo + G (cells below lo + G are recomputed
                    // alike); the first round's reads go out beside the narrow pass's
                    const int q0 = (lo + G) & ~3;
                    const int nq = wide ? (hi - q0) / (4 * G) + 1 : 0;
                    const int nqw = group_max<G>(nq);
                    const QuadIn q1 = quad_load(q0 + 4 * lane);
                    narrow();
                    quad(q1);
                    for (int j = 1; j < nqw; j++)
                        quad(quad_load(q0 + 4 * (G * j + lane)));
                } else {
                    narrow();
                }
                const int m = group_min<G>(rmin);
                if (act) {
                    mq = m;
                    loq = lo;
                    hiq = hi;
                    started = -1;
                    if (MODE != HS_SPEC && group_min<G>(diff ? 0 : 1) == 1)
                        done = true;   // stored losses agree from here on
                }
                cur ^= 1;
                wave_lds_sync();
            }
            if (MODE != HS_SPEC) {
                if (!__syncthreads_or(row_ok && !done ? 1 : 0))
                    break;   // every scanline of the block has met the stored losses
            }
            if (bt + 1 < nbt) {
                commit_cols(tb + AH2_B);
                commit_meta((bt + 1) & 1);
            }
            __syncthreads();
        }
        if (MODE == HS_FIX && traj_a && lane == 0 && row_ok)
            flag[sg] = done ? 0 : 1;
        if (MODE == HS_SEQ)
            ran = active && !done;
        __syncthreads();   // staging buffers are rewritten by the next segment
    }
}

static void agg_args(const Geometry &g, DevBuffers &b, AggArgs &hv, AggArgs &vv, int &nh, int &nv, int &maxv,
                     const uint32_t *skip)
{
    for (AggArgs *a : {&hv, &vv}) {
        a->skip = skip;
        a->cl = b.cen_l;
        a->cr = b.cen_r;
        a->win = b.win;
        a->off = b.off;
        a->lr = b.lr;
        a->lr_stride = g.lr_stride;
        a->hflag = b.hflag;
        a->W = g.W;
        a->H = g.H;
        a->D = g.D;
        a->nbits = g.nbits;
        a->p1 = g.p1;
        a->p2 = g.p2;
    }
    nh = nv = maxv = 0;
    for (int k = 0; k < g.npaths; k++) {
        if (g.ry[k] == 0) {
            hv.rx[nh] = g.rx[k];
            hv.ry[nh] = 0;
            hv.slot[nh] = (int8_t)k;
            nh++;
        } else {
            vv.rx[nv] = g.rx[k];
            vv.ry[nv] = g.ry[k];
            vv.slot[nv] = (int8_t)k;
            // chain index range: x = kc + rx*t over t in [0, H)
            vv.kmin[nv] = g.rx[k] > 0 ? -(g.H - 1) : 0;
            maxv = max(maxv, g.rx[k] == 0 ? g.W : g.W + g.H - 1);
            nv++;
        }
    }
}

// dynamic LDS beyond 64 KB must be requested per kernel (gfx950 has 160 KB per CU)
static hipError_t allow_lds(const void *fn, size_t bytes)
{
    if (bytes <= 65536)
        return hipSuccess;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

int count_horizontal_paths(const Geometry &g)
{
    int n = 0;
    for (int k = 0; k < g.npaths; k++)
        n += g.ry[k] == 0;
    return n;
}

// segmented scanlines: speculative pass, fix-up pass, cleanup pass
template <int HG>
static hipError_t launch_agg_h2(const Geometry &g, const AggArgs &hv, int nh, hipStream_t s)
{
    constexpr int NGG = AH2_T / HG;   // scanlines per block
    if (HG == 16 && g.D > 128)
        return hipErrorInvalidValue;  // 16-lane groups stage at most D = 128
    const int seg = g.hseg;
    const int nseg = (g.W + seg - 1) / seg;
    const size_t lds2 = agg_h2_lds(g.D, HG);
    hipError_t e = allow_lds((const void *)k_agg_h2<HS_SPEC, HG>, lds2);
    if (e == hipSuccess)
        e = allow_lds((const void *)k_agg_h2<HS_FIX, HG>, lds2);
    if (e == hipSuccess)
        e = allow_lds((const void *)k_agg_h2<HS_SEQ, HG>, lds2);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL((k_agg_h2<HS_SPEC, HG>), dim3((g.H + NGG - 1) / NGG, nseg, nh), dim3(AH2_T), lds2, s, hv,
                       seg, nseg);
    if (nseg > 1)
        hipLaunchKernelGGL((k_agg_h2<HS_FIX, HG>), dim3((g.H + NGG / 2 - 1) / (NGG / 2), nseg - 1, nh),
                           dim3(AH2_T), lds2, s, hv, seg, nseg);
    if (nseg > 2)
        hipLaunchKernelGGL((k_agg_h2<HS_SEQ, HG>), dim3((g.H + NGG - 1) / NGG, 1, nh), dim3(AH2_T), lds2, s, hv,
                           seg, nseg);
    return hipGetLastError();
}

hipError_t launch_agg_h(const Geometry &g, DevBuffers &b, bool dense, hipStream_t s, const uint32_t *skip)
{
    AggArgs hv, vv;
    int nh, nv, maxv;
    agg_args(g, b, hv, vv, nh, nv, maxv, skip);
    if (!nh)
        return hipSuccess;
    // Ragged windows: segmented scanlines (16 lanes per pixel at D <= 128,
    // 32 above, many waves) win for D > 64, wide windows included now that
    // they are taken in quads; at D <= 64 one register chunk per lane does.
    bool segmented = !dense && g.D > 64;
    if (!dense && g.halt)
        segmented = !segmented;
    if (segmented)
        return g.D > 128 ? launch_agg_h2<32>(g, hv, nh, s) : launch_agg_h2<16>(g, hv, nh, s);
    size_t lds = agg_h_lds(g.W);
    dim3 grd(g.H, nh);
    const int prio = dense ? 0 : 1;
    if (g.D <= 64)
        hipLaunchKernelGGL((k_agg_h<1>), grd, dim3(64), lds, s, hv, prio);
    else if (g.D <= 128)
        hipLaunchKernelGGL((k_agg_h<2>), grd, dim3(64), lds, s, hv, prio);
    else
        hipLaunchKernelGGL((k_agg_h<4>), grd, dim3(64), lds, s, hv, prio);
    return hipGetLastError();
}

hipError_t launch_agg_v(const Geometry &g, DevBuffers &b, bool dense, hipStream_t s, const uint32_t *skip)
{
    AggArgs hv, vv;
    int nh, nv, maxv;
    agg_args(g, b, hv, vv, nh, nv, maxv, skip);
    if (!nv)
        return hipSuccess;
    if (dense) {
        // every window is the full range: 16 scanlines per block, lanes by disparity
        dim3 grd((maxv + AV_NG - 1) / AV_NG, nv);
        size_t lds = agg_v_lds(g.D);
        if (g.D <= 64)
            hipLaunchKernelGGL((k_agg_v<4>), grd, dim3(AV_T), lds, s, vv);
        else if (g.D <= 128)
            hipLaunchKernelGGL((k_agg_v<8>), grd, dim3(AV_T), lds, s, vv);
        else
            hipLaunchKernelGGL((k_agg_v<16>), grd, dim3(AV_T), lds, s, vv);
        return hipGetLastError();
    }
    // ragged windows: LDS-resident state, chunk count per pixel
    // 16 lanes per vertical chain at D <= 64 (640x480: 2 % faster), 32 above
    // (1242x375, D = 128: 16 lanes are 5 % slower)
    const int vg = g.D <= 64 ? 16 : 32;
    int nbx = 0;
    for (int i = 0; i < nv; i++)
        nbx = max(nbx, vv.rx[i] == 0 ? (g.W + 256 / vg - 1) / (256 / vg) : (g.W + g.H - 1 + 15) / 16);
    const size_t lds = agg_v2_lds(g.D, 16, 8);   // the larger of 8 and 16 chains per block
    if (g.D <= 64)
        hipLaunchKernelGGL((k_agg_v2<128, 16>), dim3(nbx, nv), dim3(256), lds, s, vv);
    else if (g.D <= 128)
        hipLaunchKernelGGL((k_agg_v2<128, 32>), dim3(nbx, nv), dim3(256), lds, s, vv);
    else
        hipLaunchKernelGGL((k_agg_v2<kMaxDisp, 32>), dim3(nbx, nv), dim3(256), lds, s, vv);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// gate re-run (Section 4's innovation test): pixels that failed it in the
// first pass search the full range in a second matching pass and restart from
// that measurement.
//
// Sparse second pass.  Along one path, Eq. 1 makes a pixel's L_r depend on the
// previous pixel's only through that pixel's vector of L_r over its window
// (and its minimum).  The second pass therefore differs from the first only
// from a pixel whose window changed (a "moved" pixel: widened, and narrower
// than the full range before) up to the first later pixel whose recomputed
// vector equals the stored one; from there on the two passes agree again.
// The first pass's L_r stay in the path buffers.  One wave per scanline of
// every path walks it: it jumps from moved pixel to moved pixel, starts from
// the previous pixel's stored L_r, recomputes Eq. 1 until the vector rejoins
// the stored one, and writes what changed: in place for pixels that kept their
// window, into a full-range block after the first pass's cells for the moved
// pixels.  Pixels it wrote (and every widened pixel) are marked; the WTA and
// the correction then run on the marked pixels only, and the others keep the
// first pass's results, which a full second pass reproduces bit for bit.
// When the blocks would not fit behind the first pass's cells, the dense
// second pass (every pixel matched again) runs instead; the choice is made on
// the device, and each route's launches read a skip word.
// ---------------------------------------------------------------------------

constexpr int GW_T = 1024, GW_PER = 4, GW_BLOCK = GW_T * GW_PER;   // widening and placement: pixels per thread, block

// sum over a block of GW_T threads (every thread receives it); `red` holds
// one word per wave
__device__ __forceinline__ uint32_t block_sum(uint32_t v, uint32_t *red)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
        v += (uint32_t)__shfl_xor((int)v, m);
    __syncthreads();   // `red` may still be read from the previous call
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = v;
    __syncthreads();
    uint32_t t = 0;
#pragma unroll
    for (int w = 0; w < GW_T / 64; w++)
        t += red[w];
    return t;
}

// widen the failed pixels' windows (FULLWIN | GATEFAIL); each block of
// GW_BLOCK pixels writes its counts (widened, moved, added cells) to
// parts[3 * block]; with `moved` set, also mark the pixels for the sparse pass
__global__ __launch_bounds__(GW_T) void k_gate_widen(int N, int D, const uint8_t *__restrict__ mask,
                                                     uint8_t *__restrict__ flags, uint16_t *__restrict__ win,
                                                     const uint32_t *__restrict__ off, uint32_t *__restrict__ rr,
                                                     uint32_t *__restrict__ parts, uint8_t *__restrict__ moved,
                                                     uint8_t *__restrict__ touched)
{
    __shared__ uint32_t red[GW_T / 64];
    const int base = blockIdx.x * GW_BLOCK + threadIdx.x * GW_PER;
    uint32_t nw = 0, nm = 0, ex = 0;
#pragma unroll
    for (int i = 0; i < GW_PER; i++) {
        const int t = base + i;
        const bool fail = t < N && mask[t];
        const int w1 = fail ? (int)(win[t] >> 8) + 1 : D;
        const bool mv = fail && w1 < D;
        nw += fail ? 1u : 0u;
        nm += mv ? 1u : 0u;
        ex += (uint32_t)(D - w1);
        if (moved && t < N) {
            moved[t] = mv ? 1 : 0;
            touched[t] = fail ? 1 : 0;
        }
        if (fail) {
            flags[t] |= SGM_FLAG_FULLWIN | SGM_FLAG_GATEFAIL;
            win[t] = (uint16_t)((D - 1) << 8);
        }
    }
    nw = block_sum(nw, red);
    nm = block_sum(nm, red);
    ex = block_sum(ex, red);
    if (threadIdx.x == 0) {
        parts[3 * blockIdx.x] = nw;
        parts[3 * blockIdx.x + 1] = nm;
        parts[3 * blockIdx.x + 2] = ex;
        if (blockIdx.x == 0)
            rr[RR_M1] = off[N];
    }
}

// totals of the widening's block counts (few: every block reads them all);
// with `sparse`, the full-range block of every moved pixel at M1 + rank * D
// (rank: raster order among the moved pixels) when they all fit in a path
// buffer (`cap` cells).  The skip words pick the route, and the sparse route's
// cell count (first pass + widening) goes to off[N].
__global__ __launch_bounds__(GW_T) void k_gate_place(int N, int D, int nparts, size_t cap, int sparse, int force_dense,
                                                     const uint32_t *__restrict__ parts,
                                                     const uint8_t *__restrict__ moved, uint32_t *__restrict__ woff,
                                                     uint32_t *__restrict__ rr, uint32_t *__restrict__ off)
{
    __shared__ uint32_t red[GW_T / 64];
    __shared__ uint32_t tot;
    uint32_t nw = 0, nm = 0, ex = 0, before = 0;
    for (int i = threadIdx.x; i < nparts; i += GW_T) {
        nw += parts[3 * i];
        nm += parts[3 * i + 1];
        ex += parts[3 * i + 2];
        before += i < (int)blockIdx.x ? parts[3 * i + 1] : 0u;
    }
    nw = block_sum(nw, red);
    nm = block_sum(nm, red);
    ex = block_sum(ex, red);
    before = block_sum(before, red);
    const uint32_t m1 = rr[RR_M1];
    const bool fits = sparse && !force_dense && (size_t)m1 + (size_t)nm * (size_t)D <= cap;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        rr[RR_NW] = nw;
        rr[RR_NMOVED] = nm;
        rr[RR_EXTRA] = ex;
        rr[RR_SKIP_DENSE] = fits ? 0u : nw;
        rr[RR_SKIP_SPARSE] = fits ? nw : 0u;
        if (fits)
            off[N] = m1 + ex;
    }
    if (!fits)
        return;   // uniform over the grid
    // ranks: moved pixels of the blocks before, then of the threads before, then of this thread's
    const int base = blockIdx.x * GW_BLOCK + threadIdx.x * GW_PER;
    bool mv[GW_PER];
    uint32_t cnt = 0;
#pragma unroll
    for (int i = 0; i < GW_PER; i++) {
        mv[i] = base + i < N && moved[base + i];
        cnt += mv[i] ? 1u : 0u;
    }
    uint32_t rank = before + block_excl_scan(cnt, &tot);
#pragma unroll
    for (int i = 0; i < GW_PER; i++)
        if (mv[i])
            woff[base + i] = m1 + (rank++) * (uint32_t)D;
}

int gate_parts(const Geometry &g) { return (g.N + GW_BLOCK - 1) / GW_BLOCK; }

hipError_t launch_gate_widen(const Geometry &g, DevBuffers &b, bool sparse, hipStream_t s)
{
    const int np = gate_parts(g);
    uint32_t *parts = b.rerun + RR_WORDS;
    hipLaunchKernelGGL(k_gate_widen, dim3(np), dim3(GW_T), 0, s, g.N, g.D, b.mask, b.flags, b.win, b.off, b.rerun,
                       parts, sparse ? b.moved : (uint8_t *)nullptr, sparse ? b.touched : (uint8_t *)nullptr);
    hipLaunchKernelGGL(k_gate_place, dim3(np), dim3(GW_T), 0, s, g.N, g.D, np, g.lr_stride, sparse ? 1 : 0,
                       g.rr_dense ? 1 : 0, (const uint32_t *)parts, b.moved, b.woff, b.rerun, b.off);
    return hipGetLastError();
}

struct WalkArgs {
    const uint64_t *cl, *cr;
    const uint16_t *win;
    const uint32_t *off, *woff;
    const uint8_t *moved;
    uint8_t *touched;
    uint8_t *lr;
    size_t lr_stride;
    int W, H, nbits, p1, p2, npaths;
    int8_t rx[kMaxPaths], ry[kMaxPaths], slot[kMaxPaths];
    int cbase[kMaxPaths + 1];   // first scanline of each listed path; cbase[npaths] = all scanlines
    const uint32_t *skip;
};

constexpr int RW_T = 64;   // one wave (one scanline) per block: a finished scanline frees its slot at once

// Eq. 1 at one pixel for a whole wave (lanes by disparity, chunk j holds
// d = 64 j + lane): Ln = LBIG outside the window [lo, hi]
template <int MAXCH>
__device__ __forceinline__ void eq1_wave(const Chain<MAXCH> &st, int lane, bool first, uint64_t clp, int x, int lo,
                                         int hi, const uint64_t (&crv)[MAXCH], int jlo, int jhi, int p1, int p2,
                                         int nbits, int (&Ln)[MAXCH])
{
    const int mq = st.mq;
    const int cap = first ? LBIG : mq + p2;
    const int base = first ? 0 : -mq;
#pragma unroll
    for (int j = 0; j < MAXCH; j++) {
        Ln[j] = LBIG;
        if (j < jlo || j > jhi)
            continue;
        const int d = j * 64 + lane;
        int pm = from_prev_lane<64>(st.Lp[j]);
        int pp = from_next_lane<64>(st.Lp[j]);
        if (j > 0) {
            const int edge = __builtin_amdgcn_readlane(st.Lp[j - 1], 63);
            pm = lane == 0 ? edge : pm;
        }
        if (j < MAXCH - 1) {
            const int edge = __builtin_amdgcn_readlane(st.Lp[j + 1], 0);
            pp = lane == 63 ? edge : pp;
        }
        const int best = first ? 0 : min(min(st.Lp[j], cap), min(pm, pp) + p1);
        const int c = d > x ? nbits : __popcll(clp ^ crv[j]);
        const bool in = (unsigned)(d - lo) <= (unsigned)(hi - lo);
        Ln[j] = in ? c + best + base : LBIG;
    }
}

// loads of one step of the walk: the right census at x - d and, for a pixel
// that kept its window, its stored L_r, for every disparity of [lo, hi]
template <int MAXCH>
__device__ __forceinline__ void walk_loads(const uint64_t *crow, const uint8_t *lrk, int x, int lo, int hi,
                                           uint32_t o, bool mvp, int lane, uint64_t (&crv)[MAXCH], int (&old)[MAXCH])
{
    const int jlo = lo >> 6, jhi = hi >> 6;
#pragma unroll
    for (int j = 0; j < MAXCH; j++) {
        crv[j] = 0;
        old[j] = LBIG;
        if (j < jlo || j > jhi)
            continue;
        const int d = j * 64 + lane;
        const bool in = (unsigned)(d - lo) <= (unsigned)(hi - lo);
        if (in && d <= x)
            crv[j] = crow[x - d];
        if (in && !mvp)
            old[j] = lrk[o + (uint32_t)(d - lo)];
    }
}

template <int MAXCH, int P>
__global__ __launch_bounds__(RW_T) void k_rerun_walk(WalkArgs a)
{
    if (pass_skipped(a.skip))
        return;
    const int c = blockIdx.x * (RW_T / 64) + (int)(threadIdx.x >> 6);
    if (c >= a.cbase[a.npaths])
        return;   // the whole wave
    int pi = 0;
    while (pi + 1 < a.npaths && c >= a.cbase[pi + 1])
        pi++;
    const int rx = a.rx[pi], ry = a.ry[pi], cc = c - a.cbase[pi];
    const int W = a.W, H = a.H;
    // the scanline's first pixel lies on the border the path enters from
    const int x0 = rx > 0 ? 0 : W - 1, y0 = ry > 0 ? 0 : H - 1;
    int sx, sy, len;
    if (ry == 0) {
        sx = x0, sy = cc, len = W;
    } else if (rx == 0) {
        sx = cc, sy = y0, len = H;
    } else if (cc < W) {
        sx = cc, sy = y0, len = min(H, rx > 0 ? W - cc : cc + 1);
    } else {
        sx = x0, sy = y0 + ry * (cc - W + 1);
        len = min(W, ry > 0 ? H - sy : sy + 1);
    }
    const int p0 = sy * W + sx, dp = ry * W + rx;
    const int lane = threadIdx.x & 63;
    uint8_t *lrk = a.lr + (size_t)a.slot[pi] * a.lr_stride;
    const int p1 = a.p1, p2 = a.p2, nbits = a.nbits;
    Chain<MAXCH> st;
#pragma unroll
    for (int j = 0; j < MAXCH; j++)
        st.Lp[j] = LBIG;
    st.mq = 0;
    bool dirty = false;   // the previous pixel's L_r differ from the first pass's
    for (int t0 = 0; t0 < len; t0 += 64) {
        // this batch's pixels, one per lane
        const int tl = min(t0 + lane, len - 1);
        const int pl = p0 + tl * dp;
        const bool mvl = t0 + lane < len && a.moved[pl];
        const uint64_t mvb = __ballot(mvl);
        if (!dirty && !mvb)
            continue;
        const uint32_t bwin = a.win[pl];
        const uint32_t boff = mvl ? a.woff[pl] : a.off[pl];
        const uint64_t bcl = a.cl[pl];
        const int n = min(64, len - t0);
        int s = 0;
        while (s < n) {
            const bool cont = dirty;   // the group continues a dirty stretch
            bool start = false;
            uint32_t qwin = 0, qoff = 0;
            if (!dirty) {
                // next moved pixel of the batch; its predecessor kept the
                // first pass's L_r (a moved predecessor would have left the
                // scanline dirty)
                const uint64_t rem = (mvb >> s) << s;
                if (!rem)
                    break;
                s = __builtin_ctzll(rem);
                start = t0 + s > 0;
                if (s > 0) {
                    qwin = (uint32_t)__builtin_amdgcn_readlane((int)bwin, s - 1);
                    qoff = (uint32_t)__builtin_amdgcn_readlane((int)boff, s - 1);
                } else if (start) {
                    const int q = p0 + (t0 - 1) * dp;
                    qwin = a.win[q];
                    qoff = a.off[q];
                }
            }
            // a group of steps whose loads are issued together (one memory
            // latency per group): P steps where the scanline is already dirty
            // (a stretch that has not rejoined tends to go on); from a moved
            // pixel, the moved pixels that follow it (the scanline stays dirty
            // through them) and two more
            // (~(mvb >> s) is 0 only when s = 0 and all 64 pixels moved)
            const uint64_t rest = ~(mvb >> s);
            const int run = rest ? __builtin_ctzll(rest) : 64;
            const int gn = min(n - s, cont ? P : min(run + 2, P));   // >= 1: every group advances s
            uint64_t crv[P][MAXCH];
            int old[P][MAXCH];
#pragma unroll
            for (int i = 0; i < P; i++) {
                if (i >= gn)
                    break;
                const int si = s + i, t = t0 + si;
                const uint32_t wv = (uint32_t)__builtin_amdgcn_readlane((int)bwin, si);
                const uint32_t o = (uint32_t)__builtin_amdgcn_readlane((int)boff, si);
                const int lo = (int)(wv & 255), hi = lo + (int)(wv >> 8);
                walk_loads<MAXCH>(a.cr + (size_t)(sy + t * ry) * W, lrk, sx + t * rx, lo, hi, o,
                                  (mvb >> si) & 1ull, lane, crv[i], old[i]);
            }
            if (start) {
                const int qlo = (int)(qwin & 255), qhi = qlo + (int)(qwin >> 8);
                int m = LBIG;
#pragma unroll
                for (int j = 0; j < MAXCH; j++) {
                    const int d = j * 64 + lane;
                    const bool in = (unsigned)(d - qlo) <= (unsigned)(qhi - qlo);
                    st.Lp[j] = in ? (int)lrk[qoff + (uint32_t)(d - qlo)] : LBIG;
                    m = min(m, st.Lp[j]);
                }
                st.mq = group_min_dpp<64>(m);
            }
            int done = gn;
#pragma unroll
            for (int i = 0; i < P; i++) {
                if (i >= gn)
                    break;
                // Eq. 1 at the pixel of lane s + i
                const int si = s + i, t = t0 + si;
                const uint32_t wv = (uint32_t)__builtin_amdgcn_readlane((int)bwin, si);
                const uint32_t o = (uint32_t)__builtin_amdgcn_readlane((int)boff, si);
                const uint64_t clp = readlane64(bcl, si);
                const bool mvp = (mvb >> si) & 1ull;
                const int lo = (int)(wv & 255), hi = lo + (int)(wv >> 8);
                int Ln[MAXCH];
                eq1_wave<MAXCH>(st, lane, t == 0, clp, sx + t * rx, lo, hi, crv[i], lo >> 6, hi >> 6, p1, p2, nbits,
                                Ln);
                bool neq = false;
                int m = LBIG;
#pragma unroll
                for (int j = 0; j < MAXCH; j++) {
                    neq |= Ln[j] != old[i][j];
                    m = min(m, Ln[j]);
                }
                // a moved pixel always writes its block; another pixel writes
                // (and is marked) only where its L_r changed
                const bool changed = mvp || __ballot(neq) != 0ull;
                if (changed) {
#pragma unroll
                    for (int j = 0; j < MAXCH; j++) {
                        const int d = j * 64 + lane;
                        if (Ln[j] != LBIG)
                            lrk[o + (uint32_t)(d - lo)] = (uint8_t)Ln[j];
                    }
                    if (!mvp && lane == 0)
                        a.touched[p0 + t * dp] = 1;
                }
                dirty = changed;
#pragma unroll
                for (int j = 0; j < MAXCH; j++)
                    st.Lp[j] = Ln[j];
                st.mq = group_min_dpp<64>(m);
                if (!dirty) {
                    done = i + 1;   // rejoined: the rest of the group is not needed
                    break;
                }
            }
            s += done;
        }
    }
}

hipError_t launch_rerun_walk(const Geometry &g, DevBuffers &b, hipStream_t s)
{
    WalkArgs a;
    a.cl = b.cen_l;
    a.cr = b.cen_r;
    a.win = b.win;
    a.off = b.off;
    a.woff = b.woff;
    a.moved = b.moved;
    a.touched = b.touched;
    a.lr = b.lr;
    a.lr_stride = g.lr_stride;
    a.W = g.W;
    a.H = g.H;
    a.nbits = g.nbits;
    a.p1 = g.p1;
    a.p2 = g.p2;
    a.skip = b.rerun + RR_SKIP_SPARSE;
    // horizontal scanlines (the longest) first in the grid
    int n = 0, tot = 0;
    for (int pass = 0; pass < 2; pass++)
        for (int k = 0; k < g.npaths; k++) {
            if ((g.ry[k] == 0) != (pass == 0))
                continue;
            a.rx[n] = g.rx[k];
            a.ry[n] = g.ry[k];
            a.slot[n] = (int8_t)k;
            a.cbase[n] = tot;
            tot += g.ry[k] == 0 ? g.H : g.rx[k] == 0 ? g.W : g.W + g.H - 1;
            n++;
        }
    a.cbase[n] = tot;
    a.npaths = n;
    const dim3 grd((tot + RW_T / 64 - 1) / (RW_T / 64));
    if (g.D <= 64)
        hipLaunchKernelGGL((k_rerun_walk<1, 4>), grd, dim3(RW_T), 0, s, a);
    else if (g.D <= 128)
        hipLaunchKernelGGL((k_rerun_walk<2, 4>), grd, dim3(RW_T), 0, s, a);
    else if (g.D <= 192)
        hipLaunchKernelGGL((k_rerun_walk<3, 4>), grd, dim3(RW_T), 0, s, a);
    else
        hipLaunchKernelGGL((k_rerun_walk<4, 4>), grd, dim3(RW_T), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// winner-takes-all (Section 2.3) with parabolic sub-pixel fit, then the
// Kalman correction (Eq. 5-6) and the innovation test (Section 4).
// A group of WG lanes handles one pixel: lanes sum the paths' L_r over the
// window (S), keep S in LDS and reduce (S << 9 | slot), which picks the
// smallest S and then the lowest disparity.  Lane 0 then fits the parabola
// through S(d*-1), S(d*), S(d*+1) and updates the filter in double
// precision.  Reduced frames use 8 lanes (half a DPP row; up to 29 cells in
// one pass, typical reduced windows have 8-10), full-range frames 16.
// ---------------------------------------------------------------------------

constexpr int WTA_T = 256;

// min over the 8 lanes of a half DPP row; every lane receives the result
__device__ __forceinline__ int half_row_min8(int v)
{
    v = min(v, __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true));   // row_half_mirror
    v = min(v, __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true));    // quad_perm [2,3,0,1]
    v = min(v, __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true));    // quad_perm [1,0,3,2]
    return v;
}

template <int WG>
__global__ __launch_bounds__(WTA_T) void k_wta_correct(int N, int D, int npaths, CorrectConst cc, int mode,
                                                       const uint8_t *__restrict__ lr, size_t lr_stride,
                                                       const uint16_t *__restrict__ win,
                                                       const uint32_t *__restrict__ off,
                                                       const uint8_t *__restrict__ flags,
                                                       const double *__restrict__ dhat,
                                                       const double *__restrict__ pm, uint16_t *__restrict__ dbg_sum,
                                                       int32_t *__restrict__ dstar_out, double *__restrict__ dz_out,
                                                       double *__restrict__ d_state, double *__restrict__ p_state,
                                                       uint8_t *__restrict__ mask, uint8_t *__restrict__ sflags,
                                                       const float *__restrict__ rpix, double *__restrict__ nu_out,
                                                       const uint32_t *skip, float *__restrict__ rcurv_out,
                                                       int32_t *__restrict__ kappa_out,
                                                       const uint8_t *__restrict__ touched,
                                                       const uint8_t *__restrict__ moved,
                                                       const uint32_t *__restrict__ woff)
{
    if (pass_skipped(skip))
        return;
    constexpr int WNG = WTA_T / WG;   // pixels per block
    extern __shared__ uint16_t ssum_lds[];   // [WNG][D + 8] cost sums of each pixel's window
    const int grp = threadIdx.x / WG, lane = threadIdx.x % WG;
    const int t = blockIdx.x * WNG + grp;
    if (t >= N)
        return;   // the whole group leaves together
    // sparse gate re-run pass: an unmarked pixel keeps the first pass's
    // results; a moved one reads its full-range block
    if (touched && !touched[t])
        return;
    uint16_t *ssum = ssum_lds + (size_t)grp * (D + 8);
    const uint32_t o = (moved && moved[t]) ? woff[t] : off[t];
    const uint32_t wv = win[t];
    // the correction's inputs are read with the window (every lane, no branch):
    // their latency overlaps the sums
    const uint8_t fl = flags[t];
    const double dh = dhat[t], pv = pm[t];
    const int lo = (int)(wv & 255), w = (int)(wv >> 8) + 1, hi = lo + w - 1;
    // each lane sums four consecutive cells of every path from aligned
    // dwords (16-bit halves: even and odd bytes; S <= 8 * 148 < 2^16).
    // Cells before o or past o+w-1 in the dwords belong to other pixels
    // and are ignored.
    const uint32_t a0 = o & ~3u;              // first aligned dword of the window
    const int lead = (int)(o - a0);           // cells of the previous pixel in it
    const int ndw = (lead + w + 3) >> 2;
    uint32_t key = 0x7FFFFFFFu;   // above every real key (S << 9 | slot < 2^20)
    for (int q = lane; q < ndw; q += WG) {
        const uint32_t byte0 = a0 + 4u * (uint32_t)q;
        // the paths' dwords are loaded together (path index clamped, value masked)
        uint32_t v[kMaxPaths];
#pragma unroll
        for (int k = 0; k < kMaxPaths; k++)
            v[k] = *(const uint32_t *)(lr + (size_t)min(k, npaths - 1) * lr_stride + byte0);
        uint32_t ev = 0, od = 0;
#pragma unroll
        for (int k = 0; k < kMaxPaths; k++) {
            const uint32_t vm = k < npaths ? v[k] : 0u;
            ev += vm & 0x00FF00FFu;
            od += (vm >> 8) & 0x00FF00FFu;
        }
        const uint32_t s4[4] = {ev & 0xFFFFu, od & 0xFFFFu, ev >> 16, od >> 16};
#pragma unroll
        for (int b = 0; b < 4; b++) {
            const int sl = 4 * q + b - lead;      // slot within the window
            if (sl >= 0 && sl < w) {
                ssum[sl] = (uint16_t)s4[b];
                if (dbg_sum)
                    dbg_sum[o + sl] = (uint16_t)s4[b];
                key = min(key, (s4[b] << 9) | (uint32_t)sl);
            }
        }
    }
    // keys < 2^31: the signed min is the unsigned min
    key = (uint32_t)(WG == 8 ? half_row_min8((int)key) : row_min16((int)key));
    wave_lds_sync();
    if (lane != 0)
        return;
    const int slot = (int)(key & 511u);
    const int s0 = (int)(key >> 9);
    const int ds = lo + slot;
    double dz = (double)ds;
    int kappa = 0;   // curvature a + b of the parabola (0: d* on a window edge)
    if (ds - 1 >= lo && ds + 1 <= hi) {
        const int a = (int)ssum[slot - 1] - s0, b = (int)ssum[slot + 1] - s0;
        dz = (double)ds + (double)(a - b) / (double)(2 * (a + b));
        kappa = a + b;
    }
    dstar_out[t] = ds;
    dz_out[t] = dz;
    double r = rpix ? (double)rpix[t] : cc.r;
    if (cc.curv > 0.0) {
        // measurement variance from the cost curvature: curv / kappa in [1/256, 64]
        if (kappa > 0)
            r = fmin(fmax(cc.curv / (double)kappa, 1.0 / 256.0), 64.0);
        kappa_out[t] = kappa;
        rcurv_out[t] = (float)r;
    }
    if (mode == 2)
        return;
    bool moving = false;
    double nu = 0.0, S = 0.0;
    if (fl & SGM_FLAG_PRED) {
        nu = dz - dh;
        S = pv + r;
        moving = (nu * nu) / S > cc.gate;
    }
    nu_out[t] = nu;
    if (fl & SGM_FLAG_GATEFAIL) {
        // failed the first pass's innovation test and re-measured over the
        // full range: restart from that measurement, stays marked moving
        d_state[t] = dz;
        p_state[t] = cc.r;
        mask[t] = 1;
        sflags[t] = SGM_FLAG_RESET;
        return;
    }
    if (fl & SGM_FLAG_FULLWIN) {
        d_state[t] = dz;
        p_state[t] = cc.r;
    } else {
        const double K = pv / S;
        const double am = 1.0 - K;
        d_state[t] = dh + K * nu;
        p_state[t] = (am * am) * pv + (K * K) * r;
    }
    const bool sat = (ds == lo && lo > 0) || (ds == hi && hi < D - 1);
    mask[t] = moving ? 1 : 0;
    sflags[t] = (moving || sat) ? SGM_FLAG_RESET : 0;
}

hipError_t launch_wta_correct(const Geometry &g, DevBuffers &b, const CorrectConst &cc, int mode,
                              bool debug_sum, const float *rpix, hipStream_t s, const uint32_t *skip, bool sparse)
{
    const uint8_t *touched = sparse ? b.touched : nullptr, *moved = sparse ? b.moved : nullptr;
    const uint32_t *woff = sparse ? b.woff : nullptr;
    if (mode == 0)
        hipLaunchKernelGGL((k_wta_correct<16>), dim3((g.N + 15) / 16), dim3(WTA_T), (size_t)16 * (g.D + 8) * 2, s,
                           g.N, g.D, g.npaths, cc,
                       mode, b.lr, g.lr_stride, b.win, b.off, b.flags, b.dhat, b.pm,
                       debug_sum ? b.sum : (uint16_t *)nullptr, b.dstar, b.dz, b.d, b.p, b.mask, b.sflags, rpix,
                       b.nu, skip, b.rpix, b.kappa, touched, moved, woff);
    else
        hipLaunchKernelGGL((k_wta_correct<8>), dim3((g.N + 31) / 32), dim3(WTA_T), (size_t)32 * (g.D + 8) * 2, s,
                           g.N, g.D, g.npaths, cc,
                       mode, b.lr, g.lr_stride, b.win, b.off, b.flags, b.dhat, b.pm,
                       debug_sum ? b.sum : (uint16_t *)nullptr, b.dstar, b.dz, b.d, b.p, b.mask, b.sflags, rpix,
                       b.nu, skip, b.rpix, b.kappa, touched, moved, woff);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// small conversions for the read-back entry points
// ---------------------------------------------------------------------------

__global__ void k_win_to_lohi(int N, const uint16_t *win, int32_t *out, int which)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N)
        return;
    int lo = win[p] & 255;
    out[p] = which ? lo + (win[p] >> 8) : lo;
}

hipError_t launch_windows_to_lohi(const Geometry &g, const DevBuffers &b, int32_t *out, int which, hipStream_t s)
{
    hipLaunchKernelGGL(k_win_to_lohi, dim3((g.N + 255) / 256), dim3(256), 0, s, g.N, b.win, out, which);
    return hipGetLastError();
}

__global__ void k_f64_to_f32(int W, int H, const double *src, float *dst, int pitch)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= W * H)
        return;
    int y = t / W, x = t - y * W;
    dst[(size_t)y * pitch + x] = (float)src[t];
}

hipError_t launch_state_to_f32(const Geometry &g, const double *src, float *dst, int pitch, hipStream_t s)
{
    hipLaunchKernelGGL(k_f64_to_f32, dim3((g.N + 255) / 256), dim3(256), 0, s, g.W, g.H, src, dst, pitch);
    return hipGetLastError();
}

__global__ void k_copy_u8(int W, int H, const uint8_t *src, uint8_t *dst, int pitch)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= W * H)
        return;
    int y = t / W, x = t - y * W;
    dst[(size_t)y * pitch + x] = src[t];
}

hipError_t launch_copy_u8(const Geometry &g, const uint8_t *src, uint8_t *dst, int pitch, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy_u8, dim3((g.N + 255) / 256), dim3(256), 0, s, g.W, g.H, src, dst, pitch);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// injected filter state (checkpoint restore): the state must be one the
// filter can hold, d in [0, D-1] and p > 0, both finite.  The check counts
// the pixels that break it; the copy stores -0 as +0, so that the z-buffer's
// ordering of disparities by their bits agrees with their values.
// ---------------------------------------------------------------------------
__global__ void k_check_state(int N, int D, const double *__restrict__ d, const double *__restrict__ p,
                              uint32_t *bad)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    bool ok = true;
    if (t < N) {
        const double dv = d[t], pv = p[t];
        ok = isfinite(dv) && dv >= 0.0 && dv <= (double)(D - 1) && isfinite(pv) && pv > 0.0;
    }
    const unsigned long long m = __ballot(!ok);
    if (m && (threadIdx.x & 63) == 0)
        atomicAdd(bad, (uint32_t)__popcll(m));
}

__global__ void k_load_state(int N, const double *__restrict__ d, const double *__restrict__ p,
                             const uint8_t *__restrict__ sf, double *__restrict__ sd, double *__restrict__ sp,
                             uint8_t *__restrict__ ssf, double *__restrict__ nu)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N)
        return;
    const double dv = d[t];
    sd[t] = dv == 0.0 ? 0.0 : dv;
    sp[t] = p[t];
    ssf[t] = sf[t];
    nu[t] = 0.0;
}

hipError_t launch_check_state(const Geometry &g, const double *d, const double *p, uint32_t *bad, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, bad);
    hipLaunchKernelGGL(k_check_state, dim3((g.N + 255) / 256), dim3(256), 0, s, g.N, g.D, d, p, bad);
    return hipGetLastError();
}

hipError_t launch_load_state(const Geometry &g, DevBuffers &b, const double *d, const double *p, const uint8_t *sf,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_load_state, dim3((g.N + 255) / 256), dim3(256), 0, s, g.N, d, p, sf, b.d, b.p, b.sflags,
                       b.nu);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 3x3 block median of the filtered disparity (Section 2.3 post-processing,
// outside the filter loop), clamped borders, written as float32.  The median
// of 3x3 values: sort each row of three, then the median is the median of
// (max of the row minima, median of the row medians, min of the row maxima).
// Every step is a min or max, so the result is one of the nine inputs.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sort3(double &a, double &b, double &c)
{
    double lo = fmin(a, b), hi = fmax(a, b);
    a = fmin(lo, c);
    double m = fmax(lo, c);
    b = fmin(hi, m);
    c = fmax(hi, m);
}

__device__ __forceinline__ double med3(double a, double b, double c)
{
    return fmax(fmin(a, b), fmin(fmax(a, b), c));
}

__global__ void __launch_bounds__(256) k_median3x3(int W, int H, const double *__restrict__ d,
                                                   float *__restrict__ out, int pitch)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= W || y >= H)
        return;
    const int xl = x > 0 ? x - 1 : 0, xr = x < W - 1 ? x + 1 : W - 1;
    double r[3][3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        int yy = min(max(y + i - 1, 0), H - 1);
        const double *row = d + (size_t)yy * W;
        r[i][0] = row[xl];
        r[i][1] = row[x];
        r[i][2] = row[xr];
        sort3(r[i][0], r[i][1], r[i][2]);
    }
    double lo = fmax(fmax(r[0][0], r[1][0]), r[2][0]);
    double mid = med3(r[0][1], r[1][1], r[2][1]);
    double hi = fmin(fmin(r[0][2], r[1][2]), r[2][2]);
    out[(size_t)y * pitch + x] = (float)med3(lo, mid, hi);
}

hipError_t launch_median3x3(const Geometry &g, const double *src, float *dst, int pitch, hipStream_t s)
{
    hipLaunchKernelGGL(k_median3x3, dim3((g.W + 63) / 64, (g.H + 3) / 4), dim3(256), 0, s, g.W, g.H, src, dst,
                       pitch);
    return hipGetLastError();
}

}  // namespace sgmk
