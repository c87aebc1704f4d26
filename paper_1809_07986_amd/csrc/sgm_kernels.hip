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
    return __builtin_amdgcn_update_dpp(v, v, 0x120 + N, 0xF, 0xF, false);
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

hipError_t launch_scan(const Geometry &g, DevBuffers &b, hipStream_t s);

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
    return launch_scan(g, b, s);
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

__global__ void k_splat(int W, int H, int D, WarpConst wc, const double *__restrict__ d,
                        const double *__restrict__ p, int32_t *__restrict__ tgt, double *__restrict__ dprime,
                        double *__restrict__ pprime, unsigned long long *__restrict__ zkey)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= W * H)
        return;
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
                                const uint8_t *__restrict__ sflags, uint8_t *__restrict__ has,
                                double *__restrict__ dw, double *__restrict__ pw, uint8_t *__restrict__ rw)
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
    } else {
        has[t] = 0;
        dw[t] = 0.0;
        pw[t] = 0.0;
        rw[t] = 0;
    }
    zkey[t] = 0ull;
    zidx[t] = 0xFFFFFFFFu;
}

// zooming holes: a target without a winner whose left & right (or upper &
// lower) neighbours both have winners takes their mean disparity and mean
// variance; with both pairs, the mean of four (summed left, right, up, down)
__global__ void k_fill(int W, int H, const uint8_t *__restrict__ has, const double *__restrict__ dw,
                       const double *__restrict__ pw, const uint8_t *__restrict__ rw, uint8_t *__restrict__ pred,
                       double *__restrict__ dfill, double *__restrict__ pfill, uint8_t *__restrict__ rst)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= W * H)
        return;
    int y = t / W, x = t - y * W;
    uint8_t pr = has[t];
    double dv = dw[t], pv = pw[t];
    uint8_t rv = rw[t];
    if (!pr) {
        bool hp = x - 1 >= 0 && x + 1 < W && has[t - 1] && has[t + 1];
        bool vp = y - 1 >= 0 && y + 1 < H && has[t - W] && has[t + W];
        if (hp && vp) {
            dv = (((dw[t - 1] + dw[t + 1]) + dw[t - W]) + dw[t + W]) / 4.0;
            pv = (((pw[t - 1] + pw[t + 1]) + pw[t - W]) + pw[t + W]) / 4.0;
            rv = rw[t - 1] | rw[t + 1] | rw[t - W] | rw[t + W];
            pr = 1;
        } else if (hp) {
            dv = (dw[t - 1] + dw[t + 1]) / 2.0;
            pv = (pw[t - 1] + pw[t + 1]) / 2.0;
            rv = rw[t - 1] | rw[t + 1];
            pr = 1;
        } else if (vp) {
            dv = (dw[t - W] + dw[t + W]) / 2.0;
            pv = (pw[t - W] + pw[t + W]) / 2.0;
            rv = rw[t - W] | rw[t + W];
            pr = 1;
        }
    }
    pred[t] = pr;
    dfill[t] = dv;
    pfill[t] = pv;
    rst[t] = rv;
}

// discontinuity rejection (8-neighbourhood of the filled map, decided before
// any rejection) and the search limits d^ +- k sigma, rounded outward
__global__ void k_disc_windows(int W, int H, int D, CorrectConst cc, const uint8_t *__restrict__ pred,
                               const double *__restrict__ dfill, const double *__restrict__ pfill,
                               const uint8_t *__restrict__ rst, uint8_t *__restrict__ flags,
                               uint16_t *__restrict__ win, double *__restrict__ dhat, double *__restrict__ pm)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= W * H)
        return;
    int y = t / W, x = t - y * W;
    bool ok = pred[t];
    double dv = dfill[t];
    if (ok) {
        for (int yy = y - 1; yy <= y + 1; yy++) {
            for (int xx = x - 1; xx <= x + 1; xx++) {
                if (xx < 0 || xx >= W || yy < 0 || yy >= H || (xx == x && yy == y))
                    continue;
                int u = yy * W + xx;
                if (pred[u] && fabs(dv - dfill[u]) > cc.disc)
                    ok = false;
            }
        }
    }
    uint8_t fl = 0;
    if (ok)
        fl |= SGM_FLAG_PRED;
    if (rst[t])
        fl |= SGM_FLAG_RESET;
    bool full = !ok || rst[t] || !(dv >= 0.0 && dv <= (double)(D - 1));
    double pv = pfill[t];
    if (full) {
        fl |= SGM_FLAG_FULLWIN;
        win[t] = pack_win(0, D - 1);
    } else {
        double sd = sqrt(pv);
        double a = dv - cc.k_sigma * sd;
        double b = dv + cc.k_sigma * sd;
        int l = (int)floor(a), h = (int)ceil(b);
        l = l < 0 ? 0 : l;
        h = h > D - 1 ? D - 1 : h;
        win[t] = pack_win(l, h);
    }
    flags[t] = fl;
    dhat[t] = ok ? dv : 0.0;
    pm[t] = ok ? pv : 0.0;
}

hipError_t launch_predict(const Geometry &g, DevBuffers &b, const WarpConst &wc, const CorrectConst &cc,
                          hipStream_t s)
{
    dim3 blk(256), grd((g.N + 255) / 256);
    hipLaunchKernelGGL(k_splat, grd, blk, 0, s, g.W, g.H, g.D, wc, b.d, b.p, b.tgt, b.dprime, b.pprime, b.zkey);
    hipLaunchKernelGGL(k_splat_ties, grd, blk, 0, s, g.N, b.tgt, b.dprime, b.zkey, b.zidx);
    hipLaunchKernelGGL(k_splat_resolve, grd, blk, 0, s, g.N, b.zkey, b.zidx, b.dprime, b.pprime, b.sflags, b.has,
                       b.dw, b.pw, b.rw);
    hipLaunchKernelGGL(k_fill, grd, blk, 0, s, g.W, g.H, b.has, b.dw, b.pw, b.rw, b.pred, b.dfill, b.pfill, b.rst);
    hipLaunchKernelGGL(k_disc_windows, grd, blk, 0, s, g.W, g.H, g.D, cc, b.pred, b.dfill, b.pfill, b.rst, b.flags,
                       b.win, b.dhat, b.pm);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    return launch_scan(g, b, s);
}

// ---------------------------------------------------------------------------
// ragged offsets: exclusive prefix sum of the window widths.
// Three phases: per-block scan (4096 pixels per block), scan of the block
// totals in one block, add-back.  off[N] is the total cell count M.
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

__global__ __launch_bounds__(SCAN_T) void k_scan_blocks(int N, const uint16_t *__restrict__ win,
                                                        uint32_t *__restrict__ off, uint32_t *__restrict__ part)
{
    __shared__ uint32_t tot;
    const int base = blockIdx.x * SCAN_BLOCK + threadIdx.x * SCAN_PER;
    uint32_t w[SCAN_PER];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < SCAN_PER; i++) {
        int p = base + i;
        w[i] = p < N ? (uint32_t)(win[p] >> 8) + 1u : 0u;
        sum += w[i];
    }
    uint32_t ex = block_excl_scan(sum, &tot);
#pragma unroll
    for (int i = 0; i < SCAN_PER; i++) {
        int p = base + i;
        if (p < N)
            off[p] = ex;
        ex += w[i];
    }
    if (threadIdx.x == 0)
        part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_parts(int nparts, uint32_t *__restrict__ part)
{
    __shared__ uint32_t tot;
    const int base = threadIdx.x * SCAN_PER;
    uint32_t w[SCAN_PER];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < SCAN_PER; i++) {
        w[i] = base + i < nparts ? part[base + i] : 0u;
        sum += w[i];
    }
    uint32_t ex = block_excl_scan(sum, &tot);
#pragma unroll
    for (int i = 0; i < SCAN_PER; i++) {
        if (base + i < nparts)
            part[base + i] = ex;
        ex += w[i];
    }
    if (threadIdx.x == 0)
        part[nparts] = tot;
}

__global__ void k_scan_add(int N, int nparts, uint32_t *__restrict__ off, const uint32_t *__restrict__ part)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < N)
        off[p] += part[p / SCAN_BLOCK];
    else if (p == N)
        off[N] = part[nparts];
}

hipError_t launch_scan(const Geometry &g, DevBuffers &b, hipStream_t s)
{
    int nparts = (g.N + SCAN_BLOCK - 1) / SCAN_BLOCK;   // <= SCAN_BLOCK, checked at create
    hipLaunchKernelGGL(k_scan_blocks, dim3(nparts), dim3(SCAN_T), 0, s, g.N, b.win, b.off, b.scan_part);
    hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(SCAN_T), 0, s, nparts, b.scan_part);
    hipLaunchKernelGGL(k_scan_add, dim3((g.N + 1 + 255) / 256), dim3(256), 0, s, g.N, nparts, b.off, b.scan_part);
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
// One group of 16 lanes (a DPP row) walks one scanline of one path
// direction; lanes hold consecutive disparities of the current pixel's
// window (chunks of 16 for wider windows).  The predecessor's normalised
// L_r lives in LDS indexed by absolute disparity (double-buffered per
// group); a disparity outside the predecessor's window contributes nothing.
//   L_r(p,d) = C(p,d) + min(L(q,d), L(q,d-1)+P1, L(q,d+1)+P1, m_q+P2) - m_q
// with q = p - r and m_q = min over q's window; the first pixel of a
// scanline takes L_r = C.  Results are stored per path as bytes
// (L_r <= Nc + P2 <= 255, checked at create).
// ---------------------------------------------------------------------------

constexpr int AGG_G = 16, AGG_WAVES = 1, AGG_GROUPS = 4 * AGG_WAVES, AGG_T = 64 * AGG_WAVES;

struct AggArgs {
    const uint8_t *cost;
    const uint16_t *win;
    const uint32_t *off;
    uint8_t *lr;
    size_t lr_stride;
    int W, H, p1, p2, npaths;
    int8_t rx[kMaxPaths], ry[kMaxPaths];
};

template <int MAXCH>
__global__ __launch_bounds__(AGG_T) void k_aggregate(AggArgs a)
{
    __shared__ uint16_t buf[AGG_GROUPS][2][kMaxDisp + 2];
    const int k = blockIdx.y;
    const int grp = threadIdx.x >> 4, lane = threadIdx.x & 15;
    const int chain = blockIdx.x * AGG_GROUPS + grp;
    const int W = a.W, H = a.H;
    const int rx = a.rx[k], ry = a.ry[k];
    const int nch = (ry == 0) ? H : (rx == 0) ? W : W + H - 1;
    if (chain >= nch)
        return;
    // first pixel of the scanline and its length
    const int xs = rx > 0 ? 0 : W - 1, ys = ry > 0 ? 0 : H - 1;
    int x, y;
    if (ry == 0) {
        x = xs;
        y = chain;
    } else if (rx == 0) {
        x = chain;
        y = ys;
    } else if (chain < W) {
        x = chain;
        y = ys;
    } else {
        x = xs;
        y = ys + ry * (chain - W + 1);
    }
    int len;
    {
        int lx = rx > 0 ? W - x : (rx < 0 ? x + 1 : 1 << 30);
        int ly = ry > 0 ? H - y : (ry < 0 ? y + 1 : 1 << 30);
        len = min(lx, ly);
    }
    const int step = ry * W + rx;
    int p = y * W + x;
    uint8_t *lrk = a.lr + (size_t)k * a.lr_stride;
    uint16_t *bA = buf[grp][0];
    uint16_t *bB = buf[grp][1];
    const int p1 = a.p1, p2 = a.p2;
    int mq = 0, loq = 0, hiq = -1;

    // software pipeline: window/offset and costs of the next pixel are
    // loaded while the current one is processed
    uint32_t o = a.off[p];
    uint32_t wv = a.win[p];
    int cst[MAXCH];
    {
        int w = (int)(wv >> 8) + 1;
#pragma unroll
        for (int j = 0; j < MAXCH; j++)
            if (j * AGG_G + lane < w)
                cst[j] = a.cost[o + j * AGG_G + lane];
    }
    for (int i = 0; i < len; i++) {
        const int lo = (int)(wv & 255), w = (int)(wv >> 8) + 1, hi = lo + w - 1;
        const uint32_t oc = o;
        int cur[MAXCH];
#pragma unroll
        for (int j = 0; j < MAXCH; j++)
            cur[j] = cst[j];
        if (i + 1 < len) {
            const int pn = p + step;
            o = a.off[pn];
            wv = a.win[pn];
            const int wn = (int)(wv >> 8) + 1;
#pragma unroll
            for (int j = 0; j < MAXCH; j++)
                if (j * AGG_G + lane < wn)
                    cst[j] = a.cost[o + j * AGG_G + lane];
            p = pn;
        }
        int rmin = 0x7FFF;
#pragma unroll
        for (int j = 0; j < MAXCH; j++) {
            const int sidx = j * AGG_G + lane;
            if (sidx < w) {
                const int d = lo + sidx;
                int L;
                if (i == 0) {
                    L = cur[j];
                } else {
                    int best = mq + p2;
                    const int v0 = bA[d + 1], vm = bA[d], vp = bA[d + 2];
                    if (d >= loq && d <= hiq)
                        best = min(best, v0);
                    if (d - 1 >= loq && d - 1 <= hiq)
                        best = min(best, vm + p1);
                    if (d + 1 >= loq && d + 1 <= hiq)
                        best = min(best, vp + p1);
                    L = cur[j] + best - mq;
                }
                bB[d + 1] = (uint16_t)L;
                lrk[oc + sidx] = (uint8_t)L;
                rmin = min(rmin, L);
            }
        }
        mq = row_min16(rmin);
        loq = lo;
        hiq = hi;
        uint16_t *t = bA;
        bA = bB;
        bB = t;
        wave_lds_sync();
    }
}

hipError_t launch_aggregate(const Geometry &g, DevBuffers &b, hipStream_t s)
{
    AggArgs a;
    a.cost = b.cost;
    a.win = b.win;
    a.off = b.off;
    a.lr = b.lr;
    a.lr_stride = (size_t)g.N * g.D;
    a.W = g.W;
    a.H = g.H;
    a.p1 = g.p1;
    a.p2 = g.p2;
    a.npaths = g.npaths;
    for (int k = 0; k < kMaxPaths; k++) {
        a.rx[k] = g.rx[k];
        a.ry[k] = g.ry[k];
    }
    int maxch = g.W + g.H - 1;
    dim3 grd((maxch + AGG_GROUPS - 1) / AGG_GROUPS, g.npaths), blk(AGG_T);
    if (g.D <= 64)
        hipLaunchKernelGGL(k_aggregate<4>, grd, blk, 0, s, a);
    else if (g.D <= 128)
        hipLaunchKernelGGL(k_aggregate<8>, grd, blk, 0, s, a);
    else
        hipLaunchKernelGGL(k_aggregate<16>, grd, blk, 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// winner-takes-all (Section 2.3) with parabolic sub-pixel fit, then the
// Kalman correction (Eq. 5-6) and the innovation test (Section 4).
// Pass 1 (all threads, coalesced over the block's cell range): S = sum of
// the paths' L_r; per-pixel argmin via an LDS atomic on (S << 9 | slot),
// which picks the smallest S and then the lowest disparity.  Pass 2 (one
// thread per pixel): sub-pixel fit and filter update in double precision.
// ---------------------------------------------------------------------------

constexpr int WTA_PIX = 256;

__global__ __launch_bounds__(WTA_PIX) void k_wta_correct(int N, int D, int npaths, CorrectConst cc, int mode,
                                                         const uint8_t *__restrict__ lr, size_t lr_stride,
                                                         const uint16_t *__restrict__ win,
                                                         const uint32_t *__restrict__ off,
                                                         const uint8_t *__restrict__ flags,
                                                         const double *__restrict__ dhat,
                                                         const double *__restrict__ pm, uint16_t *__restrict__ dbg_sum,
                                                         int32_t *__restrict__ dstar_out, double *__restrict__ dz_out,
                                                         double *__restrict__ d_state, double *__restrict__ p_state,
                                                         uint8_t *__restrict__ mask, uint8_t *__restrict__ sflags)
{
    __shared__ uint32_t soff[WTA_PIX];
    __shared__ uint32_t skey[WTA_PIX];
    const int p0 = blockIdx.x * WTA_PIX;
    const int np = min(WTA_PIX, N - p0);
    if ((int)threadIdx.x < np) {
        soff[threadIdx.x] = off[p0 + threadIdx.x];
        skey[threadIdx.x] = 0xFFFFFFFFu;
    }
    __syncthreads();
    const uint32_t c0 = soff[0], c1 = off[p0 + np];
    for (uint32_t c = c0 + threadIdx.x; c < c1; c += WTA_PIX) {
        int i = find_pixel(soff, np, c);
        uint32_t sv = 0;
        for (int k = 0; k < npaths; k++)
            sv += lr[(size_t)k * lr_stride + c];
        if (dbg_sum)
            dbg_sum[c] = (uint16_t)sv;
        atomicMin(&skey[i], (sv << 9) | (c - soff[i]));
    }
    __syncthreads();
    if ((int)threadIdx.x >= np)
        return;
    const int t = p0 + threadIdx.x;
    const uint32_t key = skey[threadIdx.x];
    const int slot = (int)(key & 511u);
    const int s0 = (int)(key >> 9);
    const uint32_t wv = win[t];
    const int lo = (int)(wv & 255), hi = lo + (int)(wv >> 8);
    const int ds = lo + slot;
    double dz = (double)ds;
    if (ds - 1 >= lo && ds + 1 <= hi) {
        const uint32_t c = soff[threadIdx.x] + (uint32_t)slot;
        int sm = 0, sp = 0;
        for (int k = 0; k < npaths; k++) {
            sm += lr[(size_t)k * lr_stride + c - 1];
            sp += lr[(size_t)k * lr_stride + c + 1];
        }
        const int a = sm - s0, b = sp - s0;
        dz = (double)ds + (double)(a - b) / (double)(2 * (a + b));
    }
    dstar_out[t] = ds;
    dz_out[t] = dz;
    if (mode == 2)
        return;
    const uint8_t fl = flags[t];
    bool moving = false;
    double nu = 0.0, S = 0.0;
    const double dh = dhat[t], pv = pm[t];
    if (fl & SGM_FLAG_PRED) {
        nu = dz - dh;
        S = pv + cc.r;
        moving = (nu * nu) / S > cc.gate;
    }
    if (fl & SGM_FLAG_FULLWIN) {
        d_state[t] = dz;
        p_state[t] = cc.r;
    } else {
        const double K = pv / S;
        const double am = 1.0 - K;
        d_state[t] = dh + K * nu;
        p_state[t] = (am * am) * pv + (K * K) * cc.r;
    }
    const bool sat = (ds == lo && lo > 0) || (ds == hi && hi < D - 1);
    mask[t] = moving ? 1 : 0;
    sflags[t] = (moving || sat) ? SGM_FLAG_RESET : 0;
}

hipError_t launch_wta_correct(const Geometry &g, DevBuffers &b, const CorrectConst &cc, int mode,
                              bool debug_sum, hipStream_t s)
{
    hipLaunchKernelGGL(k_wta_correct, dim3((g.N + WTA_PIX - 1) / WTA_PIX), dim3(WTA_PIX), 0, s, g.N, g.D,
                       g.npaths, cc, mode, b.lr, (size_t)g.N * g.D, b.win, b.off, b.flags, b.dhat, b.pm,
                       debug_sum ? b.sum : (uint16_t *)nullptr, b.dstar, b.dz, b.d, b.p, b.mask, b.sflags);
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

}  // namespace sgmk
