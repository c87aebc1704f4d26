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
//   k_det_cols    64 columns x 16 row chunks per workgroup: difference
//                 values and their prefix down the scanned rows.
//   k_det_rows    one workgroup per scanned row: prefix of the column
//                 prefixes along the row (row r+1 of the table).
//   k_det_windows one thread per window: fired / not fired.
//   k_det_group   one workgroup of 1024 threads: ordered compaction of the
//                 fired windows, split into independent groups, greedy
//                 grouping with one wave per group, minimum-area filter,
//                 output.
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

// Column prefix of the difference values over the scanned rows.  A
// workgroup takes 64 columns (one per lane) and splits the rows into 16
// chunks (one per wave): each thread sums its chunk, the chunk sums are
// scanned through LDS, and each thread then writes the running prefix of its
// chunk (the inputs are read twice; the second read hits the cache).
constexpr int kColTile = 64, kColChunks = 16;

__device__ __forceinline__ uint32_t diff_value(const DetectGeom &dg, const double *__restrict__ dhat,
                                               const double *__restrict__ dz, const uint8_t *__restrict__ flags,
                                               int y, int x)
{
    const size_t i = (size_t)y * dg.W + x;
    const double dh = dhat[i];
    if ((flags[i] & SGM_FLAG_PRED) && (double)x - dh >= 0.0)
        return (uint32_t)fmin(floor(fabs(dh - dz[i]) * (double)dg.scale), (double)dg.cap);
    return 0;
}

__global__ void __launch_bounds__(1024) k_det_cols(DetectGeom dg, const double *__restrict__ dhat,
                                                   const double *__restrict__ dz, const uint8_t *__restrict__ flags,
                                                   uint32_t *__restrict__ colp)
{
    __shared__ uint32_t part[kColChunks][kColTile];
    const int lane = threadIdx.x & 63, c = threadIdx.x >> 6;
    const int x = blockIdx.x * kColTile + lane;
    const int per = (dg.rows + kColChunks - 1) / kColChunks;
    const int r0 = min(c * per, dg.rows), r1 = min(r0 + per, dg.rows);
    uint32_t sum = 0;
    if (x < dg.W)
        for (int r = r0; r < r1; r++)
            sum += diff_value(dg, dhat, dz, flags, dg.top + r, x);
    part[c][lane] = sum;
    __syncthreads();
    uint32_t acc = 0;
    for (int k = 0; k < c; k++)
        acc += part[k][lane];
    if (x < dg.W)
        for (int r = r0; r < r1; r++) {
            acc += diff_value(dg, dhat, dz, flags, dg.top + r, x);
            colp[(size_t)r * dg.W + x] = acc;
        }
}

// Row r+1 of the summed-area table: inclusive prefix of the column prefixes
// along row r (one workgroup per row; block 0 also writes the zero row).
__global__ void __launch_bounds__(256) k_det_rows(DetectGeom dg, const uint32_t *__restrict__ colp,
                                                  uint32_t *__restrict__ sat)
{
    __shared__ int lds[16];
    const int r = blockIdx.x;
    const size_t stride = (size_t)dg.W + 1;
    uint32_t *row = sat + (size_t)(r + 1) * stride;
    const uint32_t *src = colp + (size_t)r * dg.W;
    if (r == 0)
        for (int x = threadIdx.x; x <= dg.W; x += 256)
            sat[x] = 0;
    if (threadIdx.x == 0)
        row[0] = 0;
    int carry = 0;
    for (int x0 = 0; x0 < dg.W; x0 += 256) {
        const int x = x0 + threadIdx.x;
        const int v = x < dg.W ? (int)src[x] : 0;
        int total;
        const int ex = block_excl_scan(v, lds, &total);   // wrapping int sums: exact modulo 2^32
        if (x < dg.W)
            row[x + 1] = (uint32_t)(carry + ex + v);
        carry += total;
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

namespace {

// Union-find over box indices in LDS: parents only point to smaller
// indices, so every set ends with its smallest index as the root.
// Path halving: a non-root points to its grandparent (an ancestor, so
// concurrent walks still end at the root; roots are only written by the
// hooking compare-and-swap).
__device__ int uf_find(volatile int *par, int x)
{
    for (;;) {
        const int p = par[x];
        if (p == x)
            return x;
        const int gp = par[p];
        if (gp == p)
            return p;
        par[x] = gp;
        x = gp;
    }
}

// pair index p of the strictly lower triangle -> (a, b), a > b >= 0
__device__ __forceinline__ void tri_pair(int p, int &a, int &b)
{
    int r = (int)((1.0 + sqrt(1.0 + 8.0 * (double)p)) * 0.5);
    while ((long long)r * (r - 1) / 2 > p)
        r--;
    while ((long long)(r + 1) * r / 2 <= p)
        r++;
    a = r;
    b = p - (int)((long long)r * (r - 1) / 2);
}

__device__ void uf_unite(int *par, int a, int b)
{
    for (;;) {
        a = uf_find(par, a);
        b = uf_find(par, b);
        if (a == b)
            return;
        if (a > b) {
            int t = a;
            a = b;
            b = t;
        }
        if (atomicCAS(&par[b], b, a) == b)
            return;
    }
}

__device__ __forceinline__ bool overlap(const Box &a, const Box &b)
{
    return min(a.x1, b.x1) > max(a.x0, b.x0) && min(a.y1, b.y1) > max(a.y0, b.y0);
}

// orders this wave's LDS writes before its later LDS reads (all lanes)
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void wave_minmax(Box &b)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        b.x0 = min(b.x0, __shfl_xor(b.x0, o, 64));
        b.y0 = min(b.y0, __shfl_xor(b.y0, o, 64));
        b.x1 = max(b.x1, __shfl_xor(b.x1, o, 64));
        b.y1 = max(b.y1, __shfl_xor(b.y1, o, 64));
    }
}

// best partner of box a among the members of its group (wave-wide; every
// lane returns the same result)
__device__ void group_best(const short4 *bx, const uint8_t *alive, const short *mem, int st, int m, int a, int &BI,
                           int &BU, int &BJ)
{
    const int lane = threadIdx.x & 63;
    const Box A = get_box(bx, a);
    const int aa = area(A);
    BI = -1;
    BU = 1;
    BJ = INT_MAX;
    for (int q = lane; q < m; q += 64) {
        const int b = mem[st + q];
        if (b == a || !alive[b])
            continue;
        const Box B = get_box(bx, b);
        const int I = inter(A, B), U = aa + area(B) - I;
        if (ranks_before(I, U, b, BI, BU, BJ)) {
            BI = I;
            BU = U;
            BJ = b;
        }
    }
    wave_best(BI, BU, BJ);
}

}  // namespace

// LDS layout of k_det_group (bytes per box slot): bx 8, bI 4, bU 4, bj 2,
// par 4, mem 2, gs 4, gl 4, fl 4, alive 1.
constexpr size_t kDetGroupLds = (size_t)kDetMaxBoxes * 37;

// Ordered compaction of the fired windows, then the greedy grouping.
//
// Boxes that never overlap never merge (IoU 0 does not exceed a threshold
// >= 0), and a merged box stays inside the bounding box of the boxes it came
// from.  So the boxes are first split into groups: connected sets of
// overlapping boxes, joined further while the bounding boxes of two groups
// overlap.  No box of one group can ever overlap a box of another, and the
// greedy sequence inside a group does not depend on the others: each wave
// runs the grouping of one group at a time with wave-level synchronisation
// only, and all groups run in parallel.  Within a group every box keeps its
// best partner (highest IoU, then the lowest index); after a merge only the
// boxes whose partner was one of the pair search again, the others compare
// their partner with the merged box.
__global__ void __launch_bounds__(1024) k_det_group(DetectGeom dg, const uint8_t *__restrict__ fire,
                                                    int32_t *__restrict__ out, int32_t *__restrict__ count)
{
    extern __shared__ __align__(16) unsigned char smem[];
    short4 *bx = (short4 *)smem;
    int *bI = (int *)(bx + kDetMaxBoxes);
    int *bU = bI + kDetMaxBoxes;
    short *bj = (short *)(bU + kDetMaxBoxes);
    int *par = (int *)(bj + kDetMaxBoxes);
    short *mem = (short *)(par + kDetMaxBoxes);
    int *gs = (int *)(mem + kDetMaxBoxes);
    int *gl = gs + kDetMaxBoxes;
    int *fl = gl + kDetMaxBoxes;
    uint8_t *alive = (uint8_t *)(fl + kDetMaxBoxes);
    short4 *gbox = (short4 *)bI;   // group boxes while grouping (bI, bU unused then)
    short *roots = bj;             // group roots while grouping (bj unused then)
    __shared__ int lds[16];
    __shared__ int nroots, changed;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nwin = dg.base[dg.nsizes];

    // ---- ordered compaction (window order = size, row, column) ----------
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
    for (int i = tid; i < n; i += 1024) {
        alive[i] = 1;
        par[i] = i;
    }
    __syncthreads();

    // ---- groups: overlapping boxes, then overlapping group boxes ---------
    const int npairs = n * (n - 1) / 2;
    for (int p = tid; p < npairs; p += 1024) {
        int i, j;
        tri_pair(p, i, j);
        if (overlap(get_box(bx, i), get_box(bx, j)))
            uf_unite(par, i, j);
    }
    __syncthreads();
    const int nchunk = (n + 1023) / 1024;
    const int i0 = min(tid * nchunk, n), i1 = min(i0 + nchunk, n);
    for (;;) {
        for (int i = tid; i < n; i += 1024) {
            par[i] = uf_find(par, i);
            gl[i] = 0;
        }
        __syncthreads();
        for (int i = tid; i < n; i += 1024)
            atomicAdd(&gl[par[i]], 1);
        __syncthreads();
        // roots in ascending order and the start of each group's member list
        int nr = 0, nm = 0;
        for (int i = i0; i < i1; i++)
            if (par[i] == i) {
                nr++;
                nm += gl[i];
            }
        int tr, tm;
        int gr = block_excl_scan(nr, lds, &tr);
        int gm = block_excl_scan(nm, lds, &tm);
        for (int i = i0; i < i1; i++)
            if (par[i] == i) {
                roots[gr++] = (short)i;
                gs[i] = gm;
                fl[i] = gm;
                gm += gl[i];
            }
        if (tid == 0) {
            nroots = tr;
            changed = 0;
        }
        __syncthreads();
        for (int i = tid; i < n; i += 1024)
            mem[atomicAdd(&fl[par[i]], 1)] = (short)i;
        __syncthreads();
        const int r = nroots;
        for (int g = wave; g < r; g += 16) {
            const int root = roots[g], st = gs[root], m = gl[root];
            Box b{INT_MAX, INT_MAX, INT_MIN, INT_MIN};
            for (int q = lane; q < m; q += 64) {
                const Box c = get_box(bx, mem[st + q]);
                b.x0 = min(b.x0, c.x0);
                b.y0 = min(b.y0, c.y0);
                b.x1 = max(b.x1, c.x1);
                b.y1 = max(b.y1, c.y1);
            }
            wave_minmax(b);
            if (lane == 0)
                gbox[g] = make_short4((short)b.x0, (short)b.y0, (short)b.x1, (short)b.y1);
        }
        __syncthreads();
        const int rpairs = r * (r - 1) / 2;
        for (int p = tid; p < rpairs; p += 1024) {
            int g, h;
            tri_pair(p, g, h);
            if (overlap(get_box(gbox, g), get_box(gbox, h))) {
                uf_unite(par, roots[g], roots[h]);
                changed = 1;
            }
        }
        __syncthreads();
        if (!changed)
            break;
        __syncthreads();
    }
    const int r = nroots;
    if (dg.merge_iou == 0.0) {
        // Merging while any two boxes overlap ends in one box per group:
        // inside a group every merge keeps the overlap graph connected, so
        // the group collapses to its bounding box, and the groups are the
        // finest split whose bounding boxes do not overlap, which is the
        // end state of every merge order.  The merged box sits at the
        // group's smallest index, its root.
        for (int g = tid; g < r; g += 1024)
            bx[roots[g]] = gbox[g];
        for (int i = tid; i < n; i += 1024)
            alive[i] = par[i] == i;
        __syncthreads();
    }
    // per group index: start and size of the member list
    const int rg = dg.merge_iou == 0.0 ? 0 : r;
    int ga_st = 0, ga_m = 0, gb_st = 0, gb_m = 0;
    if (tid < rg) {
        ga_st = gs[roots[tid]];
        ga_m = gl[roots[tid]];
    }
    if (tid + 1024 < rg) {
        gb_st = gs[roots[tid + 1024]];
        gb_m = gl[roots[tid + 1024]];
    }
    __syncthreads();
    if (tid < rg) {
        gs[tid] = ga_st;
        gl[tid] = ga_m;
    }
    if (tid + 1024 < rg) {
        gs[tid + 1024] = gb_st;
        gl[tid + 1024] = gb_m;
    }
    __syncthreads();

    // ---- greedy grouping, one wave per group -----------------------------
    for (int g = wave; g < rg; g += 16) {
        const int st = gs[g], m = gl[g];
        if (m < 2)
            continue;
        for (int q = 0; q < m; q++) {
            const int a = mem[st + q];
            int BI, BU, BJ;
            group_best(bx, alive, mem, st, m, a, BI, BU, BJ);
            if (lane == 0) {
                bI[a] = BI;
                bU[a] = BU;
                bj[a] = BJ == INT_MAX ? (short)-1 : (short)BJ;
            }
        }
        wave_sync();
        for (;;) {
            int I = -1, U = 1, X = INT_MAX;
            for (int q = lane; q < m; q += 64) {
                const int a = mem[st + q];
                if (alive[a] && bj[a] >= 0 && ranks_before(bI[a], bU[a], a, I, U, X)) {
                    I = bI[a];
                    U = bU[a];
                    X = a;
                }
            }
            wave_best(I, U, X);
            if (X == INT_MAX || !((double)I > dg.merge_iou * (double)U))
                break;
            const int si = X, sj = bj[si];
            const Box A = get_box(bx, si), B = get_box(bx, sj);
            const Box mb{min(A.x0, B.x0), min(A.y0, B.y0), max(A.x1, B.x1), max(A.y1, B.y1)};
            const int am = area(mb);
            int nflag = 0;
            for (int q0 = 0; q0 < m; q0 += 64) {
                const int q = q0 + lane;
                bool flag = false;
                if (q < m) {
                    const int k = mem[st + q];
                    if (alive[k] && k != sj) {
                        if (k == si || bj[k] == si || bj[k] == sj) {
                            flag = true;
                        } else {
                            const Box b = get_box(bx, k);
                            const int Ik = inter(b, mb), Uk = area(b) + am - Ik;
                            if (ranks_before(Ik, Uk, si, bI[k], bU[k], bj[k])) {
                                bI[k] = Ik;
                                bU[k] = Uk;
                                bj[k] = (short)si;
                            }
                        }
                    }
                }
                const unsigned long long mask = __ballot(flag);
                if (flag)
                    fl[st + nflag + __popcll(mask & ((1ull << lane) - 1ull))] = mem[st + q];
                nflag += __popcll(mask);
            }
            wave_sync();
            if (lane == 0) {
                bx[si] = make_short4((short)mb.x0, (short)mb.y0, (short)mb.x1, (short)mb.y1);
                alive[sj] = 0;
            }
            wave_sync();
            for (int f = 0; f < nflag; f++) {
                const int k = fl[st + f];
                int BI, BU, BJ;
                group_best(bx, alive, mem, st, m, k, BI, BU, BJ);
                if (lane == 0) {
                    bI[k] = BI;
                    bU[k] = BU;
                    bj[k] = BJ == INT_MAX ? (short)-1 : (short)BJ;
                }
            }
            wave_sync();
        }
    }
    __syncthreads();

    // ---- drop boxes below the minimum area, keep list order -------------
    int keep = 0;
    for (int i = i0; i < i1; i++)
        keep += alive[i] && (long long)area(get_box(bx, i)) >= dg.min_area;
    int kept;
    int o = block_excl_scan(keep, lds, &kept);
    for (int i = i0; i < i1; i++) {
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
                         uint32_t *colp, uint32_t *sat, uint8_t *fire, int32_t *boxes, int32_t *count, hipStream_t s)
{
    static bool lds_ok[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= 64 || !lds_ok[dev]) {
        e = hipFuncSetAttribute((const void *)k_det_group, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)kDetGroupLds);
        if (e != hipSuccess)
            return e;
        if (dev >= 0 && dev < 64)
            lds_ok[dev] = true;
    }
    hipLaunchKernelGGL(k_det_cols, dim3((dg.W + kColTile - 1) / kColTile), dim3(1024), 0, s, dg, dhat, dz, flags,
                       colp);
    hipLaunchKernelGGL(k_det_rows, dim3(dg.rows), dim3(256), 0, s, dg, colp, sat);
    const int nwin = dg.base[dg.nsizes];
    if (nwin > 0)
        hipLaunchKernelGGL(k_det_windows, dim3((nwin + 255) / 256), dim3(256), 0, s, dg, sat, fire);
    hipLaunchKernelGGL(k_det_group, dim3(1), dim3(1024), kDetGroupLds, s, dg, fire, boxes, count);
    return hipGetLastError();
}

}  // namespace sgmk
