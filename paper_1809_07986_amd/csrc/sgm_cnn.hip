// Learned search window: a five-layer 3x3 convolutional network (channels
// 4 -> 16 -> 32 -> 32 -> 16 -> 2, ReLU between layers) that maps each
// pixel's prediction to a search half-width and a measurement variance, its
// training (backward pass, Gaussian NLL loss, Adam) and the per-pixel glue
// (network input, head, training targets).
//
// Convolutions are implicit GEMMs on the bf16 matrix cores with fp32
// accumulation: M = 16 output pixels of a row, N = output channels, K =
// (tap, input channel).  Activations are NHWC bfloat16; weights are
// pre-arranged ("fragments") so that each lane of a wave reads its K values
// of the B operand with one load.  The forward pass runs on gfx950's
// v_mfma_f32_16x16x32_bf16 (eight K values per lane, weights held in
// registers for a whole tile); the backward pass keeps the 16x16x16 form.
#include "sgm_internal.h"

namespace sgmk {

typedef short bf16x4 __attribute__((__vector_size__(4 * sizeof(short))));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((__vector_size__(4 * sizeof(float))));

constexpr int kCin[kCnnLayers] = {4, 16, 32, 32, 16};
constexpr int kCout[kCnnLayers] = {16, 32, 32, 16, 2};

__host__ __device__ constexpr int ksteps(int cin) { return (9 * cin + 15) / 16; }
__host__ __device__ constexpr int ntiles(int cout) { return (cout + 15) / 16; }
// channel count of a layer's output gradient as stored (multiple of 4)
__host__ __device__ constexpr int pad4(int c) { return (c + 3) & ~3; }

// offsets of each layer's weights W[co][ky][kx][ci] and biases b[co] in the
// flat parameter vector
__host__ __device__ constexpr int param_off(int l)
{
    int o = 0;
    for (int i = 0; i < l; i++)
        o += 9 * kCin[i] * kCout[i] + kCout[i];
    return o;
}
static_assert(param_off(kCnnLayers) == SGM_CNN_NPARAMS, "parameter count");

// fragments of the input-gradient kernel (layers 1..4; 16x16x16 form):
// [ksteps][ntiles][64 lanes] x 4 bf16 each
__host__ __device__ constexpr int bfrag_count(int l) { return ksteps(pad4(kCout[l])) * ntiles(kCin[l]) * 64; }
// start of layer l's input-gradient fragments (l >= 1); bfrag_off(kCnnLayers) is their end
__host__ __device__ constexpr int bfrag_off(int l)
{
    int o = 0;
    for (int i = 1; i < l; i++)
        o += bfrag_count(i);
    return o;
}

// forward fragments of the 16x16x32 kernel: [ksteps32][ntiles][64 lanes] x 8
// bf16 (two u64 each), after the others (at an even u64 index: 16-byte aligned)
__host__ __device__ constexpr int ksteps32(int cin) { return (9 * cin + 31) / 32; }
__host__ __device__ constexpr int f2_count(int l) { return ksteps32(kCin[l]) * ntiles(kCout[l]) * 64; }
__host__ __device__ constexpr int f2_off(int l)   // in u64
{
    int o = (bfrag_off(kCnnLayers) + 1) & ~1;
    for (int i = 0; i < l; i++)
        o += 2 * f2_count(i);
    return o;
}

size_t cnn_frag_count() { return (size_t)f2_off(kCnnLayers); }

__device__ __forceinline__ uint16_t f32_to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest, ties to even (finite inputs)
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// the same rounding (to nearest, ties to even) in one instruction (v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint16_t bf16_rne(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

// bfloat16 nearest to a double, ties to even, directly from the 52-bit
// significand (no intermediate float rounding); magnitudes below 2^-126
// give signed zero
__device__ __forceinline__ uint16_t f64_to_bf16(double x)
{
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const uint64_t sign = b >> 63;
    const uint64_t mag = b & 0x7FFFFFFFFFFFFFFFull;
    const uint64_t r = (mag + ((1ull << 44) - 1) + ((mag >> 45) & 1ull)) >> 45;
    const int64_t e = (int64_t)(r >> 7) - 1023 + 127;
    uint64_t bits = 0;
    if (e >= 1)
        bits = ((uint64_t)(e > 255 ? 255 : e) << 7) | (r & 0x7F);
    return (uint16_t)((sign << 15) | bits);
}

// ---------------------------------------------------------------------------
// fragment packing (from the fp32 parameter vector)
// ---------------------------------------------------------------------------

// B operand of the input gradient of layer l (1..4): B[k][n] = W[c][8 - tap][n]
// for k = tap * pad4(cout) + c (spatially flipped, transposed weights)
__global__ void k_pack(const float *__restrict__ theta, uint64_t *__restrict__ frag)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= bfrag_off(kCnnLayers))
        return;
    int l = 1;
    while (l + 1 < kCnnLayers && idx >= bfrag_off(l + 1))
        l++;
    const int local = idx - bfrag_off(l);
    const int cin = kCin[l], cout = kCout[l];
    const float *W = theta + param_off(l);
    const int kin = pad4(cout);                  // channels of the operand's input (the output gradient)
    const int nout = cin;
    const int nt_count = ntiles(nout);
    const int lane = local & 63;
    const int nt = (local >> 6) % nt_count;
    const int kk = (local >> 6) / nt_count;
    const int n = nt * 16 + (lane & 15);
    uint64_t packed = 0;
    for (int e = 0; e < 4; e++) {
        const int k = kk * 16 + (lane >> 4) * 4 + e;
        float v = 0.f;
        if (k < 9 * kin && n < nout) {
            const int tap = k / kin, c = k % kin;
            if (c < cout)
                v = W[(c * 9 + (8 - tap)) * cin + n];                 // W[c][flipped tap][n]
        }
        packed |= (uint64_t)f32_to_bf16(v) << (16 * e);
    }
    frag[idx] = packed;
}

// B operand of the 16x16x32 forward kernel: lane l of fragment (kk, nt)
// holds B[k][n] for n = 16 nt + l % 16 and k = 32 kk + 8 (l / 16) + j,
// j = 0..7, with k = tap * cin + c and B[k][n] = W[n][tap][c] (zero past the
// last tap or output channel)
__global__ void k_pack2(const float *__restrict__ theta, uint64_t *__restrict__ frag)
{
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    int l = 0;
    while (l < kCnnLayers && idx >= f2_count(l))
        idx -= f2_count(l++);
    if (l >= kCnnLayers)
        return;
    const int cin = kCin[l], cout = kCout[l];
    const float *W = theta + param_off(l);
    const int nt_count = ntiles(cout);
    const int lane = idx & 63;
    const int nt = (idx >> 6) % nt_count;
    const int kk = (idx >> 6) / nt_count;
    const int n = nt * 16 + (lane & 15);
    uint64_t half[2] = {0, 0};
    for (int j = 0; j < 8; j++) {
        const int k = kk * 32 + (lane >> 4) * 8 + j;
        float v = 0.f;
        if (k < 9 * cin && n < cout)
            v = W[(n * 9 + k / cin) * cin + k % cin];
        half[j >> 2] |= (uint64_t)f32_to_bf16(v) << (16 * (j & 3));
    }
    uint64_t *dst = frag + f2_off(l) + 2 * (size_t)idx;
    dst[0] = half[0];
    dst[1] = half[1];
}

hipError_t cnn_pack(const float *theta, uint64_t *frag, hipStream_t s)
{
    const int n = bfrag_off(kCnnLayers);
    hipLaunchKernelGGL(k_pack, dim3((n + 255) / 256), dim3(256), 0, s, theta, frag);
    int n2 = 0;
    for (int l = 0; l < kCnnLayers; l++)
        n2 += f2_count(l);
    hipLaunchKernelGGL(k_pack2, dim3((n2 + 255) / 256), dim3(256), 0, s, theta, frag);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 3x3 convolution of the backward pass (input gradient), implicit GEMM on
// v_mfma_f32_16x16x16_bf16: four K values per lane, one tap of four channels
// ---------------------------------------------------------------------------

constexpr int CV_TY = 8, CV_TX = 32;   // output tile of a block (4 waves x 4 M-tiles of 16 px)

enum { EPI_RELU = 0, EPI_F32 = 1, EPI_HEAD = 2 };   // forward epilogues (k_conv2)

// input gradient of a layer through the ReLU below it:
// out[p][n] = (mask[p][n] > 0) * sum_{tap, c} B[tap*CIN + c][n] * x[p + tap][c]
// (zero padding), bfloat16 out [p][COUT]
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_conv_grad(int H, int W, const uint16_t *__restrict__ x,
                                                   const uint64_t *__restrict__ frag,
                                                   const uint16_t *__restrict__ mask, uint16_t *__restrict__ y)
{
    constexpr int KS = ksteps(CIN), NT = ntiles(COUT);
    constexpr int SY = CV_TY + 2, SX = CV_TX + 2;
    __shared__ __align__(16) uint16_t tile[SY * SX * CIN];
    const int img = blockIdx.z;
    const int y0 = blockIdx.y * CV_TY, x0 = blockIdx.x * CV_TX;
    const size_t ibase = (size_t)img * H * W;
    // stage the input tile with its one-pixel halo (zeros outside the image)
    for (int e = threadIdx.x; e < SY * SX * (CIN / 4); e += 256) {
        const int q = e % (CIN / 4), px = e / (CIN / 4);
        const int sy = px / SX, sx = px % SX;
        const int gy = y0 + sy - 1, gx = x0 + sx - 1;
        uint2 v = make_uint2(0u, 0u);
        if (gy >= 0 && gy < H && gx >= 0 && gx < W)
            v = *(const uint2 *)(x + (ibase + (size_t)gy * W + gx) * CIN + 4 * q);
        *(uint2 *)(tile + px * CIN + 4 * q) = v;
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int grp = lane >> 4, col = lane & 15;
    f32x4 acc[4][NT];
#pragma unroll
    for (int m = 0; m < 4; m++)
#pragma unroll
        for (int t = 0; t < NT; t++)
            acc[m][t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int kk = 0; kk < KS; kk++) {
        const int k0 = kk * 16 + grp * 4;
        const int tap = k0 / CIN, c0 = k0 % CIN;
        const bool kval = k0 < 9 * CIN;
        const int ky = tap / 3, kx = tap % 3;
        bf16x4 b[NT];
#pragma unroll
        for (int t = 0; t < NT; t++) {
            const uint64_t f = frag[(kk * NT + t) * 64 + lane];
            b[t] = __builtin_bit_cast(bf16x4, f);
        }
#pragma unroll
        for (int m = 0; m < 4; m++) {
            const int row = wave * 2 + (m >> 1);
            const int cx = (m & 1) * 16 + col;
            uint64_t av = 0;
            if (kval)
                av = *(const uint64_t *)(tile + ((row + ky) * SX + cx + kx) * CIN + c0);
            const bf16x4 a = __builtin_bit_cast(bf16x4, av);
#pragma unroll
            for (int t = 0; t < NT; t++)
                acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b[t], acc[m][t], 0, 0, 0);
        }
    }
    // D[i][n]: lane holds rows i = 4*grp + e (pixels) of column n = col (channel)
#pragma unroll
    for (int m = 0; m < 4; m++) {
        const int gy = y0 + wave * 2 + (m >> 1);
        if (gy >= H)
            continue;
#pragma unroll
        for (int t = 0; t < NT; t++) {
            const int n = t * 16 + col;
            if (n >= COUT)
                continue;
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int gx = x0 + (m & 1) * 16 + grp * 4 + e;
                if (gx >= W)
                    continue;
                const size_t p = ibase + (size_t)gy * W + gx;
                const float v = acc[m][t][e];
                const bool pass = (mask[p * COUT + n] & 0x7FFFu) != 0;
                y[p * COUT + n] = f32_to_bf16(pass ? v : 0.f);
            }
        }
    }
}

template <int CIN, int COUT>
static hipError_t conv_grad(int nimg, int H, int W, const uint16_t *x, const uint64_t *frag, const uint16_t *mask,
                            uint16_t *y, hipStream_t s)
{
    dim3 grd((W + CV_TX - 1) / CV_TX, (H + CV_TY - 1) / CV_TY, nimg);
    hipLaunchKernelGGL((k_conv_grad<CIN, COUT>), grd, dim3(256), 0, s, H, W, x, frag, mask, y);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// per-pixel glue of the learned window
// ---------------------------------------------------------------------------

// network input of pixel t = (x, y) of a predicted frame (four bfloat16):
//  0: dhat / 64 (0 without prediction), 1: min(p^-, 16) / 4 (4 without),
//  2: (|I(x+1)-I(x-1)| + |I(y+1)-I(y-1)|) / 256, neighbours clamped,
//  3: min(|nu_w|, 8) / 4, nu_w the previous innovation of the warp winner
__device__ __forceinline__ uint2 feature_px(int W, int H, int x, int y, int t, const uint8_t *left, int pitch,
                                            const uint8_t *flags, const double *dhat, const double *pm,
                                            const double *nu_w)
{
    const bool pred = flags[t] & SGM_FLAG_PRED;
    const uint8_t *row = left + (size_t)y * pitch;
    const int gx = abs((int)row[min(x + 1, W - 1)] - (int)row[max(x - 1, 0)]);
    const int gy = abs((int)left[(size_t)min(y + 1, H - 1) * pitch + x] - (int)left[(size_t)max(y - 1, 0) * pitch + x]);
    const double f0 = pred ? dhat[t] * (1.0 / 64.0) : 0.0;
    const double f1 = pred ? fmin(pm[t], 16.0) * 0.25 : 4.0;
    const double f2 = (double)(gx + gy) * (1.0 / 256.0);
    const double f3 = fmin(fabs(nu_w[t]), 8.0) * 0.25;
    const uint32_t lo = (uint32_t)f64_to_bf16(f0) | ((uint32_t)f64_to_bf16(f1) << 16);
    const uint32_t hi = (uint32_t)f64_to_bf16(f2) | ((uint32_t)f64_to_bf16(f3) << 16);
    return make_uint2(lo, hi);
}

// head of pixel t: network output -> half-width w = max(1, k exp(o0 / 2))
// and measurement variance r = clamp(exp(o1), 1/16, 64) (o clipped to
// +-30); pixels with a finite window get [floor(dhat - w), ceil(dhat + w)]
// (double precision), or the full range when w >= 32
__device__ __forceinline__ void head_px(int t, int D, float k_sigma, float o0, float o1, const double *dhat, float *hw,
                                        float *rpix, uint8_t *flags, uint16_t *win)
{
    o0 = fminf(fmaxf(o0, -30.f), 30.f);
    o1 = fminf(fmaxf(o1, -30.f), 30.f);
    const float w = fmaxf(1.f, k_sigma * expf(0.5f * o0));
    const float r = fminf(fmaxf(expf(o1), 1.f / 16.f), 64.f);
    hw[t] = w;
    rpix[t] = r;
    const uint8_t fl = flags[t];
    if (fl & SGM_FLAG_FULLWIN)
        return;
    if (!(w < (float)SGM_LEARNED_WMAX)) {
        flags[t] = fl | SGM_FLAG_FULLWIN;
        win[t] = (uint16_t)((D - 1) << 8);
        return;
    }
    const double dv = dhat[t];
    int l = (int)floor(dv - (double)w), h = (int)ceil(dv + (double)w);
    l = l < 0 ? 0 : l;
    h = h > D - 1 ? D - 1 : h;
    win[t] = (uint16_t)(l | ((h - l) << 8));
}

// a frame's network: the first layer computes its input from the frame
// (and writes it out for the tile), the last applies the head
struct NetGlue {
    const uint8_t *left;
    int pitch;
    int D;
    float k_sigma;
    uint8_t *flags;
    const double *dhat, *pm, *nu_w;
    uint16_t *feat;
    float *hw, *rpix;
    uint16_t *win;
};

// ---------------------------------------------------------------------------
// 3x3 convolution, forward, on v_mfma_f32_16x16x32_bf16
//
// A block computes an 8 x 32 output tile: wave w takes rows 2w and 2w+1,
// two M-tiles of 16 pixels per row, all N-tiles.  The input tile and its
// one-pixel halo sit in LDS with a padded pixel stride (CIN + 8 values for
// CIN >= 16), so that the 16-byte A reads of sixteen neighbouring pixels
// fall in distinct banks; the layer's B fragments are read once into
// registers.  Lane l reads, for k-step kk, the eight K values 32 kk + 8 (l/16)
// + j: one tap and eight channels (CIN = 32), or half of one of two taps
// (CIN = 16), or two taps of four channels (CIN = 4).  The results go
// through LDS (bias, ReLU, bfloat16) and leave in 16-byte row stores.
// In a frame, the first layer stages the network input it computes itself
// (FEAT) and the last applies the head to its outputs (EPI_HEAD).
// ---------------------------------------------------------------------------

// 8 x 32 tiles: many small blocks keep the layer's staging, matrix work and
// stores of different blocks overlapping (8 x 64: 83 us per frame network,
// 4 x 64: 74, 8 x 32: 73, 4 x 128: 86)
constexpr int C2_TY = 8, C2_TX = 32, C2_SY = C2_TY + 2, C2_SX = C2_TX + 2;
constexpr int C2_RPW = C2_TY / 4;   // output rows per wave

__host__ __device__ constexpr int c2_ps(int cin) { return cin >= 16 ? cin + 8 : cin; }   // LDS pixel stride
__host__ __device__ constexpr int c2_out_bytes(int cout, int epi)
{
    return C2_TY * C2_TX * cout * (epi == EPI_RELU ? 2 : 4);
}
__host__ __device__ constexpr int c2_lds(int cin, int cout, int epi)
{
    const int in = C2_SY * C2_SX * c2_ps(cin) * 2;
    const int out = c2_out_bytes(cout, epi);
    return in > out ? in : out;
}

template <int CIN, int COUT, int EPI, bool FEAT>
__global__ __launch_bounds__(256) void k_conv2(int H, int W, const uint16_t *__restrict__ x,
                                               const uint64_t *__restrict__ frag, const float *__restrict__ bias,
                                               uint16_t *__restrict__ y, float *__restrict__ yf, NetGlue fg)
{
    static_assert(EPI == EPI_RELU || EPI == EPI_F32 || EPI == EPI_HEAD, "forward epilogues");
    static_assert(!FEAT || CIN == 4, "the network input has four channels");
    static_assert(CIN == 4 || CIN == 16 || CIN == 32, "input channels");
    constexpr int KS = ksteps32(CIN), NT = ntiles(COUT), PS = c2_ps(CIN);
    constexpr int MW = C2_RPW * (C2_TX / 16);   // M-tiles per wave
    __shared__ __align__(16) uint16_t smem[c2_lds(CIN, COUT, EPI) / 2];
    const int img = blockIdx.z;
    const int y0 = blockIdx.y * C2_TY, x0 = blockIdx.x * C2_TX;
    const size_t ibase = (size_t)img * H * W;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int kg = lane >> 4, col = lane & 15;
    // this lane's B fragments for the whole layer
    uint4 bfr[KS][NT];
    {
        const uint4 *fb = (const uint4 *)frag;
#pragma unroll
        for (int kk = 0; kk < KS; kk++)
#pragma unroll
            for (int t = 0; t < NT; t++)
                bfr[kk][t] = fb[(kk * NT + t) * 64 + lane];
    }
    // stage the input tile with its halo (zeros outside the image)
    {
        constexpr int CH = CIN >= 8 ? 8 : 4;              // channels per staged chunk
        constexpr int NCH = C2_SY * C2_SX * (CIN / CH);
        constexpr int PER = (NCH + 255) / 256;
        if (CH == 8) {
            uint4 v[PER];
#pragma unroll
            for (int i = 0; i < PER; i++) {
                const int e = threadIdx.x + 256 * i;
                const int q = e % (CIN / CH), px = e / (CIN / CH);
                const int sy = px / C2_SX, sx = px - sy * C2_SX;
                const int gy = y0 + sy - 1, gx = x0 + sx - 1;
                const bool ok = e < NCH && gy >= 0 && gy < H && gx >= 0 && gx < W;
                const size_t src = ok ? (ibase + (size_t)gy * W + gx) * CIN + CH * q : 0;
                const uint4 u = *(const uint4 *)(x + src);
                v[i] = ok ? u : make_uint4(0u, 0u, 0u, 0u);
            }
#pragma unroll
            for (int i = 0; i < PER; i++) {
                const int e = threadIdx.x + 256 * i;
                const int q = e % (CIN / CH), px = e / (CIN / CH);
                if (e < NCH)
                    *(uint4 *)(smem + px * PS + CH * q) = v[i];
            }
        } else {
            uint2 v[PER];
#pragma unroll
            for (int i = 0; i < PER; i++) {
                const int e = threadIdx.x + 256 * i;
                const int sy = e / C2_SX, sx = e - sy * C2_SX;
                const int gy = y0 + sy - 1, gx = x0 + sx - 1;
                const bool ok = e < NCH && gy >= 0 && gy < H && gx >= 0 && gx < W;
                if (FEAT) {
                    // the frame's network input, written out for the tile's own pixels
                    v[i] = make_uint2(0u, 0u);
                    if (ok) {
                        const int t = gy * W + gx;
                        v[i] = feature_px(W, H, gx, gy, t, fg.left, fg.pitch, fg.flags, fg.dhat, fg.pm, fg.nu_w);
                        if (sy >= 1 && sy <= C2_TY && sx >= 1 && sx <= C2_TX)
                            *(uint2 *)(fg.feat + (size_t)t * 4) = v[i];
                    }
                } else {
                    const size_t src = ok ? (ibase + (size_t)gy * W + gx) * CIN : 0;
                    const uint2 u = *(const uint2 *)(x + src);
                    v[i] = ok ? u : make_uint2(0u, 0u);
                }
            }
#pragma unroll
            for (int i = 0; i < PER; i++) {
                const int e = threadIdx.x + 256 * i;
                if (e < NCH)
                    *(uint2 *)(smem + e * PS) = v[i];
            }
        }
    }
    __syncthreads();
    f32x4 acc[MW][NT];
#pragma unroll
    for (int m = 0; m < MW; m++)
#pragma unroll
        for (int t = 0; t < NT; t++)
            acc[m][t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < KS; kk++) {
#pragma unroll
        for (int m = 0; m < MW; m++) {
            const int row = C2_RPW * wave + m / (C2_TX / 16);     // output row in the tile
            const int cx = (m % (C2_TX / 16)) * 16 + col;         // output column in the tile
            uint4 av;
            if (CIN == 32) {
                const int ky = kk / 3, kx = kk % 3;
                av = *(const uint4 *)(smem + ((row + ky) * C2_SX + cx + kx) * PS + 8 * kg);
            } else if (CIN == 16) {
                const int tap = 2 * kk + (kg >> 1);
                const int ky = tap / 3, kx = tap % 3;
                av = make_uint4(0u, 0u, 0u, 0u);
                if (tap < 9)
                    av = *(const uint4 *)(smem + ((row + ky) * C2_SX + cx + kx) * PS + 8 * (kg & 1));
            } else {
                const int t0 = 8 * kk + 2 * kg, t1 = t0 + 1;
                uint2 lo = make_uint2(0u, 0u), hi = make_uint2(0u, 0u);
                if (t0 < 9)
                    lo = *(const uint2 *)(smem + ((row + t0 / 3) * C2_SX + cx + t0 % 3) * PS);
                if (t1 < 9)
                    hi = *(const uint2 *)(smem + ((row + t1 / 3) * C2_SX + cx + t1 % 3) * PS);
                av = make_uint4(lo.x, lo.y, hi.x, hi.y);
            }
            const bf16x8 a = __builtin_bit_cast(bf16x8, av);
#pragma unroll
            for (int t = 0; t < NT; t++)
                acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf16x8, bfr[kk][t]),
                                                                    acc[m][t], 0, 0, 0);
        }
    }
    __syncthreads();   // every wave has read the input tile: its LDS takes the results
    // D[i][n]: lane holds pixels i = 4 kg + e of its M-tile, channel n = 16 t + col
#pragma unroll
    for (int t = 0; t < NT; t++) {
        const int n = t * 16 + col;
        if (n >= COUT)
            continue;
        const float bv = bias[n];
#pragma unroll
        for (int m = 0; m < MW; m++) {
            const int row = C2_RPW * wave + m / (C2_TX / 16);
            const int px0 = row * C2_TX + (m % (C2_TX / 16)) * 16 + 4 * kg;
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const float v = acc[m][t][e] + bv;
                if (EPI == EPI_RELU)
                    smem[(px0 + e) * COUT + n] = bf16_rne(fmaxf(v, 0.f));
                else
                    ((float *)smem)[(px0 + e) * COUT + n] = v;
            }
        }
    }
    __syncthreads();
    if (EPI == EPI_HEAD) {
        // raw outputs of each tile pixel, then its half-width, variance and window
        for (int e = threadIdx.x; e < C2_TY * C2_TX; e += 256) {
            const int r = e / C2_TX, c = e - r * C2_TX;
            const int gy = y0 + r, gx = x0 + c;
            if (gy >= H || gx >= W)
                continue;
            const int t = gy * W + gx;
            const float o0 = ((const float *)smem)[2 * e], o1 = ((const float *)smem)[2 * e + 1];
            *(float2 *)(yf + 2 * (ibase + (size_t)t)) = make_float2(o0, o1);
            head_px(t, fg.D, fg.k_sigma, o0, o1, fg.dhat, fg.hw, fg.rpix, fg.flags, fg.win);
        }
        return;
    }
    // rows of the tile to memory in 16-byte (8-byte for the fp32 head) pieces
    constexpr int PB = COUT * (EPI == EPI_F32 ? 4 : 2);   // bytes per pixel
    constexpr int CB = PB >= 16 ? 16 : PB;                 // bytes per piece
    constexpr int PPR = C2_TX * PB / CB;                   // pieces per tile row
    const int nx = min(C2_TX, W - x0);
    for (int e = threadIdx.x; e < C2_TY * PPR; e += 256) {
        const int r = e / PPR, c = e - r * PPR;
        const int gy = y0 + r;
        const int px = c * CB / PB;                        // pixel of the piece in its row
        if (gy >= H || px >= nx)
            continue;
        const uint8_t *src = (const uint8_t *)smem + (size_t)r * C2_TX * PB + (size_t)c * CB;
        uint8_t *dst = (EPI == EPI_F32 ? (uint8_t *)yf : (uint8_t *)y) +
                       ((ibase + (size_t)gy * W + x0) * PB + (size_t)c * CB);
        if (CB == 16)
            *(uint4 *)dst = *(const uint4 *)src;
        else
            *(uint2 *)dst = *(const uint2 *)src;
    }
}

template <int CIN, int COUT, int EPI, bool FEAT = false>
static hipError_t conv2(int nimg, int H, int W, const uint16_t *x, const uint64_t *frag, const float *bias,
                        uint16_t *y, float *yf, hipStream_t s, const NetGlue &fg = NetGlue{})
{
    dim3 grd((W + C2_TX - 1) / C2_TX, (H + C2_TY - 1) / C2_TY, nimg);
    hipLaunchKernelGGL((k_conv2<CIN, COUT, EPI, FEAT>), grd, dim3(256), 0, s, H, W, x, frag, bias, y, yf, fg);
    return hipGetLastError();
}

hipError_t cnn_forward(const float *theta, const uint64_t *frag, const uint16_t *x, int nimg, int H, int W,
                       uint16_t *a1, uint16_t *a2, uint16_t *a3, uint16_t *a4, float *out, hipStream_t s)
{
    hipError_t e;
#define CNN_TRY(call)                 \
    do {                              \
        if ((e = (call)) != hipSuccess) \
            return e;                 \
    } while (0)
    CNN_TRY((conv2<4, 16, EPI_RELU>(nimg, H, W, x, frag + f2_off(0), theta + param_off(0) + 9 * 4 * 16, a1,
                                    nullptr, s)));
    CNN_TRY((conv2<16, 32, EPI_RELU>(nimg, H, W, a1, frag + f2_off(1), theta + param_off(1) + 9 * 16 * 32, a2,
                                     nullptr, s)));
    CNN_TRY((conv2<32, 32, EPI_RELU>(nimg, H, W, a2, frag + f2_off(2), theta + param_off(2) + 9 * 32 * 32, a3,
                                     nullptr, s)));
    CNN_TRY((conv2<32, 16, EPI_RELU>(nimg, H, W, a3, frag + f2_off(3), theta + param_off(3) + 9 * 32 * 16, a4,
                                     nullptr, s)));
    CNN_TRY((conv2<16, 2, EPI_F32>(nimg, H, W, a4, frag + f2_off(4), theta + param_off(4) + 9 * 16 * 2, nullptr,
                                   out, s)));
    return hipSuccess;
}

hipError_t cnn_forward_frame(const Geometry &g, DevBuffers &b, const uint8_t *left, int pitch, float k_sigma,
                             hipStream_t s)
{
    hipError_t e;
    const NetGlue fg{left, pitch, g.D, k_sigma, b.flags, b.dhat, b.pm, b.nu_w, b.feat, b.hw, b.rpix, b.win};
    const float *theta = b.theta;
    const uint64_t *frag = b.frag;
    const int H = g.H, W = g.W;
    CNN_TRY((conv2<4, 16, EPI_RELU, true>(1, H, W, nullptr, frag + f2_off(0), theta + param_off(0) + 9 * 4 * 16,
                                          b.act_a, nullptr, s, fg)));
    CNN_TRY((conv2<16, 32, EPI_RELU>(1, H, W, b.act_a, frag + f2_off(1), theta + param_off(1) + 9 * 16 * 32, b.act_b,
                                     nullptr, s)));
    CNN_TRY((conv2<32, 32, EPI_RELU>(1, H, W, b.act_b, frag + f2_off(2), theta + param_off(2) + 9 * 32 * 32, b.act_a,
                                     nullptr, s)));
    CNN_TRY((conv2<32, 16, EPI_RELU>(1, H, W, b.act_a, frag + f2_off(3), theta + param_off(3) + 9 * 32 * 16, b.act_b,
                                     nullptr, s)));
    CNN_TRY((conv2<16, 2, EPI_HEAD>(1, H, W, b.act_b, frag + f2_off(4), theta + param_off(4) + 9 * 16 * 2, nullptr,
                                    b.cnn_out, s, fg)));
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// weight gradients: dW[co][tap][ci] = sum_p g[p][co] * x[p + tap][ci],
// db[co] = sum_p g[p][co]; GEMM with M = co, N = (tap, ci), K = pixels.
// Each block accumulates over row segments of 64 pixels and writes its
// partial sums; a second kernel adds the partials in a fixed order.
// ---------------------------------------------------------------------------

constexpr int WG_SEG = 64;
constexpr int kWgradBlocks = 240;

template <int CIN, int COUT, int GS>
__global__ __launch_bounds__(256) void k_wgrad(int nimg, int H, int W, const uint16_t *__restrict__ x,
                                               const uint16_t *__restrict__ g, float *__restrict__ part)
{
    constexpr int MT = ntiles(COUT), NTW = ksteps(CIN);   // (tap, ci) columns in tiles of 16
    constexpr int NPAIR = MT * NTW, PPW = (NPAIR + 3) / 4;
    constexpr int SX = WG_SEG + 2;
    constexpr int NW = 9 * CIN * COUT + COUT;
    __shared__ __align__(16) uint16_t sx[3 * SX * CIN];
    __shared__ __align__(16) uint16_t sg[WG_SEG * GS];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int grp = lane >> 4, col = lane & 15;
    f32x4 acc[PPW];
#pragma unroll
    for (int q = 0; q < PPW; q++)
        acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bacc = 0.f;
    const int segs = (W + WG_SEG - 1) / WG_SEG;
    const long ntile = (long)nimg * H * segs;
    for (long tI = blockIdx.x; tI < ntile; tI += gridDim.x) {
        const int sgi = (int)(tI % segs);
        const long rowi = tI / segs;
        const int yy = (int)(rowi % H), img = (int)(rowi / H);
        const int x0 = sgi * WG_SEG;
        const size_t ibase = (size_t)img * H * W;
        __syncthreads();   // previous tile fully consumed
        for (int e = threadIdx.x; e < 3 * SX * (CIN / 4); e += 256) {
            const int q = e % (CIN / 4), px = e / (CIN / 4);
            const int r = px / SX, c = px % SX;
            const int gy = yy + r - 1, gx = x0 + c - 1;
            uint2 v = make_uint2(0u, 0u);
            if (gy >= 0 && gy < H && gx >= 0 && gx < W)
                v = *(const uint2 *)(x + (ibase + (size_t)gy * W + gx) * CIN + 4 * q);
            *(uint2 *)(sx + px * CIN + 4 * q) = v;
        }
        for (int e = threadIdx.x; e < WG_SEG * (GS / 4); e += 256) {
            const int q = e % (GS / 4), px = e / (GS / 4);
            const int gx = x0 + px;
            uint2 v = make_uint2(0u, 0u);
            if (gx < W)
                v = *(const uint2 *)(g + (ibase + (size_t)yy * W + gx) * GS + 4 * q);
            *(uint2 *)(sg + px * GS + 4 * q) = v;
        }
        __syncthreads();
        if (threadIdx.x < COUT) {
            float s = 0.f;
            for (int px = 0; px < WG_SEG; px++)
                s += bf16_to_f32(sg[px * GS + threadIdx.x]);
            bacc += s;
        }
#pragma unroll
        for (int ks = 0; ks < WG_SEG / 16; ks++) {
            const int pbase = ks * 16 + grp * 4;
#pragma unroll
            for (int q = 0; q < PPW; q++) {
                const int pr = wave + 4 * q;
                if (pr >= NPAIR)
                    break;
                const int mt = pr / NTW, nt = pr % NTW;
                const int co = mt * 16 + col;
                const int j = nt * 16 + col;
                uint16_t av[4], bv[4];
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    av[e] = co < COUT ? sg[(pbase + e) * GS + co] : (uint16_t)0;
                    uint16_t v = 0;
                    if (j < 9 * CIN) {
                        const int tap = j / CIN, ci = j % CIN;
                        v = sx[((tap / 3) * SX + pbase + e + (tap % 3)) * CIN + ci];
                    }
                    bv[e] = v;
                }
                const uint64_t ap = (uint64_t)av[0] | ((uint64_t)av[1] << 16) | ((uint64_t)av[2] << 32) |
                                    ((uint64_t)av[3] << 48);
                const uint64_t bp = (uint64_t)bv[0] | ((uint64_t)bv[1] << 16) | ((uint64_t)bv[2] << 32) |
                                    ((uint64_t)bv[3] << 48);
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(bf16x4, ap),
                                                                    __builtin_bit_cast(bf16x4, bp), acc[q], 0, 0,
                                                                    0);
            }
        }
    }
    float *pb = part + (size_t)blockIdx.x * NW;
#pragma unroll
    for (int q = 0; q < PPW; q++) {
        const int pr = wave + 4 * q;
        if (pr >= NPAIR)
            break;
        const int mt = pr / NTW, nt = pr % NTW;
        const int j = nt * 16 + col;
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int co = mt * 16 + grp * 4 + e;
            if (co < COUT && j < 9 * CIN)
                pb[co * 9 * CIN + j] = acc[q][e];
        }
    }
    if (threadIdx.x < COUT)
        pb[9 * CIN * COUT + threadIdx.x] = bacc;
}

__global__ void k_sum_parts(int nblk, int nw, const float *__restrict__ part, float *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nw)
        return;
    float s = 0.f;
    for (int b = 0; b < nblk; b++)
        s += part[(size_t)b * nw + i];
    out[i] = s;
}

size_t cnn_part_floats()
{
    size_t m = 0;
    for (int l = 0; l < kCnnLayers; l++) {
        size_t nw = (size_t)9 * kCin[l] * kCout[l] + kCout[l];
        m = nw > m ? nw : m;
    }
    return m * kWgradBlocks;
}

template <int CIN, int COUT, int GS>
static hipError_t wgrad(int nimg, int H, int W, const uint16_t *x, const uint16_t *g, float *part, float *out,
                        hipStream_t s)
{
    constexpr int NW = 9 * CIN * COUT + COUT;
    hipLaunchKernelGGL((k_wgrad<CIN, COUT, GS>), dim3(kWgradBlocks), dim3(256), 0, s, nimg, H, W, x, g, part);
    hipLaunchKernelGGL(k_sum_parts, dim3((NW + 255) / 256), dim3(256), 0, s, kWgradBlocks, NW, part, out);
    return hipGetLastError();
}

hipError_t cnn_backward(const float *theta, const uint64_t *frag, const uint16_t *x, const uint16_t *a1,
                        const uint16_t *a2, const uint16_t *a3, const uint16_t *a4, const uint16_t *dz5, int nimg,
                        int H, int W, uint16_t *g0, uint16_t *g1, float *part, float *grad, hipStream_t s)
{
    (void)theta;
    hipError_t e;
    // layer 5 (16 -> 2): its output gradient is stored with 4 channels
    CNN_TRY((wgrad<16, 2, 4>(nimg, H, W, a4, dz5, part, grad + param_off(4), s)));
    CNN_TRY((conv_grad<4, 16>(nimg, H, W, dz5, frag + bfrag_off(4), a4, g0, s)));
    // layer 4 (32 -> 16)
    CNN_TRY((wgrad<32, 16, 16>(nimg, H, W, a3, g0, part, grad + param_off(3), s)));
    CNN_TRY((conv_grad<16, 32>(nimg, H, W, g0, frag + bfrag_off(3), a3, g1, s)));
    // layer 3 (32 -> 32)
    CNN_TRY((wgrad<32, 32, 32>(nimg, H, W, a2, g1, part, grad + param_off(2), s)));
    CNN_TRY((conv_grad<32, 32>(nimg, H, W, g1, frag + bfrag_off(2), a2, g0, s)));
    // layer 2 (16 -> 32)
    CNN_TRY((wgrad<16, 32, 32>(nimg, H, W, a1, g0, part, grad + param_off(1), s)));
    CNN_TRY((conv_grad<32, 16>(nimg, H, W, g0, frag + bfrag_off(1), a1, g1, s)));
    // layer 1 (4 -> 16)
    CNN_TRY((wgrad<4, 16, 16>(nimg, H, W, x, g1, part, grad + param_off(0), s)));
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// loss: Gaussian NLL of the prediction residual e (channel 0) and the
// measurement residual m (channel 1), each averaged over its weighted pixels;
// writes dL/do as bfloat16 with 4 channels (2, 3 zero)
// ---------------------------------------------------------------------------

constexpr float kOClampLoss = 15.f;
constexpr int kLossBlocks = 512;

__global__ void k_count(size_t P, const float *__restrict__ tgt, float *__restrict__ part)
{
    __shared__ float s0[256], s1[256];
    float a = 0.f, b = 0.f;
    for (size_t i = blockIdx.x * 256 + threadIdx.x; i < P; i += (size_t)gridDim.x * 256) {
        a += tgt[i * 4 + 2];
        b += tgt[i * 4 + 3];
    }
    s0[threadIdx.x] = a;
    s1[threadIdx.x] = b;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            s0[threadIdx.x] += s0[threadIdx.x + h];
            s1[threadIdx.x] += s1[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s0[0];
        part[2 * blockIdx.x + 1] = s1[0];
    }
}

// cnt[0..1] = max(1, sum); one thread block
__global__ void k_count_final(int nblk, const float *__restrict__ part, float *__restrict__ cnt)
{
    if (threadIdx.x >= 2)
        return;
    float s = 0.f;
    for (int b = 0; b < nblk; b++)
        s += part[2 * b + threadIdx.x];
    cnt[threadIdx.x] = fmaxf(1.f, s);
}

__global__ void k_loss(size_t P, const float *__restrict__ out, const float *__restrict__ tgt,
                       const float *__restrict__ cnt, uint16_t *__restrict__ dz, float *__restrict__ part)
{
    __shared__ float sl[256];
    const float ne = cnt[0], nm = cnt[1];
    float L = 0.f;
    for (size_t i = blockIdx.x * 256 + threadIdx.x; i < P; i += (size_t)gridDim.x * 256) {
        const float4 t = *(const float4 *)(tgt + i * 4);
        uint16_t gq[2];
        for (int c = 0; c < 2; c++) {
            const float o = out[i * 2 + c];
            const float res = c == 0 ? t.x : t.y;
            const float w = (c == 0 ? t.z : t.w) / (c == 0 ? ne : nm);
            const float oc = fminf(fmaxf(o, -kOClampLoss), kOClampLoss);
            const bool inside = o > -kOClampLoss && o < kOClampLoss;
            const float ex = expf(-oc);
            const float r2 = res * res;
            L += w * 0.5f * (oc + r2 * ex);
            gq[c] = f32_to_bf16(inside ? w * 0.5f * (1.f - r2 * ex) : 0.f);
        }
        *(uint2 *)(dz + i * 4) = make_uint2((uint32_t)gq[0] | ((uint32_t)gq[1] << 16), 0u);
    }
    sl[threadIdx.x] = L;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h)
            sl[threadIdx.x] += sl[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        part[blockIdx.x] = sl[0];
}

hipError_t cnn_loss(const float *out, const float *tgt, size_t P, float *cnt, float *part, uint16_t *dz,
                    float *loss, hipStream_t s)
{
    hipLaunchKernelGGL(k_count, dim3(kLossBlocks), dim3(256), 0, s, P, tgt, part);
    hipLaunchKernelGGL(k_count_final, dim3(1), dim3(64), 0, s, kLossBlocks, part, cnt);
    hipLaunchKernelGGL(k_loss, dim3(kLossBlocks), dim3(256), 0, s, P, out, tgt, cnt, dz, part);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, s, kLossBlocks, 1, part, loss);
    return hipGetLastError();
}

size_t cnn_loss_part_floats() { return 2 * kLossBlocks; }

// ---------------------------------------------------------------------------
// Adam (Kingma & Ba, 2015): m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
// theta <- theta - lr * (m c1) / (sqrt(v c2) + eps), c1,2 the bias corrections
// ---------------------------------------------------------------------------

__global__ void k_adam(int n, float *__restrict__ theta, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, float lr, float b1, float b2, float c1, float c2, float eps)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

hipError_t cnn_adam(float *theta, float *m, float *v, const float *g, int step, float lr, hipStream_t s)
{
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 / (1.0 - pow(b1, step))), c2 = (float)(1.0 / (1.0 - pow(b2, step)));
    hipLaunchKernelGGL(k_adam, dim3((SGM_CNN_NPARAMS + 255) / 256), dim3(256), 0, s, SGM_CNN_NPARAMS, theta, m, v,
                       g, lr, (float)b1, (float)b2, c1, c2, 1e-8f);
    return hipGetLastError();
}

// network input of every pixel (bfloat16 [N][4]; see feature_px), for
// callers that want it on its own (a frame's network computes its own)
__global__ void k_features(int W, int H, const uint8_t *__restrict__ left, int pitch,
                           const uint8_t *__restrict__ flags, const double *__restrict__ dhat,
                           const double *__restrict__ pm, const double *__restrict__ nu_w,
                           uint16_t *__restrict__ feat)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= W * H)
        return;
    const int y = t / W, x = t - y * W;
    *(uint2 *)(feat + (size_t)t * 4) = feature_px(W, H, x, y, t, left, pitch, flags, dhat, pm, nu_w);
}

hipError_t launch_features(const Geometry &g, const DevBuffers &b, const uint8_t *left, int pitch, uint16_t *feat,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_features, dim3((g.N + 255) / 256), dim3(256), 0, s, g.W, g.H, left, pitch, b.flags, b.dhat,
                       b.pm, b.nu_w, feat);
    return hipGetLastError();
}

// training targets of a predicted frame: e = dz_full - dhat, m = dz_full - gt
// (clipped to +-16), weights we = [prediction], wm = we * [gt >= 0]
__global__ void k_targets(int N, const uint8_t *__restrict__ flags, const double *__restrict__ dhat,
                          const double *__restrict__ dz_full, const float *__restrict__ gt, float *__restrict__ tgt)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N)
        return;
    const bool pred = flags[t] & SGM_FLAG_PRED;
    const bool gv = pred && gt[t] >= 0.f;
    const double e = fmin(fmax(dz_full[t] - dhat[t], -16.0), 16.0);
    const double m = fmin(fmax(dz_full[t] - (double)gt[t], -16.0), 16.0);
    *(float4 *)(tgt + (size_t)t * 4) =
        make_float4(pred ? (float)e : 0.f, gv ? (float)m : 0.f, pred ? 1.f : 0.f, gv ? 1.f : 0.f);
}

hipError_t launch_targets(const Geometry &g, const DevBuffers &b, const double *dz_full, const float *gt, float *tgt,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_targets, dim3((g.N + 255) / 256), dim3(256), 0, s, g.N, b.flags, b.dhat, dz_full, gt, tgt);
    return hipGetLastError();
}

}  // namespace sgmk
