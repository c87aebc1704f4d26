// C ABI of the gfx950 library: context management, argument checks and the
// per-frame launch sequences.  Every entry point is declared, with its
// contract, in include/sgm.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>

#include "sgm_internal.h"

using namespace sgmk;

// event pool for sgm_set_profiling: kProfFrames frames x stages x {start, end}
constexpr int kProfFrames = 256;

struct Profiler {
    bool on = false;
    hipEvent_t ev[kProfFrames][SGM_PROF_COUNT][2];
    bool created = false;
    int pending = 0;                 // frames recorded but not yet read
    double ms[SGM_PROF_COUNT];
    int64_t frames = 0;
};

struct sgm_context {
    sgm_params prm;
    Geometry g;
    DevBuffers b;
    bool started;
    bool debug;
    bool sparse_layout;         // the last frame's second pass kept the first pass's offsets (gate re-run)
    int device;
    Profiler prof;
    hipStream_t side;           // census and horizontal aggregation run here, forked from the caller's stream
    hipEvent_t fork0, cen;      // frame start on the caller's stream, census done on the side stream
    hipEvent_t fork, join;
    bool has_model;             // learned mode: sgm_set_window_model was called
};

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(SGM_EHIP, "%s: %s", what, hipGetErrorString(e));
}

const int8_t kPathDx[8] = {+1, -1, 0, 0, +1, -1, -1, +1};
const int8_t kPathDy[8] = {0, 0, +1, -1, +1, -1, +1, -1};

int validate(const sgm_params *p)
{
    if (!p)
        return fail(SGM_EINVAL, "params is NULL");
    if (p->width < 16 || p->height < 16 || p->width > 4096 || (int64_t)p->width * p->height > (1 << 24))
        return fail(SGM_EINVAL, "image size %dx%d outside 16..4096 wide, >= 16 tall, <= 2^24 pixels", p->width,
                    p->height);
    if (p->max_disp < 2 || p->max_disp > kMaxDisp)
        return fail(SGM_EINVAL, "max_disp %d outside [2, %d]", p->max_disp, kMaxDisp);
    // ragged offsets and cell counts are 32-bit
    if ((int64_t)p->width * p->height * p->max_disp > (int64_t)UINT32_MAX)
        return fail(SGM_EINVAL, "width*height*max_disp = %lld cells exceeds 2^32 - 1",
                    (long long)p->width * p->height * p->max_disp);
    if (p->census_w < 1 || p->census_h < 1 || !(p->census_w & 1) || !(p->census_h & 1) || p->census_w > 15 ||
        p->census_h > 15 || p->census_w * p->census_h - 1 > 64)
        return fail(SGM_EINVAL, "census window %dx%d must be odd, <= 15 and hold <= 64 bits", p->census_w,
                    p->census_h);
    int nbits = p->census_w * p->census_h - 1;
    if (p->p1 < 0 || p->p2 < p->p1)
        return fail(SGM_EINVAL, "penalties must satisfy 0 <= P1 <= P2 (got %d, %d)", p->p1, p->p2);
    if (nbits + p->p2 + p->p1 > 255)
        return fail(SGM_EINVAL, "census bits + P2 + P1 = %d exceeds the 8-bit path loss", nbits + p->p2 + p->p1);
    if ((p->path_mask & 0xFFu) == 0 || (p->path_mask & ~0xFFu))
        return fail(SGM_EINVAL, "path_mask 0x%x must select 1..8 of the paths 0..7", p->path_mask);
    if (!(p->k_sigma > 0) || !(p->q >= 0) || !(p->r > 0) || !(p->chi2_gate > 0) || !(p->disc_thresh >= 0))
        return fail(SGM_EINVAL, "need k_sigma > 0, q >= 0, r > 0, chi2_gate > 0, disc_thresh >= 0");
    if (!(p->f > 0) || !(p->baseline > 0) || !isfinite(p->cx) || !isfinite(p->cy))
        return fail(SGM_EINVAL, "need f > 0, baseline > 0 and a finite principal point");
    if (p->window_mode != SGM_WIN_KSIGMA && p->window_mode != SGM_WIN_LEARNED)
        return fail(SGM_EINVAL, "window_mode %d is neither SGM_WIN_KSIGMA nor SGM_WIN_LEARNED", p->window_mode);
    if (p->gate_rerun != 0 && p->gate_rerun != 1)
        return fail(SGM_EINVAL, "gate_rerun must be 0 or 1 (got %d)", p->gate_rerun);
    if (!(p->r_curv >= 0) || !isfinite(p->r_curv))
        return fail(SGM_EINVAL, "r_curv must be finite and >= 0");
    if (p->r_curv > 0 && p->window_mode == SGM_WIN_LEARNED)
        return fail(SGM_EINVAL, "r_curv > 0 needs SGM_WIN_KSIGMA windows (the learned window predicts r)");
    return SGM_OK;
}

template <class T>
hipError_t dalloc(T **ptr, size_t count)
{
    return hipMalloc((void **)ptr, count * sizeof(T) + 256);
}

void free_buffers(DevBuffers &b)
{
    void *all[] = {b.cen_l,  b.cen_r, b.win,    b.off,   b.scan_part, b.cost,  b.lr,    b.sum,     b.d,
                   b.p,      b.sflags, b.mask,  b.dhat,  b.pm,        b.flags, b.dstar, b.dz,      b.zkey,
                   b.zidx,   b.tgt,   b.dprime, b.pprime, b.has,      b.rw,    b.dw,    b.pw,      b.status,
                   b.rerun,  b.moved, b.touched, b.woff,
                   b.hflag,  b.nu,    b.nu_w,   b.feat,  b.act_a,     b.act_b, b.cnn_out, b.hw,    b.rpix,  b.kappa,
                   b.theta,  b.frag};
    for (void *p : all)
        if (p)
            (void)hipFree(p);
    memset(&b, 0, sizeof(b));
}

hipStream_t as_stream(void *s) { return (hipStream_t)s; }

int check_ctx(sgm_context *ctx)
{
    if (!ctx)
        return fail(SGM_EINVAL, "context is NULL");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != ctx->device)
        return fail(SGM_EINVAL, "context was created on device %d but device %d is current", ctx->device, dev);
    return SGM_OK;
}

int check_images(sgm_context *ctx, const uint8_t *l, const uint8_t *r, int32_t pitch)
{
    if (!l || !r)
        return fail(SGM_EINVAL, "image pointer is NULL");
    if (pitch < ctx->g.W)
        return fail(SGM_EINVAL, "pitch %d < width %d", pitch, ctx->g.W);
    return SGM_OK;
}

CorrectConst correct_const(const sgm_params &p)
{
    CorrectConst c;
    c.r = p.r;
    c.gate = p.chi2_gate;
    c.k_sigma = p.k_sigma;
    c.disc = p.disc_thresh;
    c.curv = p.r_curv;
    return c;
}

// fold the recorded frames into the totals (waits for their end events)
hipError_t prof_flush(Profiler &pf)
{
    for (int f = 0; f < pf.pending; f++) {
        for (int st = 0; st < SGM_PROF_COUNT; st++) {
            hipError_t e = hipEventSynchronize(pf.ev[f][st][1]);
            if (e != hipSuccess)
                return e;
            float t = 0.f;
            if (hipEventElapsedTime(&t, pf.ev[f][st][0], pf.ev[f][st][1]) == hipSuccess)
                pf.ms[st] += t;
        }
        pf.frames++;
    }
    pf.pending = 0;
    return hipSuccess;
}

Profiler g_noprof;   // never switched on: marks through it record nothing

// mark the start / end of a stage of the current frame (no-op unless on)
struct StageMark {
    Profiler &pf;
    hipStream_t s;
    StageMark(Profiler &p, hipStream_t st) : pf(p), s(st) {}
    void begin(int st) { if (pf.on) (void)hipEventRecord(pf.ev[pf.pending][st][0], s); }
    void end(int st) { if (pf.on) (void)hipEventRecord(pf.ev[pf.pending][st][1], s); }
};

// make every stage of a frame that skips it (full frames have no
// prediction) record an empty interval
void prof_begin_frame(Profiler &pf, hipStream_t s)
{
    if (!pf.on)
        return;
    if (pf.pending == kProfFrames)
        (void)prof_flush(pf);
    for (int st = 0; st < SGM_PROF_COUNT; st++) {
        (void)hipEventRecord(pf.ev[pf.pending][st][0], s);
        (void)hipEventRecord(pf.ev[pf.pending][st][1], s);
    }
}

void prof_end_frame(Profiler &pf)
{
    if (pf.on)
        pf.pending++;
}

// Census of the frame's images on the side stream, concurrently with the
// prediction (and the window network) on the caller's stream.
int start_census(sgm_context *ctx, const uint8_t *l, const uint8_t *r, int32_t pitch, hipStream_t s)
{
    hipError_t e = hipEventRecord(ctx->fork0, s);
    if (e == hipSuccess)
        e = hipStreamWaitEvent(ctx->side, ctx->fork0, 0);
    if (e != hipSuccess)
        return hip_fail(e, "stream fork");
    StageMark mk(ctx->prof, ctx->side);
    mk.begin(SGM_PROF_CENSUS);
    e = launch_census(ctx->g, l, r, pitch, ctx->b.cen_l, ctx->b.cen_r, ctx->side);
    mk.end(SGM_PROF_CENSUS);
    if (e == hipSuccess)
        e = hipEventRecord(ctx->cen, ctx->side);
    return e == hipSuccess ? SGM_OK : hip_fail(e, "census launch");
}

// cost (debug), aggregation, WTA (+ filter update in modes 0 and 1) on the
// census start_census launched for this frame
// skip: a gate re-run pass, whose launches do nothing when *skip == 0
int run_matcher(sgm_context *ctx, int mode, hipStream_t s, bool marks = true, const uint32_t *skip = nullptr)
{
    const Geometry &g = ctx->g;
    DevBuffers &b = ctx->b;
    // stages of a second matching pass are timed as a whole by the caller
    StageMark mk(marks ? ctx->prof : g_noprof, s);
    hipError_t e = hipStreamWaitEvent(s, ctx->cen, 0);
    if (e != hipSuccess)
        return hip_fail(e, "census wait");
    if (ctx->debug) {
        // the matching cost is computed inside the aggregation; the stand-alone
        // cost kernel only materialises it for inspection
        mk.begin(SGM_PROF_COST);
        e = launch_cost(g, b, s);
        mk.end(SGM_PROF_COST);
        if (e != hipSuccess)
            return hip_fail(e, "cost launch");
    }
    // horizontal paths on the side stream, concurrently with the others
    const bool fork = count_horizontal_paths(g) > 0;
    if (fork) {
        e = hipEventRecord(ctx->fork, s);
        if (e == hipSuccess)
            e = hipStreamWaitEvent(ctx->side, ctx->fork, 0);
        if (e != hipSuccess)
            return hip_fail(e, "stream fork");
        StageMark mh(marks ? ctx->prof : g_noprof, ctx->side);
        mh.begin(SGM_PROF_AGG_H);
        e = launch_agg_h(g, b, mode == 0, ctx->side, skip);
        mh.end(SGM_PROF_AGG_H);
        if (e != hipSuccess)
            return hip_fail(e, "horizontal aggregation launch");
    }
    mk.begin(SGM_PROF_AGG_V);
    e = launch_agg_v(g, b, mode == 0, s, skip);
    mk.end(SGM_PROF_AGG_V);
    if (e != hipSuccess)
        return hip_fail(e, "aggregation launch");
    if (fork) {
        e = hipEventRecord(ctx->join, ctx->side);
        if (e == hipSuccess)
            e = hipStreamWaitEvent(s, ctx->join, 0);
        if (e != hipSuccess)
            return hip_fail(e, "stream join");
    }
    mk.begin(SGM_PROF_WTA);
    // per-pixel measurement variance: the learned window's (read) or the cost curvature's (written)
    const float *rpix = (mode == 1 && ctx->prm.window_mode == SGM_WIN_LEARNED) ? b.rpix : nullptr;
    e = launch_wta_correct(g, b, correct_const(ctx->prm), mode, ctx->debug, rpix, s, skip);
    mk.end(SGM_PROF_WTA);
    if (e != hipSuccess)
        return hip_fail(e, "wta launch");
    return SGM_OK;
}

// one steady-state frame; the ego-motion comes from the host (by value in
// the launch) or, when Tdev is not NULL, from device memory
int reduced_frame_impl(sgm_context *ctx, const uint8_t *left, const uint8_t *right, int32_t pitch,
                       const double *Thost, const double *Tdev, hipStream_t s)
{
    const sgm_params &p = ctx->prm;
    WarpConst wc;
    for (int i = 0; i < 12; i++)
        wc.T[i] = Thost ? Thost[i] : 0.0;
    wc.f = p.f;
    wc.cx = p.cx;
    wc.cy = p.cy;
    wc.B = p.baseline;
    wc.fB = p.f * p.baseline;
    wc.zmin = 1e-9 * wc.fB;
    wc.q = p.q;
    const bool learned = p.window_mode == SGM_WIN_LEARNED;
    if (learned && !ctx->has_model)
        return fail(SGM_ESTATE, "learned-window context has no model (sgm_set_window_model)");
    ctx->sparse_layout = false;
    prof_begin_frame(ctx->prof, s);
    int rc0 = start_census(ctx, left, right, pitch, s);
    if (rc0)
        return rc0;
    StageMark mk(ctx->prof, s);
    mk.begin(SGM_PROF_PREDICT);
    hipError_t e = launch_predict_core(ctx->g, ctx->b, wc, Tdev, correct_const(p), s);
    mk.end(SGM_PROF_PREDICT);
    if (e != hipSuccess)
        return hip_fail(e, "prediction launch");
    if (learned) {
        // network input -> network -> half-widths, variances and windows
        const Geometry &g = ctx->g;
        DevBuffers &b = ctx->b;
        mk.begin(SGM_PROF_CNN);
        e = cnn_forward_frame(g, b, left, pitch, (float)p.k_sigma, s);
        mk.end(SGM_PROF_CNN);
        if (e != hipSuccess)
            return hip_fail(e, "window network launch");
    }
    e = launch_scan(ctx->g, ctx->b, s);
    if (e != hipSuccess)
        return hip_fail(e, "offset scan launch");
    int rc = run_matcher(ctx, 1, s);
    if (rc)
        return rc;
    if (p.gate_rerun) {
        // pixels that failed the innovation test search the full range in a
        // second matching pass and restart from its measurement; with no such
        // pixel the pass would reproduce the first one, and its launches read
        // the device-side count and return at once
        const Geometry &g = ctx->g;
        DevBuffers &b = ctx->b;
        mk.begin(SGM_PROF_RERUN);
        // debug contexts match every pixel again, so that the stage read-backs
        // show the second pass's plain ragged layout; the others take the
        // sparse pass, or the dense one when the full-range blocks do not fit
        const bool sparse = !ctx->debug;
        // the dense route is launched where it can be taken; its launches
        // read a skip word and return at once when the sparse route ran
        const bool dense = !sparse || g.rr_dense || !g.rr_room;
        const uint32_t *dense_skip = b.rerun + (sparse ? RR_SKIP_DENSE : RR_NW);
        e = launch_gate_widen(g, b, sparse, s);
        if (e == hipSuccess && sparse)
            e = launch_rerun_walk(g, b, s);
        if (e == hipSuccess && sparse) {
            const float *rpix = p.window_mode == SGM_WIN_LEARNED ? b.rpix : nullptr;
            e = launch_wta_correct(g, b, correct_const(p), 1, false, rpix, s, b.rerun + RR_SKIP_SPARSE, true);
        }
        if (e == hipSuccess && dense)
            e = launch_scan(g, b, s, dense_skip);
        if (e != hipSuccess)
            return hip_fail(e, "gate re-run launch");
        if (dense)
            rc = run_matcher(ctx, 1, s, false, dense_skip);
        mk.end(SGM_PROF_RERUN);
        if (rc)
            return rc;
        ctx->sparse_layout = sparse && !g.rr_dense;
    }
    prof_end_frame(ctx->prof);
    return SGM_OK;
}

int full_frame_impl(sgm_context *ctx, const uint8_t *left, const uint8_t *right, int32_t pitch, hipStream_t s)
{
    if (ctx->prm.window_mode == SGM_WIN_LEARNED && !ctx->has_model)
        return fail(SGM_ESTATE, "learned-window context has no model (sgm_set_window_model)");
    ctx->sparse_layout = false;
    prof_begin_frame(ctx->prof, s);
    int rc = start_census(ctx, left, right, pitch, s);
    if (rc)
        return rc;
    hipError_t e = launch_full_windows(ctx->g, ctx->b, s);
    if (e != hipSuccess)
        return hip_fail(e, "window launch");
    rc = run_matcher(ctx, 0, s);
    if (rc)
        return rc;
    prof_end_frame(ctx->prof);
    ctx->started = true;
    return SGM_OK;
}

}  // namespace

extern "C" {

const char *sgm_last_error(void) { return g_err; }

int sgm_default_params(sgm_params *out, int32_t width, int32_t height, int32_t max_disp)
{
    if (!out)
        return fail(SGM_EINVAL, "out is NULL");
    memset(out, 0, sizeof(*out));
    out->width = width;
    out->height = height;
    out->max_disp = max_disp;
    out->census_w = 9;
    out->census_h = 7;
    out->path_mask = 0xFF;
    out->p1 = 7;
    out->p2 = 86;
    out->k_sigma = 3.0;
    out->q = 0.5;
    out->r = 1.0;
    out->chi2_gate = 6.634896601021214;
    out->disc_thresh = 2.0;
    out->f = 0.58 * width;
    out->cx = (width - 1) / 2.0;
    out->cy = (height - 1) / 2.0;
    out->baseline = 0.54;
    return SGM_OK;
}

int sgm_paper_params(sgm_params *out, int32_t width, int32_t height, int32_t max_disp)
{
    int rc = sgm_default_params(out, width, height, max_disp);
    if (rc)
        return rc;
    out->census_w = 5;
    out->census_h = 5;
    out->p1 = 6;
    out->p2 = 65;
    return SGM_OK;
}

int sgm_create(const sgm_params *prm, sgm_context **out)
{
    if (!out)
        return fail(SGM_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(prm);
    if (rc)
        return rc;
    sgm_context *ctx = new (std::nothrow) sgm_context();
    if (!ctx)
        return fail(SGM_ENOMEM, "host allocation failed");
    ctx->prm = *prm;
    if (hipGetDevice(&ctx->device) != hipSuccess) {
        delete ctx;
        return fail(SGM_EHIP, "no HIP device");
    }
    Geometry &g = ctx->g;
    g.W = prm->width;
    g.H = prm->height;
    g.D = prm->max_disp;
    g.N = g.W * g.H;
    g.lr_stride = (((size_t)g.N * g.D) + 255) & ~(size_t)255;
    // gate re-run contexts: room behind the first pass's cells for a
    // full-range block of every pixel, so that the sparse second pass always
    // fits (as long as offsets stay below 2^32)
    g.rr_room = prm->gate_rerun && 2 * (size_t)g.N * g.D + 256 < ((size_t)1 << 32);
    if (g.rr_room)
        g.lr_stride = ((2 * (size_t)g.N * g.D) + 255) & ~(size_t)255;
    g.hseg = 72;
    g.halt = false;
    g.rr_dense = false;
    g.cw = prm->census_w;
    g.ch = prm->census_h;
    g.nbits = g.cw * g.ch - 1;
    g.p1 = prm->p1;
    g.p2 = prm->p2;
    g.npaths = 0;
    for (int k = 0; k < 8; k++)
        if (prm->path_mask & (1u << k)) {
            g.rx[g.npaths] = kPathDx[k];
            g.ry[g.npaths] = kPathDy[k];
            g.npaths++;
        }
    const size_t N = g.N, cells = N * (size_t)g.D;
    DevBuffers &b = ctx->b;
    memset(&b, 0, sizeof(b));
    hipError_t e = hipSuccess;
    auto A = [&](hipError_t r) {
        if (e == hipSuccess)
            e = r;
    };
    A(dalloc(&b.cen_l, N));
    A(dalloc(&b.cen_r, N));
    A(dalloc(&b.win, N));
    A(dalloc(&b.off, N + 1));
    A(dalloc(&b.scan_part, 4200));
    A(dalloc(&b.cost, cells));
    A(dalloc(&b.lr, g.lr_stride * g.npaths));
    A(dalloc(&b.sum, cells));
    A(dalloc(&b.d, N));
    A(dalloc(&b.p, N));
    A(dalloc(&b.sflags, N));
    A(dalloc(&b.mask, N));
    A(dalloc(&b.dhat, N));
    A(dalloc(&b.pm, N));
    A(dalloc(&b.flags, N));
    A(dalloc(&b.dstar, N));
    A(dalloc(&b.dz, N));
    A(dalloc(&b.rerun, RR_WORDS + 3 * (size_t)gate_parts(g)));
    A(dalloc(&b.moved, N));
    A(dalloc(&b.touched, N));
    A(dalloc(&b.woff, N));
    A(dalloc(&b.zkey, N));
    A(dalloc(&b.zidx, N));
    A(dalloc(&b.tgt, N));
    A(dalloc(&b.dprime, N));
    A(dalloc(&b.pprime, N));
    A(dalloc(&b.has, N));
    A(dalloc(&b.rw, N));
    A(dalloc(&b.dw, N));
    A(dalloc(&b.pw, N));
    A(dalloc(&b.status, 4));
    A(dalloc(&b.hflag, (size_t)2 * g.H * kHMaxSeg));
    A(dalloc(&b.nu, N));
    A(dalloc(&b.nu_w, N));
    if (prm->window_mode == SGM_WIN_LEARNED) {
        A(dalloc(&b.feat, N * 4));
        A(dalloc(&b.act_a, N * 32));
        A(dalloc(&b.act_b, N * 32));
        A(dalloc(&b.cnn_out, N * 2));
        A(dalloc(&b.hw, N));
        A(dalloc(&b.rpix, N));
        A(dalloc(&b.theta, (size_t)SGM_CNN_NPARAMS));
        A(dalloc(&b.frag, cnn_frag_count()));
    }
    if (prm->r_curv > 0) {
        A(dalloc(&b.rpix, N));
        A(dalloc(&b.kappa, N));
    }
    if (e != hipSuccess) {
        free_buffers(b);
        delete ctx;
        return fail(SGM_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
    }
    // z-buffer armed (key 0, no index); state zeroed; all synchronous
    A(hipMemset(b.zkey, 0, N * sizeof(unsigned long long)));
    A(hipMemset(b.zidx, 0xFF, N * sizeof(uint32_t)));
    A(hipMemset(b.d, 0, N * sizeof(double)));
    A(hipMemset(b.p, 0, N * sizeof(double)));
    A(hipMemset(b.sflags, 0, N));
    A(hipMemset(b.mask, 0, N));
    A(hipMemset(b.flags, 0, N));
    A(hipMemset(b.rerun, 0, RR_WORDS * sizeof(uint32_t)));
    A(hipMemset(b.dhat, 0, N * sizeof(double)));
    A(hipMemset(b.pm, 0, N * sizeof(double)));
    A(hipMemset(b.off, 0, (N + 1) * sizeof(uint32_t)));
    A(hipMemset(b.status, 0, sizeof(uint32_t)));
    A(hipMemset(b.nu, 0, N * sizeof(double)));
    A(hipMemset(b.hflag, 0, (size_t)2 * g.H * kHMaxSeg));
    A(hipMemset(b.nu_w, 0, N * sizeof(double)));
    A(hipDeviceSynchronize());
    if (e != hipSuccess) {
        free_buffers(b);
        delete ctx;
        return hip_fail(e, "initialisation");
    }
    e = hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipEventCreateWithFlags(&ctx->fork0, hipEventDisableTiming);
    if (e == hipSuccess)
        e = hipEventCreateWithFlags(&ctx->cen, hipEventDisableTiming);
    if (e == hipSuccess)
        e = hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming);
    if (e == hipSuccess)
        e = hipEventCreateWithFlags(&ctx->join, hipEventDisableTiming);
    if (e != hipSuccess) {
        for (hipEvent_t ev : {ctx->fork0, ctx->cen, ctx->fork, ctx->join})
            if (ev)
                (void)hipEventDestroy(ev);
        if (ctx->side)
            (void)hipStreamDestroy(ctx->side);
        free_buffers(b);
        delete ctx;
        return hip_fail(e, "stream/event creation");
    }
    ctx->started = false;
    ctx->debug = false;
    ctx->sparse_layout = false;
    ctx->has_model = false;
    *out = ctx;
    return SGM_OK;
}

void sgm_destroy(sgm_context *ctx)
{
    if (!ctx)
        return;
    (void)hipDeviceSynchronize();
    (void)hipEventDestroy(ctx->fork0);
    (void)hipEventDestroy(ctx->cen);
    (void)hipEventDestroy(ctx->fork);
    (void)hipEventDestroy(ctx->join);
    (void)hipStreamDestroy(ctx->side);
    if (ctx->prof.created)
        for (auto &f : ctx->prof.ev)
            for (auto &st : f)
                for (auto &ev : st)
                    (void)hipEventDestroy(ev);
    free_buffers(ctx->b);
    delete ctx;
}

int sgm_set_profiling(sgm_context *ctx, int32_t on)
{
    int rc = check_ctx(ctx);
    if (rc)
        return rc;
    Profiler &pf = ctx->prof;
    if (on && !pf.created) {
        for (auto &f : pf.ev)
            for (auto &st : f)
                for (auto &ev : st)
                    if (hipEventCreate(&ev) != hipSuccess)
                        return fail(SGM_EHIP, "event creation failed");
        pf.created = true;
    }
    if (on) {
        (void)hipDeviceSynchronize();
        pf.pending = 0;
        pf.frames = 0;
        for (double &m : pf.ms)
            m = 0.0;
    }
    pf.on = on != 0;
    return SGM_OK;
}

int sgm_read_profile(sgm_context *ctx, double *ms, int64_t *frames, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc)
        return rc;
    if (!ms || !frames)
        return fail(SGM_EINVAL, "output pointer is NULL");
    hipError_t e = hipStreamSynchronize(as_stream(stream));
    if (e == hipSuccess && ctx->prof.created)
        e = prof_flush(ctx->prof);
    if (e != hipSuccess)
        return hip_fail(e, "profile read");
    for (int i = 0; i < SGM_PROF_COUNT; i++)
        ms[i] = ctx->prof.ms[i];
    *frames = ctx->prof.frames;
    return SGM_OK;
}

int sgm_set_debug(sgm_context *ctx, int32_t on)
{
    if (!ctx)
        return fail(SGM_EINVAL, "context is NULL");
    if (on & ~(SGM_DEBUG_STAGES | SGM_DEBUG_SHORT_SEGMENTS | SGM_DEBUG_ALT_HORIZONTAL | SGM_DEBUG_DENSE_RERUN))
        return fail(SGM_EINVAL, "unknown debug bits 0x%x", on);
    ctx->debug = (on & SGM_DEBUG_STAGES) != 0;
    ctx->g.hseg = (on & SGM_DEBUG_SHORT_SEGMENTS) ? 48 : 72;
    ctx->g.halt = (on & SGM_DEBUG_ALT_HORIZONTAL) != 0;
    ctx->g.rr_dense = (on & SGM_DEBUG_DENSE_RERUN) != 0;
    return SGM_OK;
}

int sgm_full_frame(sgm_context *ctx, const uint8_t *left, const uint8_t *right, int32_t pitch, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc || (rc = check_images(ctx, left, right, pitch)))
        return rc;
    return full_frame_impl(ctx, left, right, pitch, as_stream(stream));
}

int sgm_reduced_frame(sgm_context *ctx, const uint8_t *left, const uint8_t *right, int32_t pitch,
                      const double T[16], void *stream)
{
    int rc = check_ctx(ctx);
    if (rc || (rc = check_images(ctx, left, right, pitch)))
        return rc;
    if (!T)
        return fail(SGM_EINVAL, "T_k_km1 is NULL");
    for (int i = 0; i < 16; i++)
        if (!isfinite(T[i]))
            return fail(SGM_EINVAL, "T_k_km1[%d] is not finite", i);
    if (!ctx->started)
        return fail(SGM_ESTATE, "reduced frame requested before a full frame or set_state");
    if (ctx->prm.window_mode == SGM_WIN_LEARNED && !ctx->has_model)
        return fail(SGM_ESTATE, "learned-window context has no model (sgm_set_window_model)");
    return reduced_frame_impl(ctx, left, right, pitch, T, nullptr, as_stream(stream));
}

int sgm_match_windows(sgm_context *ctx, const uint8_t *left, const uint8_t *right, int32_t pitch,
                      const int32_t *lo, const int32_t *hi, int32_t *dstar, double *dz, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc || (rc = check_images(ctx, left, right, pitch)))
        return rc;
    if (!lo || !hi || !dstar || !dz)
        return fail(SGM_EINVAL, "window or output pointer is NULL");
    hipStream_t s = as_stream(stream);
    ctx->sparse_layout = false;
    prof_begin_frame(ctx->prof, s);
    rc = start_census(ctx, left, right, pitch, s);
    if (rc)
        return rc;
    hipError_t e = launch_given_windows(ctx->g, ctx->b, lo, hi, s);
    if (e != hipSuccess)
        return hip_fail(e, "window launch");
    rc = run_matcher(ctx, 2, s);
    if (rc)
        return rc;
    prof_end_frame(ctx->prof);
    const size_t N = ctx->g.N;
    e = hipMemcpyAsync(dstar, ctx->b.dstar, N * sizeof(int32_t), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dz, ctx->b.dz, N * sizeof(double), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess)
        return hip_fail(e, "output copy");
    return SGM_OK;
}

int sgm_get_disparity(sgm_context *ctx, float *out, int32_t out_pitch, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc)
        return rc;
    if (!out || out_pitch < ctx->g.W)
        return fail(SGM_EINVAL, "bad output pointer or pitch");
    hipError_t e = launch_state_to_f32(ctx->g, ctx->b.d, out, out_pitch, as_stream(stream));
    return e == hipSuccess ? SGM_OK : hip_fail(e, "conversion launch");
}

int sgm_get_variance(sgm_context *ctx, float *out, int32_t out_pitch, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc)
        return rc;
    if (!out || out_pitch < ctx->g.W)
        return fail(SGM_EINVAL, "bad output pointer or pitch");
    hipError_t e = launch_state_to_f32(ctx->g, ctx->b.p, out, out_pitch, as_stream(stream));
    return e == hipSuccess ? SGM_OK : hip_fail(e, "conversion launch");
}

int sgm_get_disparity_median(sgm_context *ctx, float *out, int32_t out_pitch, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc)
        return rc;
    if (!out || out_pitch < ctx->g.W)
        return fail(SGM_EINVAL, "bad output pointer or pitch");
    hipError_t e = launch_median3x3(ctx->g, ctx->b.d, out, out_pitch, as_stream(stream));
    return e == hipSuccess ? SGM_OK : hip_fail(e, "median launch");
}

int sgm_get_motion_mask(sgm_context *ctx, uint8_t *out, int32_t out_pitch, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc)
        return rc;
    if (!out || out_pitch < ctx->g.W)
        return fail(SGM_EINVAL, "bad output pointer or pitch");
    hipError_t e = launch_copy_u8(ctx->g, ctx->b.mask, out, out_pitch, as_stream(stream));
    return e == hipSuccess ? SGM_OK : hip_fail(e, "copy launch");
}

int sgm_get_state(sgm_context *ctx, double *d, double *p, uint8_t *sflags, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc)
        return rc;
    if (!d || !p || !sflags)
        return fail(SGM_EINVAL, "state pointer is NULL");
    const size_t N = ctx->g.N;
    hipStream_t s = as_stream(stream);
    hipError_t e = hipMemcpyAsync(d, ctx->b.d, N * sizeof(double), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p, ctx->b.p, N * sizeof(double), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(sflags, ctx->b.sflags, N, hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? SGM_OK : hip_fail(e, "state copy");
}

int sgm_set_state(sgm_context *ctx, const double *d, const double *p, const uint8_t *sflags, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc)
        return rc;
    if (!d || !p || !sflags)
        return fail(SGM_EINVAL, "state pointer is NULL");
    hipStream_t s = as_stream(stream);
    // validate before touching the context: a rejected state leaves it as it was
    uint32_t bad = 0;
    hipError_t e = launch_check_state(ctx->g, d, p, ctx->b.status + 1, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&bad, ctx->b.status + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return hip_fail(e, "state check");
    if (bad)
        return fail(SGM_EINVAL, "%u pixels of the state have d outside [0, %d], a non-finite d or p, or p <= 0",
                    bad, ctx->g.D - 1);
    e = launch_load_state(ctx->g, ctx->b, d, p, sflags, s);
    if (e != hipSuccess)
        return hip_fail(e, "state copy");
    ctx->started = true;
    return SGM_OK;
}

int sgm_cost_cells(sgm_context *ctx, int64_t *cells, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc)
        return rc;
    if (!cells)
        return fail(SGM_EINVAL, "cells is NULL");
    uint32_t m = 0;
    hipStream_t s = as_stream(stream);
    hipError_t e = hipMemcpyAsync(&m, ctx->b.off + ctx->g.N, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return hip_fail(e, "cell count read-back");
    *cells = m;
    return SGM_OK;
}

int sgm_get_stage(sgm_context *ctx, int32_t stage, void *out, size_t bytes, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc)
        return rc;
    if (!out)
        return fail(SGM_EINVAL, "out is NULL");
    const Geometry &g = ctx->g;
    const DevBuffers &b = ctx->b;
    const size_t N = g.N;
    hipStream_t s = as_stream(stream);
    const void *src = nullptr;
    size_t need = 0;
    size_t M = 0;
    if (ctx->sparse_layout && (stage == SGM_STAGE_OFFSETS || (stage >= SGM_STAGE_PATH0 && stage < SGM_STAGE_PATH0 + 8)))
        return fail(SGM_EINVAL, "stage %d: the last frame's gate re-run kept the first pass's offsets and stored the "
                    "widened pixels' losses apart; sgm_set_debug(ctx, SGM_DEBUG_STAGES) keeps the plain layout", stage);
    if (stage == SGM_STAGE_COST || stage == SGM_STAGE_SUM ||
        (stage >= SGM_STAGE_PATH0 && stage < SGM_STAGE_PATH0 + 8)) {
        int64_t m = 0;
        rc = sgm_cost_cells(ctx, &m, stream);
        if (rc)
            return rc;
        M = (size_t)m;
    }
    switch (stage) {
    case SGM_STAGE_CENSUS_L: src = b.cen_l; need = N * 8; break;
    case SGM_STAGE_CENSUS_R: src = b.cen_r; need = N * 8; break;
    case SGM_STAGE_OFFSETS: src = b.off; need = (N + 1) * 4; break;
    case SGM_STAGE_COST:
        if (!ctx->debug)
            return fail(SGM_EINVAL, "SGM_STAGE_COST needs sgm_set_debug(ctx, 1) before the frame");
        src = b.cost; need = M; break;
    case SGM_STAGE_SUM:
        if (!ctx->debug)
            return fail(SGM_EINVAL, "SGM_STAGE_SUM needs sgm_set_debug(ctx, 1) before the frame");
        src = b.sum; need = M * 2; break;
    case SGM_STAGE_DHAT: src = b.dhat; need = N * 8; break;
    case SGM_STAGE_PM: src = b.pm; need = N * 8; break;
    case SGM_STAGE_FLAGS: src = b.flags; need = N; break;
    case SGM_STAGE_DSTAR: src = b.dstar; need = N * 4; break;
    case SGM_STAGE_DZ: src = b.dz; need = N * 8; break;
    case SGM_STAGE_STATUS: src = b.status; need = 4; break;
    case SGM_STAGE_NU: src = b.nu; need = N * 8; break;
    case SGM_STAGE_NU_W: src = b.nu_w; need = N * 8; break;
    case SGM_STAGE_FEATURES:
    case SGM_STAGE_CNN_OUT:
    case SGM_STAGE_HALFWIDTH:
    case SGM_STAGE_RPIX:
        if (ctx->prm.window_mode != SGM_WIN_LEARNED && !(stage == SGM_STAGE_RPIX && ctx->prm.r_curv > 0))
            return fail(SGM_EINVAL, "stage %d exists in learned-window contexts only", stage);
        src = stage == SGM_STAGE_FEATURES ? (const void *)b.feat
              : stage == SGM_STAGE_CNN_OUT ? (const void *)b.cnn_out
              : stage == SGM_STAGE_HALFWIDTH ? (const void *)b.hw : (const void *)b.rpix;
        need = stage == SGM_STAGE_FEATURES || stage == SGM_STAGE_CNN_OUT ? N * 8 : N * 4;
        break;
    case SGM_STAGE_RERUN:
        if (!ctx->prm.gate_rerun)
            return fail(SGM_EINVAL, "SGM_STAGE_RERUN exists in gate_rerun contexts only");
        src = b.rerun;   // RR_NW, RR_NMOVED, RR_EXTRA
        need = 3 * sizeof(uint32_t);
        break;
    case SGM_STAGE_KAPPA:
        if (!(ctx->prm.r_curv > 0))
            return fail(SGM_EINVAL, "SGM_STAGE_KAPPA exists in r_curv > 0 contexts only");
        src = b.kappa;
        need = N * 4;
        break;
    case SGM_STAGE_LO:
    case SGM_STAGE_HI: {
        if (bytes != N * 4)
            return fail(SGM_EINVAL, "stage %d needs %zu bytes, got %zu", stage, N * 4, bytes);
        hipError_t e = launch_windows_to_lohi(g, b, (int32_t *)out, stage == SGM_STAGE_HI, s);
        return e == hipSuccess ? SGM_OK : hip_fail(e, "window conversion");
    }
    default:
        if (stage >= SGM_STAGE_PATH0 && stage < SGM_STAGE_PATH0 + 8) {
            int k = stage - SGM_STAGE_PATH0, idx = -1, n = 0;
            for (int j = 0; j < 8; j++)
                if (ctx->prm.path_mask & (1u << j)) {
                    if (j == k)
                        idx = n;
                    n++;
                }
            if (idx < 0)
                return fail(SGM_EINVAL, "path %d is not enabled", k);
            src = b.lr + (size_t)idx * g.lr_stride;
            need = M;
            break;
        }
        return fail(SGM_EINVAL, "unknown stage %d", stage);
    }
    if (bytes != need)
        return fail(SGM_EINVAL, "stage %d needs %zu bytes, got %zu", stage, need, bytes);
    hipError_t e = hipMemcpyAsync(out, src, need, hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? SGM_OK : hip_fail(e, "stage copy");
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches of independent stereo streams (declared in include/sgm.h)
// ---------------------------------------------------------------------------

namespace {

constexpr int kMaxLanes = 16;

}  // namespace

struct sgm_batch {
    int n = 0;
    int device = 0;
    sgm_context **ctx = nullptr;
    const uint8_t **left = nullptr, **right = nullptr;   // default image buffers
    int32_t *pitch = nullptr;
    double *Tdev = nullptr;                 // n x 16, device: the last ego-motions
    bool have_T = false;                    // Tdev holds a steady-state step's ego-motions
    double *save_d = nullptr, *save_p = nullptr, *save_nu = nullptr;   // state save area for autotuning
    uint8_t *save_f = nullptr, *save_m = nullptr;
    size_t *save_off = nullptr;             // per-stream offsets into the save area
    int nlanes = 1;
    int order = 1;                          // 0: as given, 1: longest-processing-time first
    int hseg = 72, halt = 0;                // horizontal schedule of every stream
    hipStream_t lane[kMaxLanes];
    hipEvent_t fork, join[kMaxLanes];
    int *lane_of = nullptr, *seq = nullptr; // lane per stream, launch order
    hipStream_t cap = nullptr;              // the batch's own stream (autotuning)
};

namespace {

void batch_schedule(sgm_batch *b)
{
    // cost estimate: full-range work W*H*D; LPT: largest first onto the least
    // loaded lane; order 0 keeps the caller's order round-robin
    double load[kMaxLanes] = {0};
    for (int i = 0; i < b->n; i++)
        b->seq[i] = i;
    auto cost = [&](int i) {
        const sgm_params &p = b->ctx[i]->prm;
        return (double)p.width * p.height * p.max_disp;
    };
    if (b->order == 1) {
        for (int i = 1; i < b->n; i++)
            for (int j = i; j > 0 && cost(b->seq[j]) > cost(b->seq[j - 1]); j--) {
                int t = b->seq[j];
                b->seq[j] = b->seq[j - 1];
                b->seq[j - 1] = t;
            }
        for (int k = 0; k < b->n; k++) {
            int i = b->seq[k], best = 0;
            for (int l = 1; l < b->nlanes; l++)
                if (load[l] < load[best])
                    best = l;
            b->lane_of[i] = best;
            load[best] += cost(i);
        }
    } else {
        for (int i = 0; i < b->n; i++)
            b->lane_of[i] = i % b->nlanes;
    }
    for (int i = 0; i < b->n; i++) {
        b->ctx[i]->g.hseg = b->hseg;
        b->ctx[i]->g.halt = b->halt != 0;
    }
}

// a row of T whose homogeneous entry is 0 (no rigid motion) asks for a full frame
bool full_row(const double *T, int i) { return !T || T[16 * i + 15] == 0.0; }

// enqueue one frame of every stream on the lanes, forked from and joined back
// into `s`: full range where `T` says so (host T, or NULL = every stream),
// otherwise a steady-state frame with the ego-motion in b->Tdev; images from
// the arrays, or the default buffers where an array is NULL
int batch_enqueue(sgm_batch *b, const double *T, const uint8_t *const *l, const uint8_t *const *r,
                  const int32_t *pitch, hipStream_t s)
{
    hipError_t e = hipEventRecord(b->fork, s);
    for (int k = 0; k < b->nlanes && e == hipSuccess; k++)
        e = hipStreamWaitEvent(b->lane[k], b->fork, 0);
    if (e != hipSuccess)
        return hip_fail(e, "batch fork");
    for (int k = 0; k < b->n; k++) {
        const int i = b->seq[k];
        hipStream_t ls = b->lane[b->lane_of[i]];
        const uint8_t *li = l ? l[i] : b->left[i], *ri = r ? r[i] : b->right[i];
        const int32_t pi = pitch ? pitch[i] : b->pitch[i];
        int rc = full_row(T, i) ? full_frame_impl(b->ctx[i], li, ri, pi, ls)
                                : reduced_frame_impl(b->ctx[i], li, ri, pi, nullptr, b->Tdev + 16 * i, ls);
        if (rc) {
            char msg[sizeof(g_err)];
            snprintf(msg, sizeof(msg), "%s", g_err);
            return fail(rc, "stream %d: %s", i, msg);
        }
    }
    for (int k = 0; k < b->nlanes; k++) {
        e = hipEventRecord(b->join[k], b->lane[k]);
        if (e == hipSuccess)
            e = hipStreamWaitEvent(s, b->join[k], 0);
        if (e != hipSuccess)
            return hip_fail(e, "batch join");
    }
    return SGM_OK;
}

int batch_upload_T(sgm_batch *b, const double *T, hipStream_t s)
{
    for (int i = 0; i < b->n; i++) {
        if (full_row(T, i))
            continue;
        for (int j = 0; j < 16; j++)
            if (!isfinite(T[16 * i + j]))
                return fail(SGM_EINVAL, "T[%d] is not finite", 16 * i + j);
        if (!b->ctx[i]->started)
            return fail(SGM_ESTATE, "stream %d: steady-state frame before any full-range frame", i);
    }
    hipError_t e = hipMemcpyAsync(b->Tdev, T, sizeof(double) * 16 * b->n, hipMemcpyHostToDevice, s);
    if (e != hipSuccess)
        return hip_fail(e, "ego-motion upload");
    b->have_T = true;
    return SGM_OK;
}

int batch_state_copy(sgm_batch *b, bool save, hipStream_t s)
{
    hipError_t e = hipSuccess;
    for (int i = 0; i < b->n && e == hipSuccess; i++) {
        const size_t N = b->save_off[i + 1] - b->save_off[i], o = b->save_off[i];
        DevBuffers &c = b->ctx[i]->b;
        void *dst[5] = {b->save_d + o, b->save_p + o, b->save_f + o, b->save_m + o, b->save_nu + o};
        void *src[5] = {c.d, c.p, c.sflags, c.mask, c.nu};
        const size_t sz[5] = {N * 8, N * 8, N, N, N * 8};
        for (int k = 0; k < 5 && e == hipSuccess; k++)
            e = save ? hipMemcpyAsync(dst[k], src[k], sz[k], hipMemcpyDeviceToDevice, s)
                     : hipMemcpyAsync(src[k], dst[k], sz[k], hipMemcpyDeviceToDevice, s);
    }
    return e == hipSuccess ? SGM_OK : hip_fail(e, save ? "state save" : "state restore");
}

// Times steady-state steps (default images, the ego-motions in b->Tdev) for
// every schedule candidate, restoring every stream's state before each trial;
// keeps the fastest and restores the state at the end.  reps > 0: that many
// timed steps per candidate; reps == 0: as many as fit about budget_ms.
int batch_autotune(sgm_batch *b, int reps, int budget_ms, int32_t *chosen, hipStream_t s)
{
    int rc = batch_state_copy(b, true, s);
    if (rc)
        return rc;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess) {
        if (t0)
            (void)hipEventDestroy(t0);
        return fail(SGM_EHIP, "event creation failed");
    }
    struct Cand {
        int lanes, order, hseg, halt;
    };
    Cand cand[64];
    int nc = 0;
    const int lane_opts[] = {1, 2, 4, 8, 16};
    const int hs_opts[][2] = {{72, 0}, {48, 0}, {96, 0}, {128, 0}, {72, 1}};
    for (int oi = 0; oi < 2; oi++)
        for (int li = 0; li < 5; li++) {
            if (lane_opts[li] > b->n && lane_opts[li] != 1)
                continue;
            for (int hi = 0; hi < 5; hi++)
                cand[nc++] = Cand{lane_opts[li], oi, hs_opts[hi][0], hs_opts[hi][1]};
        }
    const Cand keep{b->nlanes, b->order, b->hseg, b->halt};
    float best = 1e30f;
    Cand bestc = keep;
    int r_each = reps;
    for (int c = 0; c < nc && !rc; c++) {
        b->nlanes = cand[c].lanes;
        b->order = cand[c].order;
        b->hseg = cand[c].hseg;
        b->halt = cand[c].halt;
        batch_schedule(b);
        const int nr = r_each > 0 ? r_each : 1;
        if ((rc = batch_state_copy(b, false, s)))
            break;
        double Tone[16] = {0};
        Tone[15] = 1.0;
        double *Tall = new (std::nothrow) double[16 * (size_t)b->n];
        if (!Tall) {
            rc = fail(SGM_ENOMEM, "host allocation failed");
            break;
        }
        for (int i = 0; i < b->n; i++)
            memcpy(Tall + 16 * i, Tone, sizeof(Tone));
        // every candidate starts from the saved state: warm-up, then the timed steps
        rc = batch_enqueue(b, Tall, nullptr, nullptr, nullptr, s);   // (the kernels read b->Tdev)
        (void)hipEventRecord(t0, s);
        for (int r = 0; r < nr && !rc; r++)
            rc = batch_enqueue(b, Tall, nullptr, nullptr, nullptr, s);
        (void)hipEventRecord(t1, s);
        delete[] Tall;
        if (rc)
            break;
        if (hipEventSynchronize(t1) != hipSuccess) {
            rc = fail(SGM_EHIP, "autotune timing failed");
            break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, t0, t1);
        ms /= (float)nr;
        if (r_each == 0) {
            // budget: the first candidate's step time sets the repetitions of all
            const double per = (double)ms * nc;
            r_each = per > 0 ? (int)fmin(fmax((double)budget_ms / per, 1.0), 20.0) : 1;
            if (r_each > 1) {
                c--;   // time the first candidate again with the budgeted repetitions
                continue;
            }
        }
        if (ms < best) {
            best = ms;
            bestc = cand[c];
        }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    b->nlanes = rc ? keep.lanes : bestc.lanes;
    b->order = rc ? keep.order : bestc.order;
    b->hseg = rc ? keep.hseg : bestc.hseg;
    b->halt = rc ? keep.halt : bestc.halt;
    batch_schedule(b);
    int rc2 = batch_state_copy(b, false, s);
    if (rc)
        return rc;
    if (rc2)
        return rc2;
    if (hipStreamSynchronize(s) != hipSuccess)
        return fail(SGM_EHIP, "autotune synchronisation failed");
    if (chosen) {
        chosen[0] = b->nlanes;
        chosen[1] = b->order;
        chosen[2] = b->hseg;
        chosen[3] = b->halt;
    }
    return SGM_OK;
}

void batch_free(sgm_batch *b)
{
    if (b->ctx)
        for (int i = 0; i < b->n; i++)
            if (b->ctx[i])
                sgm_destroy(b->ctx[i]);
    for (int l = 0; l < kMaxLanes; l++) {
        if (b->lane[l])
            (void)hipStreamDestroy(b->lane[l]);
        if (b->join[l])
            (void)hipEventDestroy(b->join[l]);
    }
    if (b->cap)
        (void)hipStreamDestroy(b->cap);
    if (b->fork)
        (void)hipEventDestroy(b->fork);
    for (void *p : {(void *)b->Tdev, (void *)b->save_d, (void *)b->save_p, (void *)b->save_f, (void *)b->save_m,
                    (void *)b->save_nu})
        if (p)
            (void)hipFree(p);
    delete[] b->ctx;
    delete[] b->left;
    delete[] b->right;
    delete[] b->pitch;
    delete[] b->lane_of;
    delete[] b->seq;
    delete[] b->save_off;
    delete b;
}

int check_batch(sgm_batch *b)
{
    if (!b)
        return fail(SGM_EINVAL, "batch is NULL");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != b->device)
        return fail(SGM_EINVAL, "batch was created on device %d but device %d is current", b->device, dev);
    return SGM_OK;
}

}  // namespace

extern "C" {

int sgm_batch_create(int32_t n, const sgm_params *params, const uint8_t *const *left,
                     const uint8_t *const *right, const int32_t *pitch, sgm_batch **out)
{
    if (!out)
        return fail(SGM_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || n > 1024 || !params || !left || !right || !pitch)
        return fail(SGM_EINVAL, "need 1 <= n <= 1024 and non-NULL params, image and pitch arrays");
    for (int i = 0; i < n; i++)
        if (!left[i] || !right[i] || pitch[i] < params[i].width)
            return fail(SGM_EINVAL, "stream %d: NULL image or pitch < width", i);
    sgm_batch *b = new (std::nothrow) sgm_batch();
    if (!b)
        return fail(SGM_ENOMEM, "host allocation failed");
    memset(b->lane, 0, sizeof(b->lane));
    memset(b->join, 0, sizeof(b->join));
    b->fork = nullptr;
    b->n = n;
    (void)hipGetDevice(&b->device);
    b->ctx = new (std::nothrow) sgm_context *[n]();
    b->left = new (std::nothrow) const uint8_t *[n];
    b->right = new (std::nothrow) const uint8_t *[n];
    b->pitch = new (std::nothrow) int32_t[n];
    b->lane_of = new (std::nothrow) int[n];
    b->seq = new (std::nothrow) int[n];
    b->save_off = new (std::nothrow) size_t[n + 1];
    if (!b->ctx || !b->left || !b->right || !b->pitch || !b->lane_of || !b->seq || !b->save_off) {
        batch_free(b);
        return fail(SGM_ENOMEM, "host allocation failed");
    }
    size_t tot = 0;
    for (int i = 0; i < n; i++) {
        b->left[i] = left[i];
        b->right[i] = right[i];
        b->pitch[i] = pitch[i];
        int rc = sgm_create(&params[i], &b->ctx[i]);
        if (rc) {
            char msg[512];
            snprintf(msg, sizeof(msg), "%s", g_err);
            batch_free(b);
            return fail(rc, "stream %d: %s", i, msg);
        }
        b->save_off[i] = tot;
        tot += (size_t)params[i].width * params[i].height;
    }
    b->save_off[n] = tot;
    hipError_t e = hipMalloc((void **)&b->Tdev, sizeof(double) * 16 * n);
    if (e == hipSuccess)
        e = hipMalloc((void **)&b->save_d, sizeof(double) * tot);
    if (e == hipSuccess)
        e = hipMalloc((void **)&b->save_p, sizeof(double) * tot);
    if (e == hipSuccess)
        e = hipMalloc((void **)&b->save_f, tot);
    if (e == hipSuccess)
        e = hipMalloc((void **)&b->save_m, tot);
    if (e == hipSuccess)
        e = hipMalloc((void **)&b->save_nu, sizeof(double) * tot);
    for (int l = 0; l < kMaxLanes && e == hipSuccess; l++) {
        e = hipStreamCreateWithFlags(&b->lane[l], hipStreamNonBlocking);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&b->join[l], hipEventDisableTiming);
    }
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    if (e != hipSuccess) {
        batch_free(b);
        return fail(SGM_ENOMEM, "batch allocation failed: %s", hipGetErrorString(e));
    }
    b->nlanes = n < 4 ? n : 4;
    b->order = 1;
    batch_schedule(b);
    *out = b;
    return SGM_OK;
}

void sgm_batch_destroy(sgm_batch *b)
{
    if (!b)
        return;
    (void)hipDeviceSynchronize();
    batch_free(b);
}

sgm_context *sgm_batch_context(sgm_batch *b, int32_t i)
{
    if (!b || i < 0 || i >= b->n) {
        fail(SGM_EINVAL, "no stream %d in the batch", i);
        return nullptr;
    }
    return b->ctx[i];
}

int sgm_batch_set_schedule(sgm_batch *b, int32_t lanes, int32_t order)
{
    if (!b || lanes < 1 || lanes > kMaxLanes || (order != 0 && order != 1))
        return fail(SGM_EINVAL, "need 1 <= lanes <= %d and order 0 or 1", kMaxLanes);
    b->nlanes = lanes;
    b->order = order;
    batch_schedule(b);
    return SGM_OK;
}

int sgm_batch_step(sgm_batch *b, const uint8_t *const *left, const uint8_t *const *right, const int32_t *pitch,
                   const double *T, void *stream)
{
    int rc = check_batch(b);
    if (rc)
        return rc;
    for (int i = 0; i < b->n; i++) {
        if ((left && !left[i]) || (right && !right[i]))
            return fail(SGM_EINVAL, "stream %d: NULL image", i);
        if (pitch && pitch[i] < b->ctx[i]->g.W)
            return fail(SGM_EINVAL, "stream %d: pitch %d < width %d", i, pitch[i], b->ctx[i]->g.W);
    }
    hipStream_t s = as_stream(stream);
    if (T && (rc = batch_upload_T(b, T, s)))
        return rc;
    return batch_enqueue(b, T, left, right, pitch, s);
}

int sgm_batch_full(sgm_batch *b, void *stream)
{
    return sgm_batch_step(b, nullptr, nullptr, nullptr, nullptr, stream);
}

int sgm_batch_step_graph(sgm_batch *b, const double *T, void *stream)
{
    (void)T;
    (void)stream;
    int rc = check_batch(b);
    if (rc)
        return rc;
    return fail(SGM_EINVAL, "captured-graph stepping is disabled: capturing a batch step (streams forked onto "
                            "lanes and side streams with events) crashed the host process inside "
                            "hipStreamEndCapture, and the cause has not been shown; use sgm_batch_step");
}

int sgm_batch_autotune(sgm_batch *b, const double *T, int32_t reps, int32_t *chosen, void *stream)
{
    int rc = check_batch(b);
    if (rc)
        return rc;
    if (!T || reps < 1)
        return fail(SGM_EINVAL, "T is NULL or reps < 1");
    for (int i = 0; i < b->n; i++)
        if (full_row(T, i))
            return fail(SGM_EINVAL, "stream %d: autotuning times steady-state frames", i);
    hipStream_t s = as_stream(stream);
    if ((rc = batch_upload_T(b, T, s)))
        return rc;
    return batch_autotune(b, reps, 0, chosen, s);
}

int sgm_autotune(sgm_batch *b, int32_t budget_ms)
{
    int rc = check_batch(b);
    if (rc)
        return rc;
    if (budget_ms < 1)
        return fail(SGM_EINVAL, "budget_ms must be >= 1");
    if (!b->have_T)
        return fail(SGM_ESTATE, "autotuning needs the ego-motions of a previous steady-state step");
    // the batch's own stream: ordered after the caller's work by the device-wide sync below
    if (hipDeviceSynchronize() != hipSuccess)
        return fail(SGM_EHIP, "synchronisation failed");
    return batch_autotune(b, 0, budget_ms, nullptr, b->cap);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// learned search window: model, network input, training targets, trainer
// ---------------------------------------------------------------------------

struct sgm_cnn {
    int maxn, H, W;
    int device;
    int nimg;            // images of the last forward
    bool have_loss;
    int step;            // Adam steps taken
    float *theta, *m, *v, *grad;
    uint64_t *frag;
    const uint16_t *x;   // input of the last forward (caller's buffer)
    uint16_t *a1, *a2, *a3, *a4;
    uint16_t *g0, *g1, *dz5;
    float *out, *cnt, *part, *lpart;
};

namespace {

void cnn_free(sgm_cnn *t)
{
    void *all[] = {t->theta, t->m, t->v, t->grad, t->frag, t->a1, t->a2, t->a3, t->a4,
                   t->g0,    t->g1, t->dz5, t->out, t->cnt, t->part, t->lpart};
    for (void *p : all)
        if (p)
            (void)hipFree(p);
}

int check_cnn(sgm_cnn *t)
{
    if (!t)
        return fail(SGM_EINVAL, "trainer is NULL");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != t->device)
        return fail(SGM_EINVAL, "trainer was created on device %d but device %d is current", t->device, dev);
    return SGM_OK;
}

}  // namespace

extern "C" {

int sgm_set_window_model(sgm_context *ctx, const float *params, int32_t n)
{
    int rc = check_ctx(ctx);
    if (rc)
        return rc;
    if (ctx->prm.window_mode != SGM_WIN_LEARNED)
        return fail(SGM_EINVAL, "context was not created with window_mode SGM_WIN_LEARNED");
    if (!params || n != SGM_CNN_NPARAMS)
        return fail(SGM_EINVAL, "need %d parameters (got %d)", SGM_CNN_NPARAMS, n);
    for (int i = 0; i < n; i++)
        if (!isfinite(params[i]))
            return fail(SGM_EINVAL, "parameter %d is not finite", i);
    hipError_t e = hipMemcpy(ctx->b.theta, params, (size_t)n * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = cnn_pack(ctx->b.theta, ctx->b.frag, nullptr);
    if (e == hipSuccess)
        e = hipDeviceSynchronize();
    if (e != hipSuccess)
        return hip_fail(e, "window model upload");
    ctx->has_model = true;
    return SGM_OK;
}

int sgm_get_features(sgm_context *ctx, const uint8_t *left, int32_t pitch, uint16_t *out, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc)
        return rc;
    if (!left || !out || pitch < ctx->g.W)
        return fail(SGM_EINVAL, "bad image, pitch or output");
    hipError_t e = launch_features(ctx->g, ctx->b, left, pitch, out, as_stream(stream));
    return e == hipSuccess ? SGM_OK : hip_fail(e, "feature launch");
}

int sgm_learned_targets(sgm_context *ctx, const double *dz_full, const float *gt, float *out, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc)
        return rc;
    if (!dz_full || !gt || !out)
        return fail(SGM_EINVAL, "NULL pointer");
    hipError_t e = launch_targets(ctx->g, ctx->b, dz_full, gt, out, as_stream(stream));
    return e == hipSuccess ? SGM_OK : hip_fail(e, "target launch");
}

int sgm_cnn_create(int32_t max_images, int32_t height, int32_t width, sgm_cnn **out)
{
    if (!out)
        return fail(SGM_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_images < 1 || height < 1 || width < 1 || (int64_t)max_images * height * width > (1ll << 28))
        return fail(SGM_EINVAL, "batch %d x %d x %d outside 1..2^28 pixels", max_images, height, width);
    sgm_cnn *t = new (std::nothrow) sgm_cnn();
    if (!t)
        return fail(SGM_ENOMEM, "host allocation failed");
    memset(t, 0, sizeof(*t));
    t->maxn = max_images;
    t->H = height;
    t->W = width;
    if (hipGetDevice(&t->device) != hipSuccess) {
        delete t;
        return fail(SGM_EHIP, "no HIP device");
    }
    const size_t P = (size_t)max_images * height * width;
    hipError_t e = hipSuccess;
    auto A = [&](hipError_t r) {
        if (e == hipSuccess)
            e = r;
    };
    A(dalloc(&t->theta, (size_t)SGM_CNN_NPARAMS));
    A(dalloc(&t->m, (size_t)SGM_CNN_NPARAMS));
    A(dalloc(&t->v, (size_t)SGM_CNN_NPARAMS));
    A(dalloc(&t->grad, (size_t)SGM_CNN_NPARAMS));
    A(dalloc(&t->frag, cnn_frag_count()));
    A(dalloc(&t->a1, P * 16));
    A(dalloc(&t->a2, P * 32));
    A(dalloc(&t->a3, P * 32));
    A(dalloc(&t->a4, P * 16));
    A(dalloc(&t->g0, P * 32));
    A(dalloc(&t->g1, P * 32));
    A(dalloc(&t->dz5, P * 4));
    A(dalloc(&t->out, P * 2));
    A(dalloc(&t->cnt, 2));
    A(dalloc(&t->part, cnn_part_floats()));
    A(dalloc(&t->lpart, cnn_loss_part_floats()));
    if (e == hipSuccess) {
        A(hipMemset(t->theta, 0, SGM_CNN_NPARAMS * sizeof(float)));
        A(hipMemset(t->m, 0, SGM_CNN_NPARAMS * sizeof(float)));
        A(hipMemset(t->v, 0, SGM_CNN_NPARAMS * sizeof(float)));
        A(hipMemset(t->grad, 0, SGM_CNN_NPARAMS * sizeof(float)));
        A(hipDeviceSynchronize());
    }
    if (e != hipSuccess) {
        cnn_free(t);
        delete t;
        return fail(SGM_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
    }
    *out = t;
    return SGM_OK;
}

void sgm_cnn_destroy(sgm_cnn *t)
{
    if (!t)
        return;
    (void)hipDeviceSynchronize();
    cnn_free(t);
    delete t;
}

int sgm_cnn_set_params(sgm_cnn *t, const float *params, int32_t n)
{
    int rc = check_cnn(t);
    if (rc)
        return rc;
    if (!params || n != SGM_CNN_NPARAMS)
        return fail(SGM_EINVAL, "need %d parameters (got %d)", SGM_CNN_NPARAMS, n);
    hipError_t e = hipMemcpy(t->theta, params, (size_t)n * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemset(t->m, 0, (size_t)n * sizeof(float));
    if (e == hipSuccess)
        e = hipMemset(t->v, 0, (size_t)n * sizeof(float));
    if (e == hipSuccess)
        e = cnn_pack(t->theta, t->frag, nullptr);
    if (e == hipSuccess)
        e = hipDeviceSynchronize();
    if (e != hipSuccess)
        return hip_fail(e, "parameter upload");
    t->step = 0;
    return SGM_OK;
}

int sgm_cnn_get_params(sgm_cnn *t, float *params, int32_t n)
{
    int rc = check_cnn(t);
    if (rc)
        return rc;
    if (!params || n != SGM_CNN_NPARAMS)
        return fail(SGM_EINVAL, "need room for %d parameters (got %d)", SGM_CNN_NPARAMS, n);
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess)
        e = hipMemcpy(params, t->theta, (size_t)n * sizeof(float), hipMemcpyDeviceToHost);
    return e == hipSuccess ? SGM_OK : hip_fail(e, "parameter read-back");
}

int sgm_cnn_forward(sgm_cnn *t, const uint16_t *x, int32_t nimg, float *out, void *stream)
{
    int rc = check_cnn(t);
    if (rc)
        return rc;
    if (!x || nimg < 1 || nimg > t->maxn)
        return fail(SGM_EINVAL, "need an input and 1 <= nimg <= %d (got %d)", t->maxn, nimg);
    hipStream_t s = as_stream(stream);
    hipError_t e = cnn_forward(t->theta, t->frag, x, nimg, t->H, t->W, t->a1, t->a2, t->a3, t->a4, t->out, s);
    const size_t P = (size_t)nimg * t->H * t->W;
    if (e == hipSuccess && out)
        e = hipMemcpyAsync(out, t->out, P * 2 * sizeof(float), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess)
        return hip_fail(e, "network forward");
    t->x = x;
    t->nimg = nimg;
    t->have_loss = false;
    return SGM_OK;
}

int sgm_cnn_loss(sgm_cnn *t, const float *targets, float *loss, void *stream)
{
    int rc = check_cnn(t);
    if (rc)
        return rc;
    if (!targets || !loss)
        return fail(SGM_EINVAL, "NULL targets or loss");
    if (t->nimg == 0)
        return fail(SGM_ESTATE, "loss before forward");
    const size_t P = (size_t)t->nimg * t->H * t->W;
    hipError_t e = cnn_loss(t->out, targets, P, t->cnt, t->lpart, t->dz5, loss, as_stream(stream));
    if (e != hipSuccess)
        return hip_fail(e, "loss launch");
    t->have_loss = true;
    return SGM_OK;
}

int sgm_cnn_backward(sgm_cnn *t, void *stream)
{
    int rc = check_cnn(t);
    if (rc)
        return rc;
    if (!t->have_loss)
        return fail(SGM_ESTATE, "backward before forward and loss");
    hipError_t e = cnn_backward(t->theta, t->frag, t->x, t->a1, t->a2, t->a3, t->a4, t->dz5, t->nimg, t->H, t->W,
                                t->g0, t->g1, t->part, t->grad, as_stream(stream));
    return e == hipSuccess ? SGM_OK : hip_fail(e, "network backward");
}

int sgm_cnn_get_grads(sgm_cnn *t, float *grads, int32_t n)
{
    int rc = check_cnn(t);
    if (rc)
        return rc;
    if (!grads || n != SGM_CNN_NPARAMS)
        return fail(SGM_EINVAL, "need room for %d gradients (got %d)", SGM_CNN_NPARAMS, n);
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess)
        e = hipMemcpy(grads, t->grad, (size_t)n * sizeof(float), hipMemcpyDeviceToHost);
    return e == hipSuccess ? SGM_OK : hip_fail(e, "gradient read-back");
}

int sgm_cnn_adam(sgm_cnn *t, float lr, void *stream)
{
    int rc = check_cnn(t);
    if (rc)
        return rc;
    if (!(lr > 0.f) || !isfinite(lr))
        return fail(SGM_EINVAL, "learning rate must be positive and finite");
    hipStream_t s = as_stream(stream);
    hipError_t e = cnn_adam(t->theta, t->m, t->v, t->grad, t->step + 1, lr, s);
    if (e == hipSuccess)
        e = cnn_pack(t->theta, t->frag, s);
    if (e != hipSuccess)
        return hip_fail(e, "Adam launch");
    t->step++;
    return SGM_OK;
}

int sgm_cnn_train_step(sgm_cnn *t, const uint16_t *x, const float *targets, int32_t nimg, float lr, float *loss,
                       void *stream)
{
    int rc = sgm_cnn_forward(t, x, nimg, nullptr, stream);
    if (rc == SGM_OK)
        rc = sgm_cnn_loss(t, targets, loss, stream);
    if (rc == SGM_OK)
        rc = sgm_cnn_backward(t, stream);
    if (rc == SGM_OK)
        rc = sgm_cnn_adam(t, lr, stream);
    return rc;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// moving-object detection
// ---------------------------------------------------------------------------
struct sgm_detector {
    sgm_detect_params prm;
    DetectGeom dg;
    int device;
    int64_t nwin;
    uint32_t *colp;   // column prefixes of the difference values, rows x width
    uint32_t *sat;
    uint8_t *fire;
};

namespace {

int check_det(sgm_detector *d)
{
    if (!d)
        return fail(SGM_EINVAL, "detector is NULL");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != d->device)
        return fail(SGM_EINVAL, "detector was created on device %d but device %d is current", d->device, dev);
    return SGM_OK;
}

// Validates the settings and fills the window grid; returns the window count
// or a negative error code.
int64_t detect_geometry(int32_t W, int32_t H, const sgm_detect_params *p, DetectGeom *dg)
{
    if (W < 16 || H < 16 || W > 4096 || (int64_t)W * H > (1 << 24))
        return fail(SGM_EINVAL, "image size %dx%d outside 16..4096 wide, >= 16 tall, <= 2^24 pixels", W, H);
    if (p->top < 0 || p->top >= H)
        return fail(SGM_EINVAL, "top row %d outside [0, %d)", p->top, H);
    if (p->n_sizes < 1 || p->n_sizes > SGM_DETECT_MAX_SIZES)
        return fail(SGM_EINVAL, "n_sizes %d outside 1..%d", p->n_sizes, SGM_DETECT_MAX_SIZES);
    if (p->scale < 1 || p->cap < 1 || p->thresh < 0)
        return fail(SGM_EINVAL, "need scale >= 1, cap >= 1, thresh >= 0");
    if (p->max_detections < 1 || p->max_detections > SGM_DETECT_MAX)
        return fail(SGM_EINVAL, "max_detections %d outside 1..%d", p->max_detections, SGM_DETECT_MAX);
    if (p->min_area < 0 || !(p->merge_iou >= 0.0 && p->merge_iou <= 1.0))
        return fail(SGM_EINVAL, "need min_area >= 0 and 0 <= merge_iou <= 1");
    memset(dg, 0, sizeof(*dg));
    dg->W = W;
    dg->H = H;
    dg->top = p->top;
    dg->rows = H - p->top;
    dg->nsizes = p->n_sizes;
    dg->scale = p->scale;
    dg->cap = p->cap;
    dg->thresh = p->thresh;
    dg->maxdet = p->max_detections;
    dg->min_area = p->min_area;
    dg->merge_iou = p->merge_iou;
    int64_t total = 0;
    for (int s = 0; s < p->n_sizes; s++) {
        const int w = p->sizes[s][0], h = p->sizes[s][1];
        if (w < 1 || h < 1 || w > W || h > H)
            return fail(SGM_EINVAL, "window %d x %d outside 1..%d x 1..%d", w, h, W, H);
        if ((uint64_t)w * (uint64_t)h * (uint64_t)p->cap >= (1ull << 32))
            return fail(SGM_EINVAL, "window %d x %d with cap %d can reach 2^32", w, h, p->cap);
        dg->w[s] = w;
        dg->h[s] = h;
        dg->sx[s] = w / 2 > 0 ? w / 2 : 1;
        dg->sy[s] = h / 2 > 0 ? h / 2 : 1;
        dg->nx[s] = (W - w) / dg->sx[s] + 1;
        const int ny = dg->rows >= h ? (dg->rows - h) / dg->sy[s] + 1 : 0;
        dg->base[s] = (int)total;
        total += (int64_t)dg->nx[s] * ny;
        if (total > (1 << 27))
            return fail(SGM_EINVAL, "more than 2^27 windows");
    }
    dg->base[p->n_sizes] = (int)total;
    return total;
}

}  // namespace

extern "C" {

int sgm_detect_default_params(sgm_detect_params *out, int32_t width, int32_t height)
{
    if (!out)
        return fail(SGM_EINVAL, "out is NULL");
    (void)width;
    memset(out, 0, sizeof(*out));
    out->top = height / 3;
    const int32_t sizes[5][2] = {{20, 20}, {30, 30}, {40, 40}, {50, 50}, {50, 75}};
    out->n_sizes = 5;
    memcpy(out->sizes, sizes, sizeof(sizes));
    out->scale = 16;
    out->cap = 256;
    out->thresh = 16;
    out->max_detections = SGM_DETECT_MAX;
    out->min_area = 1600;
    out->merge_iou = 0.0;
    return SGM_OK;
}

int sgm_detector_create(int32_t width, int32_t height, const sgm_detect_params *prm, sgm_detector **out)
{
    if (!out)
        return fail(SGM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!prm)
        return fail(SGM_EINVAL, "params is NULL");
    DetectGeom dg;
    int64_t nwin = detect_geometry(width, height, prm, &dg);
    if (nwin < 0)
        return (int)nwin;
    sgm_detector *d = new (std::nothrow) sgm_detector();
    if (!d)
        return fail(SGM_ENOMEM, "host allocation failed");
    d->prm = *prm;
    d->dg = dg;
    d->nwin = nwin;
    d->colp = nullptr;
    d->sat = nullptr;
    d->fire = nullptr;
    if (hipGetDevice(&d->device) != hipSuccess) {
        delete d;
        return fail(SGM_EHIP, "no HIP device");
    }
    hipError_t e = dalloc(&d->sat, (size_t)(dg.rows + 1) * (size_t)(width + 1));
    if (e == hipSuccess)
        e = dalloc(&d->colp, (size_t)dg.rows * (size_t)width);
    if (e == hipSuccess)
        e = dalloc(&d->fire, (size_t)(nwin > 0 ? nwin : 1));
    if (e != hipSuccess) {
        if (d->colp)
            (void)hipFree(d->colp);
        if (d->sat)
            (void)hipFree(d->sat);
        if (d->fire)
            (void)hipFree(d->fire);
        delete d;
        return fail(SGM_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
    }
    *out = d;
    return SGM_OK;
}

void sgm_detector_destroy(sgm_detector *det)
{
    if (!det)
        return;
    (void)hipFree(det->colp);
    (void)hipFree(det->sat);
    (void)hipFree(det->fire);
    delete det;
}

int sgm_detector_windows(sgm_detector *det, int64_t *n)
{
    if (!det || !n)
        return fail(SGM_EINVAL, "detector or output is NULL");
    *n = det->nwin;
    return SGM_OK;
}

int sgm_detect(sgm_detector *det, const double *dhat, const double *dz, const uint8_t *flags, int32_t *boxes,
               int32_t *count, void *stream)
{
    int rc = check_det(det);
    if (rc)
        return rc;
    if (!dhat || !dz || !flags || !boxes || !count)
        return fail(SGM_EINVAL, "NULL input or output pointer");
    hipError_t e = launch_detect(det->dg, dhat, dz, flags, det->colp, det->sat, det->fire, boxes, count,
                                 as_stream(stream));
    return e == hipSuccess ? SGM_OK : hip_fail(e, "detection launch");
}

int sgm_detect_frame(sgm_detector *det, sgm_context *ctx, int32_t *boxes, int32_t *count, void *stream)
{
    int rc = check_det(det);
    if (rc == SGM_OK)
        rc = check_ctx(ctx);
    if (rc)
        return rc;
    if (ctx->g.W != det->dg.W || ctx->g.H != det->dg.H)
        return fail(SGM_EINVAL, "context is %dx%d, detector %dx%d", ctx->g.W, ctx->g.H, det->dg.W, det->dg.H);
    return sgm_detect(det, ctx->b.dhat, ctx->b.dz, ctx->b.flags, boxes, count, stream);
}

int sgm_detector_stage(sgm_detector *det, int32_t stage, void *out, size_t bytes, void *stream)
{
    int rc = check_det(det);
    if (rc)
        return rc;
    const void *src = nullptr;
    size_t need = 0;
    if (stage == SGM_DSTAGE_SAT) {
        src = det->sat;
        need = (size_t)(det->dg.rows + 1) * (size_t)(det->dg.W + 1) * sizeof(uint32_t);
    } else if (stage == SGM_DSTAGE_FIRED) {
        src = det->fire;
        need = (size_t)det->nwin;
    } else {
        return fail(SGM_EINVAL, "unknown detector stage %d", stage);
    }
    if (!out || bytes < need)
        return fail(SGM_EINVAL, "stage %d needs %zu bytes", stage, need);
    if (need == 0)
        return SGM_OK;
    hipError_t e = hipMemcpyAsync(out, src, need, hipMemcpyDeviceToDevice, as_stream(stream));
    return e == hipSuccess ? SGM_OK : hip_fail(e, "stage copy");
}

}  // extern "C"

// ---------------------------------------------------------------------------
// detection without allocation: the scratch is a file-scope device array
// ---------------------------------------------------------------------------
static __device__ __align__(256) uint8_t scratch[SGM_DETECT_NOALLOC_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t *g_scratch[kMaxDevices];   // device address of `scratch` on each GPU (host-side name is not one)

// Address of the current device's copy of `scratch`, looked up once per device.
int scratch_of_current_device(uint8_t **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(SGM_EINVAL, "device %d outside 0..%d", dev, kMaxDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        g_scratch[dev] = (uint8_t *)p;
    }
    *out = g_scratch[dev];
    return SGM_OK;
}

size_t round256(size_t n) { return (n + 255) & ~(size_t)255; }

}  // namespace

extern "C" int sgm_detect_noalloc(int32_t width, int32_t height, const sgm_detect_params *prm, const double *dhat,
                                  const double *dz, const uint8_t *flags, int32_t *boxes, int32_t *count,
                                  void *stream)
{
    if (!prm)
        return fail(SGM_EINVAL, "params is NULL");
    if (!dhat || !dz || !flags || !boxes || !count)
        return fail(SGM_EINVAL, "NULL input or output pointer");
    DetectGeom dg;
    const int64_t nwin = detect_geometry(width, height, prm, &dg);
    if (nwin < 0)
        return (int)nwin;
    const size_t colp_b = round256((size_t)dg.rows * (size_t)width * sizeof(uint32_t));
    const size_t sat_b = round256((size_t)(dg.rows + 1) * (size_t)(width + 1) * sizeof(uint32_t));
    const size_t need = colp_b + sat_b + round256((size_t)(nwin > 0 ? nwin : 1));
    if (need > (size_t)SGM_DETECT_NOALLOC_BYTES)
        return fail(SGM_EINVAL, "%dx%d with top %d needs %zu bytes of scratch, more than the %u available", width,
                    height, prm->top, need, (unsigned)SGM_DETECT_NOALLOC_BYTES);
    uint8_t *base = nullptr;
    int rc = scratch_of_current_device(&base);
    if (rc)
        return rc;
    uint32_t *colp = (uint32_t *)base;
    uint32_t *sat = (uint32_t *)(base + colp_b);
    uint8_t *fire = base + colp_b + sat_b;
    hipError_t e = launch_detect(dg, dhat, dz, flags, colp, sat, fire, boxes, count, as_stream(stream));
    return e == hipSuccess ? SGM_OK : hip_fail(e, "detection launch");
}
