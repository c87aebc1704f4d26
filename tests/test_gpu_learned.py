"""Learned search window on the GPU vs the CPU oracle (oracle/cnn.py and
the learned-frame functions of the C oracle), through the C ABI.

Tolerances:
  * network input (bfloat16 bit patterns), innovations, training targets,
    windows, flags, masks, integer winners: bit for bit;
  * filter state of learned frames: bit for bit, given the GPU's half-widths
    and measurement variances (both sides then evaluate the same double
    precision operations);
  * network output against the fp64 oracle: relative L2 error <= 2e-2 per
    channel (bfloat16 weights and activations, fp32 accumulation; each layer
    rounds its output to 8 significant bits), and element by element within
    a bound propagated through the network from those roundings
    (_elementwise_bound);
  * parameter gradients: relative L2 error <= 5e-2 per layer tensor
    (bfloat16 activations and activation gradients);
  * head (exp in fp32): 1e-6 relative; loss: 1e-5 relative; Adam: 1e-6.
"""
import sys

import numpy as np
import pytest

import oracle as O
from oracle import cnn
import stereo_synth as synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1809_07986_amd as sgmk  # noqa: E402
from paper_1809_07986_amd import _native as NAT  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _np(t):
    return t.cpu().numpy()


def _rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _theta(seed, o0_bias=0.0, o1_bias=0.0, out_scale=0.05):
    """Random network whose outputs stay near the given biases."""
    rng = np.random.default_rng(seed)
    th = cnn.init_params(rng)
    params = cnn.unpack(th)
    for li, (W, b) in enumerate(params):
        b[:] = 0.05 * rng.standard_normal(b.shape)
    W5, b5 = params[-1]
    W5 *= out_scale
    b5[:] = [o0_bias, o1_bias]
    return cnn.pack(params).astype(np.float32)


def _gpu_reference_theta(theta32):
    """The parameters as the GPU applies them: bfloat16 weights, fp32 biases."""
    params = cnn.unpack(np.asarray(theta32, np.float64))
    return cnn.pack([(cnn.bf16_round(W), b) for W, b in params])


def _bf16_input(rng, shape):
    x = rng.uniform(0.0, 2.0, shape)
    x[..., 1] = rng.uniform(0.0, 4.0, shape[:-1])
    bits = cnn.bf16_bits(x)
    return bits, cnn.bf16_value(bits)


def _elementwise_bound(theta_ref, x):
    """Per-element bound on |GPU output - fp64 output| for input x (exact
    bfloat16 values) and parameters theta_ref (bfloat16 weights as the GPU
    applies them).

    Layer l of the GPU computes z_G = W a_G + b with fp32 accumulation of
    K = 9 ci + 1 terms (products of two bfloat16 values are exact in fp32),
    then a_G = bf16(relu(z_G)) (layers 1-4) or o = z_G (layer 5, fp32).  The
    oracle computes z = W a + b and a = relu(z) exactly.  With e the bound on
    |a_G - a| of the layer input:
        |z_G - z| <= |W| * e + g_K (|W| * (|a| + e) + |b|),  g_K = 2 K 2^-24
    (sequential fp32 summation bound, doubled for the matrix core's order),
    and relu is 1-Lipschitz while rounding to bfloat16 moves a value by at
    most 2^-8 of its magnitude, so the output bound of layers 1-4 is
        e' = dz + 2^-8 (relu(z) + dz).
    """
    params = cnn.unpack(theta_ref)
    a = np.asarray(x, np.float64)
    e = np.zeros_like(a)
    for li, (W, b) in enumerate(params):
        K = 9 * W.shape[3] + 1
        z = cnn.conv3x3(a, W, b)
        aw = np.abs(W)
        dz = cnn.conv3x3(e, aw) + 2.0 * K * 2.0 ** -24 * cnn.conv3x3(np.abs(a) + e, aw, np.abs(b))
        if li < len(params) - 1:
            a = np.maximum(z, 0.0)
            e = dz + 2.0 ** -8 * (a + dz)
        else:
            a, e = z, dz
    return a, e


def _check_elementwise(out, theta_ref, x, label):
    ref, bound = _elementwise_bound(theta_ref, x)
    err = np.abs(np.asarray(out, np.float64) - ref)
    ratio = float(np.max(err / np.maximum(bound, 1e-300)))
    _say(f"  {label}: max |d| {err.max():.3e}, max |d| / bound {ratio:.3f}")
    assert np.all(err <= bound), label
    return ref


# ---------------------------------------------------------------- network

SHAPES = [(2, 37, 70), (1, 16, 32), (1, 9, 5)]


@pytest.mark.parametrize("n,h,w", SHAPES)
def test_cnn_forward_matches_oracle(n, h, w):
    _say(f"cnn forward {n}x{h}x{w}")
    rng = np.random.default_rng(10 + h)
    theta = _theta(1 + w, out_scale=1.0)
    bits, xv = _bf16_input(rng, (n, h, w, 4))
    tr = sgmk.CnnTrainer(n, h, w)
    tr.set_params(theta)
    x = torch.from_numpy(bits.view(np.int16)).cuda()
    out = _np(tr.forward(x))
    torch.cuda.synchronize()
    ref, _ = cnn.forward(_gpu_reference_theta(theta), xv)
    for c in range(2):
        err = _rel_l2(out[..., c], ref[..., c])
        _say(f"  channel {c}: rel L2 {err:.2e}")
        assert err <= 2e-2
    assert np.all(np.isfinite(out))
    _check_elementwise(out, _gpu_reference_theta(theta), xv, f"{n}x{h}x{w}")


def test_cnn_forward_full_size_elementwise():
    # one 1242x375 image (the learned workload's frame size): every output
    # element within the propagated rounding bound, with the shipped network
    h, w = 375, 1242
    _say(f"cnn forward 1x{h}x{w}, shipped network")
    rng = np.random.default_rng(77)
    theta = sgmk.load_window_model()
    bits, xv = _bf16_input(rng, (1, h, w, 4))
    tr = sgmk.CnnTrainer(1, h, w)
    tr.set_params(theta)
    out = _np(tr.forward(torch.from_numpy(bits.view(np.int16)).cuda()))
    torch.cuda.synchronize()
    ref = _check_elementwise(out, _gpu_reference_theta(theta), xv, "1242x375")
    for c in range(2):
        assert _rel_l2(out[..., c], ref[..., c]) <= 2e-2


@pytest.mark.parametrize("n,h,w", SHAPES[:2])
def test_cnn_loss_gradient_and_adam_match_oracle(n, h, w):
    _say(f"cnn backward {n}x{h}x{w}")
    rng = np.random.default_rng(20 + h)
    theta = _theta(2 + w, out_scale=1.0)
    bits, xv = _bf16_input(rng, (n, h, w, 4))
    tgt = np.zeros((n, h, w, 4), np.float32)
    tgt[..., 0] = rng.standard_normal((n, h, w)) * 2
    tgt[..., 1] = rng.standard_normal((n, h, w))
    tgt[..., 2] = rng.random((n, h, w)) < 0.8
    tgt[..., 3] = tgt[..., 2] * (rng.random((n, h, w)) < 0.7)
    tr = sgmk.CnnTrainer(n, h, w)
    tr.set_params(theta)
    x = torch.from_numpy(bits.view(np.int16)).cuda()
    out = _np(tr.forward(x)).astype(np.float64)
    loss = float(_np(tr.loss_grad(torch.from_numpy(tgt).cuda()))[0])
    g_gpu = tr.grads().astype(np.float64)
    # loss at the GPU's own output, in fp64
    t64 = tgt.astype(np.float64)
    L_ref, do_gpu_out = cnn.loss(out, t64[..., 0], t64[..., 1], t64[..., 2], t64[..., 3])
    assert abs(loss - L_ref) <= 1e-5 * abs(L_ref), (loss, L_ref)
    # gradient against the oracle's fp64 backward of the same network
    th_ref = _gpu_reference_theta(theta)
    o_ref, acts = cnn.forward(th_ref, xv)
    _, do_ref = cnn.loss(o_ref, t64[..., 0], t64[..., 1], t64[..., 2], t64[..., 3])
    g_ref = cnn.backward(th_ref, acts, do_ref)
    off = 0
    for li, (ci, co) in enumerate(cnn.LAYERS):
        nw = 9 * ci * co
        ew = _rel_l2(g_gpu[off:off + nw], g_ref[off:off + nw])
        eb = _rel_l2(g_gpu[off + nw:off + nw + co], g_ref[off + nw:off + nw + co])
        _say(f"  layer {li + 1}: dW rel L2 {ew:.2e}, db rel L2 {eb:.2e}")
        assert ew <= 5e-2 and eb <= 5e-2
        off += nw + co
    # one Adam step from the GPU's gradient
    lr = 1e-3
    tr.adam(lr)
    th1 = tr.get_params().astype(np.float64)
    th_exp, _, _ = cnn.adam_step(theta.astype(np.float64), g_gpu, np.zeros_like(g_gpu), np.zeros_like(g_gpu), 1, lr)
    assert np.max(np.abs(th1 - th_exp)) <= 1e-6


def test_cnn_training_reduces_the_loss():
    _say("cnn training")
    rng = np.random.default_rng(5)
    n, h, w = 2, 48, 64
    bits, xv = _bf16_input(rng, (n, h, w, 4))
    # residual scale grows with input channel 2 (the image gradient)
    sd = 0.25 + 2.0 * xv[..., 2]
    tgt = np.zeros((n, h, w, 4), np.float32)
    tgt[..., 0] = rng.standard_normal((n, h, w)) * sd
    tgt[..., 1] = rng.standard_normal((n, h, w)) * 0.5
    tgt[..., 2] = 1.0
    tgt[..., 3] = 1.0
    tr = sgmk.CnnTrainer(n, h, w)
    tr.set_params(_theta(7))
    x = torch.from_numpy(bits.view(np.int16)).cuda()
    t = torch.from_numpy(tgt).cuda()
    losses = []
    for it in range(300):
        losses.append(float(_np(tr.train_step(x, t, 3e-3))[0]))
    _say(f"  loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    # the optimum is the mean over pixels of (log sd^2 + 1)/2 (+ the m term)
    opt = float(np.mean(0.5 * (np.log(sd ** 2) + 1)) + 0.5 * (np.log(0.25) + 1))
    assert losses[-1] < losses[0] - 0.3
    assert losses[-1] < opt + 0.15, (losses[-1], opt)


# ---------------------------------------------------------------- per-pixel glue

def _seq():
    return synth.make_sequence("tiny")


def _prm(seq, **kw):
    return O.Params(seq.cam.width, seq.cam.height, seq.max_disp, f=seq.cam.f, baseline=seq.cam.baseline, **kw)


def test_innovation_and_features_match_oracle():
    _say("innovation and features, tiny")
    seq = _seq()
    g = sgmk.ReducedSGM(seq.cam.width, seq.cam.height, seq.max_disp, f=seq.cam.f, baseline=seq.cam.baseline)
    o = O.OracleFilter(_prm(seq))
    g.full_frame(seq.left[0], seq.right[0])
    o.full_frame(seq.left[0], seq.right[0])
    assert np.all(_np(g.stage(NAT.STAGE_NU)) == 0)
    for k in (1, 2):
        # prediction of frame k from the oracle's state before it, carrying
        # the previous innovation with the warp winner
        dhat, pm, flags, lo, hi, nu_w = O.predict_aux(o.prm, o.d, o.p, o.sflags, seq.T[k], o.nu)
        g.reduced_frame(seq.left[k], seq.right[k], seq.T[k])
        o.reduced_frame(seq.left[k], seq.right[k], seq.T[k])
        torch.cuda.synchronize()
        assert np.array_equal(_np(g.stage(NAT.STAGE_NU)), o.nu), k
        assert np.array_equal(_np(g.stage(NAT.STAGE_NU_W)), nu_w), k
        assert np.array_equal(dhat, o.dhat) and np.array_equal(flags, o.flags), k
        f = cnn.features(seq.left[k], dhat, pm, flags, nu_w)
        got = _np(g.features(seq.left[k])).view(np.uint16)
        assert np.array_equal(got, cnn.bf16_bits(f)), k
        assert k == 1 or np.any(nu_w != 0), k   # frame 0 is a full frame: no innovation yet


def test_learned_targets_match_oracle():
    _say("learned targets, tiny")
    seq = _seq()
    kw = dict(f=seq.cam.f, baseline=seq.cam.baseline)
    g = sgmk.ReducedSGM(seq.cam.width, seq.cam.height, seq.max_disp, **kw)
    full = sgmk.ReducedSGM(seq.cam.width, seq.cam.height, seq.max_disp, **kw)
    g.full_frame(seq.left[0], seq.right[0])
    g.reduced_frame(seq.left[1], seq.right[1], seq.T[1])
    full.full_frame(seq.left[1], seq.right[1])
    dz_full = full.stage(NAT.STAGE_DZ)
    gt = np.where(seq.valid[1], seq.disp_gt[1], -1).astype(np.float32)
    tg = _np(g.learned_targets(dz_full, torch.from_numpy(gt)))
    torch.cuda.synchronize()
    dhat, flags = _np(g.stage(NAT.STAGE_DHAT)), _np(g.stage(NAT.STAGE_FLAGS))
    e, m, we, wm = cnn.targets(dhat, flags, _np(dz_full), seq.disp_gt[1], seq.valid[1])
    for c, ref in enumerate((e, m, we, wm)):
        assert np.array_equal(tg[..., c], ref.astype(np.float32)), c
    assert we.sum() > 0 and wm.sum() > 0


# ---------------------------------------------------------------- learned frames

def _learned_run(seq, theta, gate_rerun, frames=(1, 2), label="", **over):
    kw = dict(f=seq.cam.f, baseline=seq.cam.baseline)
    g = sgmk.ReducedSGM(seq.cam.width, seq.cam.height, seq.max_disp, window_mode=NAT.WIN_LEARNED,
                        gate_rerun=int(gate_rerun), **kw, **over)
    g.set_window_model(theta)
    o = O.OracleFilter(_prm(seq, **over))
    g.full_frame(seq.left[0], seq.right[0])
    o.full_frame(seq.left[0], seq.right[0])
    th_ref = _gpu_reference_theta(theta)
    stats = []
    for k in frames:
        g.reduced_frame(seq.left[k], seq.right[k], seq.T[k])
        torch.cuda.synchronize()
        f = o.predict_learned(seq.left[k], seq.T[k])
        feat = _np(g.stage(NAT.STAGE_FEATURES)).view(np.uint16)
        assert np.array_equal(feat, cnn.bf16_bits(f)), (label, k)
        out = _np(g.stage(NAT.STAGE_CNN_OUT)).astype(np.float64)
        o_ref, _ = cnn.forward(th_ref, cnn.bf16_value(feat)[None])
        for c in range(2):
            assert _rel_l2(out[..., c], o_ref[0, ..., c]) <= 2e-2, (label, k, c)
        _check_elementwise(out[None], th_ref, cnn.bf16_value(feat)[None], f"{label} frame {k}")
        hw = _np(g.stage(NAT.STAGE_HALFWIDTH)).astype(np.float64)
        rp = _np(g.stage(NAT.STAGE_RPIX)).astype(np.float64)
        hw_ref, rp_ref = cnn.head(out, o.prm.k_sigma)
        np.testing.assert_allclose(hw, hw_ref, rtol=1e-6)
        np.testing.assert_allclose(rp, rp_ref, rtol=1e-6)
        o.finish_learned(seq.left[k], seq.right[k], hw, rp, gate_rerun)
        d, p, sf = (_np(t) for t in g.get_state())
        assert np.array_equal(_np(g.stage(NAT.STAGE_FLAGS)), o.flags), (label, k)
        assert np.array_equal(_np(g.stage(NAT.STAGE_LO)), o.lo), (label, k)
        assert np.array_equal(_np(g.stage(NAT.STAGE_HI)), o.hi), (label, k)
        assert np.array_equal(_np(g.stage(NAT.STAGE_DSTAR)), o.dstar), (label, k)
        assert np.array_equal(_np(g.stage(NAT.STAGE_DZ)), o.dz), (label, k)
        assert np.array_equal(d, o.d) and np.array_equal(p, o.p) and np.array_equal(sf, o.sflags), (label, k)
        assert np.array_equal(_np(g.motion_mask()), o.mask), (label, k)
        assert np.array_equal(_np(g.stage(NAT.STAGE_NU)), o.nu), (label, k)
        stats.append(dict(cells=g.cost_cells(), gatefail=int(o.gatefail.sum()),
                          full=int(((o.flags & O.FULLWIN) != 0).sum())))
    _say(f"  {label}: {stats}")
    return stats


@pytest.mark.parametrize("gate_rerun", [False, True])
def test_learned_frames_match_oracle(gate_rerun):
    _say(f"learned frames, tiny, gate_rerun={gate_rerun}")
    seq = _seq()
    stats = _learned_run(seq, _theta(3, o0_bias=0.5, o1_bias=-1.0), gate_rerun, label=f"rerun={gate_rerun}")
    if gate_rerun:
        assert any(s["gatefail"] > 0 for s in stats), "the moving box should fail the innovation test"


def test_learned_rerun_without_failures_matches_oracle():
    # no pixel can fail the innovation test (the gate is out of reach), so the
    # second matching pass has nothing to widen: the library's re-run launches
    # return at once, the oracle re-runs, and the two must still agree
    _say("learned frames, tiny, gate_rerun=True, unreachable gate")
    seq = _seq()
    stats = _learned_run(seq, _theta(3, o0_bias=0.5, o1_bias=-1.0), True, label="rerun, no failure",
                         chi2_gate=1e300)
    assert all(s["gatefail"] == 0 for s in stats)


def test_learned_frame_full_size_matches_oracle():
    # the learned workload at full size (1242x375, D = 256) with the shipped
    # network and the gate re-run: features, network output, windows, both
    # matching passes and the filter state against the oracle
    _say("learned frame, 1242x375x256, shipped network, gate re-run")
    seq = synth.make_sequence("learned", frames=2, seed=4100)
    O.use_threads(True)     # identical to the one-thread build (tests/test_oracle_threads.py)
    try:
        stats = _learned_run(seq, sgmk.load_window_model(), True, frames=(1,), label="learned full size")
    finally:
        O.use_threads(False)
    n = seq.cam.width * seq.cam.height
    assert 0 < stats[0]["full"] < n and stats[0]["cells"] < n * seq.max_disp


def test_saturated_half_width_searches_the_full_range():
    _say("saturated half-width, tiny")
    seq = _seq()
    stats = _learned_run(seq, _theta(4, o0_bias=12.0), False, frames=(1,), label="saturated")
    assert stats[0]["full"] == seq.cam.width * seq.cam.height
    assert stats[0]["cells"] == seq.cam.width * seq.cam.height * seq.max_disp


def test_learned_context_needs_a_model():
    seq = _seq()
    g = sgmk.ReducedSGM(seq.cam.width, seq.cam.height, seq.max_disp, window_mode=NAT.WIN_LEARNED)
    with pytest.raises(sgmk.SgmError) as ei:
        g.full_frame(seq.left[0], seq.right[0])
    assert ei.value.code == NAT.SGM_ESTATE
    plain = sgmk.ReducedSGM(seq.cam.width, seq.cam.height, seq.max_disp)
    with pytest.raises(sgmk.SgmError) as ei:
        plain.set_window_model(np.zeros(NAT.CNN_NPARAMS, np.float32))
    assert ei.value.code == NAT.SGM_EINVAL
    with pytest.raises(sgmk.SgmError):
        g.set_window_model(np.zeros(10, np.float32))


# ---------------------------------------------------------------- trained network

def _run_variant(seq, theta=None, **kw):
    g = sgmk.ReducedSGM(seq.cam.width, seq.cam.height, seq.max_disp, f=seq.cam.f, baseline=seq.cam.baseline, **kw)
    if theta is not None:
        g.set_window_model(theta)
    g.full_frame(seq.left[0], seq.right[0])
    cells = bad = valid = 0.0
    for k in range(1, seq.frames):
        g.reduced_frame(seq.left[k], seq.right[k], seq.T[k])
        gt = torch.from_numpy(seq.disp_gt[k].astype(np.float32)).cuda()
        ok = torch.from_numpy(seq.valid[k]).cuda()
        cells += g.cost_cells()
        bad += float(((g.disparity() - gt).abs() > 3)[ok].sum())
        valid += float(ok.sum())
    return cells / (seq.frames - 1), bad / valid


def test_trained_window_beats_k_sigma_on_a_held_out_sequence():
    """The shipped network (trained on seeds 4000-4039) against the k-sigma
    rule on held-out seed 4104: fewer matched cells than k = 8 and fewer bad
    pixels than k = 3 and k = 8; within 1 percentage point of full range."""
    _say("trained window vs k-sigma, learned seed 4104, 16 frames")
    seq = synth.make_sequence("learned", frames=16, seed=4104)
    theta = sgmk.load_window_model()
    c3, b3 = _run_variant(seq)
    c8, b8 = _run_variant(seq, k_sigma=8.0)
    cl, bl = _run_variant(seq, theta, window_mode=NAT.WIN_LEARNED)
    g = sgmk.ReducedSGM(seq.cam.width, seq.cam.height, seq.max_disp, f=seq.cam.f, baseline=seq.cam.baseline)
    bad = valid = 0.0
    for k in range(1, seq.frames):
        g.full_frame(seq.left[k], seq.right[k])
        gt = torch.from_numpy(seq.disp_gt[k].astype(np.float32)).cuda()
        ok = torch.from_numpy(seq.valid[k]).cuda()
        bad += float(((g.disparity() - gt).abs() > 3)[ok].sum())
        valid += float(ok.sum())
    bf = bad / valid
    _say(f"  k=3: {c3 / 1e6:.2f} M cells, {b3:.4%}; k=8: {c8 / 1e6:.2f} M, {b8:.4%}; "
         f"learned: {cl / 1e6:.2f} M, {bl:.4%}; full: {seq.cam.width * seq.cam.height * seq.max_disp / 1e6:.1f} M, "
         f"{bf:.4%}")
    assert cl < c8
    assert bl < b3 and bl < b8
    assert bl <= bf + 0.01
