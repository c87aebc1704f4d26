"""Pins of the learned-window oracle (oracle/cnn.py and the learned-frame
functions of the C oracle) against library routines, closed forms, finite
differences and special cases that reduce to the plain method."""
import numpy as np
import pytest
import scipy.signal
import torch

import oracle
from oracle import cnn
from stereo_synth import make_sequence


def _rng(seed):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------- bfloat16

def test_bf16_matches_torch_on_float32_values():
    rng = _rng(1)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000),
                        rng.uniform(0, 4, 20000)]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().astype(np.uint16)
    got = cnn.bf16_bits(x.astype(np.float64))
    tiny = np.abs(x) < 2.0 ** -126
    assert np.array_equal(got[~tiny], ref[~tiny])


def test_bf16_ties_go_to_even():
    # 1 + k/128 are consecutive bfloat16 values; the midpoints round to the even one
    k = np.arange(0, 127)
    mid = 1.0 + (k + 0.5) / 128.0
    got = cnn.bf16_value(cnn.bf16_bits(mid))
    even = 1.0 + np.where(k % 2 == 0, k, k + 1) / 128.0
    assert np.array_equal(got, even)
    # just above a midpoint rounds up, just below rounds down
    assert np.array_equal(cnn.bf16_value(cnn.bf16_bits(mid + 1e-12)), 1.0 + (k + 1) / 128.0)
    assert np.array_equal(cnn.bf16_value(cnn.bf16_bits(mid - 1e-12)), 1.0 + k / 128.0)


def test_bf16_carry_into_exponent_and_zero():
    x = np.array([0.0, -0.0, 2.0 - 2.0 ** -10, 1.9999999, 2.0 ** -127, 3.0e38])
    v = cnn.bf16_value(cnn.bf16_bits(x))
    assert v[0] == 0.0 and v[1] == 0.0
    assert v[2] == 2.0 and v[3] == 2.0
    assert v[4] == 0.0
    assert np.isfinite(v[5])


# ---------------------------------------------------------------- convolution

def test_conv3x3_single_channel_is_scipy_correlate2d():
    rng = _rng(2)
    x = rng.standard_normal((1, 9, 13, 1))
    W = rng.standard_normal((1, 3, 3, 1))
    out = cnn.conv3x3(x, W, np.array([0.25]))
    ref = scipy.signal.correlate2d(x[0, :, :, 0], W[0, :, :, 0], mode="same", boundary="fill") + 0.25
    np.testing.assert_allclose(out[0, :, :, 0], ref, rtol=0, atol=1e-12)


def test_conv3x3_channels_are_sums_of_single_channel_correlations():
    rng = _rng(3)
    x = rng.standard_normal((2, 6, 7, 3))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    out = cnn.conv3x3(x, W, b)
    for n in range(2):
        for co in range(4):
            ref = b[co] + sum(scipy.signal.correlate2d(x[n, :, :, ci], W[co, :, :, ci], mode="same",
                                                       boundary="fill") for ci in range(3))
            np.testing.assert_allclose(out[n, :, :, co], ref, rtol=0, atol=1e-12)


def test_conv3x3_transpose_is_the_adjoint():
    rng = _rng(4)
    x = rng.standard_normal((2, 5, 8, 3))
    g = rng.standard_normal((2, 5, 8, 6))
    W = rng.standard_normal((6, 3, 3, 3))
    lhs = np.sum(cnn.conv3x3(x, W) * g)
    rhs = np.sum(x * cnn.conv3x3_transpose(g, W))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_conv3x3_wgrad_matches_directional_derivative():
    # the map W -> sum(g * conv(x, W, b)) is linear: its derivative along any V is exact
    rng = _rng(5)
    x = rng.standard_normal((2, 4, 5, 3))
    g = rng.standard_normal((2, 4, 5, 2))
    dW, db = cnn.conv3x3_wgrad(x, g)
    for _ in range(5):
        V = rng.standard_normal((2, 3, 3, 3))
        c = rng.standard_normal(2)
        lhs = np.sum(g * cnn.conv3x3(x, V, c))
        rhs = np.sum(dW * V) + np.sum(db * c)
        assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


# ---------------------------------------------------------------- network gradients

def _fd(f, theta, idx, h=1e-6):
    out = []
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        out.append((f(tp) - f(tm)) / (2 * h))
    return np.array(out)


def test_backward_matches_central_differences():
    rng = _rng(6)
    theta = cnn.init_params(rng)
    theta += 0.05 * rng.standard_normal(theta.shape)   # non-zero biases
    x = rng.uniform(0, 2, (1, 5, 6, 4))
    do = rng.standard_normal((1, 5, 6, 2))
    o, acts = cnn.forward(theta, x)
    g = cnn.backward(theta, acts, do)
    assert g.shape == (cnn.N_PARAMS,)
    idx = np.concatenate([rng.choice(cnn.N_PARAMS, 250, replace=False), np.arange(cnn.N_PARAMS - 20,
                                                                                 cnn.N_PARAMS)])
    fd = _fd(lambda t: float(np.sum(do * cnn.forward(t, x)[0])), theta, idx)
    err = np.abs(fd - g[idx]) / np.maximum(1e-3, np.abs(g[idx]))
    assert np.max(err) < 1e-6, np.max(err)


def test_loss_gradient_and_chain_match_central_differences():
    rng = _rng(7)
    theta = cnn.init_params(rng) * 0.5
    x = rng.uniform(0, 2, (1, 4, 5, 4))
    e = rng.standard_normal((1, 4, 5)) * 2
    m = rng.standard_normal((1, 4, 5))
    we = (rng.random((1, 4, 5)) < 0.8).astype(float)
    wm = we * (rng.random((1, 4, 5)) < 0.7)

    def total(t):
        return cnn.loss(cnn.forward(t, x)[0], e, m, we, wm)[0]

    o, acts = cnn.forward(theta, x)
    L, do = cnn.loss(o, e, m, we, wm)
    g = cnn.backward(theta, acts, do)
    idx = rng.choice(cnn.N_PARAMS, 200, replace=False)
    fd = _fd(total, theta, idx)
    err = np.abs(fd - g[idx]) / np.maximum(1e-4, np.abs(g[idx]))
    assert np.max(err) < 1e-5, np.max(err)
    # dL/do itself
    oo = rng.standard_normal((1, 4, 5, 2)) * 3
    _, d_o = cnn.loss(oo, e, m, we, wm)
    flat = oo.reshape(-1)
    for i in rng.choice(flat.size, 20, replace=False):
        op, om = flat.copy(), flat.copy()
        op[i] += 1e-6
        om[i] -= 1e-6
        fd_i = (cnn.loss(op.reshape(oo.shape), e, m, we, wm)[0] -
                cnn.loss(om.reshape(oo.shape), e, m, we, wm)[0]) / 2e-6
        assert abs(fd_i - d_o.reshape(-1)[i]) < 1e-7


def test_loss_is_minimised_at_the_log_squared_residual():
    e = np.array([[0.5, 1.0, 3.0, 7.5]])
    m = np.array([[2.0, 0.25, 1.0, 4.0]])
    o = np.stack([np.log(e ** 2), np.log(m ** 2)], axis=-1)
    w = np.ones_like(e)
    L, do = cnn.loss(o, e, m, w, w)
    assert np.max(np.abs(do)) < 1e-15
    # the minimum value: mean of (log r^2 + 1) / 2 per channel
    expect = np.mean(0.5 * (np.log(e ** 2) + 1)) + np.mean(0.5 * (np.log(m ** 2) + 1))
    assert abs(L - expect) < 1e-12
    # outside the clip range the gradient is zero
    _, do2 = cnn.loss(np.full((1, 4, 2), 20.0), e, m, w, w)
    assert np.all(do2 == 0)


def test_adam_first_steps_closed_form():
    rng = _rng(8)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    t1, m1, v1 = cnn.adam_step(th, g, m, v, 1, 1e-3)
    # bias-corrected moments of one step are g and g^2
    np.testing.assert_allclose(t1, th - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    g2 = rng.standard_normal(50)
    t2, _, _ = cnn.adam_step(t1, g2, m1, v1, 2, 1e-3)
    mh = (0.9 * 0.1 * g + 0.1 * g2) / (1 - 0.81)
    vh = (0.999 * 0.001 * g * g + 0.001 * g2 * g2) / (1 - 0.999 ** 2)
    np.testing.assert_allclose(t2, t1 - 1e-3 * mh / (np.sqrt(vh) + 1e-8), rtol=1e-13, atol=1e-15)


def test_head_closed_forms():
    o = np.array([[[np.log(4.0), np.log(2.0)], [-50.0, -50.0], [50.0, 50.0], [0.0, 0.0]]])
    hw, r = cnn.head(o, 3.0)
    np.testing.assert_allclose(hw[0], [6.0, 1.0, 3.0 * np.exp(15.0), 3.0], rtol=1e-15)
    np.testing.assert_allclose(r[0], [2.0, 1 / 16, 64.0, 1.0], rtol=1e-15)


def test_parameter_count_and_packing():
    assert cnn.N_PARAMS == 19394
    # 2 * 9 * (4*16 + 16*32 + 32*32 + 32*16 + 16*2) flops per pixel
    assert 2 * 9 * sum(ci * co for ci, co in cnn.LAYERS) == 38592
    th = np.arange(cnn.N_PARAMS, dtype=float)
    assert np.array_equal(cnn.pack(cnn.unpack(th)), th)


# ---------------------------------------------------------------- features and windows

def test_features_on_a_ramp():
    H, W = 6, 9
    yy, xx = np.mgrid[0:H, 0:W]
    I = (3 * xx + 5 * yy).astype(np.uint8)
    dhat = np.full((H, W), 20.0)
    pm = np.full((H, W), 1.5)
    flags = np.full((H, W), oracle.PRED, np.uint8)
    flags[0, 0] = oracle.FULLWIN
    nu = np.zeros((H, W))
    nu[2, 3] = -3.0
    nu[2, 4] = 100.0
    f = cnn.features(I, dhat, pm, flags, nu)
    # interior: central differences 2*3 and 2*5
    assert f[3, 4, 2] == (6 + 10) / 256
    # left border column: clamped neighbour gives a one-sided difference 3 (x) and 10 (y)
    assert f[3, 0, 2] == (3 + 10) / 256
    # corner: 3 + 5
    assert f[0, 0, 2] == (3 + 5) / 256
    assert f[3, 4, 0] == 20.0 / 64 and f[3, 4, 1] == 1.5 / 4
    assert f[0, 0, 0] == 0.0 and f[0, 0, 1] == 4.0
    assert f[2, 3, 3] == 0.75 and f[2, 4, 3] == 2.0


def _prm(W, H, D):
    return oracle.Params(width=W, height=H, max_disp=D)


def test_learned_windows_cover_the_half_width_minimally():
    rng = _rng(9)
    H, W, D = 7, 11, 64
    prm = _prm(W, H, D)
    dhat = rng.uniform(0, D - 1, (H, W))
    hw = rng.uniform(1, 40, (H, W))
    flags = np.full((H, W), oracle.PRED, np.uint8)
    flags[0, :3] |= oracle.FULLWIN
    lo0 = np.zeros((H, W), np.int32)
    hi0 = np.full((H, W), D - 1, np.int32)
    fl, lo, hi = oracle.learned_windows(prm, dhat, hw, flags, lo0, hi0)
    for y in range(H):
        for x in range(W):
            if flags[y, x] & oracle.FULLWIN or hw[y, x] >= 32:
                assert fl[y, x] & oracle.FULLWIN and lo[y, x] == 0 and hi[y, x] == D - 1
                continue
            a, b = dhat[y, x] - hw[y, x], dhat[y, x] + hw[y, x]
            assert lo[y, x] == max(0, int(np.floor(a))) and hi[y, x] == min(D - 1, int(np.ceil(b)))
            assert not fl[y, x] & oracle.FULLWIN


def test_identity_warp_carries_aux_to_the_same_pixel():
    H, W, D = 12, 20, 32
    prm = _prm(W, H, D)
    rng = _rng(10)
    d = np.full((H, W), 8.0)
    d[:, 10:] = 8.5            # no discontinuity above the 2 px threshold
    p = np.ones((H, W))
    aux = rng.standard_normal((H, W))
    out = oracle.predict_aux(prm, d, p, np.zeros((H, W), np.uint8), np.eye(4), aux)
    dhat, flags, aux_out = out[0], out[2], out[5]
    assert np.all(flags & oracle.PRED)
    assert np.array_equal(dhat, d)
    assert np.array_equal(aux_out, aux)


def test_correct_ex_with_constant_r_is_the_plain_correction():
    rng = _rng(11)
    H, W, D = 8, 10, 32
    prm = _prm(W, H, D)
    dhat = rng.uniform(2, 30, (H, W))
    pm = rng.uniform(0.2, 3, (H, W))
    flags = rng.choice([oracle.FULLWIN, oracle.PRED, oracle.PRED | oracle.FULLWIN, oracle.PRED | oracle.RESET |
                        oracle.FULLWIN], (H, W)).astype(np.uint8)
    lo = np.maximum(0, np.floor(dhat - 3)).astype(np.int32)
    hi = np.minimum(D - 1, np.ceil(dhat + 3)).astype(np.int32)
    dstar = rng.integers(lo, hi + 1).astype(np.int32)
    dz = dstar + rng.uniform(-0.5, 0.5, (H, W))
    ref = oracle.correct(prm, dhat, pm, flags, lo, hi, dstar, dz)
    got = oracle.correct_ex(prm, dhat, pm, flags, lo, hi, dstar, dz, np.full((H, W), prm.r))
    for a, b in zip(ref, got[:4]):
        assert np.array_equal(a, b)
    pred = (flags & oracle.PRED) != 0
    assert np.array_equal(got[4], np.where(pred, dz - dhat, 0.0))
    # a per-pixel r enters the gain and the gate: K = p / (p + r)
    rp = rng.uniform(0.1, 5, (H, W))
    d2, p2, mask2, _, _ = oracle.correct_ex(prm, dhat, pm, flags, lo, hi, dstar, dz, rp)
    kal = pred & ((flags & oracle.FULLWIN) == 0)
    K = pm / (pm + rp)
    np.testing.assert_allclose(d2[kal], (dhat + K * (dz - dhat))[kal], rtol=1e-14)
    np.testing.assert_allclose(p2[kal], ((1 - K) ** 2 * pm + K ** 2 * rp)[kal], rtol=1e-14)
    assert np.array_equal(mask2.astype(bool), pred & ((dz - dhat) ** 2 / (pm + rp) > prm.chi2_gate))
    # GATEFAIL: restart from the measurement, moving, RESET
    fl3 = flags | oracle.GATEFAIL | oracle.FULLWIN
    d3, p3, m3, s3, _ = oracle.correct_ex(prm, dhat, pm, fl3, lo, hi, dstar, dz, rp)
    assert np.array_equal(d3, dz) and np.all(p3 == prm.r) and np.all(m3 == 1) and np.all(s3 == oracle.RESET)


def test_learned_frame_with_k_sigma_half_widths_is_the_plain_frame():
    seq = make_sequence("tiny")
    prm = oracle.Params(width=seq.cam.width, height=seq.cam.height, max_disp=seq.max_disp, f=seq.cam.f,
                        baseline=seq.cam.baseline)
    a, b = oracle.OracleFilter(prm), oracle.OracleFilter(prm)
    a.full_frame(seq.left[0], seq.right[0])
    b.full_frame(seq.left[0], seq.right[0])
    for k in (1, 2):
        a.reduced_frame(seq.left[k], seq.right[k], seq.T[k])
        b.predict_learned(seq.left[k], seq.T[k])
        hw = prm.k_sigma * np.sqrt(b.pm)
        assert np.all(hw[(b.flags & oracle.FULLWIN) == 0] < 32)
        b.finish_learned(seq.left[k], seq.right[k], hw, np.full(hw.shape, prm.r), gate_rerun=False)
        for name in ("d", "p", "mask", "sflags", "lo", "hi", "dstar", "dz", "flags", "nu"):
            assert np.array_equal(getattr(a, name), getattr(b, name)), name


def test_gate_rerun_measures_failed_pixels_over_the_full_range():
    seq = make_sequence("tiny")
    prm = oracle.Params(width=seq.cam.width, height=seq.cam.height, max_disp=seq.max_disp, f=seq.cam.f,
                        baseline=seq.cam.baseline)
    a = oracle.OracleFilter(prm)
    a.full_frame(seq.left[0], seq.right[0])
    a.predict_learned(seq.left[1], seq.T[1])
    # windows wide enough (and r small enough) for the innovation test to fire
    hw = np.full(a.pm.shape, 8.0)
    a.finish_learned(seq.left[1], seq.right[1], hw, np.full(hw.shape, 0.25), gate_rerun=True)
    failed = a.gatefail
    assert failed.any(), "the moving box should fail the innovation test"
    # failed pixels: full range, GATEFAIL, restart from the measurement, moving
    assert np.all(a.lo[failed] == 0) and np.all(a.hi[failed] == prm.max_disp - 1)
    assert np.all(a.flags[failed] & oracle.GATEFAIL)
    assert np.array_equal(a.d[failed], a.dz[failed]) and np.all(a.mask[failed] == 1)
    # the second pass is a plain match over the final windows
    dstar, dz = oracle.match(prm, seq.left[1], seq.right[1], a.lo, a.hi)
    assert np.array_equal(dstar, a.dstar) and np.array_equal(dz, a.dz)
    # without failures nothing changes: a gate that nobody fails
    b = oracle.OracleFilter(oracle.Params(width=prm.width, height=prm.height, max_disp=prm.max_disp, f=prm.f,
                                          baseline=prm.baseline, chi2_gate=1e300))
    b.full_frame(seq.left[0], seq.right[0])
    b.predict_learned(seq.left[1], seq.T[1])
    b.finish_learned(seq.left[1], seq.right[1], hw, np.full(hw.shape, 0.25), gate_rerun=True)
    assert not b.gatefail.any() and not np.any(b.flags & oracle.GATEFAIL)


def test_targets_hand_worked():
    # training targets of a predicted frame, worked by hand:
    #   e = dz_full - dhat (measurement minus prediction), m = dz_full - gt,
    #   both clipped to +-16 px; we = prediction exists; wm = we and valid truth
    dhat = np.array([[10.0, 10.0, 5.0, 0.0, 20.0, 3.25]])
    flags = np.array([[oracle.PRED, oracle.PRED | oracle.RESET, 0, oracle.PRED, oracle.PRED,
                       oracle.PRED | oracle.FULLWIN]], np.uint8)
    dz_full = np.array([[12.5, 40.0, 7.0, 3.0, 0.0, 3.0]])
    gt = np.array([[12.0, 13.0, 7.0, -1.0, 19.0, 20.0]])
    valid = np.array([[True, True, True, False, True, True]])
    e, m, we, wm = cnn.targets(dhat, flags, dz_full, gt, valid)
    # pixel 0: +2.5 / +0.5; pixel 1: +30 -> +16 / +27 -> +16 (RESET keeps the prediction);
    # pixel 2: no prediction -> all zero even though the truth is valid;
    # pixel 3: +3 and no valid truth; pixel 4: -20 -> -16 / -19 -> -16;
    # pixel 5: -0.25 and 3 - 20 = -17 -> -16
    assert np.array_equal(e, [[2.5, 16.0, 0.0, 3.0, -16.0, -0.25]])
    assert np.array_equal(m, [[0.5, 16.0, 0.0, 0.0, -16.0, -16.0]])
    assert np.array_equal(we, [[1.0, 1.0, 0.0, 1.0, 1.0, 1.0]])
    assert np.array_equal(wm, [[1.0, 1.0, 0.0, 0.0, 1.0, 1.0]])
    # the clip is exactly +-16: 16 stays, 16.5 becomes 16
    e, m, _, _ = cnn.targets(np.array([[0.0, 0.0]]), np.array([[oracle.PRED] * 2], np.uint8),
                             np.array([[16.0, 16.5]]), np.array([[0.0, 0.5]]), np.array([[True, True]]))
    assert np.array_equal(e, [[16.0, 16.0]]) and np.array_equal(m, [[16.0, 16.0]])
