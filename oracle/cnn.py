"""Plain CPU oracle of the learned search window (test infrastructure only).

Double-precision numpy, written from the definitions, for the learned-window
extension of the reduced-space method:

* ``features``  -- the four per-pixel network inputs (predicted disparity,
  its variance, the left image's gradient magnitude, the previous innovation
  carried by the warp), and ``bf16_round`` / ``bf16_bits``, the
  round-to-nearest-even conversion the GPU applies to them;
* ``forward`` / ``backward`` -- five 3x3 convolutions (zero padding, ReLU
  between layers), channel widths 4 -> 16 -> 32 -> 32 -> 16 -> 2;
* ``loss`` -- Gaussian negative log-likelihood of two residuals under the
  network's two log-variances;
* ``adam_step`` -- Adam (Kingma & Ba, 2015) with bias correction;
* ``head`` -- the map from the two outputs to a half-width and a per-pixel
  measurement variance.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this module; the GPU library never does.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np

PRED, RESET, FULLWIN = 1, 2, 4

# (input channels, output channels) of the five 3x3 layers
LAYERS: Tuple[Tuple[int, int], ...] = ((4, 16), (16, 32), (32, 32), (32, 16), (16, 2))
N_PARAMS = sum(9 * ci * co + co for ci, co in LAYERS)   # 19394

# scaling of the inputs (every feature lands in about [0, 4])
F_DISP = 1.0 / 64.0          # predicted disparity per px
F_VAR_CAP, F_VAR = 16.0, 0.25   # min(p^-, 16) / 4; 4 where there is no prediction
F_GRAD = 1.0 / 256.0         # (|dI/dx| + |dI/dy|) with central differences
F_NU_CAP, F_NU = 8.0, 0.25   # min(|nu|, 8) / 4

WMAX = 32.0                  # a half-width at or above this means "full range"
O_CLAMP_LOSS = 15.0          # loss and gradient use o clipped to [-15, 15]
O_CLAMP_HEAD = 30.0
R_MIN, R_MAX = 1.0 / 16.0, 64.0
TARGET_CLAMP = 16.0          # residual targets are clipped to +-16 px


# ---------------------------------------------------------------------------
# parameters: flat vector <-> per-layer (W[co, ky, kx, ci], b[co])
# ---------------------------------------------------------------------------

def unpack(theta: np.ndarray) -> List[Tuple[np.ndarray, np.ndarray]]:
    theta = np.asarray(theta, np.float64)
    assert theta.shape == (N_PARAMS,)
    out, o = [], 0
    for ci, co in LAYERS:
        n = 9 * ci * co
        W = theta[o:o + n].reshape(co, 3, 3, ci)
        o += n
        b = theta[o:o + co]
        o += co
        out.append((W, b))
    return out


def pack(params) -> np.ndarray:
    return np.concatenate([np.concatenate([W.reshape(-1), b.reshape(-1)]) for W, b in params])


def init_params(rng: np.random.Generator) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases."""
    params = []
    for ci, co in LAYERS:
        W = rng.standard_normal((co, 3, 3, ci)) * np.sqrt(2.0 / (9 * ci))
        params.append((W, np.zeros(co)))
    return pack(params)


# ---------------------------------------------------------------------------
# bfloat16: nearest value with an 8-bit significand, ties to even
# ---------------------------------------------------------------------------

def bf16_bits(x: np.ndarray) -> np.ndarray:
    """bfloat16 bit patterns of x (float64), rounded to nearest, ties to
    even, directly from double precision.  Magnitudes below 2^-126 (the
    smallest normal bfloat16) become signed zero; x must be finite."""
    x = np.asarray(x, np.float64)
    b = x.view(np.uint64).astype(np.uint64)
    sign = (b >> np.uint64(63)) & np.uint64(1)
    mag = b & np.uint64(0x7FFFFFFFFFFFFFFF)
    # keep 7 of the 52 stored significand bits; the 45 dropped bits round
    # to nearest with ties to the even kept value (a carry may reach the
    # exponent, which is the correct result)
    keep_lsb = (mag >> np.uint64(45)) & np.uint64(1)
    r = (mag + np.uint64((1 << 44) - 1) + keep_lsb) >> np.uint64(45)
    exp = (r >> np.uint64(7)).astype(np.int64) - 1023 + 127
    man = r & np.uint64(0x7F)
    ok = exp >= 1
    bits = np.where(ok, (exp.clip(0, 255).astype(np.uint64) << np.uint64(7)) | man, np.uint64(0))
    return ((sign << np.uint64(15)) | bits).astype(np.uint16)


def bf16_value(bits: np.ndarray) -> np.ndarray:
    """float64 values of bfloat16 bit patterns."""
    b = np.asarray(bits, np.uint16).astype(np.uint32) << np.uint32(16)
    return b.view(np.float32).astype(np.float64)


def bf16_round(x: np.ndarray) -> np.ndarray:
    return bf16_value(bf16_bits(x))


# ---------------------------------------------------------------------------
# inputs
# ---------------------------------------------------------------------------

def features(left: np.ndarray, dhat: np.ndarray, pm: np.ndarray, flags: np.ndarray,
             nu_w: np.ndarray) -> np.ndarray:
    """[H, W, 4] float64 network input of a predicted frame.

    0: dhat / 64 where a prediction exists, else 0;
    1: min(p^-, 16) / 4 where a prediction exists, else 4;
    2: (|I(x+1,y) - I(x-1,y)| + |I(x,y+1) - I(x,y-1)|) / 256 on the left image,
       neighbours clamped to the image;
    3: min(|nu|, 8) / 4 with nu the previous frame's innovation of the pixel's
       warp winner (0 for filled holes and pixels without prediction).
    """
    I = np.asarray(left, np.float64)
    H, W = I.shape
    pred = (np.asarray(flags) & PRED) != 0
    xm = I[:, np.maximum(np.arange(W) - 1, 0)]
    xp = I[:, np.minimum(np.arange(W) + 1, W - 1)]
    ym = I[np.maximum(np.arange(H) - 1, 0), :]
    yp = I[np.minimum(np.arange(H) + 1, H - 1), :]
    f = np.zeros((H, W, 4))
    f[..., 0] = np.where(pred, np.asarray(dhat, np.float64) * F_DISP, 0.0)
    f[..., 1] = np.where(pred, np.minimum(np.asarray(pm, np.float64), F_VAR_CAP) * F_VAR, F_VAR_CAP * F_VAR)
    f[..., 2] = (np.abs(xp - xm) + np.abs(yp - ym)) * F_GRAD
    f[..., 3] = np.minimum(np.abs(np.asarray(nu_w, np.float64)), F_NU_CAP) * F_NU
    return f


# ---------------------------------------------------------------------------
# 3x3 convolution (cross-correlation, zero padding 1), NHWC
# ---------------------------------------------------------------------------

def conv3x3(x: np.ndarray, W: np.ndarray, b=None) -> np.ndarray:
    """out[n, y, x, co] = b[co] + sum_{ky, kx, ci} W[co, ky, kx, ci] * x[n, y+ky-1, x+kx-1, ci]."""
    N, H, Wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    out = np.zeros((N, H, Wd, W.shape[0]))
    for ky in range(3):
        for kx in range(3):
            out += xp[:, ky:ky + H, kx:kx + Wd, :] @ W[:, ky, kx, :].T
    if b is not None:
        out += b
    return out


def conv3x3_transpose(g: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Adjoint of the linear part of conv3x3 with respect to its input:
    out[n, y, x, ci] = sum_{ky, kx, co} W[co, ky, kx, ci] * g[n, y-ky+1, x-kx+1, co]."""
    N, H, Wd, _ = g.shape
    gp = np.pad(g, ((0, 0), (1, 1), (1, 1), (0, 0)))
    out = np.zeros((N, H, Wd, W.shape[3]))
    for ky in range(3):
        for kx in range(3):
            out += gp[:, 2 - ky:2 - ky + H, 2 - kx:2 - kx + Wd, :] @ W[:, ky, kx, :]
    return out


def conv3x3_wgrad(x: np.ndarray, g: np.ndarray):
    """Gradients of sum(g * conv3x3(x, W, b)) with respect to W and b."""
    N, H, Wd, ci = x.shape
    co = g.shape[3]
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dW = np.zeros((co, 3, 3, ci))
    g2 = g.reshape(-1, co)
    for ky in range(3):
        for kx in range(3):
            dW[:, ky, kx, :] = g2.T @ xp[:, ky:ky + H, kx:kx + Wd, :].reshape(-1, ci)
    return dW, g2.sum(axis=0)


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------

def forward(theta: np.ndarray, x: np.ndarray):
    """x [N, H, W, 4] -> (o [N, H, W, 2], cache).  ReLU after layers 1-4."""
    params = unpack(theta)
    acts = [np.asarray(x, np.float64)]
    a = acts[0]
    for li, (W, b) in enumerate(params):
        z = conv3x3(a, W, b)
        if li < len(params) - 1:
            a = np.maximum(z, 0.0)
            acts.append(a)
        else:
            a = z
    return a, acts


def backward(theta: np.ndarray, acts, do: np.ndarray) -> np.ndarray:
    """Gradient of sum(do * o) with respect to the flat parameter vector."""
    params = unpack(theta)
    grads = [None] * len(params)
    g = np.asarray(do, np.float64)
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        dW, db = conv3x3_wgrad(acts[li], g)
        grads[li] = (dW, db)
        if li > 0:
            # through the convolution, then through the ReLU of layer li
            # (its output acts[li] is positive exactly where it passed)
            g = conv3x3_transpose(g, W) * (acts[li] > 0.0)
    return pack(grads)


def loss(o: np.ndarray, e: np.ndarray, m: np.ndarray, we: np.ndarray, wm: np.ndarray):
    """Negative log-likelihood of the residuals e (prediction) and m
    (measurement) under zero-mean Gaussians of variance exp(o0), exp(o1):

        L = sum we * (o0 + e^2 exp(-o0)) / 2 / max(1, sum we)
          + sum wm * (o1 + m^2 exp(-o1)) / 2 / max(1, sum wm)

    with o clipped to [-15, 15] (zero gradient outside).  Returns (L, dL/do).
    """
    o = np.asarray(o, np.float64)
    ne = max(1.0, float(np.sum(we)))
    nm = max(1.0, float(np.sum(wm)))
    L = 0.0
    do = np.zeros_like(o)
    for c, (res, w, n) in enumerate(((e, we, ne), (m, wm, nm))):
        oc = np.clip(o[..., c], -O_CLAMP_LOSS, O_CLAMP_LOSS)
        inside = (o[..., c] > -O_CLAMP_LOSS) & (o[..., c] < O_CLAMP_LOSS)
        r2 = np.asarray(res, np.float64) ** 2
        ex = np.exp(-oc)
        L += float(np.sum(w * 0.5 * (oc + r2 * ex))) / n
        do[..., c] = np.where(inside, w * 0.5 * (1.0 - r2 * ex) / n, 0.0)
    return L, do


def adam_step(theta, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (step number t >= 1) -> (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def head(o: np.ndarray, k_sigma: float):
    """Network output -> (half-width, measurement variance).

    The first output is the log-variance of the prediction residual: the
    half-width is k_sigma standard deviations, at least 1 px.  The second is
    the log of the measurement variance, kept in [1/16, 64] px^2.
    """
    o = np.asarray(o, np.float64)
    hw = np.maximum(1.0, k_sigma * np.exp(0.5 * np.clip(o[..., 0], -O_CLAMP_HEAD, O_CLAMP_HEAD)))
    r = np.clip(np.exp(np.clip(o[..., 1], -O_CLAMP_HEAD, O_CLAMP_HEAD)), R_MIN, R_MAX)
    return hw, r


def targets(dhat, flags, dz_full, disp_gt, valid):
    """Training targets of one predicted frame: (e, m, we, wm).

    e = dz_full - dhat (the full-range measurement against the prediction),
    m = dz_full - d_gt (the full-range measurement against the ground truth),
    both clipped to +-16 px; we marks pixels with a prediction, wm those that
    also have valid ground truth.
    """
    pred = (np.asarray(flags) & PRED) != 0
    e = np.clip(np.asarray(dz_full, np.float64) - np.asarray(dhat, np.float64), -TARGET_CLAMP, TARGET_CLAMP)
    m = np.clip(np.asarray(dz_full, np.float64) - np.asarray(disp_gt, np.float64), -TARGET_CLAMP, TARGET_CLAMP)
    we = pred.astype(np.float64)
    wm = (pred & np.asarray(valid, bool)).astype(np.float64)
    return np.where(pred, e, 0.0), np.where(wm > 0, m, 0.0), we, wm
