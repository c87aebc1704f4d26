"""The OpenMP build of the oracle (the CPU baseline) against the one-thread
build (the parity reference): every output identical, bit for bit."""
import numpy as np
import pytest

import oracle as O
import stereo_synth as synth


@pytest.fixture
def threaded():
    n = O.use_threads(True)
    yield n
    O.use_threads(False)


def _run(fn):
    O.use_threads(False)
    a = fn()
    O.use_threads(True)
    b = fn()
    O.use_threads(False)
    return a, b


def test_threaded_build_uses_several_threads(threaded):
    assert threaded >= 1
    assert O.use_threads(False) == 1


@pytest.mark.parametrize("mask", [0xFF, 0x0F, 0xF0, 0x02])
def test_ragged_match_identical(mask):
    rng = np.random.default_rng(40 + mask)
    H, W, D = 23, 57, 40
    left = rng.integers(0, 256, (H, W)).astype(np.uint8)
    right = np.roll(left, -3, axis=1)
    lo, hi = synth.random_windows(rng, H, W, D, max_width=9, full_frac=0.2)
    prm = O.Params(W, H, D, path_mask=mask, f=100.0)

    def go():
        dstar, dz, C, S = O.match(prm, left, right, lo, hi, want_cs=True)
        C2 = np.where(C >= 0, C, 0)
        S2, Lr = O.aggregate(C2, lo, hi, prm.p1, prm.p2, mask, want_lr=True)
        return dstar, dz, C, S, S2, Lr

    a, b = _run(go)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_filter_sequence_identical():
    seq = synth.make_sequence("tiny")

    def go():
        F = O.OracleFilter(O.Params(seq.cam.width, seq.cam.height, seq.max_disp, f=seq.cam.f,
                                    baseline=seq.cam.baseline))
        out = []
        F.full_frame(seq.left[0], seq.right[0])
        for k in range(1, seq.frames):
            F.reduced_frame(seq.left[k], seq.right[k], seq.T[k])
            out += [F.d.copy(), F.p.copy(), F.mask.copy(), F.sflags.copy(), F.dz.copy(), F.lo.copy()]
        return out

    a, b = _run(go)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
