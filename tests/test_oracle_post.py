"""Pins of the post-processing oracle: the 3x3 block median (Section 2.3)."""
import numpy as np

import oracle


def test_median_is_numpy_median_of_clamped_neighbourhoods():
    rng = np.random.default_rng(0)
    d = rng.uniform(0, 60, (7, 11))
    got = oracle.median3x3(d)
    pad = np.pad(d, 1, mode="edge")
    for y in range(7):
        for x in range(11):
            assert got[y, x] == np.median(pad[y:y + 3, x:x + 3])


def test_median_removes_isolated_impulses_and_keeps_planes():
    d = np.full((9, 12), 20.25)
    d[4, 5] = 90.0
    d[0, 0] = -5.0
    out = oracle.median3x3(d)
    assert np.all(out == 20.25)
    # the median of a 3x3 patch of a plane is its centre value; a clamped
    # corner of f = x/2 + y/4 takes the median of
    # {0,0,0,0,.25,.25,.5,.5,.75} = 0.25
    yy, xx = np.mgrid[0:9, 0:12]
    ramp = 0.5 * xx + 0.25 * yy
    out = oracle.median3x3(ramp)
    assert np.array_equal(out[1:-1, 1:-1], ramp[1:-1, 1:-1])
    assert out[0, 0] == 0.25


def test_median_of_a_step_keeps_the_edge():
    d = np.zeros((6, 10))
    d[:, 5:] = 30.0
    assert np.array_equal(oracle.median3x3(d), d)
