"""Host-side pieces of the evaluation tools (no GPU): the noise statistics
of Section 3 and the ego-motion perturbation."""
import math

import numpy as np

from paper_1809_07986_amd.estimate_noise import noise_stats, perturb


def test_noise_stats_gaussian_and_uniform():
    rng = np.random.default_rng(0)
    e = rng.normal(0.0, 0.5, 400000)
    s = noise_stats(e)
    # truncation at 6 sigma changes nothing at this sample size; SE of the
    # mean square is sigma^2 * sqrt(2 / n) ~ 5.6e-4
    assert abs(s["variance"] - 0.25) < 3e-3
    assert abs(s["within_1px"] - math.erf(1.0 / (0.5 * math.sqrt(2)))) < 3e-3
    u = rng.uniform(-2.0, 2.0, 400000)
    su = noise_stats(u)
    assert abs(su["variance"] - 4.0 / 3.0) < 1e-2      # E[u^2] = a^2 / 3
    assert abs(su["within_1px"] - 0.5) < 3e-3
    assert su["outliers"] == 0.0


def test_noise_stats_counts_outliers_and_ignores_them():
    e = np.array([0.5, -0.5, 0.5, -0.5, 10.0, -7.0])
    s = noise_stats(e, inlier=3.0)
    assert s["variance"] == 0.25 and s["mean"] == 0.0
    assert abs(s["outliers"] - 2 / 6) < 1e-12
    assert sum(s["hist"]) == 4


def test_perturb_keeps_a_rigid_motion():
    T = np.eye(4)
    T[:3, 3] = [0.1, 0.0, -1.0]
    rng = np.random.default_rng(1)
    assert np.array_equal(perturb(T, rng, 0.0, 0.0), T)
    P = perturb(T, rng, 0.5, 0.02)
    R = P[:3, :3]
    assert np.allclose(R @ R.T, np.eye(3), atol=1e-12)
    assert abs(np.linalg.det(R) - 1.0) < 1e-12
    assert np.array_equal(P[3], [0, 0, 0, 1])
    assert not np.allclose(P, T)


def test_curvature_scale_recovers_tau():
    # errors drawn as N(0, tau / kappa): the maximum-likelihood scale mean(e^2 kappa)
    # returns tau within its sampling error (relative sd sqrt(2/n))
    from paper_1809_07986_amd.estimate_noise import curvature_scale
    rng = np.random.default_rng(3)
    n, tau = 200000, 7.5
    kappa = rng.integers(20, 400, n)
    err = rng.normal(0.0, np.sqrt(tau / kappa))
    kappa[:1000] = 0                       # undefined curvature: not used
    err[1000:1100] = 50.0                  # gross errors beyond the inlier bound: not used
    res = curvature_scale(err, kappa, inlier=3.0)
    assert res["n"] == n - 1100
    assert abs(res["tau"] / tau - 1) < 5 * np.sqrt(2 / res["n"])
