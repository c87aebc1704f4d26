"""Pins of the CPU oracle to things other than itself (no GPU needed).

Each test checks the oracle against a closed form, a brute-force enumeration,
an independent reformulation, an invariant, or a hand-worked example, chosen so
that a plausible slip (dropped term, wrong sign or index, transposed operand)
fails at least one of them.
"""
import itertools
import os

import numpy as np
import pytest

import oracle as O
import stereo_synth as synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    vals, rows = {}, []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#")[0].strip()
        if not line:
            continue
        if "=" in line:
            k, v = [s.strip() for s in line.split("=", 1)]
            vals[k] = v
        else:
            rows.append([int(t) for t in line.split()])
    return vals, rows


# ---------------------------------------------------------------- census / cost

def test_census_worked_example():
    vals, rows = _read_golden("census_3x3_example.txt")
    img = np.array(rows, np.uint8)
    c = O.census(img, 3, 3)
    assert int(c[1, 1]) == int(vals["expected_centre_census"])


def test_census_constant_image_is_zero():
    img = np.full((12, 20), 77, np.uint8)
    assert not O.census(img, 9, 7).any()


@pytest.mark.parametrize("axis", [0, 1])
def test_census_ramp_closed_form(axis):
    # On a strictly increasing ramp the darker neighbours are exactly those on
    # the lower side; with clamp-to-edge, every interior pixel (and every pixel
    # at least one step from the low border) sees the full pattern.
    H, W = 15, 21
    yy, xx = np.mgrid[0:H, 0:W]
    img = (5 * (xx if axis == 1 else yy)).astype(np.uint8)
    c = O.census(img, 9, 7)
    expected = 0
    for dy in range(-3, 4):
        for dx in range(-4, 5):
            if dx == 0 and dy == 0:
                continue
            darker = (dx < 0) if axis == 1 else (dy < 0)
            expected = (expected << 1) | int(darker)
    interior = c[1:, 1:]
    assert np.all(interior == np.uint64(expected))
    # the pixels on the low border have no darker neighbour at all
    border = c[:, 0] if axis == 1 else c[0, :]
    assert not border.any()


def test_census_bit_count_and_cost_range():
    rng = np.random.default_rng(0)
    img = rng.integers(0, 256, (20, 30)).astype(np.uint8)
    c = O.census(img, 9, 7)
    assert int(c.max()) < (1 << 62)
    c5 = O.census(img, 5, 5)
    assert int(c5.max()) < (1 << 24)


def test_cost_zero_at_true_shift_and_max_outside():
    # right = left shifted by s: interior census strings coincide at d = s
    rng = np.random.default_rng(1)
    H, W, D, s = 16, 48, 16, 5
    left = rng.integers(0, 256, (H, W)).astype(np.uint8)
    right = np.zeros_like(left)
    right[:, : W - s] = left[:, s:]
    right[:, W - s:] = rng.integers(0, 256, (H, s))
    cl, cr = O.census(left, 9, 7), O.census(right, 9, 7)
    lo = np.zeros((H, W), np.int32)
    hi = np.full((H, W), D - 1, np.int32)
    C = O.cost(cl, cr, D, 62, lo, hi)
    assert np.all(C[3:H - 3, s + 4:W - 4, s] == 0)
    # x - d < 0 -> the largest cost, the number of census bits
    for x in range(0, D - 1):
        assert np.all(C[:, x, x + 1:] == 62)
    # Hamming distance is symmetric and bounded
    assert C.min() >= 0 and C.max() <= 62


# ---------------------------------------------------------------- aggregation

def _pen(a, b, p1, p2):
    return 0 if a == b else (p1 if abs(a - b) == 1 else p2)


@pytest.mark.parametrize("seed", range(6))
def test_single_path_equals_exhaustive_dp(seed):
    # One path along a row is an exact dynamic programme: the normalised
    # L_r at the last pixel equals the minimal energy over all label
    # sequences ending in d, minus the overall minimum.
    rng = np.random.default_rng(seed)
    n, D = 6, 5
    p1, p2 = 7, 86 if seed % 2 else 20
    C = rng.integers(0, 63, (1, n, D)).astype(np.int32)
    lo = np.zeros((1, n), np.int32)
    hi = np.full((1, n), D - 1, np.int32)
    S, Lr = O.aggregate(C, lo, hi, p1, p2, path_mask=0x01, want_lr=True)
    best = np.full(D, 10 ** 9)
    for seq in itertools.product(range(D), repeat=n):
        e = sum(int(C[0, i, seq[i]]) for i in range(n))
        e += sum(_pen(seq[i], seq[i - 1], p1, p2) for i in range(1, n))
        best[seq[-1]] = min(best[seq[-1]], e)
    got = Lr[0, 0, n - 1].astype(np.int64)
    assert np.array_equal(got - got.min(), best - best.min())
    assert np.array_equal(S[0, n - 1], Lr[0, 0, n - 1])


@pytest.mark.parametrize("seed", range(6))
def test_ragged_single_path_equals_exhaustive_dp(seed):
    # Same identity with per-pixel label sets (reduced search windows): the
    # label of pixel i is restricted to [lo_i, hi_i].
    rng = np.random.default_rng(100 + seed)
    n, D = 6, 7
    p1, p2 = 6, 65
    lo = rng.integers(0, D - 1, (1, n)).astype(np.int32)
    hi = np.minimum(lo + rng.integers(0, 4, (1, n)), D - 1).astype(np.int32)
    C = rng.integers(0, 63, (1, n, D)).astype(np.int32)
    S, Lr = O.aggregate(C, lo, hi, p1, p2, path_mask=0x02, want_lr=True)   # right-to-left path
    # path 1 runs right to left: its last pixel is x = 0
    order = list(range(n - 1, -1, -1))
    sets = [range(lo[0, x], hi[0, x] + 1) for x in order]
    best = {}
    for seq in itertools.product(*sets):
        e = sum(int(C[0, x, d]) for x, d in zip(order, seq))
        e += sum(_pen(seq[i], seq[i - 1], p1, p2) for i in range(1, n))
        best[seq[-1]] = min(best.get(seq[-1], 10 ** 9), e)
    dom = list(range(lo[0, 0], hi[0, 0] + 1))
    got = np.array([Lr[1, 0, 0, d] for d in dom], np.int64)
    want = np.array([best[d] for d in dom], np.int64)
    assert np.array_equal(got - got.min(), want - want.min())


def _dense_sgm_big(C, lo, hi, p1, p2, path_mask, big=10 ** 6):
    """Independent second formulation: dense SGM over all D disparities where
    every cell outside the pixel's window costs `big` (far above any in-window
    loss).  Plain per-pixel loops, numpy over the disparity axis."""
    H, W, D = C.shape
    d_idx = np.arange(D)
    inwin = (d_idx[None, None, :] >= lo[:, :, None]) & (d_idx[None, None, :] <= hi[:, :, None])
    Cb = np.where(inwin, C, big).astype(np.int64)
    S = np.zeros((H, W, D), np.int64)
    for k in range(8):
        if not (path_mask >> k) & 1:
            continue
        rx, ry = O.PATH_DX[k], O.PATH_DY[k]
        L = np.zeros((H, W, D), np.int64)
        ys = range(H) if ry >= 0 else range(H - 1, -1, -1)
        xs = list(range(W)) if rx >= 0 else list(range(W - 1, -1, -1))
        for y in ys:
            for x in xs:
                qx, qy = x - rx, y - ry
                if not (0 <= qx < W and 0 <= qy < H):
                    L[y, x] = Cb[y, x]
                    continue
                prev = L[qy, qx]
                m = prev.min()
                up = np.concatenate([prev[1:], [np.iinfo(np.int64).max // 4]])
                dn = np.concatenate([[np.iinfo(np.int64).max // 4], prev[:-1]])
                best = np.minimum(np.minimum(prev, np.minimum(up, dn) + p1), m + p2)
                L[y, x] = Cb[y, x] + best - m
        S += L
    return S, inwin


@pytest.mark.parametrize("seed,mask", [(0, 0xFF), (1, 0xFF), (2, 0x0F), (3, 0xF0), (4, 0x81)])
def test_ragged_aggregation_equals_dense_big_sentinel(seed, mask):
    rng = np.random.default_rng(200 + seed)
    H, W, D = 9, 13, 12
    C = rng.integers(0, 63, (H, W, D)).astype(np.int32)
    lo, hi = synth.random_windows(rng, H, W, D, max_width=6, full_frac=0.15)
    S = O.aggregate(C, lo, hi, 7, 86, path_mask=mask)
    Sd, inwin = _dense_sgm_big(C, lo, hi, 7, 86, mask)
    assert np.array_equal(S[inwin], Sd[inwin])


def test_full_windows_equal_dense_sgm():
    rng = np.random.default_rng(7)
    H, W, D = 8, 11, 9
    C = rng.integers(0, 63, (H, W, D)).astype(np.int32)
    lo = np.zeros((H, W), np.int32)
    hi = np.full((H, W), D - 1, np.int32)
    S = O.aggregate(C, lo, hi, 7, 86)
    Sd, _ = _dense_sgm_big(C, lo, hi, 7, 86, 0xFF)
    assert np.array_equal(S, Sd)


def test_aggregation_bounds():
    # C <= L_r <= C + P2 and min_d C <= min_d L_r <= min_d C + P2, S <= 8 (Nc + P2)
    rng = np.random.default_rng(8)
    H, W, D = 10, 14, 16
    p1, p2 = 7, 86
    C = rng.integers(0, 63, (H, W, D)).astype(np.int32)
    lo, hi = synth.random_windows(rng, H, W, D, max_width=8, full_frac=0.2)
    S, Lr = O.aggregate(C, lo, hi, p1, p2, want_lr=True)
    d_idx = np.arange(D)
    inwin = (d_idx[None, None, :] >= lo[:, :, None]) & (d_idx[None, None, :] <= hi[:, :, None])
    for k in range(8):
        L = Lr[k]
        assert np.all(L[inwin] >= C[inwin])
        assert np.all(L[inwin] <= C[inwin] + p2)
        Lm = np.where(inwin, L, 10 ** 9).min(axis=2)
        Cm = np.where(inwin, C, 10 ** 9).min(axis=2)
        assert np.all(Lm >= Cm) and np.all(Lm <= Cm + p2)
    assert S[inwin].max() <= 8 * (62 + p2) and 8 * (62 + p2) < 2 ** 16
    assert Lr[:, inwin].max() <= 62 + p2 < 2 ** 8


@pytest.mark.parametrize("mask", [0xFF, 0x0F, 0xF0])
def test_aggregation_dihedral_symmetry(mask):
    # the path sets are closed under transposition and horizontal flips
    rng = np.random.default_rng(9)
    H, W, D = 9, 12, 10
    C = rng.integers(0, 63, (H, W, D)).astype(np.int32)
    lo, hi = synth.random_windows(rng, H, W, D, max_width=5, full_frac=0.1)
    S = O.aggregate(C, lo, hi, 7, 86, path_mask=mask)
    St = O.aggregate(C.transpose(1, 0, 2).copy(), lo.T.copy(), hi.T.copy(), 7, 86, path_mask=mask)
    Sf = O.aggregate(C[:, ::-1].copy(), lo[:, ::-1].copy(), hi[:, ::-1].copy(), 7, 86, path_mask=mask)
    Sv = O.aggregate(C[::-1].copy(), lo[::-1].copy(), hi[::-1].copy(), 7, 86, path_mask=mask)
    assert np.array_equal(St.transpose(1, 0, 2), S)
    assert np.array_equal(Sf[:, ::-1], S)
    assert np.array_equal(Sv[::-1], S)


def test_single_direction_geometry():
    # a path only sees its predecessors: a cost spike at one pixel reaches the
    # pixels downstream along that path and no pixel upstream of it
    H, W, D = 7, 9, 4
    C = np.zeros((H, W, D), np.int32)
    C[3, 4, :] = [50, 0, 50, 50]
    lo = np.zeros((H, W), np.int32)
    hi = np.full((H, W), D - 1, np.int32)
    for k in range(8):
        _, Lr = O.aggregate(C, lo, hi, 7, 86, path_mask=1 << k, want_lr=True)
        L = Lr[k]
        touched = {(y, x) for y in range(H) for x in range(W) if L[y, x].any()}
        rx, ry = O.PATH_DX[k], O.PATH_DY[k]
        expect = set()
        y, x = 3, 4
        while 0 <= y < H and 0 <= x < W:
            expect.add((y, x))
            y, x = y + ry, x + rx
        assert touched == expect, (k, sorted(touched))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_second_pass_differs_only_until_losses_rejoin(seed):
    # Gate re-run (Section 4's innovation test, then a second matching pass):
    # the second pass widens some pixels to the full range.  Eq. 1 sees the
    # previous pixel on a path only through its vector of L_r, so a pixel that
    # kept its window and whose predecessor's L_r did not change has unchanged
    # L_r: the two passes differ from a widened pixel up to the first pixel
    # whose losses agree again, and nowhere else.
    rng = np.random.default_rng(300 + seed)
    H, W, D = 10, 14, 16
    C = rng.integers(0, 63, (H, W, D)).astype(np.int32)
    lo1, hi1 = synth.random_windows(rng, H, W, D, max_width=6, full_frac=0.1)
    moved = rng.random((H, W)) < 0.08
    lo2 = np.where(moved, 0, lo1).astype(np.int32)
    hi2 = np.where(moved, D - 1, hi1).astype(np.int32)
    _, L1 = O.aggregate(C, lo1, hi1, 7, 86, want_lr=True)
    _, L2 = O.aggregate(C, lo2, hi2, 7, 86, want_lr=True)
    d = np.arange(D)
    in1 = (d >= lo1[..., None]) & (d <= hi1[..., None])
    kept = rejoined = differ = 0
    for k in range(8):
        rx, ry = O.PATH_DX[k], O.PATH_DY[k]
        same = np.all(np.where(in1, L1[k] == L2[k], True), axis=2)
        for y in range(H):
            for x in range(W):
                if moved[y, x]:
                    continue
                qy, qx = y - ry, x - rx
                first = not (0 <= qy < H and 0 <= qx < W)
                if first or (not moved[qy, qx] and same[qy, qx]):
                    assert same[y, x], (k, y, x)
                    kept += 1
                elif same[y, x]:
                    rejoined += 1
                else:
                    differ += 1
    assert kept > 0 and rejoined > 0 and differ > 0, (kept, rejoined, differ)


# ---------------------------------------------------------------- WTA / subpixel

def test_wta_argmin_lowest_on_ties():
    rng = np.random.default_rng(10)
    H, W, D = 6, 7, 9
    S = rng.integers(0, 20, (H, W, D)).astype(np.int32)
    lo = np.zeros((H, W), np.int32)
    hi = np.full((H, W), D - 1, np.int32)
    dstar, _ = O.wta(S, lo, hi)
    assert np.array_equal(dstar, np.argmin(S, axis=2))
    lo2, hi2 = synth.random_windows(rng, H, W, D, max_width=4, full_frac=0.0)
    dstar2, _ = O.wta(S, lo2, hi2)
    for y in range(H):
        for x in range(W):
            seg = S[y, x, lo2[y, x]:hi2[y, x] + 1]
            assert dstar2[y, x] == lo2[y, x] + int(np.argmin(seg))


def test_subpixel_worked_example():
    vals, _ = _read_golden("subpixel_example.txt")
    S = np.full((1, 1, 8), 500, np.int32)
    S[0, 0, 3:6] = [int(vals["S_minus"]), int(vals["S_star"]), int(vals["S_plus"])]
    lo = np.zeros((1, 1), np.int32)
    hi = np.full((1, 1), 7, np.int32)
    dstar, dz = O.wta(S, lo, hi)
    assert dstar[0, 0] == 4
    assert dz[0, 0] == 4 + float(vals["offset"])


@pytest.mark.parametrize("shift", [-0.375, -0.25, 0.0, 0.125, 0.375, 0.5])
def test_subpixel_recovers_parabola_vertex(shift):
    # integer samples of 64 (d - d0 - shift)^2 + 3 (exact for these shifts)
    d0 = 6
    D = 12
    dd = np.arange(D)
    vals = 64 * (dd - d0 - shift) ** 2 + 3
    assert np.all(vals == np.round(vals))
    S = vals.astype(np.int32)
    _, dz = O.wta(S.reshape(1, 1, D), np.zeros((1, 1), np.int32), np.full((1, 1), D - 1, np.int32))
    assert dz[0, 0] == d0 + shift


def test_subpixel_edges_and_range():
    # no fit at a window edge; offset always in (-0.5, 0.5]
    rng = np.random.default_rng(11)
    H, W, D = 10, 10, 16
    S = rng.integers(0, 50, (H, W, D)).astype(np.int32)
    lo, hi = synth.random_windows(rng, H, W, D, max_width=6, full_frac=0.0)
    dstar, dz = O.wta(S, lo, hi)
    off = dz - dstar
    assert np.all(off > -0.5) and np.all(off <= 0.5)
    edge = (dstar == lo) | (dstar == hi)
    assert np.all(off[edge] == 0.0)


# ------------------------------------------------- cost-curvature measurement variance

@pytest.mark.parametrize("c,e", [(1, 0), (3, 2), (7, -5), (40, 39), (200, -17)])
def test_curvature_of_a_parabola_is_its_second_difference(c, e):
    # S(d) = 50 + c (d - m)^2 + e (d - m) with |e| < c has its integer minimum
    # at m, and the three samples around it have a = c - e, b = c + e: the
    # curvature a + b = 2c whatever the slope e, and r = r_curv / (2c)
    D, m = 16, 7
    dd = np.arange(D)
    S = (50 + c * (dd - m) ** 2 + e * (dd - m)).astype(np.int32).reshape(1, 1, D)
    lo, hi = np.zeros((1, 1), np.int32), np.full((1, 1), D - 1, np.int32)
    dstar, _ = O.wta(S, lo, hi)
    assert dstar[0, 0] == m
    tau = 3.5
    rpix, kappa = O.curvature_r(S, lo, hi, dstar, tau, 1.0)
    assert kappa[0, 0] == 2 * c
    want = min(max(tau / (2 * c), 1 / 256), 64.0)
    assert rpix[0, 0] == want


def test_curvature_edges_ties_and_clamps():
    D = 8
    lo = np.array([[0, 2, 0, 0, 3]], np.int32)
    hi = np.array([[7, 2, 7, 7, 5]], np.int32)
    S = np.full((1, 5, D), 90, np.int32)
    S[0, 0, 0:3] = [10, 20, 30]                  # minimum on the lower edge: no parabola
    S[0, 1, 2] = 5                                # one-cell window
    S[0, 2, 2:6] = [40, 30, 30, 60]               # tie: d* = 3 (lowest), a = 10, b = 0
    S[0, 3, 3:6] = [12, 11, 12]                   # kappa = 2: r_curv / 2 above 64 -> 64
    S[0, 4, 3:6] = [80, 70, 60]                   # minimum on the upper edge
    dstar, _ = O.wta(S, lo, hi)
    assert dstar.tolist() == [[0, 2, 3, 4, 5]]
    rpix, kappa = O.curvature_r(S, lo, hi, dstar, 1000.0, 0.75)
    assert kappa.tolist() == [[0, 0, 10, 2, 0]]
    assert rpix[0, 0] == 0.75 and rpix[0, 1] == 0.75 and rpix[0, 4] == 0.75
    assert rpix[0, 2] == 64.0 and rpix[0, 3] == 64.0
    rpix, _ = O.curvature_r(S, lo, hi, dstar, 0.001, 0.75)
    assert rpix[0, 2] == 1 / 256 and rpix[0, 3] == 1 / 256


def test_curvature_filter_uses_the_per_pixel_variance():
    # a filter run with r_curv: the correction of each pixel is the Kalman
    # closed form with that pixel's r = clamp(r_curv / kappa)
    seq = synth.make_sequence("tiny")
    H, W, D = seq.cam.height, seq.cam.width, seq.max_disp
    F = O.OracleFilter(O.Params(W, H, D, f=seq.cam.f, baseline=seq.cam.baseline, r_curv=20.0))
    F.full_frame(seq.left[0], seq.right[0])
    assert np.all(F.p == F.prm.r) and np.all(F.d == F.dz)
    k = F.kappa
    assert np.all((k == 0) | (k >= 1))
    F.reduced_frame(seq.left[1], seq.right[1], seq.T[1])
    r = np.where(F.kappa > 0, np.clip(20.0 / np.maximum(F.kappa, 1), 1 / 256, 64.0), F.prm.r)
    assert np.array_equal(F.rpix, r)
    use = ((F.flags & O.PRED) != 0) & ((F.flags & O.FULLWIN) == 0)
    assert use.sum() > 1000
    r, pm, dh, dz = r[use], F.pm[use], F.dhat[use], F.dz[use]
    assert np.max(np.abs(F.d[use] - (r * dh + pm * dz) / (pm + r))) < 1e-9
    assert np.max(np.abs(F.p[use] / (pm * r / (pm + r)) - 1)) < 1e-9


# ---------------------------------------------------------------- prediction

def _prm(H=24, W=32, D=64, **kw):
    return O.Params(W, H, D, f=kw.pop("f", 300.0), baseline=kw.pop("baseline", 0.5), **kw)


def test_warp_identity():
    prm = _prm()
    H, W = prm.height, prm.width
    rng = np.random.default_rng(12)
    d = np.full((H, W), 20.0) + rng.uniform(-0.4, 0.4, (H, W))
    p = rng.uniform(0.3, 1.0, (H, W))
    dh, pm, fl, lo, hi = O.predict(prm, d, p, np.zeros((H, W), np.uint8), np.eye(4))
    assert np.all(fl & O.PRED)
    assert np.max(np.abs(dh - d)) < 1e-12
    assert np.max(np.abs(pm - (p + prm.q))) < 1e-12


def test_warp_forward_translation_closed_form():
    # fronto-parallel plane at depth Z, camera moves v forward:
    # d' = fB / (Z - v), x' = cx + (x - cx) Z / (Z - v), Phi = Z / (Z - v)
    prm = _prm(H=31, W=41, D=64)
    H, W = prm.height, prm.width
    fB = prm.f * prm.baseline
    Z, v = 10.0, 1.0
    d0 = fB / Z
    d = np.full((H, W), d0)
    p = np.full((H, W), 0.8)
    T = np.eye(4)
    T[2, 3] = -v
    dh, pm, fl, lo, hi = O.predict(prm, d, p, np.zeros((H, W), np.uint8), T)
    phi = Z / (Z - v)
    ok = (fl & O.PRED) > 0
    assert ok.mean() > 0.9
    assert np.max(np.abs(dh[ok] - fB / (Z - v))) < 1e-9
    assert np.max(np.abs(pm[ok] - (phi * phi * 0.8 + prm.q))) < 1e-9
    # one marked source pixel (slightly nearer, so it wins its target)
    xs, ys = 30, 22
    d2 = d.copy()
    d2[ys, xs] = d0 + 0.5
    Zs = fB / d2[ys, xs]
    dh2, _, fl2, _, _ = O.predict(prm, d2, p, np.zeros((H, W), np.uint8), T)
    tx = int(np.floor(prm.cx + (xs - prm.cx) * Zs / (Zs - v) + 0.5))
    ty = int(np.floor(prm.cy + (ys - prm.cy) * Zs / (Zs - v) + 0.5))
    assert abs(dh2[ty, tx] - fB / (Zs - v)) < 1e-9


def test_warp_lateral_translation_closed_form():
    prm = _prm(H=20, W=40, D=64)
    H, W = prm.height, prm.width
    fB = prm.f * prm.baseline
    Z = 6.0
    d = np.full((H, W), fB / Z)
    d[7, 10] += 0.3
    p = np.full((H, W), 0.5)
    tx_m = 0.1   # moves points by +0.1 m in x: x' = x + f * 0.1 / Z = x + 5 px
    T = np.eye(4)
    T[0, 3] = tx_m
    dh, pm, fl, _, _ = O.predict(prm, d, p, np.zeros((H, W), np.uint8), T)
    shift = prm.f * tx_m / (fB / d[7, 10])
    assert abs(dh[7, 10 + int(round(shift))] - d[7, 10]) < 1e-12
    ok = (fl & O.PRED) > 0
    assert np.max(np.abs(pm[ok] - (0.5 + prm.q))) < 1e-12      # Phi = 1
    # columns that no source reaches (the left strip) have no prediction
    assert not np.any(fl[:, :5] & O.PRED)


def test_zero_disparity_stays_zero_with_unit_phi_under_forward_motion():
    prm = _prm(H=16, W=16, D=32)
    H, W = prm.height, prm.width
    d = np.zeros((H, W))
    p = np.full((H, W), 0.7)
    T = np.eye(4)
    T[2, 3] = -2.0
    dh, pm, fl, _, _ = O.predict(prm, d, p, np.zeros((H, W), np.uint8), T)
    ok = (fl & O.PRED) > 0
    assert ok.all()
    assert np.all(dh == 0.0)
    assert np.max(np.abs(pm - (0.7 + prm.q))) < 1e-12


def _predict_identity(prm, d, p, sflags=None):
    H, W = d.shape
    if sflags is None:
        sflags = np.zeros((H, W), np.uint8)
    return O.predict(prm, d, p, sflags, np.eye(4))


def test_hole_fill_cases():
    # With T = I every source lands on itself; a source with d > D-1 is dropped
    # and leaves a hole.
    prm = _prm(H=5, W=5, D=16, q=0.0)
    big = 15.5
    d = np.full((5, 5), 8.0)
    d[0, :] = [8.0, 8.2, 8.4, 8.6, 8.8]
    p = np.full((5, 5), 0.5)
    # (a) interior hole with both pairs: mean of four, variance mean of four
    d1 = d.copy()
    d1[2, 2] = big
    p1 = p.copy()
    p1[1, 2], p1[3, 2], p1[2, 1], p1[2, 3] = 0.2, 0.4, 0.6, 0.8
    d1[1, 2], d1[3, 2], d1[2, 1], d1[2, 3] = 8.0, 8.4, 8.8, 9.2
    dh, pm, fl, lo, hi = _predict_identity(prm, d1, p1)
    assert fl[2, 2] & O.PRED
    assert abs(dh[2, 2] - (8.0 + 8.4 + 8.8 + 9.2) / 4) < 1e-12
    assert abs(pm[2, 2] - 0.5) < 1e-12
    # (b) hole on the left border: only the vertical pair exists
    d2 = d.copy()
    d2[2, 0] = big
    d2[1, 0], d2[3, 0] = 7.5, 8.5
    dh, pm, fl, _, _ = _predict_identity(prm, d2, p)
    assert fl[2, 0] & O.PRED and abs(dh[2, 0] - 8.0) < 1e-12
    # (c) corner hole: no pair at all -> no prediction, full window
    d3 = d.copy()
    d3[0, 0] = big
    dh, pm, fl, lo, hi = _predict_identity(prm, d3, p)
    assert not fl[0, 0] & O.PRED and fl[0, 0] & O.FULLWIN
    assert lo[0, 0] == 0 and hi[0, 0] == prm.max_disp - 1
    # (d) two adjacent holes in a row: each uses its vertical pair
    d4 = d.copy()
    d4[2, 1] = big
    d4[2, 2] = big
    d4[1, 1], d4[3, 1], d4[1, 2], d4[3, 2] = 7.0, 8.0, 8.0, 9.0
    dh, pm, fl, _, _ = _predict_identity(prm, d4, p)
    assert abs(dh[2, 1] - 7.5) < 1e-12 and abs(dh[2, 2] - 8.5) < 1e-12
    # (e) a filled hole carries RESET if a contributor had it
    sf = np.zeros((5, 5), np.uint8)
    sf[1, 2] = O.RESET
    dh, pm, fl, _, _ = _predict_identity(prm, d1, p1, sf)
    assert fl[2, 2] & O.RESET and fl[2, 2] & O.FULLWIN


def test_discontinuity_rejection_cases():
    prm = _prm(H=6, W=8, D=32, q=0.0, disc_thresh=2.0)
    p = np.full((6, 8), 0.5)
    d = np.full((6, 8), 10.0)
    d[:, 4:] = 13.0          # step of 3 > 2 between columns 3 and 4
    dh, pm, fl, lo, hi = _predict_identity(prm, d, p)
    rej = (fl & O.PRED) == 0
    assert np.all(rej[:, 3:5]) and not np.any(rej[:, :3]) and not np.any(rej[:, 5:])
    assert np.all(fl[:, 3:5] & O.FULLWIN)
    # a step of exactly the threshold is kept
    d2 = np.full((6, 8), 10.0)
    d2[:, 4:] = 12.0
    _, _, fl2, _, _ = _predict_identity(prm, d2, p)
    assert np.all(fl2 & O.PRED)
    # diagonal-only contact also counts (8-neighbourhood)
    d3 = np.full((6, 8), 10.0)
    d3[2, 2] = 20.0
    d3[1, 2] = d3[3, 2] = d3[2, 1] = d3[2, 3] = 20.0
    d3[1, 1] = 10.0
    _, _, fl3, _, _ = _predict_identity(prm, d3, p)
    assert not fl3[2, 2] & O.PRED        # neighbours 20 in cross, 10 on the diagonals
    assert fl3[0, 5] & O.PRED


def test_window_limits_examples():
    # p^- = 1 (p = 0.5, q = 0.5), k = 3: d^ = 10.0 -> [7, 13]; 10.3 -> [7, 14]; 1.0 -> [0, 4]
    prm = _prm(H=3, W=3, D=16, q=0.5, disc_thresh=1e9)
    p = np.full((3, 3), 0.5)
    for dv, (l, h) in [(10.0, (7, 13)), (10.3, (7, 14)), (1.0, (0, 4)), (14.5, (11, 15))]:
        d = np.full((3, 3), dv)
        dh, pm, fl, lo, hi = _predict_identity(prm, d, p)
        assert lo[1, 1] == l and hi[1, 1] == h, (dv, lo[1, 1], hi[1, 1])
        assert not fl[1, 1] & O.FULLWIN


# ---------------------------------------------------------------- correction

def test_kalman_closed_form():
    prm = _prm(H=4, W=5, D=32, r=1.0)
    rng = np.random.default_rng(13)
    dh = rng.uniform(5, 20, (4, 5))
    pm = rng.uniform(0.5, 3.0, (4, 5))
    dz = dh + rng.uniform(-1.5, 1.5, (4, 5))
    fl = np.full((4, 5), O.PRED, np.uint8)
    lo = np.zeros((4, 5), np.int32)
    hi = np.full((4, 5), 31, np.int32)
    dstar = np.round(dz).astype(np.int32)
    d, p, mask, sf = O.correct(prm, dh, pm, fl, lo, hi, dstar, dz)
    r = prm.r
    assert np.max(np.abs(d - (r * dh + pm * dz) / (pm + r))) < 1e-12
    assert np.max(np.abs(p / (pm * r / (pm + r)) - 1)) < 1e-12


def test_kalman_static_pixel_converges_to_fixed_point():
    # static pixel, Phi = 1, q = 0.5, r = 1: p = 1 -> 0.6 -> 0.5238... -> 0.5
    q, r = 0.5, 1.0
    prm = _prm(H=3, W=3, D=32, q=q, r=r)
    d = np.full((3, 3), 12.0)
    p = np.full((3, 3), r)
    sf = np.zeros((3, 3), np.uint8)
    seq = []
    for _ in range(12):
        dh, pm, fl, lo, hi = O.predict(prm, d, p, sf, np.eye(4))
        dstar = np.full((3, 3), 12, np.int32)
        d, p, mask, sf = O.correct(prm, dh, pm, fl, lo, hi, dstar, dh.copy())
        seq.append(p[1, 1])
    assert abs(seq[0] - 0.6) < 1e-12
    assert abs(seq[1] - 1.1 / 2.1) < 1e-12
    assert abs(seq[2] - (1.1 / 2.1 + 0.5) / (1.1 / 2.1 + 1.5)) < 1e-12
    p_inf = (-q + np.sqrt(q * q + 4 * q * r)) / 2
    assert abs(p_inf - 0.5) < 1e-15
    assert abs(seq[-1] - p_inf) < 1e-6
    assert not mask.any()


def test_chi2_gate_constant_and_decision():
    from scipy.stats import chi2
    assert abs(O.Params(4, 4, 8).chi2_gate - chi2.ppf(0.99, 1)) < 1e-9
    prm = _prm(H=1, W=2, D=32, r=1.0)
    pm = np.array([[1.0, 1.0]])
    S = pm + prm.r
    nu = np.sqrt(prm.chi2_gate * S)
    dh = np.array([[10.0, 10.0]])
    dz = dh + nu * np.array([[0.999, 1.001]])
    fl = np.full((1, 2), O.PRED, np.uint8)
    lo = np.zeros((1, 2), np.int32)
    hi = np.full((1, 2), 31, np.int32)
    d, p, mask, sf = O.correct(prm, dh, pm, fl, lo, hi, np.full((1, 2), 13, np.int32), dz)
    assert mask.tolist() == [[0, 1]]
    assert sf.tolist() == [[0, O.RESET]]


def test_full_window_pixels_restart_and_edge_saturation_resets():
    prm = _prm(H=1, W=4, D=32, r=1.0)
    dh = np.array([[10.0, 10.0, 10.0, 0.0]])
    pm = np.array([[1.0, 1.0, 1.0, 0.0]])
    fl = np.array([[O.PRED, O.PRED, O.PRED | O.RESET | O.FULLWIN, O.FULLWIN]], np.uint8)
    lo = np.array([[7, 7, 0, 0]], np.int32)
    hi = np.array([[13, 13, 31, 31]], np.int32)
    dstar = np.array([[7, 10, 20, 5]], np.int32)
    dz = np.array([[7.0, 10.2, 20.0, 5.0]])
    d, p, mask, sf = O.correct(prm, dh, pm, fl, lo, hi, dstar, dz)
    assert sf[0, 0] == O.RESET and sf[0, 1] == 0          # minimum on the lower edge
    assert d[0, 2] == 20.0 and p[0, 2] == prm.r           # full window -> restart
    assert mask[0, 2] == 1                                 # innovation 10 vs the prediction
    assert d[0, 3] == 5.0 and mask[0, 3] == 0             # no prediction -> no test


# ---------------------------------------------------------------- paper preset

def test_paper_table1_preset_runs():
    vals, _ = _read_golden("table1_params.txt")
    cw, ch = [int(t) for t in vals["census_window"].split("x")]
    seq = synth.make_sequence("tiny", frames=1)
    prm = O.Params(seq.cam.width, seq.cam.height, int(vals["max_disp"]), census_w=cw, census_h=ch,
                   p1=int(vals["P1"]), p2=int(vals["P2"]), f=seq.cam.f, baseline=seq.cam.baseline)
    assert prm.nbits == 24
    F = O.OracleFilter(prm)
    F.full_frame(seq.left[0], seq.right[0])
    v = seq.valid[0]
    bad = (np.abs(F.dz - seq.disp_gt[0]) > 3) & v
    assert bad.sum() / v.sum() < 0.03


def test_end_to_end_tiny_sequence_accuracy():
    seq = synth.make_sequence("tiny")
    prm = O.Params(seq.cam.width, seq.cam.height, seq.max_disp, f=seq.cam.f, baseline=seq.cam.baseline)
    F = O.OracleFilter(prm)
    F.full_frame(seq.left[0], seq.right[0])
    v = seq.valid[0]
    assert ((np.abs(F.d - seq.disp_gt[0]) > 3) & v).sum() / v.sum() < 0.02
    for k in range(1, seq.frames):
        F.reduced_frame(seq.left[k], seq.right[k], seq.T[k])
        w = F.hi - F.lo + 1
        assert w.mean() < 0.5 * seq.max_disp        # the search space shrinks


def test_wrong_ego_motion_is_detected_and_recovered():
    # Section 2.4 / Section 4: with a wrong ego-motion (1.5 m of extra forward
    # motion at frame 2) the prediction disagrees with the measurement: many
    # predicted pixels are flagged moving and reset; the reset pixels search
    # the full range in frame 3, and by frame 4 the estimate is no worse than
    # that of the run that never had the error
    seq = synth.make_sequence("tiny", frames=5)
    prm = O.Params(seq.cam.width, seq.cam.height, seq.max_disp, f=seq.cam.f, baseline=seq.cam.baseline)

    def run(corrupt):
        F = O.OracleFilter(prm)
        F.full_frame(seq.left[0], seq.right[0])
        stats = []
        for k in range(1, 5):
            T = seq.T[k].copy()
            if corrupt and k == 2:
                T[2, 3] -= 1.5
            F.reduced_frame(seq.left[k], seq.right[k], T)
            v = seq.valid[k]
            pred = (F.flags & O.PRED) != 0
            stats.append(dict(bad=float(np.mean(np.abs(F.d - seq.disp_gt[k])[v] > 3)),
                              mask=float(F.mask[pred].mean()), reset=float((F.sflags & O.RESET).astype(bool).mean()),
                              full=float(((F.flags & O.FULLWIN) != 0).mean())))
        return stats

    clean, bad = run(False), run(True)
    assert bad[0] == clean[0]
    assert bad[1]["mask"] > 0.2 and bad[1]["mask"] > 5 * clean[1]["mask"]
    assert bad[1]["reset"] > 0.1 and bad[1]["bad"] > 3 * clean[1]["bad"]
    assert bad[2]["full"] > clean[2]["full"] + 0.1          # frame 3 re-measures the reset pixels
    assert bad[3]["bad"] <= clean[3]["bad"] + 0.01          # recovered by frame 4
