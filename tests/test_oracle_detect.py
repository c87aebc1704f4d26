"""Pins of the moving-object detection oracle (Section 4).

Hand-worked values for the difference map, brute-force box sums for the
summed-area table and the sliding windows, hand-worked greedy groupings (one
where merging the highest intersection-over-union pair first gives a
different answer than merging the first overlapping pair), and closed-form
end-to-end cases.
"""
import numpy as np

import oracle as O


def test_motion_values_hand_worked():
    dhat = np.array([[3.0, 10.5, 30.0, 1.0], [6.0, 6.0, 6.0, 6.0]])
    dz = np.array([[2.9375, 0.0, 5.0, 0.5], [6.0, 6.0, 6.0, 6.0]])
    flags = np.array([[O.PRED, O.PRED, O.PRED, 0], [0, 0, 0, 0]], np.uint8)
    # column 0: x - d^ = -3 < 0 (no correspondence), column 1: x - d^ < 0 too
    dhat[0, 0] = 0.0      # x - d^ = 0: inside
    dz[0, 0] = 0.0625     # 0.0625 * 16 = 1
    v = O.motion_values(dhat, dz, flags, scale=16, cap=256)
    assert v[0, 0] == 1
    assert v[0, 1] == 0             # 1 - 10.5 < 0
    assert v[0, 2] == 0             # 2 - 30 < 0
    assert v[0, 3] == 0             # no prediction
    assert np.all(v[1] == 0)
    dhat2 = np.array([[0.0, 0.0, 1.0, 2.0]])
    dz2 = np.array([[20.0, 0.99, 1.0, 2.0 + 1.0 / 32]])
    v2 = O.motion_values(dhat2, dz2, np.full((1, 4), O.PRED, np.uint8), scale=16, cap=256)
    assert v2.tolist() == [[256, 15, 0, 0]]   # 320 capped; floor(15.84); 0; floor(0.5)


def test_integral_box_sums_match_brute_force():
    rng = np.random.default_rng(3)
    v = rng.integers(0, 300, (13, 17)).astype(np.int32)
    S = O.integral(v)
    assert S.shape == (14, 18)
    for (x0, y0, x1, y1) in [(0, 0, 17, 13), (3, 2, 9, 11), (16, 12, 17, 13), (5, 5, 5, 9)]:
        got = S[y1, x1] - S[y0, x1] - S[y1, x0] + S[y0, x0]
        assert got == v[y0:y1, x0:x1].sum()


def _windows_brute(v, dp):
    H, W = v.shape
    top = H // 3 if dp.top is None else dp.top
    out = []
    for (w, h) in dp.sizes:
        sx, sy = max(w // 2, 1), max(h // 2, 1)
        for y0 in range(top, H - h + 1, sy):
            for x0 in range(0, W - w + 1, sx):
                if v[y0:y0 + h, x0:x0 + w].sum() >= dp.thresh * w * h:
                    out.append((x0, y0, x0 + w, y0 + h))
    return out


def test_sliding_windows_match_brute_force_in_order():
    rng = np.random.default_rng(4)
    v = (rng.random((90, 140)) < 0.2).astype(np.int32) * rng.integers(0, 200, (90, 140)).astype(np.int32)
    v[40:70, 30:80] = 40
    dp = O.DetectParams(sizes=((20, 20), (30, 20), (11, 7)), thresh=16, max_detections=100000)
    boxes, fired = O.detect_windows(O.integral(v), dp)
    want = _windows_brute(v, dp)
    assert fired == len(want)
    assert [tuple(b) for b in boxes] == want


def test_window_count_on_a_constant_map_and_the_cap():
    H, W = 120, 200
    v = np.full((H, W), 16, np.int32)
    dp = O.DetectParams(max_detections=100000)
    _, fired = O.detect_windows(O.integral(v), dp)
    top = H // 3
    n = 0
    for (w, h) in dp.sizes:
        n += ((W - w) // (w // 2) + 1) * ((H - top - h) // (h // 2) + 1)
    assert fired == n
    capped, fired2 = O.detect_windows(O.integral(v), O.DetectParams(max_detections=7))
    assert fired2 == n and len(capped) == 7
    # one below the level fires nothing
    _, none = O.detect_windows(O.integral(v - 1), dp)
    assert none == 0


def test_merge_two_overlapping_boxes():
    out = O.merge_boxes([(0, 0, 10, 10), (5, 0, 15, 10)])
    assert out.tolist() == [[0, 0, 15, 10]]


def test_disjoint_and_touching_boxes_stay():
    boxes = [(0, 0, 10, 10), (10, 0, 20, 10), (30, 30, 40, 45)]
    assert O.merge_boxes(boxes).tolist() == [list(b) for b in boxes]


def test_merge_takes_the_highest_iou_pair_first():
    # IoU(A,B) = 50/150, IoU(B,C) = 80/120, IoU(A,C) = 30/170; threshold 0.3.
    # B,C merge first into (5,0,17,10); IoU with A is then 50/170 < 0.3.
    # (Merging the first pair above the threshold, A,B, would end in one box.)
    boxes = [(0, 0, 10, 10), (5, 0, 15, 10), (7, 0, 17, 10)]
    assert O.merge_boxes(boxes, merge_iou=0.3).tolist() == [[0, 0, 10, 10], [5, 0, 17, 10]]


def test_merged_box_takes_the_earlier_place_and_chains_grow():
    # C overlaps nothing at first; the union of A and B reaches it
    boxes = [(0, 0, 10, 10), (50, 0, 60, 10), (8, 0, 52, 4), (100, 100, 110, 110)]
    # IoU(A,C) = 8/(100+176-8); IoU(B,C) = 8/268 too: tie -> the pair (A,C) first
    out = O.merge_boxes(boxes)
    assert out.tolist() == [[0, 0, 60, 10], [100, 100, 110, 110]]


def test_small_boxes_are_discarded_in_order():
    boxes = [(0, 0, 10, 10), (50, 50, 90, 90), (200, 0, 230, 30)]
    assert O.merge_boxes(boxes, min_area=900).tolist() == [[50, 50, 90, 90], [200, 0, 230, 30]]


def _scene(W, H, rects, diff):
    dhat = np.full((H, W), 0.0)
    dz = dhat.copy()
    for (x0, y0, x1, y1) in rects:
        dz[y0:y1, x0:x1] = diff
    return dhat, dz, np.full((H, W), O.PRED, np.uint8)


def test_one_object_gives_one_box_spanning_the_fired_windows():
    W, H = 260, 150
    obj = (100, 80, 160, 125)
    dhat, dz, fl = _scene(W, H, [obj], 4.0)
    dp = O.DetectParams()
    boxes, fired = O.detect(dhat, dz, fl, dp)
    v = O.motion_values(dhat, dz, fl)
    want = np.array(_windows_brute(v, dp))
    assert fired == len(want) > 0
    assert boxes.tolist() == [[want[:, 0].min(), want[:, 1].min(), want[:, 2].max(), want[:, 3].max()]]
    x0, y0, x1, y1 = boxes[0]
    assert x0 <= obj[0] and y0 <= obj[1] and x1 >= obj[2] and y1 >= obj[3]


def test_two_objects_two_boxes_and_the_top_third_is_ignored():
    W, H = 400, 180
    a, b, top = (40, 100, 100, 150), (280, 90, 340, 140), (180, 5, 240, 55)
    dhat, dz, fl = _scene(W, H, [a, b, top], 5.0)
    boxes, _ = O.detect(dhat, dz, fl)
    assert len(boxes) == 2
    # list order follows the first window of each group: b starts higher
    (r, l) = boxes
    assert l[0] <= a[0] and l[2] >= a[2] and l[2] < b[0]
    assert r[0] <= b[0] and r[2] >= b[2]
    assert boxes[:, 1].min() >= H // 3


def test_static_scene_and_missing_predictions_give_nothing():
    W, H = 200, 120
    dhat, dz, fl = _scene(W, H, [(50, 60, 120, 110)], 6.0)
    assert O.detect(dhat, dhat.copy(), fl)[0].shape == (0, 4)
    assert O.detect(dhat, dz, np.zeros_like(fl))[0].shape == (0, 4)


def test_merging_every_overlap_ends_in_disjoint_bounding_boxes():
    # with merge_iou = 0 the grouping stops only when no two boxes overlap;
    # every input lies in exactly one result, and each result is the
    # bounding box of the inputs inside it
    rng = np.random.default_rng(11)
    for _ in range(40):
        n = int(rng.integers(1, 40))
        xy = rng.integers(0, 150, (n, 2))
        wh = rng.integers(1, 35, (n, 2))
        boxes = np.concatenate([xy, xy + wh], axis=1).astype(np.int32)
        out = O.merge_boxes(boxes)
        for a in range(len(out)):
            for b in range(a + 1, len(out)):
                ia = min(out[a][2], out[b][2]) - max(out[a][0], out[b][0])
                ib = min(out[a][3], out[b][3]) - max(out[a][1], out[b][1])
                assert not (ia > 0 and ib > 0)
        inside = [[k for k in range(n) if out[j][0] <= boxes[k][0] and out[j][1] <= boxes[k][1]
                   and boxes[k][2] <= out[j][2] and boxes[k][3] <= out[j][3]] for j in range(len(out))]
        assert sorted(k for ks in inside for k in ks) == list(range(n))
        for j, ks in enumerate(inside):
            sub = boxes[ks]
            assert out[j].tolist() == [sub[:, 0].min(), sub[:, 1].min(), sub[:, 2].max(), sub[:, 3].max()]
