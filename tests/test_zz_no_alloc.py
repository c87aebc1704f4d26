"""Allocation-free detection (sgm_detect_noalloc) against sgm_detect, through the C ABI.

The allocation-free entry point runs the same kernels on scratch held in a
library-wide device array; its boxes and counts must equal those of the
detector-object entry point bit for bit (integer work), on two calls in a row
where the second has a smaller input, so stale scratch contents of the first
call would show.  The boxes are also checked against the oracle.
"""
import ctypes
import sys

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1809_07986_amd as sgmk  # noqa: E402
from paper_1809_07986_amd import _native as NAT  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _scene(W, H, seed, n_obj):
    rng = np.random.default_rng(seed)
    dhat = rng.uniform(0, 60, (H, W))
    dz = dhat + rng.normal(0, 0.6, (H, W))
    for _ in range(n_obj):
        w, h = int(rng.integers(20, 90)), int(rng.integers(20, 80))
        x0, y0 = int(rng.integers(0, W - w)), int(rng.integers(H // 3, H - h))
        dz[y0:y0 + h, x0:x0 + w] += rng.uniform(2, 8) * rng.choice([-1, 1])
    fl = np.full((H, W), O.PRED, np.uint8)
    fl[rng.random((H, W)) < 0.05] = 0
    return dhat, dz, fl


def _noalloc(W, H, prm, dhat, dz, fl, boxes, count):
    lib = NAT.load()
    dh = torch.as_tensor(dhat).cuda().contiguous()
    z = torch.as_tensor(dz).cuda().contiguous()
    f = torch.as_tensor(fl).cuda().contiguous()
    s = torch.cuda.current_stream().cuda_stream
    rc = lib.sgm_detect_noalloc(W, H, ctypes.byref(prm), dh.data_ptr(), z.data_ptr(), f.data_ptr(),
                                boxes.data_ptr(), count.data_ptr(), ctypes.c_void_p(s))
    assert rc == 0, NAT.load().sgm_last_error()
    torch.cuda.synchronize()
    n, fired = (int(v) for v in count.cpu())
    return boxes[:n].cpu().numpy(), fired


def test_noalloc_detection_equals_the_detector_on_two_calls():
    boxes = torch.full((NAT.DETECT_MAX, 4), -7, dtype=torch.int32, device="cuda")
    count = torch.full((2,), -7, dtype=torch.int32, device="cuda")
    # the larger input first, then a smaller one: scratch holds the first call's data
    for (W, H, seed, kw) in ((1242, 375, 11, dict()),
                             (333, 170, 12, dict(thresh=6, merge_iou=0.05, min_area=100,
                                                 sizes=((12, 12), (20, 20), (20, 36))))):
        _say(f"noalloc detection {W}x{H} seed={seed} {kw}")
        dhat, dz, fl = _scene(W, H, seed, 8)
        det = sgmk.Detector(W, H, **kw)
        want_boxes, want_fired = det.detect(dhat, dz, fl)
        torch.cuda.synchronize()
        want_boxes = want_boxes.cpu().numpy()
        got_boxes, got_fired = _noalloc(W, H, det.params, dhat, dz, fl, boxes, count)
        assert got_fired == want_fired
        assert np.array_equal(got_boxes, want_boxes), (got_boxes, want_boxes)
        p = det.params
        dp = O.DetectParams(sizes=tuple((p.sizes[k][0], p.sizes[k][1]) for k in range(p.n_sizes)), top=p.top,
                            scale=p.scale, cap=p.cap, thresh=p.thresh, max_detections=p.max_detections,
                            min_area=p.min_area, merge_iou=p.merge_iou)
        ob, of = O.detect(dhat, dz, fl, dp)
        assert of == got_fired and np.array_equal(ob, got_boxes)
        assert got_fired > 0 and len(got_boxes) > 0
        _say(f"  {got_fired} windows fired, {len(got_boxes)} boxes")
        det.close()


def test_noalloc_rejects_a_scratch_need_beyond_the_maximum():
    lib = NAT.load()
    prm = sgmk.detect_params(4096, 4096, top=0)
    t = torch.zeros(16, dtype=torch.float64, device="cuda")
    out = torch.zeros(16, dtype=torch.int32, device="cuda")
    rc = lib.sgm_detect_noalloc(4096, 4096, ctypes.byref(prm), t.data_ptr(), t.data_ptr(), t.data_ptr(),
                                out.data_ptr(), out.data_ptr(), None)
    assert rc == NAT.SGM_EINVAL
    assert b"scratch" in lib.sgm_last_error()
    assert lib.sgm_detect_noalloc(100, 100, None, t.data_ptr(), t.data_ptr(), t.data_ptr(), out.data_ptr(),
                                  out.data_ptr(), None) == NAT.SGM_EINVAL
