"""Gate re-run (Section 4's innovation test, then a second matching pass):
the sparse second pass against the dense one, through the C ABI.

A context without debug stages recomputes, along each path, only from the
widened pixels until the path losses rejoin the first pass's, and runs the
WTA and the correction on the pixels it changed.  Its per-pixel results must
equal, bit for bit, those of the two dense routes: the device-side fallback
(SGM_DEBUG_DENSE_RERUN) and a debug-stages context, which matches every pixel
again exactly as before.  The dense second pass itself is compared with the
oracle in tests/test_gpu_learned.py (tiny and 1242x375x256 learned frames),
which now run the sparse route as well.

Tolerance: bit for bit on flags, windows, winners, sub-pixel measurements,
innovations, filter state, masks and the cell count.
"""
import sys

import numpy as np
import pytest

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


def _outputs(g):
    d, p, sf = (_np(t) for t in g.get_state())
    out = {k: _np(g.stage(s)) for k, s in (("flags", NAT.STAGE_FLAGS), ("lo", NAT.STAGE_LO), ("hi", NAT.STAGE_HI),
                                            ("dstar", NAT.STAGE_DSTAR), ("dz", NAT.STAGE_DZ), ("nu", NAT.STAGE_NU))}
    out.update(d=d, p=p, sflags=sf, mask=_np(g.motion_mask()), cells=np.array([g.cost_cells()]))
    return out


def _compare_routes(seq, D, frames=(1, 2, 3), label="", model=None, extra=(), **over):
    """Run the three routes on the same frames and compare them; return the
    number of widened pixels over those frames and the three contexts."""
    W, H = seq.cam.width, seq.cam.height
    _say(f"gate re-run routes, {W}x{H}x{D} {label}, frames {frames}")
    routes = {"plain": NAT.DEBUG_STAGES, "sparse": 0, "fallback": NAT.DEBUG_DENSE_RERUN}
    ctx = {}
    for name, dbg in routes.items():
        g = sgmk.ReducedSGM(W, H, D, f=seq.cam.f, baseline=seq.cam.baseline, gate_rerun=1, **over)
        g.set_debug(dbg)
        if model is not None:
            g.set_window_model(model)
        g.full_frame(seq.left[0], seq.right[0])
        ctx[name] = g
    failed = 0
    for k in frames:
        outs = {}
        for name, g in ctx.items():
            g.reduced_frame(seq.left[k], seq.right[k], seq.T[k])
            torch.cuda.synchronize()
            outs[name] = _outputs(g)
            outs[name].update({f"stage{st}": _np(g.stage(st)) for st in extra})
        ref = outs["plain"]
        for name in ("sparse", "fallback"):
            for key, v in ref.items():
                assert np.array_equal(outs[name][key], v), (D, label, k, name, key)
        nfail = int(((ref["flags"] & NAT.FLAG_GATEFAIL) != 0).sum())
        # the device-side counts: widened = GATEFAIL pixels, moved <= widened,
        # added cells <= widened * (D - 1); equal on every route
        counts = [_np(g.stage(NAT.STAGE_RERUN)).tolist() for g in ctx.values()]
        assert counts[0][0] == nfail and counts[0][1] <= nfail and counts[0][2] <= nfail * (D - 1), counts
        assert counts[1] == counts[0] and counts[2] == counts[0], counts
        failed += nfail
    _say(f"  widened pixels: {failed} of {len(frames) * W * H}")
    return failed, ctx


# D = 37, 64, 128, 160, 256: one to four 64-disparity chunks per lane in the walk
# (37: full-range blocks at offsets that are not multiples of four)
@pytest.mark.parametrize("D", [37, 64, 128, 160, 256])
def test_sparse_rerun_equals_dense(D):
    seq = synth.make_sequence("driving", frames=4, width=640, height=192, seed=7)
    W, H = seq.cam.width, seq.cam.height
    failed, ctx = _compare_routes(seq, D)
    assert failed > 0, "the moving cars should fail the innovation test"
    # the sparse route kept the first pass's offsets: their read-back is refused
    with pytest.raises(sgmk.SgmError):
        ctx["sparse"].stage(NAT.STAGE_OFFSETS)
    with pytest.raises(sgmk.SgmError):
        ctx["sparse"].stage(NAT.STAGE_PATH0)
    # the dense routes keep the plain layout
    assert ctx["fallback"].stage(NAT.STAGE_OFFSETS).numel() == W * H + 1
    for g in ctx.values():
        g.close()


def test_sparse_rerun_when_every_pixel_fails():
    # a gate nothing passes: every predicted pixel is widened, whole 64-pixel
    # batches of every scanline are moved, and the full-range blocks fill most
    # of the room reserved behind the first pass's cells
    seq = synth.make_sequence("driving", frames=3, width=640, height=192, seed=7)
    failed, ctx = _compare_routes(seq, 128, frames=(1, 2), label="gate 1e-12", chi2_gate=1e-12)
    n = seq.cam.width * seq.cam.height
    assert failed > 1.6 * n, "nearly every pixel should fail the innovation test"
    for g in ctx.values():
        g.close()


@pytest.mark.parametrize("mask", [0x0F, 0xF0, 0x41])
def test_sparse_rerun_path_subsets(mask):
    # subsets of the paths (Table 2's sets and a pair) with the paper's census
    # and penalties (Table 1)
    seq = synth.make_sequence("driving", frames=3, width=640, height=192, seed=7)
    failed, ctx = _compare_routes(seq, 128, frames=(1, 2), label=f"paths 0x{mask:02x}", path_mask=mask,
                                  census_w=5, census_h=5, p1=6, p2=65)
    assert failed > 0
    for g in ctx.values():
        g.close()


def test_sparse_rerun_tall_image():
    # taller than wide: most diagonal scanlines enter through the side borders
    seq = synth.make_sequence("tiny", frames=3, width=40, height=120, seed=5)
    failed, ctx = _compare_routes(seq, 32, frames=(1, 2), label="40x120", chi2_gate=0.5)
    assert failed > 0
    for g in ctx.values():
        g.close()


def test_sparse_rerun_small_image():
    # scanlines shorter than one 64-pixel batch, and more disparities than columns
    seq = synth.make_sequence("tiny", frames=3, width=37, height=19, seed=3)
    failed, ctx = _compare_routes(seq, 64, frames=(1, 2), label="37x19", chi2_gate=0.5)
    assert failed > 0
    for g in ctx.values():
        g.close()


def test_sparse_rerun_full_hd_learned():
    # the combined workload's stream size: 1920x1080, D = 256, learned windows
    # (shipped network) and near cars; many placement blocks, long scanlines
    seq = synth.make_sequence("learned", frames=3, width=1920, height=1080, seed=11, cars=10, near=2.4,
                              f=0.58 * 1920)
    failed, ctx = _compare_routes(seq, 256, frames=(1, 2), label="learned", model=sgmk.load_window_model(),
                                  window_mode=NAT.WIN_LEARNED)
    assert failed > 0
    for g in ctx.values():
        g.close()


def test_sparse_rerun_with_curvature_variance():
    # per-pixel measurement variance from the cost curvature (r_curv): the
    # sparse pass's WTA writes kappa and r only for the pixels it changed
    seq = synth.make_sequence("driving", frames=3, width=640, height=192, seed=7)
    failed, ctx = _compare_routes(seq, 128, frames=(1, 2), label="r_curv", r_curv=8.31,
                                  extra=(NAT.STAGE_KAPPA, NAT.STAGE_RPIX))
    assert failed > 0
    for g in ctx.values():
        g.close()


def test_sparse_rerun_in_a_batch():
    # the batched step runs every stream's frame, second pass included, on
    # concurrent lanes: each stream against a single context on the dense route
    streams = [dict(width=320, height=96, max_disp=64, f=350.0, seed=11),
               dict(width=256, height=128, max_disp=96, f=300.0, seed=13),
               dict(width=200, height=72, max_disp=160, f=160.0, seed=12)]
    seqs = [synth.make_sequence("tiny", frames=3, seed=st["seed"], width=st["width"], height=st["height"],
                                max_disp=st["max_disp"], f=st["f"]) for st in streams]
    prm = [dict(width=st["width"], height=st["height"], max_disp=st["max_disp"], f=st["f"], baseline=0.54,
                gate_rerun=1, chi2_gate=0.5) for st in streams]
    _say("gate re-run in a batch of 3 uneven streams vs single dense-route contexts")
    b = sgmk.SgmBatch(prm)
    singles = []
    for i, (pr, q) in enumerate(zip(prm, seqs)):
        b.load(i, q.left[0], q.right[0])
        g = sgmk.ReducedSGM(**pr)
        g.set_debug(NAT.DEBUG_STAGES)
        g.full_frame(q.left[0], q.right[0])
        singles.append(g)
    b.full()
    failed = 0
    for k in (1, 2):
        for i, q in enumerate(seqs):
            b.load(i, q.left[k], q.right[k])
        b.step(np.stack([q.T[k] for q in seqs]))
        for g, q in zip(singles, seqs):
            g.reduced_frame(q.left[k], q.right[k], q.T[k])
        torch.cuda.synchronize()
        for i, (c, g) in enumerate(zip(b.contexts, singles)):
            got, ref = _outputs(c), _outputs(g)
            for key, v in ref.items():
                assert np.array_equal(got[key], v), (k, i, key)
            failed += int(((ref["flags"] & NAT.FLAG_GATEFAIL) != 0).sum())
    _say(f"  widened pixels: {failed}")
    assert failed > 0
    for g in singles:
        g.close()
