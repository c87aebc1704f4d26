"""Batched streams (concurrent lanes) against independent contexts."""
import sys

import numpy as np
import pytest

import stereo_synth as synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle as O  # noqa: E402
import paper_1809_07986_amd as sgmk  # noqa: E402
from paper_1809_07986_amd import _native as NAT  # noqa: E402

D_TOL = 1e-4
P_TOL = 1e-4


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


STREAMS = [  # uneven sizes and disparity ranges
    dict(width=320, height=96, max_disp=64, f=350.0, seed=11),
    dict(width=200, height=72, max_disp=32, f=160.0, seed=12),
    dict(width=256, height=128, max_disp=96, f=300.0, seed=13),
    dict(width=180, height=64, max_disp=48, f=250.0, seed=14),
]


def _sequences(frames=3):
    out = []
    for st in STREAMS:
        out.append(synth.make_sequence("tiny", frames=frames, seed=st["seed"], width=st["width"],
                                       height=st["height"], max_disp=st["max_disp"], f=st["f"]))
    return out


def _states(ctxs):
    res = []
    for c in ctxs:
        d, p, f = (t.cpu().numpy() for t in c.get_state())
        res.append((d, p, f, c.motion_mask().cpu().numpy()))
    return res


def _batch(seqs):
    b = sgmk.SgmBatch([dict(width=st["width"], height=st["height"], max_disp=st["max_disp"], f=st["f"],
                            baseline=0.54) for st in STREAMS])
    for i, q in enumerate(seqs):
        b.load(i, q.left[0], q.right[0])
    b.full()
    return b


def test_batch_matches_independent_contexts():
    seqs = _sequences()
    _say("case: batch of 4 uneven streams vs single contexts")
    b = _batch(seqs)
    singles = []
    for st, q in zip(STREAMS, seqs):
        g = sgmk.ReducedSGM(st["width"], st["height"], st["max_disp"], f=st["f"], baseline=0.54)
        g.full_frame(q.left[0], q.right[0])
        singles.append(g)
    for k in (1, 2, 1):        # the third step revisits frame 1 (same motion as the first)
        Ts = [q.T[2] if k == 2 else q.T[1] for q in seqs]
        for i, q in enumerate(seqs):
            b.load(i, q.left[k], q.right[k])
        b.step(np.stack(Ts))
        for g, q, T in zip(singles, seqs, Ts):
            g.reduced_frame(q.left[k], q.right[k], T)
        torch.cuda.synchronize()
        for i, (a, s) in enumerate(zip(_states(b.contexts), _states(singles))):
            for x, y in zip(a, s):
                assert np.array_equal(x, y), (k, i)
        _say(f"step {k}: identical")


def test_batch_streams_match_oracle():
    # every stream of an uneven batch against its own oracle filter, frame by
    # frame: state, mask, windows, winners and measurements (Section 2.4,
    # Eq. 2-6 per stream; the batch only changes where the work runs)
    seqs = _sequences()
    _say("case: batch of 4 uneven streams vs the oracle")
    b = _batch(seqs)
    oracles = []
    for st, q in zip(STREAMS, seqs):
        F = O.OracleFilter(O.Params(st["width"], st["height"], st["max_disp"], f=st["f"], baseline=0.54))
        F.full_frame(q.left[0], q.right[0])
        oracles.append(F)
    for k in (1, 2):
        Ts = [q.T[k] for q in seqs]
        for i, q in enumerate(seqs):
            b.load(i, q.left[k], q.right[k])
        b.step(np.stack(Ts))
        for F, q, T in zip(oracles, seqs, Ts):
            F.reduced_frame(q.left[k], q.right[k], T)
        torch.cuda.synchronize()
        for i, (c, F) in enumerate(zip(b.contexts, oracles)):
            d, p, sf = (t.cpu().numpy() for t in c.get_state())
            assert np.max(np.abs(d - F.d)) <= D_TOL, (k, i)
            assert np.max(np.abs(p - F.p) / np.maximum(F.p, 1e-12)) <= P_TOL, (k, i)
            assert np.array_equal(sf, F.sflags), (k, i)
            assert np.array_equal(c.motion_mask().cpu().numpy(), F.mask), (k, i)
            assert np.array_equal(c.stage(NAT.STAGE_LO).cpu().numpy(), F.lo), (k, i)
            assert np.array_equal(c.stage(NAT.STAGE_HI).cpu().numpy(), F.hi), (k, i)
            assert np.array_equal(c.stage(NAT.STAGE_DSTAR).cpu().numpy(), F.dstar), (k, i)
            assert np.array_equal(c.stage(NAT.STAGE_FLAGS).cpu().numpy(), F.flags), (k, i)
            assert np.max(np.abs(c.stage(NAT.STAGE_DZ).cpu().numpy() - F.dz)) <= D_TOL, (k, i)
        _say(f"step {k}: every stream matches its oracle")


@pytest.mark.skip(reason="captured-graph stepping is disabled in the library: its first run crashed the host "
                         "process inside stream capture and the cause has not been shown")
def test_batch_graph_replays_equal_eager():
    seqs = _sequences()
    _say("case: graph replays vs eager batch steps")
    b1 = _batch(seqs)
    b2 = _batch(seqs)
    Ts = np.stack([q.T[1] for q in seqs])
    for r in range(4):
        for i, q in enumerate(seqs):
            b1.load(i, q.left[1 + r % 2], q.right[1 + r % 2])
            b2.load(i, q.left[1 + r % 2], q.right[1 + r % 2])
        b1.step_graph(Ts)
        b2.step(Ts)
        torch.cuda.synchronize()
        _ = b1.contexts[0].disparity().sum().item()    # eager work between replays
        for a, s in zip(_states(b1.contexts), _states(b2.contexts)):
            for x, y in zip(a, s):
                assert np.array_equal(x, y), r


def test_batch_graph_stepping_reports_disabled():
    b = sgmk.SgmBatch([dict(width=32, height=16, max_disp=16)])
    with pytest.raises(sgmk.SgmError) as e:
        b.step_graph(np.eye(4)[None])
    assert e.value.code == -1


def test_batch_schedules_give_identical_results():
    seqs = _sequences()
    Ts = np.stack([q.T[1] for q in seqs])
    ref = None
    for lanes, order in ((1, 0), (2, 1), (4, 0), (3, 1)):
        b = _batch(seqs)
        b.set_schedule(lanes, order)
        for i, q in enumerate(seqs):
            b.load(i, q.left[1], q.right[1])
        b.step(Ts)
        torch.cuda.synchronize()
        st = _states(b.contexts)
        if ref is None:
            ref = st
        else:
            for a, s in zip(ref, st):
                for x, y in zip(a, s):
                    assert np.array_equal(x, y), (lanes, order)


def test_batch_autotune_keeps_state_and_schedule_is_valid():
    seqs = _sequences()
    b = _batch(seqs)
    Ts = np.stack([q.T[1] for q in seqs])
    for i, q in enumerate(seqs):
        b.load(i, q.left[1], q.right[1])
    torch.cuda.synchronize()
    before = _states(b.contexts)
    lanes, order = b.autotune(Ts, reps=2)
    torch.cuda.synchronize()
    after = _states(b.contexts)
    assert 1 <= lanes <= 16 and order in (0, 1)
    for a, s in zip(before, after):
        for x, y in zip(a, s):
            assert np.array_equal(x, y)
    # stepping after tuning still matches an untuned batch
    b2 = _batch(seqs)
    for i, q in enumerate(seqs):
        b2.load(i, q.left[1], q.right[1])
    b.step(Ts)
    b2.step(Ts)
    torch.cuda.synchronize()
    for a, s in zip(_states(b.contexts), _states(b2.contexts)):
        for x, y in zip(a, s):
            assert np.array_equal(x, y)


def test_batch_step_before_full_is_an_error():
    b = sgmk.SgmBatch([dict(width=32, height=16, max_disp=16)])
    with pytest.raises(sgmk.SgmError) as e:
        b.step(np.eye(4)[None])
    assert e.value.code == -4
