"""Batched streams (concurrent lanes, captured graphs) against independent contexts and the oracle."""
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


GRAPH_OFF = ("captured-graph stepping is disabled in the library: capturing a batch step crashed the host "
             "process inside hipStreamEndCapture and the cause has not been shown")


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


@pytest.mark.skip(reason=GRAPH_OFF)
@pytest.mark.parametrize("side_stream", [False, True])
def test_batch_graph_replays_equal_eager(side_stream):
    # the captured step replayed several times (new frames copied into the
    # default buffers before each replay, eager work and synchronisations in
    # between), on the current torch stream or a created one; every replay
    # must equal an eager step of a second batch
    seqs = _sequences()
    _say(f"case: graph replays vs eager batch steps (side stream {side_stream})")
    b1 = _batch(seqs)
    b2 = _batch(seqs)
    st = torch.cuda.Stream() if side_stream else torch.cuda.current_stream()
    for r in range(4):
        k = 1 + r % 2
        Ts = np.stack([q.T[k] for q in seqs])
        with torch.cuda.stream(st):
            for i, q in enumerate(seqs):
                b1.load(i, q.left[k], q.right[k])
            b1.step_graph(Ts)
        for i, q in enumerate(seqs):
            b2.load(i, q.left[k], q.right[k])
        b2.step(Ts)
        torch.cuda.synchronize()
        _ = b1.contexts[0].disparity().sum().item()    # eager work between replays
        for i, (a, s_) in enumerate(zip(_states(b1.contexts), _states(b2.contexts))):
            for x, y in zip(a, s_):
                assert np.array_equal(x, y), (r, i)
        _say(f"  replay {r}: identical to the eager step")


@pytest.mark.skip(reason=GRAPH_OFF)
def test_batch_graph_replay_matches_oracle():
    seqs = _sequences()
    _say("case: graph replays vs the oracle")
    b = _batch(seqs)
    oracles = []
    for st, q in zip(STREAMS, seqs):
        F = O.OracleFilter(O.Params(st["width"], st["height"], st["max_disp"], f=st["f"], baseline=0.54))
        F.full_frame(q.left[0], q.right[0])
        oracles.append(F)
    for k in (1, 2):
        Ts = np.stack([q.T[k] for q in seqs])
        for i, q in enumerate(seqs):
            b.load(i, q.left[k], q.right[k])
        b.step_graph(Ts)
        torch.cuda.synchronize()
        for i, (c, F, q) in enumerate(zip(b.contexts, oracles, seqs)):
            F.reduced_frame(q.left[k], q.right[k], q.T[k])
            d, p, sf = (t.cpu().numpy() for t in c.get_state())
            assert np.max(np.abs(d - F.d)) <= D_TOL, (k, i)
            assert np.max(np.abs(p - F.p) / np.maximum(F.p, 1e-12)) <= P_TOL, (k, i)
            assert np.array_equal(sf, F.sflags), (k, i)
            assert np.array_equal(c.motion_mask().cpu().numpy(), F.mask), (k, i)
            assert np.array_equal(c.stage(NAT.STAGE_DSTAR).cpu().numpy(), F.dstar), (k, i)


def test_batch_graph_stepping_reports_disabled():
    b = sgmk.SgmBatch([dict(width=32, height=16, max_disp=16)])
    b.full()
    with pytest.raises(sgmk.SgmError) as e:
        b.step_graph(np.eye(4)[None])
    assert e.value.code == NAT.SGM_EINVAL


def test_batch_step_with_images_and_full_rows():
    # per-step image arrays (not the default buffers) and a row asking one
    # stream for a full-range frame, against single contexts
    seqs = _sequences()
    _say("case: batch step with per-step images and a full-range row")
    b = _batch(seqs)
    singles = []
    for st, q in zip(STREAMS, seqs):
        g = sgmk.ReducedSGM(st["width"], st["height"], st["max_disp"], f=st["f"], baseline=0.54)
        g.full_frame(q.left[0], q.right[0])
        singles.append(g)
    Ts = np.stack([q.T[1] for q in seqs])
    Ts[2, 3, 3] = 0.0                       # stream 2: full range
    images = [(torch.as_tensor(q.left[1]).cuda(), torch.as_tensor(q.right[1]).cuda()) for q in seqs]
    b.step(Ts, images=images)
    for i, (g, q) in enumerate(zip(singles, seqs)):
        if i == 2:
            g.full_frame(q.left[1], q.right[1])
        else:
            g.reduced_frame(q.left[1], q.right[1], q.T[1])
    torch.cuda.synchronize()
    for i, (a, s_) in enumerate(zip(_states(b.contexts), _states(singles))):
        for x, y in zip(a, s_):
            assert np.array_equal(x, y), i


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


@pytest.mark.parametrize("budget", [False, True])
def test_batch_autotune_keeps_state_and_schedule_is_valid(budget):
    seqs = _sequences()
    b = _batch(seqs)
    Ts = np.stack([q.T[1] for q in seqs])
    for i, q in enumerate(seqs):
        b.load(i, q.left[1], q.right[1])
    if budget:
        b.step(Ts)                            # sgm_autotune uses the last ego-motions
    torch.cuda.synchronize()
    before = _states(b.contexts)
    if budget:
        b.autotune_budget(200)
    else:
        lanes, order, seg, alt = b.autotune(Ts, reps=2)
        assert 1 <= lanes <= 16 and order in (0, 1) and seg in (48, 72, 96, 128) and alt in (0, 1)
    torch.cuda.synchronize()
    after = _states(b.contexts)
    for a, s_ in zip(before, after):
        for x, y in zip(a, s_):
            assert np.array_equal(x, y)
    # stepping after tuning still matches an untuned batch
    b2 = _batch(seqs)
    for i, q in enumerate(seqs):
        b2.load(i, q.left[1], q.right[1])
    if budget:
        b2.step(Ts)
    b.step(Ts)
    b2.step(Ts)
    torch.cuda.synchronize()
    for a, s_ in zip(_states(b.contexts), _states(b2.contexts)):
        for x, y in zip(a, s_):
            assert np.array_equal(x, y)


def test_batch_step_before_full_is_an_error():
    b = sgmk.SgmBatch([dict(width=32, height=16, max_disp=16)])
    with pytest.raises(sgmk.SgmError) as e:
        b.step(np.eye(4)[None])
    assert e.value.code == -4
