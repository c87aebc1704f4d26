"""Train the learned search window on the GPU with the library's kernels.

Data: seeded "learned" sequences (1242x375, disparities 0-255, 50 frames,
cars as near as 1.6 m).  For every frame k >= 1 of a training sequence the
k-sigma filter's prediction supplies the network input (sgm_get_features)
and a full-range match of the same frame supplies the targets
(sgm_learned_targets): the residual of the prediction against the
full-range measurement and the residual of the full-range measurement
against the scene's ground truth.  Training runs forward, loss, backward and
Adam through sgm_cnn_train_step.

Evaluation on held-out sequences compares, per frame, the matched cells and
the fraction of valid pixels whose filtered disparity is off by more than
3 px for: the k-sigma windows, the learned windows, the learned windows with
the gate re-run, and full-range matching of every frame.

    python -m paper_1809_07986_amd.train_window --out gpurun_out/window_cnn

Writes <out>/window_cnn.f32 (the parameters, little-endian float32, layout
of include/sgm.h) and <out>/window_cnn.json (settings, losses, evaluation).
Rendering runs in a pool of CPU worker processes forked before the GPU is
first used.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

import stereo_synth

LAYERS = ((4, 16), (16, 32), (32, 32), (32, 16), (16, 2))


def _render(job):
    seed, frames = job
    seq = stereo_synth.make_sequence("learned", frames=frames, seed=seed, cache=False)
    gt = np.where(seq.valid, seq.disp_gt, -1).astype(np.float32)
    return seed, seq.left, seq.right, gt, seq.T, seq.cam.f, seq.cam.baseline, seq.max_disp


def init_params(seed: int) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    out = []
    for ci, co in LAYERS:
        out.append((rng.standard_normal((co, 3, 3, ci)) * math.sqrt(2.0 / (9 * ci))).reshape(-1))
        out.append(np.zeros(co))
    return np.concatenate(out).astype(np.float32)


def _log(msg):
    print(msg, flush=True)


def collect(pool, seeds, frames, torch, sgmk, N, keep_data=True):
    """Network inputs and targets of every frame k >= 1 of the sequences."""
    feats, tgts = [], []
    ctx = full = None
    jobs = [(s, frames) for s in seeds]
    for seed, L, R, GT, T, f, B, D in pool.map(_render, jobs):
        H, W = L.shape[1:]
        if ctx is None:
            ctx = sgmk.ReducedSGM(W, H, D, f=f, baseline=B)
            full = sgmk.ReducedSGM(W, H, D, f=f, baseline=B)
        ctx.full_frame(L[0], R[0])
        for k in range(1, L.shape[0]):
            ctx.reduced_frame(L[k], R[k], T[k])
            feats.append(ctx.features(L[k]).clone())
            full.full_frame(L[k], R[k])
            tgts.append(ctx.learned_targets(full.stage(N.STAGE_DZ), torch.from_numpy(GT[k])).clone())
        torch.cuda.synchronize()
        _log(f"  sequence {seed}: {len(feats)} frames collected")
    return torch.stack(feats), torch.stack(tgts)


def evaluate(pool, seeds, frames, theta, torch, sgmk, N, ks=(3.0,)):
    """Per-variant mean cells per frame and bad-pixel rates (> 3 px)."""
    variants = {}
    for k in ks:
        variants["ksigma" if k == 3.0 else f"ksigma_{k:g}"] = dict(k_sigma=k)
    variants.update({"learned": dict(window_mode=N.WIN_LEARNED),
                     "learned_rerun": dict(window_mode=N.WIN_LEARNED, gate_rerun=1), "full": None})
    acc = {v: dict(cells=0.0, bad_d=0.0, bad_dz=0.0, valid=0.0, frames=0) for v in variants}
    ctxs = {}
    for seed, L, R, GT, T, f, B, D in pool.map(_render, [(s, frames) for s in seeds]):
        H, W = L.shape[1:]
        for name, kw in variants.items():
            if name not in ctxs:
                ctxs[name] = sgmk.ReducedSGM(W, H, D, f=f, baseline=B, **(kw or {}))
                if kw and kw.get("window_mode") == N.WIN_LEARNED:
                    ctxs[name].set_window_model(theta)
            g = ctxs[name]
            g.full_frame(L[0], R[0])
            for k in range(1, L.shape[0]):
                if kw is None:
                    g.full_frame(L[k], R[k])
                else:
                    g.reduced_frame(L[k], R[k], T[k])
                gt = torch.from_numpy(GT[k]).cuda()
                valid = gt >= 0
                d = g.disparity()
                dz = g.stage(N.STAGE_DZ)
                a = acc[name]
                a["cells"] += g.cost_cells()
                a["bad_d"] += float(((d - gt).abs() > 3)[valid].sum())
                a["bad_dz"] += float(((dz - gt.double()).abs() > 3)[valid].sum())
                a["valid"] += float(valid.sum())
                a["frames"] += 1
        _log(f"  evaluated sequence {seed}")
    res = {}
    for name, a in acc.items():
        res[name] = dict(cells_per_frame=a["cells"] / a["frames"], bad_px_d=a["bad_d"] / a["valid"],
                         bad_px_dz=a["bad_dz"] / a["valid"], frames=a["frames"])
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--train-seeds", default="4000-4039")
    ap.add_argument("--test-seeds", default="4100-4104")
    ap.add_argument("--frames", type=int, default=50)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--batch", type=int, default=2, help="frames per step")
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--out", default=os.path.join("gpurun_out", "window_cnn"))
    ap.add_argument("--eval-only", default=None, metavar="WEIGHTS",
                    help="evaluate these parameters instead of training")
    ap.add_argument("--eval-k", default="3", help="comma-separated k_sigma values to evaluate")
    args = ap.parse_args(argv)

    def seeds(spec):
        a, b = spec.split("-") if "-" in spec else (spec, spec)
        return list(range(int(a), int(b) + 1))

    t0 = time.time()
    # the render pool is forked before anything touches the GPU
    pool = cf.ProcessPoolExecutor(max_workers=args.workers, mp_context=mp.get_context("fork"))
    list(pool.map(time.sleep, [0.5] * args.workers))   # every worker started now
    import torch
    import paper_1809_07986_amd as sgmk
    from paper_1809_07986_amd import _native as N
    os.makedirs(args.out, exist_ok=True)
    train_seeds, test_seeds = seeds(args.train_seeds), seeds(args.test_seeds)
    ks = tuple(float(k) for k in args.eval_k.split(","))
    if args.eval_only:
        theta = np.fromfile(args.eval_only, dtype="<f4")
        ev = evaluate(pool, test_seeds, args.frames, theta, torch, sgmk, N, ks)
        for k, v in ev.items():
            _log(f"  {k}: {v}")
        with open(os.path.join(args.out, "evaluation.json"), "w") as fh:
            json.dump(dict(weights=args.eval_only, test_seeds=args.test_seeds, frames=args.frames, evaluation=ev),
                      fh, indent=1)
        pool.shutdown()
        return
    _log(f"collecting {len(train_seeds)} training sequences x {args.frames} frames")
    X, Y = collect(pool, train_seeds, args.frames, torch, sgmk, N)
    Xv, Yv = collect(pool, test_seeds[:1], args.frames, torch, sgmk, N)
    F, H, W = X.shape[:3]
    _log(f"  {F} training frames {H}x{W}, {time.time() - t0:.0f} s")
    tr = sgmk.CnnTrainer(args.batch, H, W)
    theta0 = init_params(args.seed)
    tr.set_params(theta0)
    rng = np.random.default_rng(args.seed)
    hist = []
    t1 = time.time()

    def val_loss():
        tot = 0.0
        nb = 0
        for i in range(0, Xv.shape[0] - args.batch + 1, args.batch):
            tr.forward(Xv[i:i + args.batch])
            tot += float(tr.loss_grad(Yv[i:i + args.batch]).item())
            nb += 1
        return tot / max(nb, 1)

    for step in range(args.steps):
        i = int(rng.integers(0, F - args.batch + 1))
        lr = args.lr * 0.5 * (1.0 + math.cos(math.pi * step / args.steps))
        loss = tr.train_step(X[i:i + args.batch], Y[i:i + args.batch], lr)
        if step % 100 == 0 or step == args.steps - 1:
            lv = float(loss.item())
            hist.append(dict(step=step, train_loss=lv))
            _log(f"  step {step}: loss {lv:.4f} lr {lr:.2e}")
    torch.cuda.synchronize()
    train_s = time.time() - t1
    theta = tr.get_params()
    v_end = val_loss()
    tr.set_params(theta0)
    v_start = val_loss()
    tr.set_params(theta)
    _log(f"held-out loss {v_start:.4f} -> {v_end:.4f}; training {train_s:.1f} s")
    theta.astype("<f4").tofile(os.path.join(args.out, "window_cnn.f32"))
    _log("evaluating on held-out sequences")
    ev = evaluate(pool, test_seeds, args.frames, theta, torch, sgmk, N, ks)
    for k, v in ev.items():
        _log(f"  {k}: {v}")
    meta = dict(train_seeds=args.train_seeds, test_seeds=args.test_seeds, frames=args.frames, steps=args.steps,
                batch=args.batch, lr=args.lr, init_seed=args.seed, training_frames=F, train_seconds=train_s,
                heldout_loss_init=v_start, heldout_loss_final=v_end, history=hist, evaluation=ev,
                command="python -m paper_1809_07986_amd.train_window " + " ".join(argv or sys.argv[1:]))
    with open(os.path.join(args.out, "window_cnn.json"), "w") as fh:
        json.dump(meta, fh, indent=1)
    pool.shutdown()
    _log(f"done in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
