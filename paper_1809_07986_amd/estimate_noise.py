"""Process and measurement noise from ground truth (Section 3).

Process noise q: the ground truth of frame k-1 is put into the filter state
and warped to frame k with the ego-motion (the prediction of Eq. 2-4); the
difference between that prediction and the ground truth of frame k, on
static pixels whose prediction came from a ground-truth pixel, is the
disparity error the ego-motion step introduces.  The ego-motion can be
perturbed (rotation and translation noise, standing in for an estimated
ego-motion) to see how q grows with ego-motion error.

Measurement noise r: every frame is matched over the full disparity range
(as at the filter's initialisation) and d_z is compared with the ground
truth on static pixels.

Both variances are the mean squared error of the errors within +-`inlier`
pixels (gross mismatches and warp outliers are counted separately), with the
fraction of errors inside +-1 px and the histograms.

    python -m paper_1809_07986_amd.estimate_noise --out gpurun_out/noise.json
"""
from __future__ import annotations

import argparse
import json
import math
import os

import numpy as np

RESET = 2


def noise_stats(err: np.ndarray, inlier: float = 3.0, bins: int = 60) -> dict:
    """Variance estimate (mean square of |e| <= inlier), bias, spread and histogram."""
    err = np.asarray(err, np.float64).ravel()
    if err.size == 0:
        return {"n": 0}
    inl = err[np.abs(err) <= inlier]
    hist, edges = np.histogram(err, bins=bins, range=(-inlier, inlier))
    return {"n": int(err.size), "variance": float(np.mean(inl * inl)) if inl.size else float("nan"),
            "mean": float(np.mean(inl)) if inl.size else float("nan"),
            "within_1px": float(np.mean(np.abs(err) <= 1.0)),
            "outliers": float(1.0 - inl.size / err.size),
            "hist": hist.tolist(), "hist_edges": [float(edges[0]), float(edges[-1])]}


def perturb(T: np.ndarray, rng: np.random.Generator, rot_deg: float, trans_m: float) -> np.ndarray:
    """T with a small random rotation (Rodrigues, angle ~ N(0, rot_deg)) and
    translation offset (~ N(0, trans_m) per axis)."""
    if rot_deg <= 0 and trans_m <= 0:
        return T
    axis = rng.normal(size=3)
    axis /= np.linalg.norm(axis)
    ang = math.radians(rng.normal(0.0, rot_deg)) if rot_deg > 0 else 0.0
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    dR = np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * (K @ K)
    out = T.copy()
    out[:3, :3] = dR @ T[:3, :3]
    out[:3, 3] = dR @ T[:3, 3] + (rng.normal(0.0, trans_m, 3) if trans_m > 0 else 0.0)
    return out


def process_errors(g, seq, k: int, T: np.ndarray, torch, N) -> np.ndarray:
    """Prediction of frame k from the ground truth of k-1 minus the truth of k."""
    gt0 = seq.disp_gt[k - 1].astype(np.float64)
    v0 = seq.valid[k - 1]
    d = np.where(v0, gt0, 0.0)
    p = np.ones_like(d)
    sf = np.where(v0, 0, RESET).astype(np.uint8)
    g.set_state(d, p, sf)
    g.reduced_frame(seq.left[k], seq.right[k], T)
    dhat = g.stage(N.STAGE_DHAT).cpu().numpy()
    fl = g.stage(N.STAGE_FLAGS).cpu().numpy()
    use = (fl & 1).astype(bool) & ~(fl & RESET).astype(bool) & seq.valid[k] & ~seq.mover[k] & ~seq.mover[k - 1]
    return (dhat - seq.disp_gt[k].astype(np.float64))[use]


def measurement_errors(g, seq, k: int, N) -> np.ndarray:
    g.full_frame(seq.left[k], seq.right[k])
    dz = g.stage(N.STAGE_DZ).cpu().numpy()
    use = seq.valid[k] & ~seq.mover[k]
    return (dz - seq.disp_gt[k].astype(np.float64))[use]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--seeds", default="2,3,4")
    ap.add_argument("--frames", type=int, default=20)
    ap.add_argument("--preset", default="default")
    ap.add_argument("--ego-rot-deg", default="0,0.02,0.05", help="rotation noise levels (deg)")
    ap.add_argument("--ego-trans-m", type=float, default=0.01, help="translation noise when rotation noise > 0")
    ap.add_argument("--inlier", type=float, default=3.0)
    ap.add_argument("--out", default=os.path.join("gpurun_out", "noise.json"))
    args = ap.parse_args(argv)
    import torch
    import paper_1809_07986_amd as sgmk
    from paper_1809_07986_amd import _native as N
    from stereo_synth import make_sequence
    seeds = [int(s) for s in args.seeds.split(",")]
    levels = [float(v) for v in args.ego_rot_deg.split(",")]
    proc = {lv: [] for lv in levels}
    meas = []
    for seed in seeds:
        seq = make_sequence("driving", frames=args.frames, seed=seed)
        H, W, D = seq.cam.height, seq.cam.width, seq.max_disp
        g = sgmk.ReducedSGM(W, H, D, preset=args.preset, f=seq.cam.f, baseline=seq.cam.baseline)
        rng = np.random.default_rng(seed)
        for k in range(1, seq.frames):
            for lv in levels:
                T = perturb(seq.T[k], rng, lv, args.ego_trans_m if lv > 0 else 0.0)
                proc[lv].append(process_errors(g, seq, k, T, torch, N))
            meas.append(measurement_errors(g, seq, k, N))
        g.close()
        print(f"  sequence {seed} done", flush=True)
    res = {"seeds": seeds, "frames": args.frames, "preset": args.preset, "inlier_px": args.inlier,
           "process": {f"rot {lv:g} deg" + (f", trans {args.ego_trans_m:g} m" if lv > 0 else " (exact ego-motion)"):
                       noise_stats(np.concatenate(v), args.inlier) for lv, v in proc.items()},
           "measurement": noise_stats(np.concatenate(meas), args.inlier)}
    for k, v in res["process"].items():
        print(f"  q [{k}]: {v['variance']:.4f} px^2, within 1 px {v['within_1px']:.4f}, outliers {v['outliers']:.4f}")
    m = res["measurement"]
    print(f"  r: {m['variance']:.4f} px^2, within 1 px {m['within_1px']:.4f}, outliers {m['outliers']:.4f}")
    os.makedirs(os.path.dirname(args.out) or ".", exist_ok=True)
    with open(args.out, "w") as fh:
        json.dump(res, fh, indent=1)


if __name__ == "__main__":
    main()
