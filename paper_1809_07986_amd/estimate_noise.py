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

Per-pixel measurement noise from the cost curvature (the approach Section 3
attributes to the authors' earlier method): the library's r_curv mode gives
each measurement the variance r_curv / kappa, kappa the curvature of the
sub-pixel parabola.  With the errors e of the full-range measurements taken
as N(0, tau / kappa), the maximum-likelihood tau is mean(e^2 kappa) over the
inliers; it is reported with the constant r.  --compare then runs the filter
on the same sequences with the constant default r, the constant estimated r
and the curvature variance with the estimated tau, and reports the
bad-pixel rates (> 3 px on valid truth) of the filtered disparity.

    python -m paper_1809_07986_amd.estimate_noise --compare --out gpurun_out/noise.json
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


def measurement_errors(g, seq, k: int, N):
    """Full-range measurement minus the truth on static pixels, and the
    curvature kappa of each of those measurements (g has r_curv > 0)."""
    g.full_frame(seq.left[k], seq.right[k])
    dz = g.stage(N.STAGE_DZ).cpu().numpy()
    kappa = g.stage(N.STAGE_KAPPA).cpu().numpy()
    use = seq.valid[k] & ~seq.mover[k]
    return (dz - seq.disp_gt[k].astype(np.float64))[use], kappa[use]


def curvature_scale(err: np.ndarray, kappa: np.ndarray, inlier: float = 3.0) -> dict:
    """Maximum-likelihood tau of e ~ N(0, tau / kappa) over the inliers with a
    defined curvature: tau = mean(e^2 kappa)."""
    use = (kappa > 0) & (np.abs(err) <= inlier)
    e, k = err[use].astype(np.float64), kappa[use].astype(np.float64)
    tau = float(np.mean(e * e * k))
    return {"tau": tau, "n": int(use.sum()), "kappa_median": float(np.median(k)),
            "r_median": float(np.median(np.clip(tau / k, 1 / 256, 64.0)))}


def filter_accuracy(sgmk, N, seqs, torch, label: str, **params) -> dict:
    """Bad-pixel rate (> 3 px on valid truth) and mean |error| of the filtered
    disparity and of the measurement, frames 1.. of each sequence."""
    bad_d = bad_z = n = 0
    abs_d = 0.0
    for seq in seqs:
        H, W, D = seq.cam.height, seq.cam.width, seq.max_disp
        g = sgmk.ReducedSGM(W, H, D, f=seq.cam.f, baseline=seq.cam.baseline, **params)
        g.full_frame(seq.left[0], seq.right[0])
        for k in range(1, seq.frames):
            g.reduced_frame(seq.left[k], seq.right[k], seq.T[k])
            d = g.get_state()[0].cpu().numpy()
            dz = g.stage(N.STAGE_DZ).cpu().numpy()
            gt = seq.disp_gt[k].astype(np.float64)
            v = seq.valid[k]
            bad_d += int((np.abs(d - gt)[v] > 3).sum())
            bad_z += int((np.abs(dz - gt)[v] > 3).sum())
            abs_d += float(np.abs(d - gt)[v].sum())
            n += int(v.sum())
        g.close()
    res = {"bad_px_gt3_d": bad_d / n, "bad_px_gt3_dz": bad_z / n, "mean_abs_err_d": abs_d / n, "pixels": n}
    print(f"  {label}: bad d {res['bad_px_gt3_d']:.5f}, bad dz {res['bad_px_gt3_dz']:.5f}, "
          f"mean |d - gt| {res['mean_abs_err_d']:.4f}", flush=True)
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--seeds", default="2,3,4")
    ap.add_argument("--frames", type=int, default=20)
    ap.add_argument("--preset", default="default")
    ap.add_argument("--ego-rot-deg", default="0,0.02,0.05", help="rotation noise levels (deg)")
    ap.add_argument("--ego-trans-m", type=float, default=0.01, help="translation noise when rotation noise > 0")
    ap.add_argument("--inlier", type=float, default=3.0)
    ap.add_argument("--compare", action="store_true",
                    help="filter accuracy with constant r, estimated r and the curvature variance")
    ap.add_argument("--out", default=os.path.join("gpurun_out", "noise.json"))
    args = ap.parse_args(argv)
    import torch
    import paper_1809_07986_amd as sgmk
    from paper_1809_07986_amd import _native as N
    from stereo_synth import make_sequence
    seeds = [int(s) for s in args.seeds.split(",")]
    levels = [float(v) for v in args.ego_rot_deg.split(",")]
    proc = {lv: [] for lv in levels}
    meas, kap = [], []
    seqs = []
    for seed in seeds:
        seq = make_sequence("driving", frames=args.frames, seed=seed)
        seqs.append(seq)
        H, W, D = seq.cam.height, seq.cam.width, seq.max_disp
        g = sgmk.ReducedSGM(W, H, D, preset=args.preset, f=seq.cam.f, baseline=seq.cam.baseline)
        gc = sgmk.ReducedSGM(W, H, D, preset=args.preset, f=seq.cam.f, baseline=seq.cam.baseline, r_curv=1.0)
        rng = np.random.default_rng(seed)
        for k in range(1, seq.frames):
            for lv in levels:
                T = perturb(seq.T[k], rng, lv, args.ego_trans_m if lv > 0 else 0.0)
                proc[lv].append(process_errors(g, seq, k, T, torch, N))
            e, kp = measurement_errors(gc, seq, k, N)
            meas.append(e)
            kap.append(kp)
        g.close()
        gc.close()
        print(f"  sequence {seed} done", flush=True)
    res = {"seeds": seeds, "frames": args.frames, "preset": args.preset, "inlier_px": args.inlier,
           "process": {f"rot {lv:g} deg" + (f", trans {args.ego_trans_m:g} m" if lv > 0 else " (exact ego-motion)"):
                       noise_stats(np.concatenate(v), args.inlier) for lv, v in proc.items()},
           "measurement": noise_stats(np.concatenate(meas), args.inlier),
           "curvature": curvature_scale(np.concatenate(meas), np.concatenate(kap), args.inlier)}
    for k, v in res["process"].items():
        print(f"  q [{k}]: {v['variance']:.4f} px^2, within 1 px {v['within_1px']:.4f}, outliers {v['outliers']:.4f}")
    m = res["measurement"]
    print(f"  r: {m['variance']:.4f} px^2, within 1 px {m['within_1px']:.4f}, outliers {m['outliers']:.4f}")
    c = res["curvature"]
    print(f"  curvature: tau {c['tau']:.3f} (cost x px^2), median kappa {c['kappa_median']:g}, "
          f"median r {c['r_median']:.4f} px^2", flush=True)
    if args.compare:
        res["compare"] = {
            "constant r = 1 (default)": filter_accuracy(sgmk, N, seqs, torch, "constant r = 1", preset=args.preset),
            f"constant r = {m['variance']:.4f} (estimated)": filter_accuracy(
                sgmk, N, seqs, torch, "constant estimated r", preset=args.preset, r=m["variance"]),
            f"curvature, tau = {c['tau']:.3f}": filter_accuracy(
                sgmk, N, seqs, torch, "curvature r", preset=args.preset, r_curv=c["tau"]),
        }
    os.makedirs(os.path.dirname(args.out) or ".", exist_ok=True)
    with open(args.out, "w") as fh:
        json.dump(res, fh, indent=1)


if __name__ == "__main__":
    main()
