"""Accuracy and speed of the aggregation path sets (Section 5, Tables 1-2).

The paper evaluates its matcher with 8 paths and with the 4 nondiagonal
paths, and reports that 4 diagonal paths give more outliers.  This script
repeats that comparison on seeded synthetic driving sequences with ground
truth, for the paper's Table 1 settings (census 5x5, P1=6, P2=65, 128
disparities) and for the library defaults (census 9x7, P1=7, P2=86):

  full range  every frame matched over all disparities (the setting the
              paper's parameters were tuned in): bad pixels (> 3 px) and
              mean absolute error of d_z against the truth;
  reduced     the Kalman-filtered stream (full first frame, then reduced
              frames): bad pixels of the filter output d, and frames/s.

    python -m paper_1809_07986_amd.evaluate_paths --out gpurun_out/paths.json
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

MASKS = {"8 paths": 0xFF, "4 nondiagonal": 0x0F, "4 diagonal": 0xF0}


def _log(msg):
    print(msg, flush=True)


def run(seeds, frames, presets, torch, sgmk, make_sequence):
    dev = torch.device("cuda", torch.cuda.current_device())
    res = {}
    for preset in presets:
        for name, mask in MASKS.items():
            acc = dict(full_bad=0.0, full_abs=0.0, red_bad=0.0, valid=0.0, full_s=0.0, red_s=0.0, nf=0, nr=0)
            for seed in seeds:
                seq = make_sequence("driving", frames=frames, seed=seed)
                H, W, D = seq.cam.height, seq.cam.width, seq.max_disp
                L = torch.from_numpy(seq.left).to(dev)
                R = torch.from_numpy(seq.right).to(dev)
                gts = [torch.from_numpy(seq.disp_gt[k].astype(np.float64)).to(dev) for k in range(seq.frames)]
                vals = [torch.from_numpy(seq.valid[k]).to(dev) for k in range(seq.frames)]
                kw = dict(f=seq.cam.f, baseline=seq.cam.baseline, path_mask=mask, preset=preset)
                gf = sgmk.ReducedSGM(W, H, D, **kw)
                gr = sgmk.ReducedSGM(W, H, D, **kw)
                gf.full_frame(L[0], R[0])
                gr.full_frame(L[0], R[0])
                torch.cuda.synchronize()
                for k in range(1, seq.frames):
                    t0 = time.perf_counter()
                    gf.full_frame(L[k], R[k])
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    gr.reduced_frame(L[k], R[k], seq.T[k])
                    torch.cuda.synchronize()
                    t2 = time.perf_counter()
                    acc["full_s"] += t1 - t0
                    acc["red_s"] += t2 - t1
                    acc["nf"] += 1
                    v = vals[k]
                    ez = (gf.stage(sgmk.N.STAGE_DZ) - gts[k]).abs()[v]
                    ed = (gr.disparity().double() - gts[k]).abs()[v]
                    acc["full_bad"] += float((ez > 3).sum())
                    acc["full_abs"] += float(ez.sum())
                    acc["red_bad"] += float((ed > 3).sum())
                    acc["valid"] += float(v.sum())
                gf.close()
                gr.close()
            key = f"{preset} / {name}"
            res[key] = {"full_bad_px_gt3": round(acc["full_bad"] / acc["valid"], 6),
                        "full_mean_abs_err": round(acc["full_abs"] / acc["valid"], 5),
                        "reduced_bad_px_gt3": round(acc["red_bad"] / acc["valid"], 6),
                        "full_ms_per_frame": round(acc["full_s"] / acc["nf"] * 1e3, 4),
                        "reduced_ms_per_frame": round(acc["red_s"] / acc["nf"] * 1e3, 4),
                        "frames": acc["nf"]}
            _log(f"  {key}: {res[key]}")
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--seeds", default="2,3,4")
    ap.add_argument("--frames", type=int, default=20)
    ap.add_argument("--presets", default="paper,default")
    ap.add_argument("--out", default=os.path.join("gpurun_out", "paths.json"))
    args = ap.parse_args(argv)
    import torch
    import paper_1809_07986_amd as sgmk
    from stereo_synth import make_sequence
    seeds = [int(s) for s in args.seeds.split(",")]
    res = run(seeds, args.frames, args.presets.split(","), torch, sgmk, make_sequence)
    os.makedirs(os.path.dirname(args.out) or ".", exist_ok=True)
    with open(args.out, "w") as fh:
        json.dump(dict(seeds=seeds, frames=args.frames, results=res,
                       note="per-frame times include a device synchronisation"), fh, indent=1)


if __name__ == "__main__":
    main()
