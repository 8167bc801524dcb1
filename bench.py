"""Benchmark of the 2D-LUT hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Headline (`value`): svdlut_apply on one 3840x2160 float32 frame (33x33 LUTs at rank 8,
reconstruction fused, 480x270 spatial map), in Mpix/s, with inputs resident in HBM.
Each timed step is one launch; four disjoint buffer sets rotate so that the 256 MB
Infinity Cache cannot serve a step from the previous one.  The other hot-path rows are
measured in the same run and reported under "rows".  Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N_ROT = 4


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--rows", default="all", help="comma list of extra rows to time (c1,c3,c4,c5) or 'none'")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget of the oracle CPU baseline")
    return ap.parse_args()


def event_time(fn, steps, warmup, torch):
    """Average ms per call of fn(i) over `steps` calls, timed with HIP events on the current stream."""
    for i in range(warmup):
        fn(i)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(steps):
        fn(i)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def cpu_baseline(case, budget_s):
    """The fp64 oracle timed on row bands of the same frame until about budget_s of work."""
    from oracle import lut as ol
    x, U, s, V, m = case.x[0], case.U[0], case.s[0], case.V[0], case.smap[0]
    H, W = x.shape[1:]
    T = ol.reconstruct(U, s, V)
    band = 64
    px, t_total, rows = 0, 0.0, 0
    y0 = 0
    while t_total < budget_s and y0 < H:
        ys = np.repeat(np.arange(y0, min(y0 + band, H)), W)
        xs = np.tile(np.arange(W), min(band, H - y0))
        t = time.perf_counter()
        ol.transform_at(x, T, m, ys, xs)
        t_total += time.perf_counter() - t
        px += ys.size
        rows += min(band, H - y0)
        y0 += band
    return {"value": px / t_total / 1e6, "unit": "Mpix/s", "cores": 1, "kind": "oracle",
            "sample": f"{rows} of 2160 rows of the 3840x2160 frame (fp64 NumPy, single thread), {t_total:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import synth
    c2 = synth.frame_4k()                         # host inputs first, before the GPU is touched
    import torch
    import paper_2508_16121_amd as svd

    B, H, W, D, R, h, w = c2.shape
    npx = H * W
    sets = []
    for k in range(N_ROT):
        sets.append(dict(x=torch.from_numpy(c2.x).cuda(), U=torch.from_numpy(c2.U).cuda(),
                         s=torch.from_numpy(c2.s).cuda(), V=torch.from_numpy(c2.V).cuda(),
                         m=torch.from_numpy(c2.smap).cuda(), y=torch.empty_like(torch.from_numpy(c2.x)).cuda()))
    torch.cuda.synchronize()

    def step(i):
        b = sets[i % N_ROT]
        svd.apply(b["x"], b["U"], b["s"], b["V"], b["m"], out=b["y"])

    ms = event_time(step, args.steps, args.warmup, torch)
    bytes_alg = npx * (12 + 12) + 9 * h * w * 4 + 9 * D * R * 2 * 4 + 9 * R * 4
    achieved = bytes_alg / (ms * 1e-3) / 1e9
    value = npx / (ms * 1e-3) / 1e6
    out = {
        "metric": "Mpix/s of 2D-LUT apply at 4K (fwd, fwd+bwd, batched); % of HBM peak",
        "value": round(value, 1), "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "svdlut_apply 1x3x2160x3840 fp32, D=33 R=8, map 9x270x480 fp32, fused reconstruction",
                   "global_batch": 1, "pixels": npx},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None},
    }
    out["cpu_baseline"] = cpu_baseline(c2, args.cpu_seconds) if args.cpu_seconds > 0 else None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
