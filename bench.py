#!/usr/bin/env python3
"""Throughput of the camera operator pair A x + A^T y on one MI355X.

One step = one forward projection y = A x and one backprojection A^T y of
the 128^3 flame volume seen by the 1024^2 plenoptic camera (64^2 lenslets,
2x2 rays/pixel, 256 samples/ray), inputs resident in HBM.  The value is
valid ray-samples per second over both operators (a sample is valid when its
ray is unoccluded and crosses the grid).

Prints one JSON line (see the repository's benchmark contract).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP32 operations of one sample (FMA counted as 2):
#   forward: position 3 FMA (6), cell fraction 3 sub (3), 7 lerps of
#            sub + FMA (21), accumulate (1)                            -> 31
#   adjoint: position (6), fraction (3), 3 complements, 2 + 4 + 8
#            weight products (17), 8 additions into the voxels (8)    -> 34
FLOP_PER_SAMPLE = {"project": 31.0, "backproject": 34.0}
# FP32 vector peak without packed-FP32 dual issue (disabled in this build):
# 256 CUs x 4 SIMD x 16 lanes x 2 flop/FMA x 2.4 GHz
PEAK_FP32_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
GATHER_BYTES_PER_SAMPLE = 32.0   # 8 FP32 voxels per trilinear sample


def cpu_baseline(g, cams, x, valid_fraction, target_s=12.0):
    """The FP64 oracle on the host cores: forward on a random pixel subset,
    then the backprojection of an image holding only those pixels."""
    import numpy as np

    import oracle

    cam = cams[0]
    npix = cam["det_nu"] * cam["det_nv"]
    R = cam["rays_u"] * cam["rays_v"]
    S = cam["samples"]
    threads = oracle.default_threads()
    rng = np.random.default_rng(0)
    x64 = np.asarray(x, np.float64).reshape(-1)
    n = 2048
    while True:
        pix = rng.choice(npix, size=min(n, npix), replace=False)
        t0 = time.perf_counter()
        yv = oracle.project_pixels(g, cam, x64, pix, threads)
        t_fwd = time.perf_counter() - t0
        if t_fwd * 2.2 >= target_s or n >= npix:
            break
        n = int(min(npix, n * max(2.0, 0.5 * target_s / max(t_fwd, 1e-3))))
    img = np.zeros(npix)
    img[pix] = yv + 1.0
    t0 = time.perf_counter()
    oracle.backproject(g, [cam], img, threads)
    t_adj = time.perf_counter() - t0
    nominal = len(pix) * R * S
    valid = nominal * valid_fraction
    return {"value": 2.0 * valid / (t_fwd + t_adj) / 1e9, "unit": "Gsamples/s",
            "cores": threads, "kind": "oracle",
            "sample": (f"{len(pix)} random pixels of the same camera: FP64 forward on them, "
                       f"then FP64 backprojection of an image holding only them; "
                       f"valid samples = {len(pix)} px x {R} rays x {S} samples x valid-ray "
                       f"fraction {valid_fraction:.4f}; {t_fwd:.1f} s + {t_adj:.1f} s")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU path is a design, not a build", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1812_03358_amd import ltm, workloads as W

    cfg = W.config_plenoptic()
    g, cams = cfg["grid"], cfg["cameras"]
    x_host = cfg["volume"]()
    plan = ltm.Plan(g, cams)
    x = torch.from_numpy(x_host.reshape(-1)).cuda()
    y = plan.project(x)
    xt = torch.empty_like(x)
    torch.cuda.synchronize()
    valid = plan.valid_samples()
    nominal = sum(ltm_nominal(c) for c in cams)

    for _ in range(args.warmup):
        plan.project(x, y)
        plan.backproject(y, xt)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    start.record(stream)
    for k in range(args.steps):
        ev[k][0].record(stream)
        plan.project(x, y)
        ev[k][1].record(stream)
        plan.backproject(y, xt)
        ev[k][2].record(stream)
    stop.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    total_ms = start.elapsed_time(stop)
    fwd_ms = sum(e[0].elapsed_time(e[1]) for e in ev) / args.steps
    adj_ms = sum(e[1].elapsed_time(e[2]) for e in ev) / args.steps
    ms_step = total_ms / args.steps
    value = 2.0 * valid / (ms_step * 1e-3) / 1e9

    dominant = "backproject" if adj_ms >= fwd_ms else "project"
    dom_ms = max(adj_ms, fwd_ms)
    achieved = FLOP_PER_SAMPLE[dominant] * valid / (dom_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_FP32_TFLOPS, 2),
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                "traffic": None, "kernel": "k_backproject" if dominant == "backproject" else "k_project",
                "ms_per_launch": round(dom_ms, 4)}
    gather = {d: round(valid / (ms * 1e-3) * GATHER_BYTES_PER_SAMPLE / 1e9 / HBM_PEAK_GBS, 4)
              for d, ms in (("project", fwd_ms), ("backproject", adj_ms))}

    out = {
        "metric": "ray-samples/s for A x + A^T y (% HBM roofline)",
        "value": round(value, 3),
        "unit": "Gsamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "plenoptic_128: 128^3 flame volume (1.25 mm voxels), 1 plenoptic "
                               "camera 1024^2 px behind 64^2 lenslets, 2x2 rays/pixel, 256 "
                               "samples/ray; one A x + one A^T y per step",
                   "valid_samples_per_direction": valid, "nominal_samples_per_direction": nominal,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "gather_equivalent_hbm_frac": gather,
        "ms_project": round(fwd_ms, 4),
        "ms_backproject": round(adj_ms, 4),
        "wall_s_timed": round(t_wall, 3),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, cams, x_host, valid / nominal, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def ltm_nominal(cam):
    return cam["det_nu"] * cam["det_nv"] * cam["rays_u"] * cam["rays_v"] * cam["samples"]


if __name__ == "__main__":
    main()
