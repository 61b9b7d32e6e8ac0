#!/usr/bin/env python3
"""Throughput of the camera operator pair A x + A^T y on one MI355X.

Default workload (batched_48): 48 flame frames (12 each of 96^3, 128^3,
160^3 and 192^3 voxels) seen by 4 plenoptic cameras at 0/30/60/90 degrees
(1024^2 pixels behind 64^2 lenslets, 2x2 rays per pixel, 2n samples per
ray).  One step = one replay of a hipGraph holding the persistent forward
sweep over all frames and cameras, then the persistent adjoint sweep; inputs
resident in HBM.  The value is valid ray-samples per second over both
directions (a sample is valid when its ray is unoccluded and crosses the
grid).  Other workloads (--workload) time single plans, reconstructions,
the learned warm start and the paper's own transport discretization.

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
# MI355X's published FP32 vector peak, 157.3 TFLOP/s = 256 CUs x 4 SIMD x 16
# lanes x 2 flop/FMA x 2 (packed dual issue) x 2.4 GHz.  The kernels are
# compiled without packed FP32, so 78.6 TFLOP/s is the ceiling they can reach;
# the roofline fraction is still taken against the published figure.
PEAK_FP32_TFLOPS = 256 * 4 * 16 * 2 * 2 * 2.4e9 / 1e12
PEAK_FP32_NON_PACKED_TFLOPS = PEAK_FP32_TFLOPS / 2
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
    # a sample that is the whole image finishes early: repeat the pair until
    # about target_s of CPU time has been measured
    reps = 1
    while t_fwd + t_adj < 0.8 * target_s and reps < 20:
        t0 = time.perf_counter()
        oracle.project_pixels(g, cam, x64, pix, threads)
        t_fwd += time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.backproject(g, [cam], img, threads)
        t_adj += time.perf_counter() - t0
        reps += 1
    nominal = len(pix) * R * S * reps
    valid = nominal * valid_fraction
    return {"value": 2.0 * valid / (t_fwd + t_adj) / 1e9, "unit": "Gsamples/s",
            "cores": threads, "kind": "oracle",
            "sample": (f"{len(pix)} random pixels of the same camera ({reps} pass(es)): FP64 forward "
                       f"on them, then FP64 backprojection of an image holding only them; valid "
                       f"samples = {len(pix)} px x {R} rays x {S} samples x valid-ray fraction "
                       f"{valid_fraction:.4f} per pass; {t_fwd:.1f} s + {t_adj:.1f} s")}


def time_pair(plan, x, y, xt, steps, warmup):
    """Event-timed steps of (project, backproject) on torch's current stream."""
    import torch

    for _ in range(warmup):
        plan.project(x, y)
        plan.backproject(y, xt)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    start.record(stream)
    for k in range(steps):
        ev[k][0].record(stream)
        plan.project(x, y)
        ev[k][1].record(stream)
        plan.backproject(y, xt)
        ev[k][2].record(stream)
    stop.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    total_ms = start.elapsed_time(stop)
    fwd_ms = sum(e[0].elapsed_time(e[1]) for e in ev) / steps
    adj_ms = sum(e[1].elapsed_time(e[2]) for e in ev) / steps
    return total_ms / steps, fwd_ms, adj_ms, t_wall


def counter_traffic(plan, direction):
    """HBM bytes per launch of k_march from the committed FETCH_SIZE and
    WRITE_SIZE summary, or None when the kernel source or the camera's default
    tiling differs from the ones the counters were taken with."""
    import hashlib

    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                        "k_march_plenoptic_128_hbm_counters.md")
    try:
        line = [l for l in open(path) if l.startswith("provenance: ")][0]
        prov = json.loads(line[len("provenance: "):])
        src = os.path.join(os.path.dirname(os.path.abspath(__file__)), prov["kernel_source"])
        if hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != prov["sha256_16"]:
            return None
        key = "tiling_forward" if direction == "project" else "tiling_adjoint"
        t = plan.get_tiling(0 if direction == "project" else 1, 0)
        if [t.tile_u, t.tile_v, t.order, t.splits, t.brick_floats, round(t.chunk_mm, 6)] != prov[key]:
            return None
        return prov["traffic_bytes"][direction]
    except (OSError, IndexError, KeyError, ValueError):
        return None


def counter_traffic_batch(adjoint):
    """HBM bytes per launch of k_batch on the 48-frame sweep from the
    committed FETCH_SIZE/WRITE_SIZE summary, or None when the kernel source
    or the tuned table changed since the counters were taken."""
    import hashlib

    base = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(base, "profiles", "k_batch_batched_48_hbm_counters.md")
    try:
        line = [l for l in open(path) if l.startswith("provenance: ")][0]
        prov = json.loads(line[len("provenance: "):])
        for rel, h in prov["sha256_16"].items():
            if hashlib.sha256(open(os.path.join(base, rel), "rb").read()).hexdigest()[:16] != h:
                return None
        return prov["traffic_bytes"]["backproject" if adjoint else "project"]
    except (OSError, IndexError, KeyError, ValueError):
        return None


def roofline_of(valid, fwd_ms, adj_ms):
    dominant = "backproject" if adj_ms >= fwd_ms else "project"
    dom_ms = max(adj_ms, fwd_ms)
    achieved = FLOP_PER_SAMPLE[dominant] * valid / (dom_ms * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_FP32_TFLOPS, 2),
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": None,
            "kernel": "k_march<true> (adjoint)" if dominant == "backproject" else "k_march<false> (forward)",
            "ms_per_launch": round(dom_ms, 4),
            "frac_of_non_packed_fp32": round(achieved / PEAK_FP32_NON_PACKED_TFLOPS, 4)}
    gather = {d: round(valid / (ms * 1e-3) * GATHER_BYTES_PER_SAMPLE / 1e9 / HBM_PEAK_GBS, 4)
              for d, ms in (("project", fwd_ms), ("backproject", adj_ms))}
    return roof, gather


def base_record(args, value, ms_step, workload, extra_config):
    return {
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
        "config": dict({"workload": workload, "parallelism": "single GPU"}, **extra_config),
    }


def copy_probe():
    """A plain 256 MiB device copy, so counter runs can scale their byte
    counts against a kernel of known traffic."""
    import torch

    src = torch.ones(64 << 20, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()


def run_single(args, cfg, workload, tune=False):
    """One A x + one A^T y per step over the configuration's cameras; with
    tune (and without --no-autotune) every camera's tilings are autotuned
    first, outside the timed region."""
    import torch

    from paper_1812_03358_amd import autotune, ltm

    g, cams = cfg["grid"], cfg["cameras"]
    x_host = cfg["volume"]()
    plan = ltm.Plan(g, cams)
    x = torch.from_numpy(x_host.reshape(-1)).cuda()
    y = plan.project(x)
    xt = torch.empty_like(x)
    torch.cuda.synchronize()
    tuned = None
    if tune and not args.no_autotune:
        t0 = time.perf_counter()
        tuned = autotune.autotune_plan(plan, x, y, reps=2,
                                       cache=args.autotune_cache or autotune.TUNED_TABLE)
        t_tune = time.perf_counter() - t0
        plan.project(x, y)
        torch.cuda.synchronize()
    valid = plan.valid_samples()
    nominal = sum(ltm_nominal(c) for c in cams)
    ms_step, fwd_ms, adj_ms, t_wall = time_pair(plan, x, y, xt, args.steps, args.warmup)
    value = 2.0 * valid / (ms_step * 1e-3) / 1e9
    out = base_record(args, value, ms_step, workload,
                      {"valid_samples_per_direction": valid, "nominal_samples_per_direction": nominal})
    out["roofline"], out["gather_equivalent_hbm_frac"] = roofline_of(valid, fwd_ms, adj_ms)
    out["config"]["tilings"] = [
        {d: {k: (round(v, 4) if isinstance(v, float) else v)
             for k, v in plan.get_tiling(i, ci).as_dict().items()}
         for i, d in ((0, "project"), (1, "backproject"))}
        for ci in range(len(cams))]
    if cfg["name"] == "plenoptic_128":
        dom = "backproject" if adj_ms >= fwd_ms else "project"
        out["roofline"]["traffic"] = counter_traffic(plan, dom)
    if tuned is not None:
        out["autotune_s"] = round(t_tune, 2)
        out["autotune"] = [{"ms": round(r["ms"], 4), "default_ms": round(r["default_ms"], 4)}
                           for r in tuned]
    out["ms_project"] = round(fwd_ms, 4)
    out["ms_backproject"] = round(adj_ms, 4)
    out["gsamples_per_s_project"] = round(valid / (fwd_ms * 1e-3) / 1e9, 2)
    out["gsamples_per_s_backproject"] = round(valid / (adj_ms * 1e-3) / 1e9, 2)
    out["wall_s_timed"] = round(t_wall, 3)
    if args.copy_probe:
        copy_probe()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, cams, x_host, valid / nominal, args.cpu_seconds)
    return out


def host_cpu():
    """CPU model, logical CPUs of the host and the CPUs this process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, os.cpu_count() or 1, usable


def oracle_threads():
    """Threads the oracle may use: OMP_NUM_THREADS when set (a GPU job's
    share of the host), else every CPU this process may use."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    _, _, usable = host_cpu()
    return max(1, int(env)) if env.isdigit() and int(env) > 0 else usable


def cpu_baseline_frames(units, threads, target_s):
    """The FP64 oracle on a sample of a multi-frame, multi-camera workload.
    units: (grid, cameras, volume, valid samples per direction of the frame);
    for each frame the same fraction f of every camera's pixels is drawn,
    projected (oracle.project_pixels per camera) and backprojected (one
    oracle.backproject of the frame's image holding only those pixels, so its
    per-thread volumes are reduced once per frame).  f doubles from a small
    calibration pass until the sample takes about target_s.  Returns
    (Gsamples/s over both directions, valid samples per direction in the
    sample, forward s, adjoint s, f)."""
    import numpy as np

    import oracle

    f = 1.0 / 512
    while True:
        t_fwd = t_adj = 0.0
        valid = 0.0
        for k, (g, cams, vol, frame_valid) in enumerate(units):
            rng = np.random.default_rng(1000 + k)
            x64 = np.asarray(vol, np.float64).reshape(-1)
            img = []
            for c in cams:
                npix = c["det_nu"] * c["det_nv"]
                pix = rng.choice(npix, size=max(1, int(round(f * npix))), replace=False)
                t0 = time.perf_counter()
                yv = oracle.project_pixels(g, c, x64, pix, threads)
                t_fwd += time.perf_counter() - t0
                im = np.zeros(npix)
                im[pix] = yv + 1.0
                img.append(im)
            t0 = time.perf_counter()
            oracle.backproject(g, cams, np.concatenate(img), threads)
            t_adj += time.perf_counter() - t0
            valid += f * frame_valid
        if t_fwd + t_adj >= 0.45 * target_s or f >= 1.0:
            break
        f = min(1.0, f * max(2.0, min(16.0, 0.8 * target_s / max(t_fwd + t_adj, 1e-3))))
    return 2.0 * valid / (t_fwd + t_adj) / 1e9, valid, t_fwd, t_adj, f


def run_batched(args):
    """48 frames x 4 plenoptic cameras: tuned tilings, one graph replay of the
    persistent A sweep then A^T sweep per step."""
    import numpy as np
    import torch

    from paper_1812_03358_amd import autotune, ltm, workloads as W

    frames = W.config_batched()
    cache = args.autotune_cache or autotune.TUNED_TABLE
    plans, xs, ys, xts, vols = [], [], [], [], {}
    tuned = {}
    t0 = time.perf_counter()
    for f in frames:
        n = f["grid"]["nx"]
        p = ltm.Plan(f["grid"], f["cameras"])
        vol = W.flame(n, f["volume_seed"])
        vols.setdefault(n, (f, vol))
        x = torch.from_numpy(vol.reshape(-1)).cuda()
        y = torch.empty(p.n_meas, device="cuda")
        if not args.no_autotune:
            if n not in tuned:
                # one parity-gated tuning per volume size (the frames of a size
                # share grid and cameras, hence their operator)
                p.project(x, y)
                tuned[n] = (p, autotune.autotune_plan(p, x, y, reps=2, cache=cache))
            else:
                src = tuned[n][0]
                for ci in range(len(f["cameras"])):
                    for d in (ltm.FORWARD, ltm.ADJOINT):
                        p.set_tiling(d, ci, src.get_tiling(d, ci), rebind=False)
                p.bind()
        plans.append(p)
        xs.append(x)
        ys.append(y)
        xts.append(torch.empty_like(x))
    t_setup = time.perf_counter() - t0
    valid = sum(p.valid_samples() for p in plans)
    nominal = sum(ltm_nominal(c) for f in frames for c in f["cameras"])
    batch = ltm.Batch(plans, xs, ys, xts)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        batch.sweep(s)
        s.synchronize()
        batch.capture(s)
        for _ in range(args.warmup):
            batch.replay(s)
        s.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t_wall = time.perf_counter()
        a.record(s)
        for _ in range(args.steps):
            batch.replay(s)
        b.record(s)
        s.synchronize()
        t_wall = time.perf_counter() - t_wall
        # each direction's sweep alone, eagerly on the same stream: the
        # persistent kernel's launch time (plus the adjoint's accumulator
        # clear and FP32 conversion kernels, under 0.5% of it)
        reps = max(2, min(args.steps, 5))
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(reps)]
        for e in ev:
            e[0].record(s)
            batch.project(s)
            e[1].record(s)
            batch.backproject(s)
            e[2].record(s)
        s.synchronize()
    ms = a.elapsed_time(b) / args.steps
    fwd_ms = sum(e[0].elapsed_time(e[1]) for e in ev) / reps
    adj_ms = sum(e[1].elapsed_time(e[2]) for e in ev) / reps
    value = 2.0 * valid / (ms * 1e-3) / 1e9
    out = base_record(args, value, ms, "batched_48: 48 flame frames (12 each of 96/128/160/192^3, "
                      "160 mm cube) x 4 plenoptic cameras at 0/30/60/90 deg, 1024^2 px, 64^2 "
                      "lenslets, 2x2 rays, S = 2n; one hipGraph replay of the persistent A sweep "
                      "and A^T sweep per step" +
                      ("" if args.no_autotune else "; tilings from the committed tuned table, "
                       "each passed through the tuner's parity gate at set-up"),
                      {"valid_samples_per_direction": valid, "nominal_samples_per_direction": nominal,
                       "frames": len(frames), "cameras_per_frame": 4})
    roof, gather = roofline_of(valid, fwd_ms, adj_ms)
    roof["kernel"] = "k_batch<true> (adjoint sweep)" if adj_ms >= fwd_ms else "k_batch<false> (forward sweep)"
    roof["traffic"] = counter_traffic_batch(adj_ms >= fwd_ms)
    out["roofline"] = roof
    out["gather_equivalent_hbm_frac_not_a_roofline"] = gather
    out["ms_project_sweep"] = round(fwd_ms, 3)
    out["ms_backproject_sweep"] = round(adj_ms, 3)
    out["gsamples_per_s_project"] = round(valid / (fwd_ms * 1e-3) / 1e9, 2)
    out["gsamples_per_s_backproject"] = round(valid / (adj_ms * 1e-3) / 1e9, 2)
    out["wall_s_timed"] = round(t_wall, 3)
    out["setup_s"] = round(t_setup, 2)
    if args.copy_probe:
        copy_probe()
    if tuned:
        out["autotune"] = {str(n): [{"cam": r["camera"], "dir": r["direction"], "ms": round(r["ms"], 4),
                                     "default_ms": round(r["default_ms"], 4)} for r in res]
                           for n, (_, res) in tuned.items()}
    if not args.no_cpu_baseline:
        # one frame per volume size, all four cameras, extrapolated to the
        # 48-frame sweep by valid-sample count
        import oracle

        model, logical, usable = host_cpu()
        threads = oracle_threads()
        units = []
        for n in sorted(vols):
            f, vol = vols[n]
            frame_valid = sum(oracle.count_valid_rays(f["grid"], c, threads) * c["samples"]
                              for c in f["cameras"])
            units.append((f["grid"], f["cameras"], vol, frame_valid))
        v_all, s_all, tf_all, ta_all, f_all = cpu_baseline_frames(units, threads, args.cpu_seconds)
        v_one, s_one, tf_one, ta_one, f_one = cpu_baseline_frames(units, 1, args.cpu_seconds * 0.5)
        out["cpu_baseline"] = {
            "value": round(v_all, 4), "unit": "Gsamples/s", "cores": threads, "kind": "oracle",
            "sample": (f"one frame of each size (96/128/160/192^3), all 4 cameras: a random "
                       f"{f_all:.4f} of every camera's pixels, FP64 forward on them and FP64 "
                       f"backprojection of the frame's image holding only them; {s_all:.3e} valid "
                       f"samples per direction (that fraction of each frame's valid samples, "
                       f"counted by the oracle); {tf_all:.1f} s + {ta_all:.1f} s on {threads} threads; "
                       f"extrapolated by valid-sample count to the 48-frame sweep: "
                       f"{2.0 * valid / (v_all * 1e9):.0f} s per A + A^T sweep"),
            "one_core_value": round(v_one, 5),
            "one_core_sample": (f"the same frames, fraction {f_one:.4f} of the pixels, 1 thread: "
                                f"{tf_one:.1f} s + {ta_one:.1f} s; "
                                f"{2.0 * valid / (v_one * 1e9) / 60:.0f} min per sweep extrapolated"),
            "cpu_model": model, "host_logical_cpus": logical, "cpus_usable": usable}
    return out


def run_recon(args):
    """Reconstruction on the 128^3 plenoptic workload: FISTA with the
    hyperbola potential on Poisson data, per-iteration time and final rho."""
    import numpy as np
    import torch

    from paper_1812_03358_amd import ltm, workloads as W

    cfg = W.config_plenoptic()
    g, cams = cfg["grid"], cfg["cameras"]
    plan = ltm.Plan(g, cams)
    xt = torch.from_numpy(cfg["volume"]().reshape(-1)).cuda()
    y_clean = plan.project(xt).cpu().numpy()
    y = torch.from_numpy(W.poisson_noise(y_clean, seed=cfg["noise_seed"])).cuda()
    # majorizer scale for the edge-preserving weight: 36 beta = 1% of median D
    d = plan.backproject(plan.project(torch.ones(plan.n_voxels, device="cuda")))
    dpos = d[d > 0]
    beta = 0.01 * float(dpos.median()) / 36.0
    solver = ltm.Solver(plan, y, beta=beta, psi_kind=ltm.PSI_HYPERBOLA, delta=0.02, momentum=True)
    solver.step(2)
    torch.cuda.synchronize()
    solver.reset()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    solver.step(args.iters)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    rho, it = solver.residual()
    x = solver.x()
    err = float(torch.linalg.norm(x - xt) / torch.linalg.norm(xt))
    out = base_record(args, 1000.0 * args.iters / ms, ms / args.iters,
                      f"recon_plenoptic_128: FISTA, hyperbola potential (delta 0.02), "
                      f"{args.iters} iterations, Poisson data at peak 1000", {"beta": beta})
    out["metric"] = "reconstruction iterations/s"
    out["unit"] = "iterations/s"
    out["final_rho"] = rho
    out["iterations"] = it
    out["rel_error_to_truth"] = err
    return out


def run_recon_three(args):
    """The paper's three-camera reconstruction at its sizes: plenoptic 2048^2
    (128^2 lenslets) head-on plus single-lens 1024^2 cameras at +-30 deg, an
    8x8 angular grid each, 200 samples per ray, 100^3 at 1 mm; FISTA with
    per-camera gain estimation on images whose gains are planted at 0.8 and
    1.3.  Reports iterations/s and the time of one iteration."""
    import numpy as np
    import torch

    from paper_1812_03358_amd import ltm, workloads as W

    cfg = W.config_three_camera()
    g, cams = cfg["grid"], cfg["cameras"]
    plan = ltm.Plan(g, cams)
    xt = torch.from_numpy(cfg["volume"]().reshape(-1)).cuda()
    y = plan.project(xt)
    off = 0
    for cam, gain in zip(cams, cfg["gains"]):
        m = W.n_pixels(cam)
        y[off:off + m] /= gain
        off += m
    solver = ltm.Solver(plan, y, gains=True, momentum=True)
    solver.step(2)
    torch.cuda.synchronize()
    solver.reset()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    solver.step(args.iters)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    rho, it = solver.residual()
    *_, gains = solver.save()
    x = solver.x()
    err = float(torch.linalg.norm(x - xt) / torch.linalg.norm(xt))
    valid = plan.valid_samples()
    out = base_record(args, 1000.0 * args.iters / ms, ms / args.iters,
                      f"recon_three_camera_100: FISTA with gain estimation, {args.iters} iterations, "
                      f"noiseless images with planted gains {cfg['gains']}",
                      {"valid_samples_per_direction": valid})
    out["metric"] = "reconstruction iterations/s"
    out["unit"] = "iterations/s"
    out["s_per_iteration"] = ms / args.iters / 1000.0
    out["paper_s_per_iteration"] = {"value": 49.0, "hardware": "NVIDIA Quadro K5200, OpenCL, FP32",
                                    "note": "context only: the paper's operator is a different "
                                            "discretization of the same optics"}
    out["final_rho"] = rho
    out["iterations"] = it
    out["gains"] = gains
    out["rel_error_to_truth"] = err
    return out


def run_transport(args):
    """The paper's own discretization (L2-projected light-field transport) at
    the three-camera experiment's single-lens size: 1024^2 px of 5 um, 100^3
    flame at 1 mm, 8x8 pillbox cells; one A x + one A^T y per step.  Then the
    angular-discretization study: the normalized difference of Dirac and
    pillbox images at K = 2^2 .. 32^2 from a Dirac 64^2 image, beside the
    ray-driven operator (8x8 rays, 400 samples)."""
    import numpy as np
    import torch

    from paper_1812_03358_amd import ltm, workloads as W

    g = W.grid(100, 1.0)
    cam = W.single_lens_camera(1024, (8, 8), 1, phi_deg=args.phi)
    x = torch.from_numpy(W.flame(100, 5).reshape(-1)).cuda()
    t0 = time.perf_counter()
    op = ltm.Transport(g, cam, ltm.BASIS_PILLBOX)
    t_tables = time.perf_counter() - t0
    y = op.project(x)
    xt = torch.empty_like(x)
    for _ in range(args.warmup):
        op.project(x, y)
        op.backproject(y, xt)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    f_ms = a_ms = 0.0
    t_wall = time.perf_counter()
    for _ in range(args.steps):
        ev[0].record()
        op.project(x, y)
        ev[1].record()
        op.backproject(y, xt)
        ev[2].record()
        torch.cuda.synchronize()
        f_ms += ev[0].elapsed_time(ev[1])
        a_ms += ev[1].elapsed_time(ev[2])
    t_wall = time.perf_counter() - t_wall
    f_ms /= args.steps
    a_ms /= args.steps
    ms = f_ms + a_ms
    # algorithmic HBM bytes per direction: the FP32 intermediate written once
    # and read once, the input read once, the output written once
    mid = 100 * 8 * 1024 * 100 * 4
    nbytes = 2 * mid + 4 * (100 ** 3 + 1024 ** 2)
    out = base_record(args, 1000.0 / ms, ms,
                      "transport_100: paper's L2-projected light-field transport, pillbox basis, "
                      f"single-lens 1024^2 {pose_text(args.phi)}, 100^3 flame at 1 mm, 8x8 angular "
                      "cells; one A x + one A^T y per step",
                      {"bands": op.bands(), "table_build_s": round(t_tables, 3), "phi_deg": args.phi})
    out["metric"] = "transport A x + A^T y pairs/s"
    out["unit"] = "pairs/s"
    gbs = 2 * nbytes / (ms * 1e-3) / 1e9
    out["roofline"] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None}
    out["ms_project"] = round(f_ms, 4)
    out["ms_backproject"] = round(a_ms, 4)
    out["wall_s_timed"] = round(t_wall, 3)
    if args.no_study or args.phi:
        return out
    out["angular_study"] = angular_study(g, x)
    return out


def angular_study(g, x):
    """The angular-discretization experiment: single-lens images of the
    100^3 flame and of 48 point sources in the Dirac and pillbox angular bases
    at K = 2^2 .. 32^2 cells against the Dirac 64^2 image, and the ray-driven
    operator (8x8 rays, 400 samples) against both.  Two apertures: the single-lens table's
    (r 5 mm: the defocus blur at the volume's faces stays under a voxel) and
    r 15 mm (about two voxels of blur there, so the angular sampling shows).
    Each K keeps a different fraction of cells inside the lens disc, a global
    scale the camera gains absorb, so each image is also compared after its
    least-squares scale onto the reference (`nsd_scaled`)."""
    import torch

    from paper_1812_03358_amd import ltm, workloads as W

    def nsd(a, b):
        return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))

    def nsd_scaled(a, b):
        s = float(torch.dot(a, b) / torch.dot(a, a))
        return float(torch.linalg.norm(s * a - b) / torch.linalg.norm(b))

    import numpy as np

    # 48 seeded single-voxel point sources off the focal plane: a defocused
    # point images to the lens disc (pillbox cells) or to K^2 dots (Dirac)
    rng = np.random.default_rng(17)
    pts = np.zeros((g["nz"], g["ny"], g["nx"]), np.float32)
    for _ in range(48):
        k, j, i = (int(v) for v in rng.integers(10, 90, 3))
        pts[k, j, i] = 1.0
    volumes = (("flame", x), ("points", torch.from_numpy(pts.reshape(-1)).cuda()))
    rows = []
    for r_main in (5.0, 15.0):
        cam = lambda K: W.single_lens_camera(1024, (K, K), 1, r_main=r_main)
        ops = {(b, K): ltm.Transport(g, cam(K), b) for b in (ltm.BASIS_DIRAC, ltm.BASIS_PILLBOX)
               for K in (2, 4, 8, 16, 32)}
        ref_op = ltm.Transport(g, cam(64), ltm.BASIS_DIRAC)
        plan = ltm.Plan(g, [W.single_lens_camera(1024, (8, 8), 400, r_main=r_main)])
        for vname, v in volumes:
            ref = ref_op.project(v).double()
            ray = plan.project(v).double()
            for basis, name in ((ltm.BASIS_DIRAC, "dirac"), (ltm.BASIS_PILLBOX, "pillbox")):
                for K in (2, 4, 8, 16, 32):
                    yk = ops[(basis, K)].project(v).double()
                    rows.append({"volume": vname, "r_main_mm": r_main, "basis": name, "K": f"{K}x{K}",
                                 "nsd": round(nsd(yk, ref), 5),
                                 "nsd_scaled": round(nsd_scaled(yk, ref), 5),
                                 "nsd_scaled_vs_ray_driven": round(nsd_scaled(yk, ray), 5)})
            rows.append({"volume": vname, "r_main_mm": r_main,
                         "basis": "ray-driven 8x8 rays, 400 samples", "K": "8x8",
                         "nsd": round(nsd(ray, ref), 5), "nsd_scaled": round(nsd_scaled(ray, ref), 5)})
        del ops, ref_op, plan
    torch.cuda.synchronize()
    return rows


def pose_text(phi):
    """The camera pose in a workload name; a posed camera's roofline bytes
    stay those of the head-on operator (the rotated grid's intermediates and
    the shear passes are extra work, not counted as algorithmic)."""
    return "head-on" if not phi else f"at azimuth {phi:g} deg (roofline bytes of the head-on operator)"


def run_plenoptic_transport(args):
    """The paper's factorized plenoptic transport (slices onto the lenslet
    array plane per angular cell, the aperture mask, each lenslet onto the
    detector) for the default benchmark's camera: 128^3 flame at 1.25 mm,
    1024^2 pixels behind 64^2 lenslets, 4x4 pillbox cells; one A x + one A^T y
    per step.  Beside it, the normalized difference to the ray-driven
    operator's image (8x8 rays per pixel, 256 samples per ray)."""
    import torch

    from paper_1812_03358_amd import ltm, workloads as W

    n, K = 128, 4
    g = W.grid(n, 1.25)
    cam = W.plenoptic_camera(1024, 64, (K, K), 1, phi_deg=args.phi)
    x = torch.from_numpy(W.flame(n, 2).reshape(-1)).cuda()
    t0 = time.perf_counter()
    op = ltm.Transport(g, cam, ltm.BASIS_PILLBOX)
    t_tables = time.perf_counter() - t0
    y = op.project(x)
    xt = torch.empty_like(x)
    for _ in range(args.warmup):
        op.project(x, y)
        op.backproject(y, xt)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    f_ms = a_ms = 0.0
    for _ in range(args.steps):
        ev[0].record()
        op.project(x, y)
        ev[1].record()
        op.backproject(y, xt)
        ev[2].record()
        torch.cuda.synchronize()
        f_ms += ev[0].elapsed_time(ev[1])
        a_ms += ev[1].elapsed_time(ev[2])
    f_ms /= args.steps
    a_ms /= args.steps
    ms = f_ms + a_ms
    # algorithmic HBM bytes per direction: input and output once, each of the
    # three FP32 intermediates written once and read once
    r = cam["r_main"]
    d0 = 2.0 * r / K
    cells = sum(((i + 0.5) * d0 - r) ** 2 + ((j + 0.5) * d0 - r) ** 2 <= r * r
                for i in range(K) for j in range(K))
    inter = n * K * 1024 * n + 2 * cells * 1024 * 1024
    nbytes = 4 * (n ** 3 + 1024 ** 2) + 2 * 4 * inter
    ray = ltm.Plan(g, [W.plenoptic_camera(1024, 64, (8, 8), 256, phi_deg=args.phi)])
    yr = ray.project(x).double()
    nsd = float(torch.linalg.norm(y.double() - yr) / torch.linalg.norm(yr))
    out = base_record(args, 1000.0 / ms, ms,
                      "plenoptic_transport_128: paper's factorized plenoptic transport, pillbox "
                      f"basis, 1024^2 behind 64^2 lenslets {pose_text(args.phi)}, 128^3 flame at "
                      "1.25 mm, 4x4 angular cells; one A x + one A^T y per step",
                      {"bands": op.bands(), "table_build_s": round(t_tables, 3), "cells": cells,
                       "phi_deg": args.phi})
    out["metric"] = "transport A x + A^T y pairs/s"
    out["unit"] = "pairs/s"
    gbs = 2 * nbytes / (ms * 1e-3) / 1e9
    out["roofline"] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None}
    out["ms_project"] = round(f_ms, 4)
    out["ms_backproject"] = round(a_ms, 4)
    out["nsd_vs_ray_driven_8x8"] = nsd
    return out


MFMA_BF16_PEAK_TFLOPS = 2500.0   # dense BF16 MFMA, MI355X


def run_warm_start_net(args):
    """The warm-start network at 128^3 (one channel in, 16/32/64/128
    channels): each 3x3x3 convolution's forward kernel timed with HIP events
    on the stream it runs on, FLOPs = 2 x output voxels x cout x 27 x cin
    (BF16 MFMA, FP32 accumulation); then one whole training step (forward,
    MSE, backward, Adam, weight packing).  Inputs are random, weights He
    initialized."""
    import ctypes

    import numpy as np
    import torch

    from paper_1812_03358_amd import ltm, nn

    n = 128
    net = nn.UNet(seed=0)
    x = torch.from_numpy(np.random.default_rng(0).uniform(0, 1, n ** 3).astype(np.float32)).cuda()
    xin = net.prep_input(x)
    target = torch.from_numpy(np.random.default_rng(1).uniform(0, 1, n ** 3).astype(np.float32)).cuda()
    for _ in range(args.warmup):
        net.forward(xin, n, n, n)
    torch.cuda.synchronize()
    # per-layer forward convolutions, each input as the full forward leaves it
    A = net.acts
    lib = ltm.lib()
    rows, tot_flop, tot_ms = [], 0.0, 0.0
    for name in nn.ORDER:
        if name.startswith("p"):
            continue
        L = net.layers[name]
        d, h, w = net._dims(name, n, n, n)
        last = name == "out"
        out = torch.empty(d * h * w * L.cout, dtype=torch.float32 if last else torch.int16, device="cuda")
        desc = nn.conv_desc(L.ks, d, h, w, L.c0, L.c1, L.cout, L.up, 1, int(last))
        in1 = A[L.ins[1]] if len(L.ins) > 1 else None
        call = lambda: ltm._check(lib.ltm_nn_conv3d_forward(
            ctypes.byref(desc), ctypes.c_void_p(A[L.ins[0]].data_ptr()),
            ctypes.c_void_p(in1.data_ptr() if in1 is not None else 0), ctypes.c_void_p(L.wf.data_ptr()),
            ctypes.c_void_p(L.b.data_ptr()), ctypes.c_void_p(out.data_ptr()), None, ltm._stream(None)))
        call()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            call()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        flop = 2.0 * d * h * w * L.cout * L.ks ** 3 * L.cin
        tot_flop += flop
        tot_ms += ms
        rows.append({"layer": name, "dhw": d, "cin": L.cin, "cout": L.cout, "ms": round(ms, 4),
                     "tflops": round(flop / (ms * 1e-3) / 1e12, 1)})
    # one training step
    for _ in range(2):
        net.zero_grad()
        net.forward(xin, n, n, n)
        _, g = net.loss_and_grad(target)
        net.backward(g)
        net.step(lr=1e-4)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        net.zero_grad()
        net.forward(xin, n, n, n)
        _, g = net.loss_and_grad(target)
        net.backward(g)
        net.step(lr=1e-4)
    e1.record()
    torch.cuda.synchronize()
    step_ms = e0.elapsed_time(e1) / args.steps
    dom = max(rows, key=lambda r: r["ms"])
    dom_flop = 2.0 * (dom["dhw"] ** 3) * dom["cout"] * 27 * dom["cin"]
    out = base_record(args, tot_flop / (tot_ms * 1e-3) / 1e12, tot_ms,
                      "warm_start_net_128: the warm-start network's 3x3x3 BF16 convolutions at 128^3 "
                      "(forward kernels of one network pass, each timed alone), then one training step",
                      {"layers": rows})
    out["metric"] = "warm-start network forward convolutions, TFLOP/s"
    out["unit"] = "TFLOP/s"
    out["dtype"] = "bf16"
    ach = dom_flop / (dom["ms"] * 1e-3) / 1e12
    out["roofline"] = {"bound": "mfma", "achieved": round(ach, 1), "peak": MFMA_BF16_PEAK_TFLOPS,
                       "unit": "TFLOP/s", "frac": round(ach / MFMA_BF16_PEAK_TFLOPS, 4), "traffic": None,
                       "kernel": f"conv3d forward, layer {dom['layer']}"}
    out["ms_forward_convs"] = round(tot_ms, 4)
    out["ms_train_step"] = round(step_ms, 4)
    return out


def run_warm_start(args):
    """Learned warm start (2 plenoptic cameras at 0/90 deg, 128^3): train the
    network on projector-generated pairs for a time budget, then time the
    solver to relative data residual <= 1e-3 from zero and from the network
    output on held-out volumes (noiseless images)."""
    import torch

    from paper_1812_03358_amd import nn, warmstart as WS

    n = 128
    plan, cfg = WS.make_plan()
    net = nn.UNet(seed=0)
    log = (lambda m: print(m, file=sys.stderr, flush=True))
    tr = WS.train(net, plan, n, range(0, 20000), lr=args.lr, time_limit=args.train_seconds,
                  workers=12, log=log)
    rows = WS.compare(net, plan, n, range(200000, 200000 + args.eval_volumes), 1e-3, args.max_iter,
                      10, log=log, workers=8)
    zs = [r["zero"]["seconds"] for r in rows]
    ws = [r["warm"]["seconds"] for r in rows]
    zi = [r["zero"]["iterations"] for r in rows]
    wi = [r["warm"]["iterations"] for r in rows]
    out = base_record(args, sum(ws) / len(ws), sum(ws) / len(ws) * 1e3,
                      "warm_start_128: 128^3 flame volumes, 2 plenoptic cameras 1024^2 at 0/90 deg, "
                      "noiseless images; FISTA (beta = nu = 0) to relative data residual 1e-3 from the "
                      "network's estimate vs from zero", {"train_steps": tr["steps"],
                                                          "train_seconds": round(tr["seconds"], 1)})
    out["metric"] = "recon s to 1e-3 residual (warm start)"
    out["unit"] = "s"
    out["higher_is_better"] = False
    out["zero_start_s"] = round(sum(zs) / len(zs), 3)
    out["warm_start_s"] = round(sum(ws) / len(ws), 3)
    out["zero_start_iterations"] = zi
    out["warm_start_iterations"] = wi
    out["converged"] = [bool(r["zero"]["converged"] and r["warm"]["converged"]) for r in rows]
    out["network_rel_error"] = [round(r["net_rel_error"], 4) for r in rows]
    out["eval_volumes"] = len(rows)
    out["zero_start_s_median"] = round(sorted(zs)[len(zs) // 2], 3)
    out["warm_start_s_median"] = round(sorted(ws)[len(ws) // 2], 3)
    out["warm_faster_on"] = sum(1 for a, b in zip(ws, zs) if a < b)
    out["warm_start_accepted"] = sum(1 for r in rows if r["warm"]["accepted"])
    out["train_loss"] = tr["losses"][-3:]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_zero_start(cfg, sum(zi) / len(zi))
    return out


def cpu_baseline_zero_start(cfg, iterations):
    """The FP64 oracle's zero-start FISTA on the same problem: its majorizer
    set-up and two iterations are timed on the host threads, and the total is
    extrapolated to the GPU's mean zero-start iteration count."""
    import numpy as np

    import oracle
    from paper_1812_03358_amd import workloads as W

    g, cams = cfg["grid"], cfg["cameras"]
    threads = oracle_threads()
    model, logical, usable = host_cpu()
    x = W.flame(g["nx"], 200000).astype(np.float64).reshape(-1)
    ys = [oracle.project(g, [c], x, threads) for c in cams]
    t0 = time.perf_counter()
    sol = oracle.Solver(g, cams, ys, momentum=True, threads=threads)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    sol.run(2)
    t_iter = (time.perf_counter() - t0) / 2
    total = t_setup + iterations * t_iter
    return {"value": round(total, 2), "unit": "s", "cores": threads, "kind": "oracle",
            "sample": (f"FP64 oracle FISTA (beta = nu = 0) on held-out volume 200000's noiseless "
                       f"images: majorizer set-up {t_setup:.1f} s and 2 iterations timed "
                       f"({t_iter:.2f} s each) on {threads} threads, extrapolated to the GPU's mean "
                       f"zero-start count of {iterations:.1f} iterations"),
            "cpu_model": model, "host_logical_cpus": logical, "cpus_usable": usable}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="batched_48",
                    choices=["plenoptic_128", "thin_lens_32", "differentiable_256", "batched_48",
                             "recon_plenoptic_128", "recon_three_camera_100", "warm_start_128",
                             "hex_plenoptic_100", "transport_100",
                             "plenoptic_transport_128", "warm_start_net_128"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=16.0)
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--autotune-cache", default=None)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--iters", type=int, default=100)
    ap.add_argument("--train-seconds", type=float, default=240.0)
    ap.add_argument("--eval-volumes", type=int, default=64)
    ap.add_argument("--max-iter", type=int, default=4000)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--no-study", action="store_true", help="transport_100: skip the angular study")
    ap.add_argument("--phi", type=float, default=0.0,
                    help="transport workloads: camera azimuth in degrees (posed transport)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU path is a design, not a build", file=sys.stderr)
        sys.exit(2)

    from paper_1812_03358_amd import workloads as W

    if args.workload == "plenoptic_128":
        out = run_single(args, W.config_plenoptic(), "plenoptic_128: 128^3 flame volume (1.25 mm "
                         "voxels), 1 plenoptic camera 1024^2 px behind 64^2 lenslets, 2x2 rays/pixel, "
                         "256 samples/ray; one A x + one A^T y per step")
    elif args.workload == "thin_lens_32":
        out = run_single(args, W.config_thin_lens(), "thin_lens_32: 32^3 blobs, single-lens camera "
                         "64^2, 1 ray/pixel, 64 samples/ray; one A x + one A^T y per step")
    elif args.workload == "differentiable_256":
        out = run_single(args, W.config_differentiable(), "differentiable_256: 256^3 flame, 4 "
                         "plenoptic cameras 2048^2 (128^2 lenslets) at 0/30/60/90 deg, 2x1 rays, "
                         "512 samples; one A x + one A^T y per step" +
                         ("" if args.no_autotune else ", autotuned tilings"), tune=True)
    elif args.workload == "hex_plenoptic_100":
        out = run_single(args, W.config_hex_plenoptic(), "hex_plenoptic_100: 100^3 flame (1 mm "
                         "voxels), plenoptic camera 2048^2 px of 5 um behind a hexagonal 53x61 "
                         "array of 2.8/3.0/3.2 mm lenslets, light summed over all lenslets (3x3 "
                         "visited per pixel), 2x2 rays/lenslet, 200 samples/ray; one A x + one "
                         "A^T y per step")
    elif args.workload == "transport_100":
        out = run_transport(args)
    elif args.workload == "plenoptic_transport_128":
        out = run_plenoptic_transport(args)
    elif args.workload == "warm_start_net_128":
        out = run_warm_start_net(args)
    elif args.workload == "batched_48":
        out = run_batched(args)
    elif args.workload == "warm_start_128":
        out = run_warm_start(args)
    elif args.workload == "recon_three_camera_100":
        out = run_recon_three(args)
    else:
        out = run_recon(args)
    print(json.dumps(out), flush=True)


def ltm_nominal(cam):
    return cam["det_nu"] * cam["det_nv"] * cam["rays_u"] * cam["rays_v"] * cam["samples"]


if __name__ == "__main__":
    main()
