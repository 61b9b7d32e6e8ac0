"""Tile-shape autotuner for the projector and its adjoint.

For one camera of a plan and one direction, every candidate tiling is
applied, checked against the output of the plan's current tiling (relative
L2 <= 1e-6: every tiling computes the same samples, only the FP64 summation
order differs) and timed with HIP events; the fastest candidate that passes
is kept.  Results can be cached in a JSON file keyed by the GPU
architecture and the camera/grid shape.
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import ltm as _ltm

PARITY = 1e-6


def _key(plan, cam_index: int, direction: int) -> str:
    g = plan.grid
    c = plan.cameras[cam_index]
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    phi = round(float(c.get("phi_deg", 0.0)), 3)
    return (f"{arch}|dir{direction}|kind{c['kind']}|grid{g['nx']}x{g['ny']}x{g['nz']}"
            f"|det{c['det_nu']}x{c['det_nv']}|mla{c['mla_nu']}|R{c['rays_u']}x{c['rays_v']}"
            f"|S{c['samples']}|phi{phi}")


def candidates(plan, cam_index: int, direction: int):
    """Candidate tilings (dicts of ltm_tiling fields) for one camera."""
    c = plan.cameras[cam_index]
    pitch = plan.grid["pitch"]
    R = c["rays_u"] * c["rays_v"] * (9 if c["kind"] == 2 else 1)   # hexagonal: 3x3 lenslets
    out = []
    plen = c["kind"] == 1
    k = (c["det_nu"] // c["mla_nu"]) * (c["det_nv"] // c["mla_nv"]) if plen else 1
    if direction == _ltm.FORWARD:
        tiles = [1, 2] if plen else [1]
        blocks = [16, 8] if not plen else [16]
        for t in tiles:
            for blk in blocks:
                items = t * t * (k if plen else blk * blk)
                for splits in (1, 4):
                    if items % splits or items // splits > 2048 or items // splits * R > 8192:
                        continue
                    for order in (0, 2):
                        for chunk in (16, 32, 64):
                            for brick in (4096, 8192):
                                out.append(dict(tile_u=t, tile_v=t, block_u=blk, block_v=blk,
                                                order=order, splits=splits, brick_floats=brick,
                                                chunk_mm=chunk * pitch))
    else:
        tiles = [2, 4] if plen else [1, 2]
        blocks = [16] if plen else [8, 16]
        for t in tiles:
            for blk in blocks:
                items = t * t * (k if plen else blk * blk)
                for per in (64, 256):
                    splits = max(1, items // per)
                    if items % splits or items // splits > 2048 or items // splits * R > 8192:
                        continue
                    # bit 3 staggers sample walks, bit 4 merges a cell's samples,
                    # bit 5 keeps two-plane windows along the dominant axis
                    for order in (3, 26, 27, 42, 43):
                        for chunk in (16, 32):
                            for brick in (8192, 12288):
                                out.append(dict(tile_u=t, tile_v=t, block_u=blk, block_v=blk,
                                                order=order, splits=splits, brick_floats=brick,
                                                chunk_mm=chunk * pitch))
    return out


def _time(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def autotune(plan, cam_index: int, direction: int, x: torch.Tensor, y: torch.Tensor,
             reps: int = 3, cache: str | None = None, cands=None) -> dict:
    """Pick and apply the fastest parity-passing tiling for one camera.

    x: an N-float volume (forward input); y: an M-float image (adjoint input).
    Only camera `cam_index` is timed: the other cameras keep their tilings.
    Returns {"tiling": ..., "ms": ..., "default_ms": ..., "tried": n}."""
    key = _key(plan, cam_index, direction)
    store = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            store = json.load(f)
    if key in store:
        plan.set_tiling(direction, cam_index, store[key]["tiling"])
        return dict(store[key], cached=True)

    sub = _ltm.Plan(plan.grid, [plan.cameras[cam_index]], device=x.device)
    sub.set_tiling(direction, 0, plan.get_tiling(direction, cam_index))
    off = sum(c["det_nu"] * c["det_nv"] for c in plan.cameras[:cam_index])
    npx = plan.cameras[cam_index]["det_nu"] * plan.cameras[cam_index]["det_nv"]
    yc = y[off:off + npx].contiguous()
    if direction == _ltm.FORWARD:
        out = torch.empty(npx, dtype=torch.float32, device=x.device)
        run = lambda: sub.project(x, out)
    else:
        out = torch.empty(plan.n_voxels, dtype=torch.float32, device=x.device)
        run = lambda: sub.backproject(yc, out)
    default_ms = _time(run, reps)
    ref = out.clone()
    nref = float(torch.linalg.norm(ref.double())) or 1.0
    best = (default_ms, sub.get_tiling(direction, 0).as_dict())
    tried = 0
    for cand in (cands if cands is not None else candidates(plan, cam_index, direction)):
        try:
            sub.set_tiling(direction, 0, cand)
        except _ltm.LtmError:
            continue
        tried += 1
        ms = _time(run, reps)
        err = float(torch.linalg.norm((out - ref).double())) / nref
        if err <= PARITY and ms < best[0]:
            best = (ms, sub.get_tiling(direction, 0).as_dict())
    plan.set_tiling(direction, cam_index, best[1])
    result = {"tiling": best[1], "ms": best[0], "default_ms": default_ms, "tried": tried}
    if cache:
        store[key] = result
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(store, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return result


def autotune_plan(plan, x: torch.Tensor, y: torch.Tensor, reps: int = 3,
                  cache: str | None = None) -> list:
    """Autotune every camera of a plan in both directions."""
    res = []
    for ci in range(len(plan.cameras)):
        for d in (_ltm.FORWARD, _ltm.ADJOINT):
            res.append(autotune(plan, ci, d, x, y, reps, cache))
    return res
