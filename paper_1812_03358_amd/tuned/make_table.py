"""Write the tuned-tiling table for the benchmark workloads (run on the GPU).

For one frame of each volume size of the 48-frame workload (four plenoptic
cameras each) and for the 256^3 four-camera workload, every camera and
direction is searched by ltm_autotune (parity gate against the default
tiling, HIP-event timing) and the winners are written to the table, keyed by
GPU architecture, grid and camera descriptor.  Keys already in the table are
re-checked, not searched again; delete the file to search afresh.

The 48-frame workload runs as one persistent sweep per direction, launched
with the largest LDS any member needs, so a camera tuned alone to a larger
brick or to padded occupancy would lower the workgroups per CU of the whole
sweep.  Its tilings in both directions are therefore capped at
BATCH_BRICK_CAP brick floats with no occupancy padding (5 workgroups per CU),
at the slab depth (full, 1/2 or 1/4) that runs fastest, each capped tiling
checked against the searched one through the same parity bar and re-timed.

    python -m paper_1812_03358_amd.tuned.make_table [path]
"""
from __future__ import annotations

import os
import sys
import time

import torch

from paper_1812_03358_amd import autotune, ltm, workloads as W

BATCH_BRICK_CAP = 6144


def workloads():
    seen = set()
    for f in W.config_batched():
        n = f["grid"]["nx"]
        if n not in seen:
            seen.add(n)
            yield f"batched_48 frame {n}^3", f["grid"], f["cameras"], W.flame(n, f["volume_seed"]), True
    cfg = W.config_differentiable()
    yield "differentiable_256", cfg["grid"], cfg["cameras"], cfg["volume"](), False


def _fnv1a(data: bytes, h: int) -> int:
    for b in data:
        h = ((h ^ b) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


def table_key(arch: str, g: dict, cam: dict, direction: int) -> str:
    """The table key ltm_autotune files a camera's tiling under: the readable
    fields, then FNV-1a (64-bit) over the raw ltm_grid and ltm_camera structs
    (neither has padding)."""
    gs = ltm.make_grid(g)
    cs = ltm.make_cameras([cam])[0]
    h = _fnv1a(bytes(cs), _fnv1a(bytes(gs), 1469598103934665603))
    return (f"{arch}|{'A' if direction == ltm.FORWARD else 'AT'}|kind{cs.kind}|grid{gs.nx}x{gs.ny}x{gs.nz}"
            f"|det{cs.det_nu}x{cs.det_nv}|mla{cs.mla_nu}x{cs.mla_nv}|R{cs.rays_u}x{cs.rays_v}"
            f"|S{cs.samples}|{h:016x}")


def _apply(plan, direction: int, x, y, out):
    return plan.project(x, out) if direction == ltm.FORWARD else plan.backproject(y, out)


def time_direction(plan, direction: int, x, y, out, reps: int = 5) -> float:
    _apply(plan, direction, x, y, out)
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        _apply(plan, direction, x, y, out)
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return sorted(ts)[len(ts) // 2]


FIELDS = ("tile_u", "tile_v", "block_u", "block_v", "order", "splits", "brick_floats", "groups_per_cu",
          "chunk_mm")


def read_table(path: str) -> dict:
    """key -> tiling dict of every line of a table file."""
    out = {}
    if not os.path.exists(path):
        return out
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        key, tiling = line.rstrip("\n").split("\t")[:2]
        vals = tiling.split()
        out[key] = {f: (float(v) if f == "chunk_mm" else int(v)) for f, v in zip(FIELDS, vals)}
    return out


def batch_capped(plan, direction: int, x, y, tiling: dict):
    """A table tiling under the batch cap, parity-checked against the plan's
    current (tuned) output in that direction and timed.  A smaller brick may
    not hold the tiling's slabs, which then fall back to global memory, so
    the slab depth is also tried at 1/2 and 1/4; the fastest is kept (a
    tiling already within the cap keeps its depth unless a shallower one is
    faster)."""
    capped = dict(tiling, brick_floats=min(tiling["brick_floats"], BATCH_BRICK_CAP), groups_per_cu=0)
    ref = _apply(plan, direction, x, y, None).double()
    best = None
    for f in (1.0, 0.5, 0.25):
        t = dict(capped, chunk_mm=capped["chunk_mm"] * f)
        plan.set_tiling(direction, 0, t)
        out = _apply(plan, direction, x, y, None)
        err = float(torch.linalg.norm(out.double() - ref) / torch.linalg.norm(ref))
        if not err <= autotune.PARITY:
            raise RuntimeError(f"capped tiling {t} fails the parity bar ({err:.2e})")
        ms = time_direction(plan, direction, x, y, out)
        if best is None or ms < best[1]:
            best = (t, ms)
    return best


def rewrite(path: str, caps: dict) -> None:
    """Replace the tilings of the capped cameras in the table."""
    lines = open(path).read().splitlines()
    for i, line in enumerate(lines):
        if line.startswith("#"):
            continue
        key, tiling, times = line.split("\t")
        if key in caps:
            t, ms = caps[key]
            text = " ".join(str(t[f]) for f in FIELDS[:-1])
            lines[i] = f"{key}\t{text} {t['chunk_mm']!r}\t{ms:.5f} {times.split()[1]}"
    with open(path + ".tmp", "w") as f:
        f.write("\n".join(lines) + "\n")
    os.replace(path + ".tmp", path)


def main(path: str) -> None:
    caps = {}
    for name, g, cams, vol, batched in workloads():
        x = torch.from_numpy(vol.reshape(-1)).cuda()
        # one camera at a time (the table is keyed per camera and grid)
        for k, cam in enumerate(cams):
            t0 = time.perf_counter()
            plan = ltm.Plan(g, [cam])
            y = plan.project(x)
            res = autotune.autotune_plan(plan, x, y, reps=3, cache=path)
            torch.cuda.synchronize()
            print(f"{name} camera {k}: {time.perf_counter() - t0:.1f} s", flush=True)
            for r in res:
                print(f"  {'A ' if r['direction'] == 0 else 'AT'} {r['ms']:.4f} ms "
                      f"(default {r['default_ms']:.4f}) {r['tiling']}", flush=True)
            if not batched:
                continue
            # the table's line decides: the tuner applies it whenever it beats
            # the default alone
            for d in (ltm.FORWARD, ltm.ADJOINT):
                key = table_key("gfx950", g, cam, d)
                filed = read_table(path).get(key)
                got = batch_capped(plan, d, x, y, filed) if filed else None
                if got is not None and got[0] != filed:
                    caps[key] = got
                    print(f"  {'A ' if d == ltm.FORWARD else 'AT'} {got[1]:.4f} ms under the batch cap {got[0]}",
                          flush=True)
    if caps:
        rewrite(path, caps)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else autotune.TUNED_TABLE)
