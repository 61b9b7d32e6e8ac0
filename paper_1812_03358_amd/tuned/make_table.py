"""Write the tuned-tiling table for the benchmark workloads (run on the GPU).

For one frame of each volume size of the 48-frame workload (four plenoptic
cameras each) and for the 256^3 four-camera workload, every camera and
direction is searched by ltm_autotune (parity gate against the default
tiling, HIP-event timing) and the winners are written to the table, keyed by
GPU architecture, grid and camera descriptor.  Keys already in the table are
re-checked, not searched again; delete the file to search afresh.

    python -m paper_1812_03358_amd.tuned.make_table [path]
"""
from __future__ import annotations

import sys
import time

import torch

from paper_1812_03358_amd import autotune, ltm, workloads as W


def workloads():
    seen = set()
    for f in W.config_batched():
        n = f["grid"]["nx"]
        if n not in seen:
            seen.add(n)
            yield f"batched_48 frame {n}^3", f["grid"], f["cameras"], W.flame(n, f["volume_seed"])
    cfg = W.config_differentiable()
    yield "differentiable_256", cfg["grid"], cfg["cameras"], cfg["volume"]()


def main(path: str) -> None:
    for name, g, cams, vol in workloads():
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


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else autotune.TUNED_TABLE)
