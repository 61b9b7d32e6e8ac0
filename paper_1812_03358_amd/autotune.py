"""Tile-shape autotuner for the projector and its adjoint: argument
marshalling for ltm_autotune (include/ltm.h), which searches, gates every
candidate on parity with the current tiling (relative L2 <= 1e-6), times it
with HIP events and caches the result in a text file.

TUNED_TABLE is the committed table of tilings measured on MI355X for the
benchmark workloads; pass it as `cache` to apply them without a search.
"""
from __future__ import annotations

import ctypes
import os

import torch

from . import ltm as _ltm

PARITY = 1e-6
TUNED_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned", "gfx950.tsv")


def candidates(plan, cam_index: int, direction: int):
    """The stage-1 candidate tilings ltm_autotune tries for one camera (dicts
    of ltm_tiling fields); stage 2 adds groups_per_cu = 2 and 3 to the three
    fastest."""
    lib = _ltm.lib()
    n = ctypes.c_uint32()
    _ltm._check(lib.ltm_autotune_candidates(plan.handle, direction, cam_index, None, 0,
                                            ctypes.byref(n)))
    arr = (_ltm.Tiling * max(1, n.value))()
    _ltm._check(lib.ltm_autotune_candidates(plan.handle, direction, cam_index, arr, n.value,
                                            ctypes.byref(n)))
    return [arr[i].as_dict() for i in range(n.value)]


def autotune_plan(plan, x: torch.Tensor, y: torch.Tensor, reps: int = 3,
                  cache: str | None = None, stream=None) -> list:
    """Autotune every camera of a bound plan in both directions and rebind
    it.  x: an N-float volume (forward input); y: an M-float image (adjoint
    input).  Returns one dict per (camera, direction): tiling, ms, default_ms."""
    lib = _ltm.lib()
    nb = ctypes.c_uint64()
    _ltm._check(lib.ltm_autotune_workspace_bytes(plan.handle, ctypes.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=x.device)
    ms = (ctypes.c_double * (4 * len(plan.cameras)))()
    path = cache.encode() if cache else None
    _ltm._check(lib.ltm_autotune(plan.handle, _ltm._ptr(x, numel=plan.n_voxels),
                                 _ltm._ptr(y, numel=plan.n_meas), ctypes.c_void_p(ws.data_ptr()),
                                 nb.value, path, reps, ms, _ltm._stream(stream)))
    plan.bind(stream)
    out = []
    for ci in range(len(plan.cameras)):
        for d in (_ltm.FORWARD, _ltm.ADJOINT):
            out.append({"camera": ci, "direction": d,
                        "tiling": plan.get_tiling(d, ci).as_dict(),
                        "ms": ms[4 * ci + 2 * d], "default_ms": ms[4 * ci + 2 * d + 1]})
    return out
