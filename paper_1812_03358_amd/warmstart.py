"""Learned warm start for the reconstruction: training and evaluation.

Training pairs are made by the projector itself: a seeded flame volume x
(generated on host worker processes), its noiseless images y = A x from the
two-camera plenoptic plan, and the network input A^T y / max.  The loss is
the mean squared error between the network output and x; Adam updates the
FP32 master weights.  Every arithmetic step runs in libltm kernels.

Evaluation: for held-out volumes, the wall-clock time from "images on the
device, plan bound" to a confirmed relative data residual <= target, for
the plain solver started at zero and for the solver started at the network
output (time includes A^T y and the network forward).  Both solves are the
same FISTA (beta = nu = 0, nonnegativity only).
"""
from __future__ import annotations

import multiprocessing as mp
import time

import numpy as np
import torch

from . import ltm as _ltm
from . import nn as _nn
from . import workloads as W


def _flame(args):
    n, seed = args
    return seed, W.flame(n, seed)


class VolumeStream:
    """Seeded flame volumes produced by host worker processes, in order."""

    def __init__(self, n, seeds, workers=8):
        self.n = n
        self.seeds = list(seeds)
        ctx = mp.get_context("fork")
        self.pool = ctx.Pool(workers)
        self.it = self.pool.imap(_flame, [(n, s) for s in self.seeds], chunksize=1)

    def __iter__(self):
        for _ in self.seeds:
            yield next(self.it)

    def close(self):
        self.pool.terminate()
        self.pool.join()


def make_plan(device="cuda"):
    cfg = W.config_warm_start()
    return _ltm.Plan(cfg["grid"], cfg["cameras"], device=device), cfg


def infer(net, plan, y, n, stream=None, final_relu=True):
    """Network estimate of the volume from images y (FP32 on the device)."""
    aty = plan.backproject(y)
    inp = net.prep_input(aty, stream)
    return net.forward(inp, n, n, n, stream, final_relu=final_relu)


def train(net, plan, n, seeds, lr=1e-3, time_limit=None, workers=8, log=None, warmup=100):
    """One pass over the given seeds (or until time_limit seconds).  The
    learning rate ramps linearly over the first `warmup` steps: Adam's first
    steps move every weight by about lr at once, which at lr 1e-3 raises the
    loss of the freshly initialized network several-fold."""
    stream = VolumeStream(n, seeds, workers)
    t0 = time.perf_counter()
    losses = []
    count = 0
    try:
        for seed, vol in stream:
            x = torch.from_numpy(vol.reshape(-1)).to(net.device)
            y = plan.project(x)
            infer(net, plan, y, n, final_relu=False)      # the loss sees the linear output
            loss, g = net.loss_and_grad(x)
            net.backward(g)
            net.step(lr * min(1.0, (count + 1) / max(1, warmup)))
            count += 1
            if count % 25 == 0 or count == 1:
                losses.append((count, float(loss)))
                if log:
                    log(f"train step {count} seed {seed} loss {float(loss):.4e} "
                        f"{time.perf_counter() - t0:.1f}s")
            if time_limit and time.perf_counter() - t0 > time_limit:
                break
    finally:
        stream.close()
    torch.cuda.synchronize()
    return {"steps": count, "seconds": time.perf_counter() - t0, "losses": losses}


def held_out_loss(net, plan, n, seeds):
    """Mean loss of the network's linear output over fixed volumes (no
    weight update): the same volumes before and after training compare the
    network itself, where single training steps see a different volume each."""
    total = 0.0
    for seed in seeds:
        x = torch.from_numpy(W.flame(n, seed).reshape(-1)).to(net.device)
        infer(net, plan, plan.project(x), n, final_relu=False)
        loss, _ = net.loss_and_grad(x)
        total += float(loss)
    return total / len(seeds)


def solve_to(plan, y, x0=None, rho_target=1e-3, max_iter=5000, check_every=10, prelude=None):
    """FISTA (beta = nu = 0) from x0 (None: zero) until rho(x) <= target.

    The stop rule and the judgement of a warm start run in the library
    (ltm_solver_solve, ltm_solver_reset_warm): a candidate start is rescaled
    by the least-squares factor of its image and replaced by zero when it is
    non-finite or does not lower the data residual below rho(0) = 1, so the
    plain zero-start solver stays the fallback.  Wall-clock from the call
    (plan bound, y on the device) to the confirmed residual of the iterate x;
    `prelude` (a callable returning x0) is timed inside.  Returns
    dict(iterations, seconds, rho, converged, accepted, alpha, rho0)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if prelude is not None:
        x0 = prelude()
    s = _ltm.Solver(plan, y, momentum=True, rho_target=rho_target, max_iter=max_iter,
                    check_every=check_every)
    accepted, alpha, rho0 = None, None, 1.0
    if x0 is not None:
        accepted, alpha, rho0 = s.reset_warm(x0)
    it, converged, rho = s.solve()
    torch.cuda.synchronize()
    return {"iterations": it, "seconds": time.perf_counter() - t0, "rho": rho, "converged": converged,
            "accepted": accepted, "alpha": alpha, "rho0": rho0}


def compare(net, plan, n, seeds, rho_target=1e-3, max_iter=5000, check_every=10, log=None,
            workers=1):
    """Zero start vs warm start on held-out seeds (volumes made by `workers`
    host processes when workers > 1)."""
    rows = []
    stream = VolumeStream(n, seeds, workers) if workers > 1 else None
    vols = stream if stream is not None else ((s, W.flame(n, s)) for s in seeds)
    try:
        for seed, vol in vols:
            rows.append(_compare_one(net, plan, n, seed, vol, rho_target, max_iter, check_every, log))
    finally:
        if stream is not None:
            stream.close()
    return rows


def _compare_one(net, plan, n, seed, vol, rho_target, max_iter, check_every, log):
    """One held-out volume: the zero-start and warm-start solves of its images."""
    x = torch.from_numpy(vol.reshape(-1)).to(net.device)
    y = plan.project(x).clone()
    zero = solve_to(plan, y, None, rho_target, max_iter, check_every)
    warm = solve_to(plan, y, None, rho_target, max_iter, check_every,
                    prelude=lambda: infer(net, plan, y, n).contiguous())
    x0 = infer(net, plan, y, n)
    err0 = float(torch.linalg.norm(x0 - x) / torch.linalg.norm(x))
    row = {"seed": seed, "zero": zero, "warm": warm, "net_rel_error": err0}
    if log:
        log(f"seed {seed}: zero {zero['iterations']} it {zero['seconds']:.2f}s rho {zero['rho']:.2e} | "
            f"warm {warm['iterations']} it {warm['seconds']:.2f}s rho {warm['rho']:.2e} | "
            f"network error {err0:.3f}")
    return row
