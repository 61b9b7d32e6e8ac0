"""Learned warm start at small scale: the network trained on projector-made
pairs lowers its loss, and started from its estimate the plain solver needs
fewer iterations to the same data residual than from zero.

The comparison is the relative claim only: the network's output has no
ground truth to be pinned against (parity unpinned); the zero-start solver
is the reference, and both solves run the same FISTA to the same residual.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1812_03358_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_warm_start_small():
    from paper_1812_03358_amd import ltm, nn, warmstart as WS
    n = 32
    g = W.grid(n, 160.0 / n)
    cams = [W.plenoptic_camera(256, 16, (2, 2), 64, phi) for phi in (0.0, 90.0)]
    plan = ltm.Plan(g, cams)
    net = nn.UNet(seed=1)
    tr = WS.train(net, plan, n, range(0, 400), lr=2e-3, workers=4)
    first, last = tr["losses"][0][1], tr["losses"][-1][1]
    print("train", tr["steps"], "steps, loss", first, "->", last, flush=True)
    assert tr["steps"] == 400
    assert last < 0.5 * first
    rows = WS.compare(net, plan, n, [900001, 900002, 900003], rho_target=1e-3, max_iter=3000,
                      check_every=5, log=print)
    zero = sum(r["zero"]["iterations"] for r in rows)
    warm = sum(r["warm"]["iterations"] for r in rows)
    assert all(r["zero"]["converged"] and r["warm"]["converged"] for r in rows)
    assert warm < zero
