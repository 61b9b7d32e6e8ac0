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
    held_out = [900101, 900102, 900103, 900104]
    before = WS.held_out_loss(net, plan, n, held_out)
    tr = WS.train(net, plan, n, range(0, 400), lr=2e-3, workers=4)
    after = WS.held_out_loss(net, plan, n, held_out)
    print("train", tr["steps"], "steps, held-out loss", before, "->", after, flush=True)
    assert tr["steps"] == 400
    assert after < 0.5 * before
    rows = WS.compare(net, plan, n, [900001, 900002, 900003], rho_target=1e-3, max_iter=3000,
                      check_every=5, log=print)
    zero = sum(r["zero"]["iterations"] for r in rows)
    warm = sum(r["warm"]["iterations"] for r in rows)
    assert all(r["zero"]["converged"] and r["warm"]["converged"] for r in rows)
    assert warm < zero


def test_warm_start_fallback_and_rescale():
    """The plain solver judges a candidate start: a NaN-holding one, a
    negative one and one the cameras cannot see are replaced by the zero start
    (the zero start's iterations); one scaled by 1e6 is brought back by the
    least-squares factor of its image and still beats the zero start."""
    from paper_1812_03358_amd import ltm, warmstart as WS
    n = 32
    g = W.grid(n, 160.0 / n)
    cams = [W.plenoptic_camera(256, 16, (2, 2), 64, phi) for phi in (0.0, 90.0)]
    plan = ltm.Plan(g, cams)
    xt = torch.from_numpy(W.flame(n, 900004).reshape(-1)).cuda()
    y = plan.project(xt).clone()
    every = 5
    kw = dict(rho_target=1e-3, max_iter=3000, check_every=every)
    zero = WS.solve_to(plan, y, None, **kw)
    print("zero start", zero, flush=True)
    assert zero["converged"] and zero["accepted"] is None and zero["rho"] <= 1e-3
    # a fair estimate: the truth times noise of 10%
    rng = np.random.default_rng(5)
    noisy = xt * torch.from_numpy(rng.uniform(0.9, 1.1, xt.numel()).astype(np.float32)).cuda()
    good = WS.solve_to(plan, y, noisy, **kw)
    print("fair start", good, flush=True)
    assert good["accepted"] and abs(good["alpha"] - 1.0) < 0.05 and good["rho0"] < 0.2
    assert good["converged"] and good["iterations"] < zero["iterations"]
    # the same estimate at the wrong exposure: rescaled, the same solve
    big = WS.solve_to(plan, y, noisy * 1e6, **kw)
    print("fair start x 1e6", big, flush=True)
    assert big["accepted"] and abs(big["alpha"] * 1e6 - good["alpha"]) < 1e-3 * good["alpha"]
    assert abs(big["rho0"] - good["rho0"]) < 1e-4
    assert big["converged"] and abs(big["iterations"] - good["iterations"]) <= every
    # rejected starts run the zero start's solve
    bad = noisy.clone()
    bad[123] = float("nan")
    D = plan.backproject(plan.project(torch.ones_like(xt)))
    unseen = (D == 0).float()
    assert float(unseen.sum()) > 0
    for name, x0 in (("nan", bad), ("negative", -noisy), ("unseen", unseen)):
        r = WS.solve_to(plan, y, x0, **kw)
        print(name, r, flush=True)
        assert r["accepted"] is False and r["rho0"] == 1.0
        assert r["converged"] and abs(r["iterations"] - zero["iterations"]) <= every
