"""The dot-identity noise model of tests/dotbar.py against real FP32
rounding: for exact FP64 outputs of the oracle (so <Ax, y> = <x, A^T y> up
to 1e-16), scale both by the same random factor in [1, 2) -- which moves the
values across their binades -- round them to FP32 and measure the dot
statistic.  Its spread over many draws must sit below the model's sigma
(which assumes the worst binade position) and above a third of it, and no
draw may exceed the bar."""
import numpy as np

from dotbar import dot_bar, output_rounding_sigma
from paper_1812_03358_amd import workloads as W


def test_output_rounding_model(orc):
    g = W.grid((20, 24, 18), 6.0)
    cam = W.plenoptic_camera(96, 6, (2, 2), 37, phi_deg=30.0)
    x = W.flame(24, seed=7)[:18, :24, :20].astype(np.float64).reshape(-1)
    y = W.uniform_random(96 * 96, seed=32).astype(np.float64)
    Ax = orc.project(g, [cam], x)
    Aty = orc.backproject(g, [cam], y)
    sigma = output_rounding_sigma(x, Aty, y, Ax)
    bar = dot_bar(x, Aty, y, Ax)
    rng = np.random.default_rng(0)
    stats = []
    for _ in range(300):
        s = rng.uniform(1.0, 2.0)
        a = (s * Ax).astype(np.float32).astype(np.float64)
        b = (s * Aty).astype(np.float32).astype(np.float64)
        stats.append((a @ y - x @ b) / (np.linalg.norm(a) * np.linalg.norm(y)))
    std = float(np.std(stats))
    assert sigma / 3 < std <= sigma
    assert max(abs(v) for v in stats) < bar
    # this grid's noise is above the workload bar 1e-9: the small-grid bar is needed
    assert sigma > 1e-9 and bar > 1e-9
