"""Dot-identity bar for the GPU operators on small grids.

The statistic |<A x, y> - <x, A^T y>| / (||A x|| ||y||) is limited by FP32
rounding even when A and A^T use identical FP32 weights: each output value
is rounded to FP32 once (relative error uniform within half an ulp, standard
deviation at most u / sqrt(3), u = 2^-24), and every FP32 intermediate an
operator stores is rounded the same way.  For the outputs alone the
statistic's standard deviation is

    sigma = u / sqrt(3) * sqrt(sum_i (y_i (Ax)_i)^2 + sum_j (x_j (A^T y)_j)^2)
            / (||A x|| ||y||),

i.e. u / sqrt(3 N_eff) with N_eff the effective number of terms.  At the
workload sizes sigma is 1e-11 or less; on grids of a few thousand voxels and
pixels with concentrated volumes it reaches 1e-9.  The bar is four such
standard deviations, each FP32 store of the operator counted as one more
independent rounding of comparable size (``stored``: the number of FP32
arrays one direction writes, its output included -- conservative, since
intermediates hold more values than the output), and never below the
workload bar 1e-9.
"""
import math

import numpy as np

U32 = 2.0 ** -24


def output_rounding_sigma(x, Aty, y, Ax) -> float:
    x, Aty, y, Ax = (np.asarray(a, np.float64).reshape(-1) for a in (x, Aty, y, Ax))
    t1, t2 = y * Ax, x * Aty
    num = math.sqrt(float(np.dot(t1, t1) + np.dot(t2, t2)))
    return U32 / math.sqrt(3.0) * num / (float(np.linalg.norm(Ax)) * float(np.linalg.norm(y)))


def dot_bar(x, Aty, y, Ax, stored: int = 1, k: float = 4.0, floor: float = 1e-9) -> float:
    """x, y: the inputs; Ax, Aty: the FP64 oracle's outputs for them."""
    return max(floor, k * math.sqrt(stored) * output_rounding_sigma(x, Aty, y, Ax))
