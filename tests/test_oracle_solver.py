"""Pins of the oracle's regularizer and reconstruction algorithm.

* regularizer gradient (quadratic potential) equals beta (n_j x_j - sum of
  neighbours), built here from scipy.ndimage.convolve with free boundaries;
* the hyperbola potential tends to the quadratic one as delta -> infinity and
  to delta |t| as delta -> 0; gradients match finite differences of R;
* the 26-neighbour Hessian has largest eigenvalue at most 36 beta, and the
  paper's 26 beta is exceeded by an alternating vector (the reading that
  sets c_R = 36);
* the diagonal majorizer D = diag(A^T A 1) satisfies v^T D v >= ||A v||^2;
* the gain formula recovers a planted camera gain;
* with beta = nu = 0 FISTA converges to the nonnegative least-squares
  solution of scipy.optimize.nnls, and the KKT conditions hold.
"""
import math

import numpy as np
import pytest
from scipy import ndimage, optimize

from paper_1812_03358_amd import workloads as W


def test_quadratic_reg_gradient_matches_library_convolution(orc):
    shape = (5, 6, 7)
    x = W.uniform_random(shape, seed=3).astype(np.float64)
    k = np.ones((3, 3, 3))
    nsum = ndimage.convolve(x, k, mode="constant", cval=0.0) - x
    count = ndimage.convolve(np.ones(shape), k, mode="constant", cval=0.0) - 1.0
    beta = 0.37
    expect = beta * (count * x - nsum)
    got = orc.reg_grad(x, shape, beta, orc.PSI_QUADRATIC, 1.0).reshape(shape)
    assert np.max(np.abs(got - expect)) < 1e-13


def test_hyperbola_limits(orc):
    t = np.linspace(-3, 3, 61)
    big = orc.psi(t, orc.PSI_HYPERBOLA, 1e4)
    assert np.max(np.abs(big - 0.5 * t * t)) < 1e-6
    d = 1e-6
    small = orc.psi(t, orc.PSI_HYPERBOLA, d)
    assert np.max(np.abs(small - d * np.abs(t))) < 1e-11
    # curvature bounded by one (the paper's requirement on psi)
    h = 1e-4
    for delta in (0.02, 0.5, 3.0):
        curv = (orc.psi(t + h, 1, delta) - 2 * orc.psi(t, 1, delta) + orc.psi(t - h, 1, delta)) / h ** 2
        assert curv.max() <= 1.0 + 1e-5


@pytest.mark.parametrize("kind,delta", [(0, 1.0), (1, 0.05)])
def test_reg_gradient_matches_finite_differences(orc, kind, delta):
    shape = (4, 5, 3)
    x = W.uniform_random(shape, seed=11).astype(np.float64).reshape(-1)
    g = orc.reg_grad(x, shape, 0.8, kind, delta)
    rng = np.random.default_rng(0)
    for _ in range(5):
        v = rng.standard_normal(x.size)
        h = 1e-5
        fd = (orc.reg_value(x + h * v, shape, 0.8, kind, delta)
              - orc.reg_value(x - h * v, shape, 0.8, kind, delta)) / (2 * h)
        assert abs(fd - np.dot(g, v)) < 1e-7 * max(1.0, abs(fd))


def test_regularizer_majorizer_constant(orc):
    shape = (10, 10, 10)
    hess = lambda v: orc.reg_grad(v, shape, 1.0, orc.PSI_QUADRATIC, 1.0)  # linear for quadratic psi
    # power iteration: largest eigenvalue stays below 36
    rng = np.random.default_rng(1)
    v = rng.standard_normal(1000)
    lam = 0.0
    for _ in range(300):
        w = hess(v)
        lam = np.dot(v, w) / np.dot(v, v)
        v = w / np.linalg.norm(w)
    assert lam <= 36.0 + 1e-9
    # a vector alternating along x only exceeds 26: 26 beta does not majorize
    alt = np.tile((-1.0) ** np.arange(10), 100)
    rq = np.dot(alt, hess(alt)) / np.dot(alt, alt)
    assert rq > 26.0
    assert lam >= rq - 1e-9


def _tiny_problem(orc):
    g = W.grid(4, 30.0)
    cams = [W.plenoptic_camera(16, 2, (2, 2), 12, phi_deg=0.0),
            W.plenoptic_camera(16, 2, (2, 2), 12, phi_deg=90.0)]
    N = 64
    A = np.zeros((sum(c["det_nu"] ** 2 for c in cams), N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        A[:, j] = orc.project(g, cams, e)
    return g, cams, A


def test_majorizer_inequality(orc):
    g, cams, A = _tiny_problem(orc)
    D = orc.backproject(g, cams, orc.project(g, cams, np.ones(64)))
    assert np.allclose(D, A.T @ (A @ np.ones(64)), rtol=1e-13)
    rng = np.random.default_rng(2)
    for _ in range(20):
        v = rng.standard_normal(64)
        assert np.dot(v, D * v) >= np.dot(A @ v, A @ v) * (1 - 1e-12)


def test_gain_recovers_planted_gain(orc):
    g, cams, A = _tiny_problem(orc)
    xt = W.uniform_random(64, seed=5).astype(np.float64)
    y1 = orc.project(g, [cams[0]], xt)
    y2 = orc.project(g, [cams[1]], xt) / 2.5           # camera 2 reads 1/2.5 of the light
    s = orc.Solver(g, cams, [y1, y2], gains=True)
    assert abs(s._gain(1, orc.project(g, [cams[1]], xt)) - 2.5) < 1e-12
    assert s._gain(0, y1) == 1.0


def test_fista_converges_to_nnls(orc):
    # explicit nonnegative matrices standing in for two cameras; the grid only
    # fixes N (the regularizer is off)
    rng = np.random.default_rng(4)
    N = 27
    A1 = rng.uniform(0, 1, (40, N)) * (rng.uniform(0, 1, (40, N)) < 0.5)
    A2 = rng.uniform(0, 1, (30, N)) * (rng.uniform(0, 1, (30, N)) < 0.5)
    A = np.vstack([A1, A2])
    xt = np.maximum(rng.standard_normal(N), 0.0)
    b = A @ xt + 0.3 * rng.standard_normal(A.shape[0])
    x_ref, _ = optimize.nnls(A, b, maxiter=5000)
    ops = [(lambda v: A1 @ v, lambda r: A1.T @ r), (lambda v: A2 @ v, lambda r: A2.T @ r)]
    s = orc.Solver(W.grid(3, 1.0), [None, None], [b[:40], b[40:]], momentum=True, ops=ops)
    s.run(4000)
    obj = 0.5 * np.sum((A @ s.x - b) ** 2)
    obj_ref = 0.5 * np.sum((A @ x_ref - b) ** 2)
    assert obj <= obj_ref * (1 + 1e-10)
    assert (x_ref == 0).any()                      # some constraints are active
    # KKT: x >= 0, gradient >= 0 where x = 0, gradient ~ 0 where x > 0
    grad = A.T @ (A @ s.x - b)
    scale = np.abs(A.T @ b).max()
    assert s.x.min() >= 0.0
    assert grad[s.x == 0].min() >= -1e-7 * scale
    assert np.max(np.abs(grad[s.x > 1e-9])) <= 1e-7 * scale
    assert np.max(np.abs(s.x - x_ref)) <= 1e-6 * np.max(x_ref)
    # with momentum off (projected gradient) the same minimum is approached
    pg = orc.Solver(W.grid(3, 1.0), [None, None], [b[:40], b[40:]], momentum=False, ops=ops)
    pg.run(4000)
    assert 0.5 * np.sum((A @ pg.x - b) ** 2) <= obj_ref * (1 + 1e-6)


def test_projected_gradient_decreases_objective(orc):
    g, cams, A = _tiny_problem(orc)
    xt = W.uniform_random(64, seed=6).astype(np.float64)
    b = A @ xt
    s = orc.Solver(g, cams, [b[:256], b[256:]], momentum=False, beta=0.01,
                   psi_kind=orc.PSI_HYPERBOLA, delta=0.1)
    prev = s.objective()
    for _ in range(30):
        s.step()
        cur = s.objective()
        assert cur <= prev * (1 + 1e-12)        # majorize-minimize is monotone
        prev = cur
    assert s.x.min() >= 0.0


def test_zero_majorizer_voxels_keep_start_value(orc):
    # a voxel no ray sees has D_j = 0; with beta = 0 its step is zero
    g = W.grid(6, 10.0)
    cam = W.plenoptic_camera(16, 2, (1, 1), 10, phi_deg=0.0, distance=40.0)
    N = 216
    D = orc.backproject(g, [cam], orc.project(g, [cam], np.ones(N)))
    assert (D == 0).any() and (D > 0).any()
    x0 = np.full(N, 0.3)
    y = orc.project(g, [cam], W.uniform_random(N, seed=1).astype(np.float64))
    s = orc.Solver(g, [cam], [y], momentum=False, x0=x0)
    s.run(3)
    assert np.all(s.x[D == 0] == 0.3)
    assert math.isfinite(s.rho)
