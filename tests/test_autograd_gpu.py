"""Differentiable projector (torch.autograd.Function with the adjoint kernel
as backward) against FP64 central differences of the oracle's loss.

The loss L(x) = 1/2 ||A x - y||^2 is quadratic, so central differences have
no truncation error: (L(x + h v) - L(x - h v)) / 2h = v^T A^T (A x - y)
exactly, up to FP64 rounding.  For a direction v supported on a 16^3
sub-volume only the pixels whose rays cross it change, so the oracle loss is
evaluated on those pixels alone (found from the oracle projection of the
sub-volume's indicator, one voxel wider for the trilinear footprint).

Each mismatch |fd - v.grad| is divided by ||A v|| ||r|| on those pixels
(r = A x - y), the Cauchy-Schwarz bound of v.grad = <A v, r>.  The GPU
gradient is built from the FP32 residual, whose error is about 1e-7 ||A x||
per pixel; for a single-voxel direction whose positive and negative residual
contributions cancel, v.grad itself can be far smaller than that error, so
|v.grad| is not a usable scale there.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1812_03358_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    from paper_1812_03358_amd import autograd, ltm
    ltm.lib()
    return ltm, autograd


def _fd_check(orc, ltm, autograd, g, cams, x, y, sub_lo, sub_n, n_dirs, n_vox, seed):
    n = (g["nz"], g["ny"], g["nx"])
    # pixels that see the sub-volume (oracle only)
    ind = np.zeros(n)
    lo = [max(0, s - 1) for s in sub_lo]
    ind[lo[0]:sub_lo[0] + sub_n + 1, lo[1]:sub_lo[1] + sub_n + 1, lo[2]:sub_lo[2] + sub_n + 1] = 1.0
    offs = np.cumsum([0] + [c["det_nu"] * c["det_nv"] for c in cams])
    pix = [np.nonzero(orc.project(g, [c], ind.reshape(-1)))[0] for c in cams]
    assert all(p.size > 0 for p in pix)

    def residuals(v):
        return [orc.project_pixels(g, c, v, pix[k]) - y[offs[k] + pix[k]].astype(np.float64)
                for k, c in enumerate(cams)]

    def loss_diff(vp, vm):
        # L(vp) - L(vm) summed pixel by pixel, (r+^2 - r-^2)/2 = (r+ - r-)(r+ + r-)/2,
        # so the large equal parts of the two losses cancel before summation
        return sum(0.5 * float(np.dot(a - b, a + b)) for a, b in zip(residuals(vp), residuals(vm)))

    # GPU gradient through autograd
    xd = torch.from_numpy(x.reshape(-1).astype(np.float32)).cuda().requires_grad_(True)
    plan = ltm.Plan(g, cams)
    yd = torch.from_numpy(y.astype(np.float32)).cuda()
    pred = autograd.project(xd, plan)
    (0.5 * ((pred - yd) ** 2).sum()).backward()
    grad = xd.grad.detach().cpu().numpy().astype(np.float64)

    x64 = xd.detach().cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(seed)
    h = 1e-4
    errs = []
    dirs = []
    for _ in range(n_dirs):
        v = np.zeros(n)
        v[sub_lo[0]:sub_lo[0] + sub_n, sub_lo[1]:sub_lo[1] + sub_n, sub_lo[2]:sub_lo[2] + sub_n] = \
            rng.standard_normal((sub_n,) * 3)
        dirs.append(v.reshape(-1))
    for _ in range(n_vox):
        v = np.zeros(n)
        v[tuple(sl + rng.integers(0, sub_n) for sl in sub_lo)] = 1.0
        dirs.append(v.reshape(-1))
    r0 = np.concatenate(residuals(x64))
    for v in dirs:
        fd = loss_diff(x64 + h * v, x64 - h * v) / (2 * h)
        an = float(np.dot(grad, v))
        Av = np.concatenate([orc.project_pixels(g, c, v, pix[k]) for k, c in enumerate(cams)])
        scale = np.linalg.norm(Av) * np.linalg.norm(r0) + 1e-30
        errs.append(abs(fd - an) / scale)
    print("max FD mismatch", max(errs), flush=True)
    assert max(errs) < 1e-5
    return plan


def test_fd_small(orc, mods):
    ltm, autograd = mods
    g = W.grid((24, 22, 20), 5.0)
    cams = [W.plenoptic_camera(96, 6, (2, 1), 41, phi_deg=p) for p in (0.0, 30.0)]
    xt = W.flame(24, seed=4)[:20, :22, :24]
    x = xt + 0.05 * W.uniform_random(xt.shape, seed=5)
    y = orc.project(g, cams, xt.astype(np.float64).reshape(-1)).astype(np.float32)
    _fd_check(orc, ltm, autograd, g, cams, x, y, (2, 3, 4), 16, 8, 16, seed=1)


def test_fd_differentiable_256(orc, mods):
    ltm, autograd = mods
    cfg = W.config_differentiable()
    g, cams = cfg["grid"], cfg["cameras"]
    xt = cfg["volume"]()
    x = xt + 0.02 * W.uniform_random(xt.shape, seed=6)
    y = orc.project(g, cams, xt.astype(np.float64).reshape(-1)).astype(np.float32)
    plan = _fd_check(orc, ltm, autograd, g, cams, x, y, (120, 120, 120), 16, 32, 64, seed=2)
    # dot test of the same plan at full size
    xv = torch.from_numpy(W.uniform_random(256 ** 3, seed=7)).cuda()
    yv = torch.from_numpy(W.uniform_random(plan.n_meas, seed=8)).cuda()
    Ax = plan.project(xv).double()
    Aty = plan.backproject(yv).double()
    dot = abs(float((Ax * yv.double()).sum() - (xv.double() * Aty).sum())) / float(
        Ax.norm() * yv.double().norm())
    print("dot", dot, flush=True)
    assert dot < 1e-9


def test_gradient_descent_reduces_loss(orc, mods):
    ltm, autograd = mods
    cfg = W.config_thin_lens()
    g, cams = cfg["grid"], cfg["cameras"]
    plan = ltm.Plan(g, cams)
    y = torch.from_numpy(orc.project(g, cams, cfg["volume"]().astype(np.float64).reshape(-1))
                         .astype(np.float32)).cuda()
    x = torch.zeros(plan.n_voxels, device="cuda", requires_grad=True)
    opt = torch.optim.Adam([x], lr=0.02)
    losses = []
    for _ in range(30):
        opt.zero_grad()
        loss = 0.5 * ((autograd.project(x, plan) - y) ** 2).sum()
        loss.backward()
        opt.step()
        losses.append(float(loss))
    assert losses[-1] < 0.2 * losses[0]
    # the backward of the adjoint is the projector
    yv = torch.rand(plan.n_meas, device="cuda", requires_grad=True)
    xb = autograd.backproject(yv, plan)
    w = torch.rand(plan.n_voxels, device="cuda")
    (xb * w).sum().backward()
    assert torch.allclose(yv.grad, plan.project(w), rtol=1e-5, atol=1e-6)
