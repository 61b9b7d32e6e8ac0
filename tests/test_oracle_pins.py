"""Pins of the oracle functions that the other oracle tests reach only
indirectly.

* count_valid_rays: a brute-force count over every pixel, light path and
  angular sample, with the box intersection done here by a different
  algorithm (crossings of the six face rectangles, not the slab method), for a
  posed square-array plenoptic camera, a hexagonal camera and a single-lens
  camera, each seeing a box smaller than its field of view so that rays miss;
* the monitored residual rho = ||p - g y||_W / ||g y||_W: rho(0) = 1,
  rho(x_true) = 0 on noiseless data, and a hand-worked two-camera case with
  weights and an estimated gain (rho = sqrt(4/15));
* one projected-gradient step and two FISTA steps of the reconstruction
  algorithm table on a hand-worked 3 x 4 system, including the momentum
  factor (t - 1)/t+ with t = (1 + sqrt 5)/2 after the first step, and the
  l1 step x = [w - nu]_+;
* the network oracle's whole encoder-decoder forward against the same
  architecture assembled from torch.nn.functional primitives in float64.
"""
import math

import numpy as np
import pytest

from paper_1812_03358_amd import workloads as W


# ---------------------------------------------------------------- ray counts
def _chord_by_faces(g, O, w):
    """Length (in ray parameter) of the ray's part inside the closed box
    [-n d/2, n d/2]^3 with parameter >= 0, from the points where it crosses
    the six face rectangles (and its origin when that lies inside)."""
    h = [0.5 * g["nx"] * g["pitch"], 0.5 * g["ny"] * g["pitch"], 0.5 * g["nz"] * g["pitch"]]
    ts = []
    if all(abs(O[a]) <= h[a] for a in range(3)):
        ts.append(0.0)
    for a in range(3):
        if w[a] == 0.0:
            continue
        for side in (-1.0, 1.0):
            t = (side * h[a] - O[a]) / w[a]
            if t < 0.0:
                continue
            p = O + t * w
            if all(abs(p[b]) <= h[b] * (1 + 1e-12) for b in range(3) if b != a):
                ts.append(t)
    if len(ts) < 2:
        return 0.0
    return max(ts) - min(ts)


def _brute_count(orc, g, cam):
    count = 0
    for iv in range(cam["det_nv"]):
        for iu in range(cam["det_nu"]):
            for path in range(orc.n_paths(cam)):
                for rv in range(cam["rays_v"]):
                    for ru in range(cam["rays_u"]):
                        ok, O, w = orc.trace_path(cam, iu, iv, path, ru, rv)
                        if ok and _chord_by_faces(g, O, w) > 1e-9:
                            count += 1
    return count


@pytest.mark.parametrize("which", ["plenoptic", "hex", "single"])
def test_count_valid_rays_matches_brute_force(orc, which):
    if which == "plenoptic":
        # 32^2 px behind 2^2 lenslets see 6 mm at 1680 mm; the box is 4.8 mm
        cam = W.plenoptic_camera(32, 2, (2, 2), 8, phi_deg=30.0)
        g = W.grid(6, 0.8)
    elif which == "hex":
        # out of focus (1500 mm), so that the bundles spread over the box
        cam = W.hex_plenoptic_camera(24, (5, 5), (2, 3), 8, phi_deg=-20.0, distance=1500.0)
        g = W.grid((5, 4, 6), 0.5)
    else:
        # 48^2 px of 5 um see 5.5 mm at 722 mm
        cam = W.single_lens_camera(48, (3, 3), 8, phi_deg=45.0)
        g = W.grid((6, 5, 7), 0.7)
    got = orc.count_valid_rays(g, cam, threads=3)
    want = _brute_count(orc, g, cam)
    total = W.n_pixels(cam) * cam["rays_u"] * cam["rays_v"] * orc.n_paths(cam)
    # the geometry is chosen so that both occlusion and misses remove rays
    assert 0 < want < total
    assert got == want


# ---------------------------------------------------------------- residual
def _explicit_ops(*mats):
    return [((lambda v, A=A: A @ v), (lambda r, A=A: A.T @ r)) for A in mats]


def test_residual_is_one_at_zero_and_zero_at_the_truth(orc):
    g = W.grid((4, 5, 3), 1.0)
    cams = [W.plenoptic_camera(32, 2, (2, 2), 6, phi_deg=0.0, distance=60.0),
            W.plenoptic_camera(32, 2, (1, 2), 6, phi_deg=90.0, distance=60.0)]
    xt = W.uniform_random(60, seed=4).astype(np.float64)
    ys = [orc.project(g, [c], xt) for c in cams]
    wts = [W.uniform_random(y.size, seed=9 + k, lo=0.5, hi=2.0).astype(np.float64)
           for k, y in enumerate(ys)]
    for gains in (False, True):
        s = orc.Solver(g, cams, ys, ws=wts, gains=gains)
        assert s.residual(np.zeros(60)) == 1.0      # with gains: g_2 = 0 at p = 0
        assert s.residual(xt) < 1e-14
    s = orc.Solver(g, cams, ys, ws=wts)
    assert s.residual(np.zeros(60)) == 1.0
    # a scaled truth: rho = |a - 1| exactly when gains are off
    assert abs(s.residual(0.75 * xt) - 0.25) < 1e-14
    # with gains, camera 2's gain absorbs a camera-2-only scale: a second
    # camera reading 1/2 of the light leaves rho = 0
    s = orc.Solver(g, cams, [ys[0], 0.5 * ys[1]], ws=wts, gains=True)
    assert s.residual(xt) < 1e-14
    s = orc.Solver(g, cams, [ys[0], 0.5 * ys[1]], ws=wts, gains=False)
    assert s.residual(xt) > 0.1


def test_residual_hand_worked_weights_and_gain(orc):
    # camera 1: A1 = [[1, 0], [0, 2]], y1 = (2, 1), W1 = diag(1, 3);
    # camera 2: A2 = [[1, 1]], y2 = (4), W2 = (2); evaluated at v = (1, 1):
    #   p1 = (1, 2), p2 = (2); gain g2 = y2 W2 p2 / y2 W2 y2 = 16/32 = 1/2;
    #   numerator   1 (1-2)^2 + 3 (2-1)^2 + 2 (2 - 2)^2 = 4,
    #   denominator 1 * 4 + 3 * 1 + 2 * (1/2 * 4)^2 = 15,  rho = sqrt(4/15)
    A1 = np.array([[1.0, 0.0], [0.0, 2.0]])
    A2 = np.array([[1.0, 1.0]])
    def solver(gains):
        return orc.Solver(W.grid((2, 1, 1), 1.0), [None, None],
                          [np.array([2.0, 1.0]), np.array([4.0])],
                          ws=[np.array([1.0, 3.0]), np.array([2.0])], gains=gains,
                          ops=_explicit_ops(A1, A2))
    v = np.array([1.0, 1.0])
    assert abs(solver(True).residual(v) - math.sqrt(4.0 / 15.0)) < 1e-15
    # without gains: numerator 4 + 2 (2-4)^2 = 12, denominator 7 + 2*16 = 39
    assert abs(solver(False).residual(v) - math.sqrt(12.0 / 39.0)) < 1e-15


# ---------------------------------------------------------------- one step
# A = [[1,0,1,0],[0,1,1,0],[0,0,0,2]], y = (2, 1, 4), W = I.
#   D = A^T A 1 = (2, 2, 4, 4).
#   step 1 from x = z = 0: g = -A^T y = (-2, -1, -3, -8),
#       x1 = [0 - g / D]_+ = (1, 1/2, 3/4, 2); rho at z = 0 is 1.
#   step 2 from z1 = x1: A z1 = (7/4, 5/4, 4), r = (-1/4, 1/4, 0),
#       g = (-1/4, 1/4, 0, 0), x2 = (9/8, 3/8, 3/4, 2),
#       rho at z1 = sqrt(1/8) / sqrt(21).
#   FISTA: t1 = (1 + sqrt 5)/2 and z1 = x1 (t0 - 1 = 0); t2 = (1 + sqrt(7 + 2
#       sqrt 5))/2 (since t1^2 = t1 + 1) and z2 = x2 + ((t1 - 1)/t2)(x2 - x1).
_A = np.array([[1.0, 0.0, 1.0, 0.0], [0.0, 1.0, 1.0, 0.0], [0.0, 0.0, 0.0, 2.0]])
_Y = np.array([2.0, 1.0, 4.0])
_X1 = np.array([1.0, 0.5, 0.75, 2.0])
_X2 = np.array([1.125, 0.375, 0.75, 2.0])


def _one_camera(orc, momentum, nu=0.0):
    return orc.Solver(W.grid((4, 1, 1), 1.0), [None], [_Y], momentum=momentum, nu=nu,
                      ops=_explicit_ops(_A))


def test_projected_gradient_steps_by_hand(orc):
    s = _one_camera(orc, momentum=False)
    assert np.array_equal(s.D, [2.0, 2.0, 4.0, 4.0])
    assert s.step() == 1.0
    assert np.array_equal(s.x, _X1) and np.array_equal(s.z, _X1)
    rho = s.step()
    assert abs(rho - math.sqrt(0.125 / 21.0)) < 1e-15
    assert np.array_equal(s.x, _X2) and np.array_equal(s.z, _X2)


def test_fista_steps_by_hand(orc):
    s = _one_camera(orc, momentum=True)
    s.step()
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    assert abs(s.t - phi) < 1e-15
    assert np.array_equal(s.x, _X1) and np.array_equal(s.z, _X1)
    s.step()
    t2 = (1.0 + math.sqrt(7.0 + 2.0 * math.sqrt(5.0))) / 2.0
    assert abs(s.t - t2) < 1e-14
    mom = (phi - 1.0) / t2              # 0.2818...; (t-1)/t would give 0.382
    assert np.array_equal(s.x, _X2)
    assert np.max(np.abs(s.z - (_X2 + mom * (_X2 - _X1)))) < 1e-15
    assert abs(s.z[0] - (1.125 + 0.125 * mom)) < 1e-15 and abs(mom - 0.28176) < 1e-5


def test_l1_step_by_hand(orc):
    # nu = 1/2: x1 = [(1, 1/2, 3/4, 2) - 1/2]_+ = (1/2, 0, 1/4, 3/2)
    s = _one_camera(orc, momentum=False, nu=0.5)
    s.step()
    assert np.array_equal(s.x, [0.5, 0.0, 0.25, 1.5])


# ---------------------------------------------------------------- network
torch = pytest.importorskip("torch")


def _torch_unet(params, x):
    """The encoder-decoder of the warm start, assembled from
    torch.nn.functional in float64: per level two 3x3x3 conv + ReLU, 2x max
    pooling down; on the way up nearest 2x upsampling into a 3x3x3 conv +
    ReLU, then the channel concatenation [upsampled path, encoder skip] into
    two 3x3x3 conv + ReLU; a final linear 1x1x1 conv."""
    import torch.nn.functional as F

    def conv(name, h):
        w, b = params[name]
        cout = w.shape[0]
        ks = 1 if name == "out" else 3
        cin = w.shape[1] // ks ** 3
        wt = torch.from_numpy(w.reshape(cout, ks, ks, ks, cin).transpose(0, 4, 1, 2, 3).copy())
        return F.conv3d(h, wt, torch.from_numpy(b), padding=ks // 2)

    r = F.relu
    h = torch.from_numpy(np.asarray(x, np.float64)[None, None].copy())
    e1 = r(conv("e12", r(conv("e11", h))))
    e2 = r(conv("e22", r(conv("e21", F.max_pool3d(e1, 2)))))
    e3 = r(conv("e32", r(conv("e31", F.max_pool3d(e2, 2)))))
    e4 = r(conv("e42", r(conv("e41", F.max_pool3d(e3, 2)))))
    up = lambda t: F.interpolate(t, scale_factor=2, mode="nearest")
    d3 = r(conv("d32", r(conv("d31", torch.cat([r(conv("u3", up(e4))), e3], 1)))))
    d2 = r(conv("d22", r(conv("d21", torch.cat([r(conv("u2", up(d3))), e2], 1)))))
    d1 = r(conv("d12", r(conv("d11", torch.cat([r(conv("u1", up(d2))), e1], 1)))))
    return conv("out", d1)[0, 0].numpy(), e4[0].numpy().transpose(1, 2, 3, 0)


def test_unet_forward_matches_torch_functional():
    from oracle import nn as onn

    rng = np.random.default_rng(12)
    params = {}
    for name, _, c0, c1, cout, ks, _, _ in onn.ARCH:
        fan = ks ** 3 * (c0 + c1)
        params[name] = (rng.standard_normal((cout, fan)) * np.sqrt(2.0 / fan),
                        0.1 * rng.standard_normal(cout))
    x = rng.uniform(0, 1, (16, 8, 8))
    out, acts = onn.unet_forward(params, x[..., None])
    ref, e4 = _torch_unet(params, x)
    assert out.shape == (16, 8, 8)
    assert np.max(np.abs(acts["e42"] - e4)) <= 1e-11 * np.max(np.abs(e4))
    assert np.max(np.abs(out - ref)) <= 1e-11 * np.max(np.abs(ref))
    # a swapped concatenation order is a different network
    swapped = dict(params)
    w, b = params["d11"]
    swapped["d11"] = (np.concatenate([w.reshape(16, 27, 32)[:, :, 16:], w.reshape(16, 27, 32)[:, :, :16]],
                                     axis=2).reshape(16, -1), b)
    out2, _ = onn.unet_forward(swapped, x[..., None])
    assert np.max(np.abs(out2 - ref)) > 1e-3 * np.max(np.abs(ref))
