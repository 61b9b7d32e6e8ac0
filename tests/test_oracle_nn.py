"""Pins of the FP64 network oracle against torch.nn.functional (float64, CPU):
conv3d with zero padding, its input and weight gradients by autograd,
max pooling and nearest upsampling."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
import torch.nn.functional as F

from oracle import nn as onn


def _torch_w(w, cin, ks):
    # [cout][taps*cin] (tap-major, ci fastest) -> torch [cout][cin][kz][ky][kx]
    cout = w.shape[0]
    return torch.from_numpy(w.reshape(cout, ks, ks, ks, cin).transpose(0, 4, 1, 2, 3).copy())


@pytest.mark.parametrize("cin,cout,ks", [(1, 16, 3), (16, 8, 3), (8, 1, 1), (24, 16, 3)])
def test_conv_matches_torch(cin, cout, ks):
    rng = np.random.default_rng(cin * 100 + cout)
    x = rng.standard_normal((5, 6, 7, cin))
    w = rng.standard_normal((cout, ks ** 3 * cin))
    b = rng.standard_normal(cout)
    ref = F.conv3d(torch.from_numpy(x.transpose(3, 0, 1, 2)[None].copy()), _torch_w(w, cin, ks),
                   torch.from_numpy(b), padding=ks // 2)[0].numpy().transpose(1, 2, 3, 0)
    assert np.max(np.abs(onn.conv3d(x, w, b, ks) - ref)) < 1e-11


@pytest.mark.parametrize("cin,cout,ks", [(4, 8, 3), (8, 1, 1)])
def test_conv_gradients_match_autograd(cin, cout, ks):
    rng = np.random.default_rng(7)
    x = rng.standard_normal((4, 5, 6, cin))
    w = rng.standard_normal((cout, ks ** 3 * cin))
    g = rng.standard_normal((4, 5, 6, cout))
    xt = torch.from_numpy(x.transpose(3, 0, 1, 2)[None].copy()).requires_grad_(True)
    wt = _torch_w(w, cin, ks).requires_grad_(True)
    y = F.conv3d(xt, wt, padding=ks // 2)
    (y * torch.from_numpy(g.transpose(3, 0, 1, 2)[None].copy())).sum().backward()
    dx_ref = xt.grad[0].numpy().transpose(1, 2, 3, 0)
    dw_ref = wt.grad.numpy().transpose(0, 2, 3, 4, 1).reshape(cout, -1)
    assert np.max(np.abs(onn.conv3d_dgrad(g, w, cin, ks) - dx_ref)) < 1e-10
    assert np.max(np.abs(onn.conv3d_wgrad(x, g, ks) - dw_ref)) < 1e-10


def test_pool_and_upsample_match_torch():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((4, 6, 8, 3))
    xt = torch.from_numpy(x.transpose(3, 0, 1, 2)[None].copy())
    mp = F.max_pool3d(xt, 2)[0].numpy().transpose(1, 2, 3, 0)
    up = F.interpolate(xt, scale_factor=2, mode="nearest")[0].numpy().transpose(1, 2, 3, 0)
    assert np.array_equal(onn.maxpool2(x), mp)
    assert np.array_equal(onn.upsample2(x), up)


def test_unet_shapes_and_linear_output():
    rng = np.random.default_rng(1)
    params = {}
    for name, _, c0, c1, cout, ks, _, _ in onn.ARCH:
        fan = ks ** 3 * (c0 + c1)
        params[name] = (rng.standard_normal((cout, fan)) * np.sqrt(2.0 / fan), np.zeros(cout))
    out, acts = onn.unet_forward(params, rng.uniform(0, 1, (8, 8, 8, 1)))
    # the output layer is linear (its ReLU applies only at inference) ...
    assert out.shape == (8, 8, 8) and out.min() < 0.0 < out.max()
    # ... and every hidden activation passed its ReLU
    assert all(acts[k].min() >= 0.0 for k in acts if k not in ("in", "out"))
    assert acts["e42"].shape == (1, 1, 1, 128)
