"""FP64 reference of the warm-start network's operations.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain numpy definitions:
a "same" 3-D convolution written as a sum over the kernel taps, its input
and weight gradients written out from that sum, 2x2x2 max pooling, nearest
2x upsampling, and the encoder-decoder forward built from them.  Pinned in
tests/test_oracle_nn.py against torch.nn.functional in float64 on the CPU.

Layouts match the library: activations [D][H][W][C]; weights [Cout][taps*Cin]
with tap = dz*9 + dy*3 + dx (offsets -1..1) and the input channel fastest.
"""
from __future__ import annotations

import numpy as np


def taps_of(ks: int):
    if ks == 1:
        return [(0, 0, 0)]
    return [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def shift(x, dz, dy, dx):
    """s[z, y, x] = x[z + dz, y + dy, x + dx], zero outside the grid."""
    D, H, W = x.shape[:3]
    out = np.zeros_like(x)
    zs, ze = max(0, -dz), min(D, D - dz)
    ys, ye = max(0, -dy), min(H, H - dy)
    xs, xe = max(0, -dx), min(W, W - dx)
    out[zs:ze, ys:ye, xs:xe] = x[zs + dz:ze + dz, ys + dy:ye + dy, xs + dx:xe + dx]
    return out


def conv3d(x, w, b, ks: int):
    """out[v, co] = b[co] + sum_tap sum_ci x[v + tap, ci] w[co, tap*Cin + ci]."""
    x = np.asarray(x, np.float64)
    cin = x.shape[3]
    cout = w.shape[0]
    out = np.zeros(x.shape[:3] + (cout,))
    for t, (dz, dy, dx) in enumerate(taps_of(ks)):
        wt = np.asarray(w[:, t * cin:(t + 1) * cin], np.float64)      # (cout, cin)
        out += shift(x, dz, dy, dx) @ wt.T
    if b is not None:
        out += np.asarray(b, np.float64)
    return out


def conv3d_dgrad(g, w, cin: int, ks: int):
    """d/dx of sum(g * conv3d(x)): dx[v, ci] = sum_tap sum_co g[v - tap, co] w[co, tap*Cin + ci]."""
    g = np.asarray(g, np.float64)
    dx = np.zeros(g.shape[:3] + (cin,))
    for t, (dz, dy, dx_) in enumerate(taps_of(ks)):
        wt = np.asarray(w[:, t * cin:(t + 1) * cin], np.float64)
        dx += shift(g, -dz, -dy, -dx_) @ wt
    return dx


def conv3d_wgrad(x, g, ks: int):
    """d/dw of sum(g * conv3d(x)): dw[co, tap*Cin + ci] = sum_v g[v, co] x[v + tap, ci]."""
    x = np.asarray(x, np.float64)
    g = np.asarray(g, np.float64)
    cin, cout = x.shape[3], g.shape[3]
    dw = np.zeros((cout, len(taps_of(ks)) * cin))
    G = g.reshape(-1, cout)
    for t, (dz, dy, dx) in enumerate(taps_of(ks)):
        dw[:, t * cin:(t + 1) * cin] = G.T @ shift(x, dz, dy, dx).reshape(-1, cin)
    return dw


def maxpool2(x):
    D, H, W, C = x.shape
    r = x.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C)
    return r.max(axis=(1, 3, 5))


def upsample2(x):
    return np.repeat(np.repeat(np.repeat(x, 2, axis=0), 2, axis=1), 2, axis=2)


def relu(x):
    return np.maximum(x, 0.0)


# Encoder-decoder: (name, inputs, cin0, cin1, cout, ksize, upsample, relu)
ARCH = [
    ("e11", ("in",), 1, 0, 16, 3, False, True),
    ("e12", ("e11",), 16, 0, 16, 3, False, True),
    ("e21", ("p1",), 16, 0, 32, 3, False, True),
    ("e22", ("e21",), 32, 0, 32, 3, False, True),
    ("e31", ("p2",), 32, 0, 64, 3, False, True),
    ("e32", ("e31",), 64, 0, 64, 3, False, True),
    ("e41", ("p3",), 64, 0, 128, 3, False, True),
    ("e42", ("e41",), 128, 0, 128, 3, False, True),
    ("u3", ("e42",), 128, 0, 64, 3, True, True),
    ("d31", ("u3", "e32"), 64, 64, 64, 3, False, True),
    ("d32", ("d31",), 64, 0, 64, 3, False, True),
    ("u2", ("d32",), 64, 0, 32, 3, True, True),
    ("d21", ("u2", "e22"), 32, 32, 32, 3, False, True),
    ("d22", ("d21",), 32, 0, 32, 3, False, True),
    ("u1", ("d22",), 32, 0, 16, 3, True, True),
    ("d11", ("u1", "e12"), 16, 16, 16, 3, False, True),
    ("d12", ("d11",), 16, 0, 16, 3, False, True),
    ("out", ("d12",), 16, 0, 1, 1, False, False),
]
POOLS = {"p1": "e12", "p2": "e22", "p3": "e32"}


def unet_forward(params, x_in, round_bf16=None):
    """Forward of the encoder-decoder in FP64.  params: name -> (w, b).
    round_bf16: optional function applied to every activation stored
    between layers (to mirror BF16 storage)."""
    acts = {"in": np.asarray(x_in, np.float64)}
    rnd = round_bf16 or (lambda a: a)
    order = ["e11", "e12", "p1", "e21", "e22", "p2", "e31", "e32", "p3", "e41", "e42",
             "u3", "d31", "d32", "u2", "d21", "d22", "u1", "d11", "d12", "out"]
    spec = {a[0]: a for a in ARCH}
    for name in order:
        if name in POOLS:
            acts[name] = maxpool2(acts[POOLS[name]])
            continue
        _, ins, c0, c1, cout, ks, up, act = spec[name]
        x = acts[ins[0]]
        if up:
            x = upsample2(x)
        if len(ins) == 2:
            x = np.concatenate([x, acts[ins[1]]], axis=3)
        w, b = params[name]
        y = conv3d(x, w, b, ks)
        if act:
            y = relu(y)
        acts[name] = y if name == "out" else rnd(y)
    return acts["out"][..., 0], acts
