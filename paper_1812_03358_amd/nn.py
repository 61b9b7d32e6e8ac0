"""Warm-start encoder-decoder on the library's BF16 MFMA kernels.

A 3-D U-Net-style network (4 levels, 16/32/64/128 channels, two 3x3x3
convolutions per level with bias + ReLU, 2x max pooling down, nearest 2x
upsampling + 3x3x3 convolution up, skip concatenation, final 1x1x1
convolution + ReLU) maps the normalized backprojection A^T y / max to a
starting volume for the reconstruction.  Forward, backward and the Adam
update all run in libltm's kernels (ltm_nn_*); this module only sequences
them and owns the buffers (torch tensors as device memory).
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import ltm as _ltm

# (name, inputs, c0, c1, cout, ksize, upsample) -- every layer has bias + ReLU
ARCH = [
    ("e11", ("in",), 1, 0, 16, 3, False),
    ("e12", ("e11",), 16, 0, 16, 3, False),
    ("e21", ("p1",), 16, 0, 32, 3, False),
    ("e22", ("e21",), 32, 0, 32, 3, False),
    ("e31", ("p2",), 32, 0, 64, 3, False),
    ("e32", ("e31",), 64, 0, 64, 3, False),
    ("e41", ("p3",), 64, 0, 128, 3, False),
    ("e42", ("e41",), 128, 0, 128, 3, False),
    ("u3", ("e42",), 128, 0, 64, 3, True),
    ("d31", ("u3", "e32"), 64, 64, 64, 3, False),
    ("d32", ("d31",), 64, 0, 64, 3, False),
    ("u2", ("d32",), 64, 0, 32, 3, True),
    ("d21", ("u2", "e22"), 32, 32, 32, 3, False),
    ("d22", ("d21",), 32, 0, 32, 3, False),
    ("u1", ("d22",), 32, 0, 16, 3, True),
    ("d11", ("u1", "e12"), 16, 16, 16, 3, False),
    ("d12", ("d11",), 16, 0, 16, 3, False),
    ("out", ("d12",), 16, 0, 1, 1, False),
]
POOLS = [("p1", "e12"), ("p2", "e22"), ("p3", "e32")]
ORDER = ["e11", "e12", "p1", "e21", "e22", "p2", "e31", "e32", "p3", "e41", "e42",
         "u3", "d31", "d32", "u2", "d21", "d22", "u1", "d11", "d12", "out"]

_VP, _U32, _U64, _D = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double


ConvDesc = _ltm.ConvDesc


def _lib():
    return _ltm.lib()


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _s(stream=None):
    return _ltm._stream(stream)


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round FP32/FP64 values to the nearest BF16 (ties to even), as float32."""
    f = np.asarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def to_bf16_tensor(a: np.ndarray, device="cuda") -> torch.Tensor:
    """float array -> uint16 BF16 bit patterns on the device (int16 tensor)."""
    b = bf16_round(a).view(np.uint32) >> 16
    return torch.from_numpy(b.astype(np.uint16).view(np.int16).copy()).to(device)


def from_bf16_tensor(t: torch.Tensor) -> np.ndarray:
    u = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32)


def conv_desc(ks, d, h, w, c0, c1, cout, up, relu=1, out_f32=0, split=None):
    return ConvDesc(ks, d, h, w, c0, c1, cout, int(up), relu, out_f32,
                    cout if split is None else split, 0)


class Layer:
    def __init__(self, name, ins, c0, c1, cout, ks, up, rng, device):
        self.name, self.ins, self.c0, self.c1, self.cout, self.ks, self.up = \
            name, ins, c0, c1, cout, ks, up
        self.cin = c0 + c1
        self.K = ks ** 3 * self.cin
        fan = self.K
        w = rng.standard_normal((cout, self.K)) * math.sqrt(2.0 / fan)
        self.w = torch.from_numpy(w.astype(np.float32)).to(device)
        self.b = torch.zeros(cout, device=device)
        self.dw = torch.zeros_like(self.w)
        self.db = torch.zeros_like(self.b)
        self.mw, self.vw = torch.zeros_like(self.w), torch.zeros_like(self.w)
        self.mb, self.vb = torch.zeros_like(self.b), torch.zeros_like(self.b)
        nf, nb = _U64(), _U64()
        _ltm._check(_lib().ltm_nn_packed_sizes(cout, self.cin, ks, ctypes.byref(nf), ctypes.byref(nb)))
        self.wf = torch.zeros(nf.value, dtype=torch.int16, device=device)
        self.wb = torch.zeros(nb.value, dtype=torch.int16, device=device)

    def pack(self, stream=None):
        _ltm._check(_lib().ltm_nn_pack_weights(_p(self.w), self.cout, self.cin, self.ks, _p(self.wf),
                                               _p(self.wb), _s(stream)))


class UNet:
    """The warm-start network.  forward() keeps the activations for
    backward(); step() applies Adam.  Volumes are [D][H][W] with D, H, W
    multiples of 8."""

    def __init__(self, seed: int = 0, device="cuda"):
        rng = np.random.default_rng(seed)
        self.device = torch.device(device)
        self.layers = {a[0]: Layer(*a, rng=rng, device=self.device) for a in ARCH}
        self.acts = {}
        self.args = {}
        self.t = 0
        self.pack()
        self._scratch = torch.zeros(64, dtype=torch.int32, device=self.device)
        self._loss = torch.zeros(1, dtype=torch.float64, device=self.device)

    def pack(self, stream=None):
        for L in self.layers.values():
            L.pack(stream)

    def parameters(self):
        for L in self.layers.values():
            yield L.w
            yield L.b

    def state_dict(self):
        return {f"{n}.{k}": getattr(L, k).detach().cpu() for n, L in self.layers.items() for k in ("w", "b")}

    def load_state_dict(self, sd):
        for n, L in self.layers.items():
            L.w.copy_(sd[f"{n}.w"].to(self.device))
            L.b.copy_(sd[f"{n}.b"].to(self.device))
        self.pack()

    def _dims(self, name, D, H, W):
        lvl = {"e1": 0, "e2": 1, "e3": 2, "e4": 3, "u3": 2, "d3": 2, "u2": 1, "d2": 1, "u1": 0, "d1": 0,
               "ou": 0}[name[:2]]
        return D >> lvl, H >> lvl, W >> lvl

    def prep_input(self, aty: torch.Tensor, stream=None) -> torch.Tensor:
        """A^T y (FP32, N) -> network input (BF16 bits, N), scaled by 1/max."""
        out = torch.empty(aty.numel(), dtype=torch.int16, device=self.device)
        _ltm._check(_lib().ltm_nn_prep_input(_p(aty), _p(out), _p(self._scratch), aty.numel(), _s(stream)))
        return out

    def forward(self, x_in: torch.Tensor, D: int, H: int, W: int, stream=None,
                final_relu: bool = False) -> torch.Tensor:
        """x_in: BF16 bits [D*H*W] (one channel).  Returns the FP32 volume.
        The output layer is linear in training (a ReLU there leaves a freshly
        initialized network with almost no positive outputs, hence no
        gradient); inference passes final_relu=True for a nonnegative x0."""
        lib = _lib()
        A = {"in": x_in}
        for name in ORDER:
            if name.startswith("p"):
                src = dict(POOLS)[name]
                d, h, w = self._dims(src, D, H, W)
                C = self.layers[src].cout
                y = torch.empty((d // 2) * (h // 2) * (w // 2) * C, dtype=torch.int16, device=self.device)
                arg = torch.empty(y.numel(), dtype=torch.uint8, device=self.device)
                _ltm._check(lib.ltm_nn_maxpool2(_p(A[src]), _p(y), _p(arg), d, h, w, C, _s(stream)))
                A[name] = y
                self.args[name] = arg
                continue
            L = self.layers[name]
            d, h, w = self._dims(name, D, H, W)
            last = name == "out"
            out = torch.empty(d * h * w * L.cout, dtype=torch.float32 if last else torch.int16,
                              device=self.device)
            desc = conv_desc(L.ks, d, h, w, L.c0, L.c1, L.cout, L.up,
                             int(final_relu) if last else 1, int(last))
            in1 = A[L.ins[1]] if len(L.ins) > 1 else None
            _ltm._check(lib.ltm_nn_conv3d_forward(ctypes.byref(desc), _p(A[L.ins[0]]), _p(in1), _p(L.wf),
                                                  _p(L.b), _p(out), None, _s(stream)))
            A[name] = out
        self.acts = A
        self.dims = (D, H, W)
        return A["out"]

    def loss_and_grad(self, target: torch.Tensor, stream=None):
        """MSE against target (FP32, N); returns (loss tensor, d loss / d out)."""
        self._loss.zero_()
        g = torch.empty_like(self.acts["out"])
        _ltm._check(_lib().ltm_nn_mse(_p(self.acts["out"]), _p(target), _p(g), _p(self._loss),
                                      g.numel(), _s(stream)))
        return self._loss, g

    def backward(self, g_out: torch.Tensor, stream=None):
        """Accumulate dw, db from d loss / d out (FP32, the linear output's
        gradient as ltm_nn_mse returns it)."""
        lib = _lib()
        D, H, W = self.dims
        A = self.acts
        grads = {"out": g_out}
        first = {"out": True}

        def add_grad(name, t):
            if name in grads:
                _ltm._check(lib.ltm_nn_add(_p(grads[name]), _p(t), t.numel(), _s(stream)))
            else:
                grads[name] = t

        for name in reversed(ORDER):
            if name.startswith("p"):
                src = dict(POOLS)[name]
                d, h, w = self._dims(src, D, H, W)
                C = self.layers[src].cout
                gsrc = grads.get(src)
                if gsrc is None:
                    gsrc = torch.zeros(d * h * w * C, device=self.device)
                    grads[src] = gsrc
                _ltm._check(lib.ltm_nn_maxpool2_backward(_p(grads[name]), _p(self.args[name]), _p(gsrc),
                                                         d, h, w, C, _s(stream)))
                continue
            L = self.layers[name]
            d, h, w = self._dims(name, D, H, W)
            n = d * h * w * L.cout
            gpre = torch.empty(n, dtype=torch.int16, device=self.device)
            relu = 0 if name == "out" else 1
            _ltm._check(lib.ltm_nn_relu_backward(_p(grads[name]), _p(A[name]) if relu else None, relu,
                                                 _p(gpre), _p(L.db), n, L.cout, _s(stream)))
            desc = conv_desc(L.ks, d, h, w, L.c0, L.c1, L.cout, L.up)
            in1 = A[L.ins[1]] if len(L.ins) > 1 else None
            _ltm._check(lib.ltm_nn_conv3d_wgrad(ctypes.byref(desc), _p(A[L.ins[0]]), _p(in1), _p(gpre),
                                                _p(L.dw), _s(stream)))
            if L.ins[0] == "in":
                continue
            dx0 = torch.empty(d * h * w * L.c0, device=self.device)
            dx1 = torch.empty(d * h * w * L.c1, device=self.device) if L.c1 else None
            _ltm._check(lib.ltm_nn_conv3d_dgrad(ctypes.byref(desc), _p(gpre), _p(L.wb), _p(dx0), _p(dx1),
                                                _s(stream)))
            if L.up:
                low = torch.empty(dx0.numel() // 8, device=self.device)
                _ltm._check(lib.ltm_nn_upsample2_backward(_p(dx0), _p(low), d, h, w, L.c0, 0, _s(stream)))
                dx0 = low
            add_grad(L.ins[0], dx0)
            if L.c1:
                add_grad(L.ins[1], dx1)

    def step(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, stream=None):
        self.t += 1
        lib = _lib()
        for L in self.layers.values():
            for w, g, m, v in ((L.w, L.dw, L.mw, L.vw), (L.b, L.db, L.mb, L.vb)):
                _ltm._check(lib.ltm_nn_adam(_p(w), _p(g), _p(m), _p(v), w.numel(), lr, b1, b2, eps, self.t,
                                            _s(stream)))
        self.pack(stream)

    def zero_grad(self):
        for L in self.layers.values():
            L.dw.zero_()
            L.db.zero_()
