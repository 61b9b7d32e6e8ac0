"""Warm-start network kernels against the FP64 oracle (oracle/nn.py) on
BF16-rounded operands: conv forward (with concatenation, fused upsampling,
1x1x1 and one-channel cases), input gradient, weight gradient, pooling,
ReLU backward, MSE and Adam.  FP32 accumulation over at most a few thousand
BF16 products gives relative errors near 1e-6; tolerances are 1e-5.
Whole-network checks store activations in BF16 on the GPU, so they compare
at a few 1e-2."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
import torch.nn.functional as F

from oracle import nn as onn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nn():
    from paper_1812_03358_amd import nn as N
    N._lib()
    return N


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _rand(rng, shape, scale=1.0):
    from paper_1812_03358_amd.nn import bf16_round
    return bf16_round(rng.standard_normal(shape) * scale).astype(np.float64)


CASES = [
    # (D, H, W, c0, c1, cout, ks, up)
    (6, 5, 10, 1, 0, 16, 3, 0),
    (8, 8, 8, 16, 0, 16, 3, 0),
    (6, 8, 4, 16, 16, 16, 3, 0),
    (4, 6, 8, 32, 0, 64, 3, 0),
    (4, 4, 6, 64, 64, 64, 3, 0),
    (4, 4, 4, 128, 0, 128, 3, 0),
    (8, 6, 8, 32, 0, 16, 3, 1),
    (6, 5, 7, 16, 0, 1, 1, 0),
    (6, 6, 6, 24, 0, 40, 3, 0),
    # 8 output planes per workgroup (at most 16 input channels) over a ragged depth
    (10, 6, 12, 8, 8, 32, 3, 0),
    # row-staged weight gradient (rows of 128, 64, 32 voxels): plain,
    # concatenated (also inside a 16-channel input tile), upsampled, 3 x 3
    # (output, input) channel tiles
    (2, 3, 128, 16, 0, 16, 3, 0),
    (3, 2, 128, 8, 8, 32, 3, 0),
    (2, 3, 32, 64, 0, 32, 3, 0),
    (4, 2, 64, 32, 0, 16, 3, 1),
    (3, 2, 64, 24, 8, 16, 3, 0),
    (2, 2, 32, 32, 16, 48, 3, 1),
    # one input channel on rows of 64, 128 and 32 voxels (weight gradient from
    # row-shifted copies of the input rows), two output tiles
    (3, 4, 64, 1, 0, 16, 3, 0),
    (2, 3, 128, 1, 0, 32, 3, 0),
    (2, 2, 32, 1, 0, 16, 3, 0),
    # 1x1x1 to one output channel from 8 and 32 channels
    (4, 4, 4, 8, 0, 1, 1, 0),
    (3, 5, 7, 32, 0, 1, 1, 0),
    # power-of-two rows (the shift-indexed weight-gradient kernel): a skip
    # concatenation, an upsampled input, 128 output channels
    (4, 8, 16, 32, 32, 32, 3, 0),
    (8, 16, 8, 32, 0, 16, 3, 1),
    (2, 4, 8, 64, 0, 128, 3, 0),
]


def _layer(nn, rng, c0, c1, cout, ks):
    cin = c0 + c1
    w = _rand(rng, (cout, ks ** 3 * cin), np.sqrt(2.0 / (ks ** 3 * cin)))
    b = _rand(rng, (cout,), 0.1)
    wt = torch.from_numpy(w.astype(np.float32)).cuda()
    import ctypes
    nf, nb = ctypes.c_uint64(), ctypes.c_uint64()
    nn._lib().ltm_nn_packed_sizes(cout, cin, ks, ctypes.byref(nf), ctypes.byref(nb))
    wf = torch.zeros(nf.value, dtype=torch.int16, device="cuda")
    wbk = torch.zeros(nb.value, dtype=torch.int16, device="cuda")
    assert nn._lib().ltm_nn_pack_weights(nn._p(wt), cout, cin, ks, nn._p(wf), nn._p(wbk), None) == 0
    return w, b, wf, wbk


@pytest.mark.parametrize("case", CASES)
def test_conv_forward_dgrad_wgrad(nn, case):
    import ctypes
    D, H, W, c0, c1, cout, ks, up = case
    rng = np.random.default_rng(sum(case))
    lib = nn._lib()
    d0, h0, w0 = (D // 2, H // 2, W // 2) if up else (D, H, W)
    x0 = _rand(rng, (d0, h0, w0, c0))
    x1 = _rand(rng, (D, H, W, c1)) if c1 else None
    w, b, wf, wbk = _layer(nn, rng, c0, c1, cout, ks)
    xe = onn.upsample2(x0) if up else x0
    if c1:
        xe = np.concatenate([xe, x1], axis=3)
    ref = onn.conv3d(xe, w, b, ks)
    # forward, FP32 out without activation
    out = torch.empty(D * H * W * cout, device="cuda")
    desc = nn.conv_desc(ks, D, H, W, c0, c1, cout, up, relu=0, out_f32=1)
    t0 = nn.to_bf16_tensor(x0.reshape(-1))
    t1 = nn.to_bf16_tensor(x1.reshape(-1)) if c1 else None
    bt = torch.from_numpy(b.astype(np.float32)).cuda()
    assert lib.ltm_nn_conv3d_forward(ctypes.byref(desc), nn._p(t0), nn._p(t1), nn._p(wf), nn._p(bt),
                                     nn._p(out), None, None) == 0
    assert rel(out.cpu().numpy(), ref.reshape(-1)) < 1e-5
    # BF16 output with ReLU
    outb = torch.empty(D * H * W * cout, dtype=torch.int16, device="cuda")
    descr = nn.conv_desc(ks, D, H, W, c0, c1, cout, up, relu=1, out_f32=0)
    assert lib.ltm_nn_conv3d_forward(ctypes.byref(descr), nn._p(t0), nn._p(t1), nn._p(wf), nn._p(bt),
                                     nn._p(outb), None, None) == 0
    assert np.array_equal(nn.from_bf16_tensor(outb), nn.bf16_round(np.maximum(out.cpu().numpy(), 0)))
    # input gradient
    g = _rand(rng, (D, H, W, cout))
    gt = nn.to_bf16_tensor(g.reshape(-1))
    if not (c0 == 1 and c1 == 0):
        dx0 = torch.empty(D * H * W * c0, device="cuda")
        dx1 = torch.empty(D * H * W * c1, device="cuda") if c1 else None
        assert lib.ltm_nn_conv3d_dgrad(ctypes.byref(desc), nn._p(gt), nn._p(wbk), nn._p(dx0), nn._p(dx1),
                                       None) == 0
        dref = onn.conv3d_dgrad(g, w, c0 + c1, ks)
        d0ref = dref[..., :c0]
        got0 = dx0.cpu().numpy().reshape(D, H, W, c0)
        if up:
            low = torch.empty(d0 * h0 * w0 * c0, device="cuda")
            assert lib.ltm_nn_upsample2_backward(nn._p(dx0), nn._p(low), D, H, W, c0, 0, None) == 0
            got0 = low.cpu().numpy().reshape(d0, h0, w0, c0)
            d0ref = d0ref.reshape(d0, 2, h0, 2, w0, 2, c0).sum(axis=(1, 3, 5))
        assert rel(got0, d0ref) < 1e-5
        if c1:
            assert rel(dx1.cpu().numpy().reshape(D, H, W, c1), dref[..., c0:]) < 1e-5
    # weight gradient (accumulates)
    dw = torch.zeros(cout, ks ** 3 * (c0 + c1), device="cuda")
    for _ in range(2):
        assert lib.ltm_nn_conv3d_wgrad(ctypes.byref(desc), nn._p(t0), nn._p(t1), nn._p(gt), nn._p(dw),
                                       None) == 0
    assert rel(dw.cpu().numpy(), 2 * onn.conv3d_wgrad(xe, g, ks)) < 1e-5


def test_pool_relu_mse_adam(nn):
    import ctypes
    lib = nn._lib()
    rng = np.random.default_rng(5)
    x = _rand(rng, (4, 6, 8, 16))
    xt = nn.to_bf16_tensor(x.reshape(-1))
    y = torch.empty(x.size // 8, dtype=torch.int16, device="cuda")
    arg = torch.empty(x.size // 8, dtype=torch.uint8, device="cuda")
    assert lib.ltm_nn_maxpool2(nn._p(xt), nn._p(y), nn._p(arg), 4, 6, 8, 16, None) == 0
    assert np.array_equal(nn.from_bf16_tensor(y).reshape(2, 3, 4, 16), onn.maxpool2(x))
    gy = rng.standard_normal(x.size // 8).astype(np.float32)
    dx = torch.ones(x.size, device="cuda")
    assert lib.ltm_nn_maxpool2_backward(nn._p(torch.from_numpy(gy).cuda()), nn._p(arg), nn._p(dx),
                                        4, 6, 8, 16, None) == 0
    xx = torch.from_numpy(x.transpose(3, 0, 1, 2)[None].copy()).requires_grad_(True)
    F.max_pool3d(xx, 2).mul(torch.from_numpy(gy.reshape(2, 3, 4, 16).transpose(3, 0, 1, 2)[None].astype(
        np.float64))).sum().backward()
    ref = xx.grad[0].numpy().transpose(1, 2, 3, 0).reshape(-1) + 1.0
    assert rel(dx.cpu().numpy(), ref) < 1e-7
    # relu backward + bias gradient
    dout = rng.standard_normal(x.size).astype(np.float32)
    g = torch.empty(x.size, dtype=torch.int16, device="cuda")
    db = torch.zeros(16, device="cuda")
    assert lib.ltm_nn_relu_backward(nn._p(torch.from_numpy(dout).cuda()), nn._p(xt), 1, nn._p(g),
                                    nn._p(db), x.size, 16, None) == 0
    gref = nn.bf16_round(dout * (x.reshape(-1) > 0))
    assert np.array_equal(nn.from_bf16_tensor(g), gref)
    assert rel(db.cpu().numpy(), gref.reshape(-1, 16).astype(np.float64).sum(0)) < 1e-6
    # mse
    p = np.abs(rng.standard_normal(1000)).astype(np.float32) * (rng.uniform(size=1000) > 0.2)
    t = rng.standard_normal(1000).astype(np.float32)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    gg = torch.empty(1000, device="cuda")
    assert lib.ltm_nn_mse(nn._p(torch.from_numpy(p).cuda()), nn._p(torch.from_numpy(t).cuda()), nn._p(gg),
                          nn._p(loss), 1000, None) == 0
    assert abs(float(loss) - np.mean((p.astype(np.float64) - t) ** 2)) < 1e-12
    assert rel(gg.cpu().numpy(), 2 * (p - t) / 1000) < 1e-6
    # adam vs torch.optim.Adam (float64, CPU), three steps
    w0 = rng.standard_normal(300)
    grads = [rng.standard_normal(300) for _ in range(3)]
    wt = torch.from_numpy(w0.copy()).requires_grad_(True)
    opt = torch.optim.Adam([wt], lr=1e-2)
    w = torch.from_numpy(w0.astype(np.float32)).cuda()
    m, v = torch.zeros_like(w), torch.zeros_like(w)
    for k, gk in enumerate(grads):
        opt.zero_grad()
        wt.grad = torch.from_numpy(gk.copy())
        opt.step()
        gd = torch.from_numpy(gk.astype(np.float32)).cuda()
        assert lib.ltm_nn_adam(nn._p(w), nn._p(gd), nn._p(m), nn._p(v), 300, 1e-2, 0.9, 0.999, 1e-8,
                               k + 1, None) == 0
        assert float(gd.abs().max()) == 0.0
    assert rel(w.cpu().numpy(), wt.detach().numpy()) < 1e-6


@pytest.mark.parametrize("nvox,C,relu", [
    (999, 8, 1), (1000, 4, 1), (4096, 1, 0), (4096, 1, 1), (512, 128, 1), (64, 1024, 1),
    (3 << 18, 16, 1),   # 8-element path: C below 8 (folded), shuffled lanes, a two-pass grid-stride loop
    (105, 1, 1),        # n not a multiple of 8: one element per thread
    (100, 24, 1),       # C not a power of two
])
def test_relu_backward_shapes(nn, nvox, C, relu):
    lib = nn._lib()
    rng = np.random.default_rng(nvox + C)
    n = nvox * C
    x = _rand(rng, (n,))
    dout = rng.standard_normal(n).astype(np.float32)
    xt = nn.to_bf16_tensor(x)
    g = torch.empty(n, dtype=torch.int16, device="cuda")
    db = torch.zeros(C, device="cuda")
    assert lib.ltm_nn_relu_backward(nn._p(torch.from_numpy(dout).cuda()), nn._p(xt) if relu else None, relu,
                                    nn._p(g), nn._p(db), n, C, None) == 0
    gref = nn.bf16_round(dout * (x > 0) if relu else dout)
    assert np.array_equal(nn.from_bf16_tensor(g), gref)
    gd = gref.reshape(-1, C).astype(np.float64)
    # FP32 sums in any order: error well under 1e-5 of the sum of magnitudes
    assert np.all(np.abs(db.cpu().numpy() - gd.sum(0)) <= 1e-5 * np.abs(gd).sum(0) + 1e-30)


def _bf16(t):
    return t.to(torch.float32).to(torch.bfloat16).to(torch.float64)


class _RoundAct(torch.autograd.Function):
    """BF16 rounding of a stored activation (forward only)."""

    @staticmethod
    def forward(ctx, t):
        return _bf16(t)

    @staticmethod
    def backward(ctx, g):
        return g


class _RoundGrad(torch.autograd.Function):
    """BF16 rounding of the pre-activation gradient (backward only)."""

    @staticmethod
    def forward(ctx, t):
        return t.clone()

    @staticmethod
    def backward(ctx, g):
        return _bf16(g)


def _torch_net(params, x, n):
    """The same network in torch float64 on the CPU (autograd reference),
    rounding where the kernels store BF16: every stored activation, and the
    gradient with respect to each conv's output; accumulation stays FP64."""
    acts = {"in": x}
    spec = {a[0]: a for a in onn.ARCH}

    def tw(w, cin, ks):
        cout = w.shape[0]
        return w.reshape(cout, ks, ks, ks, cin).permute(0, 4, 1, 2, 3)

    for name in ["e11", "e12", "p1", "e21", "e22", "p2", "e31", "e32", "p3", "e41", "e42",
                 "u3", "d31", "d32", "u2", "d21", "d22", "u1", "d11", "d12", "out"]:
        if name in onn.POOLS:
            acts[name] = F.max_pool3d(acts[onn.POOLS[name]], 2)
            continue
        _, ins, c0, c1, cout, ks, up, _ = spec[name]
        h = acts[ins[0]]
        if up:
            h = F.interpolate(h, scale_factor=2, mode="nearest")
        if c1:
            h = torch.cat([h, acts[ins[1]]], dim=1)
        w, b = params[name]
        z = _RoundGrad.apply(F.conv3d(h, tw(w, c0 + c1, ks), b, padding=ks // 2))
        acts[name] = z if name == "out" else _RoundAct.apply(F.relu(z))
    return acts["out"][0, 0]


def test_network_forward_backward_vs_float64(nn):
    n = 16
    net = nn.UNet(seed=3)
    rng = np.random.default_rng(9)
    x = nn.bf16_round(rng.uniform(0, 1, (n, n, n)))
    target = rng.uniform(0, 1, (n, n, n)).astype(np.float32)
    out = net.forward(nn.to_bf16_tensor(x.reshape(-1)), n, n, n)
    loss, g = net.loss_and_grad(torch.from_numpy(target.reshape(-1)).cuda())
    net.zero_grad()
    net.backward(g)
    torch.cuda.synchronize()
    # FP64 reference with the same BF16-rounded weights (packed from the FP32 master)
    params = {}
    for name, L in net.layers.items():
        params[name] = (torch.from_numpy(nn.bf16_round(L.w.cpu().numpy()).astype(np.float64)).requires_grad_(True),
                        torch.from_numpy(L.b.cpu().numpy().astype(np.float64)).requires_grad_(True))
    xt = torch.from_numpy(x.astype(np.float64)[None, None].copy())
    ref = _torch_net(params, xt, n)
    assert rel(out.cpu().numpy(), ref.detach().numpy().reshape(-1)) < 3e-2
    rl = ((ref - torch.from_numpy(target.astype(np.float64))) ** 2).mean()
    rl.backward()
    assert abs(float(loss) - float(rl)) < 3e-2 * float(rl)
    worst = 0.0
    for name, L in net.layers.items():
        e = rel(L.dw.cpu().numpy(), params[name][0].grad.numpy())
        worst = max(worst, e)
        assert e < 0.1, (name, e)
    print("worst layer weight-gradient rel error", worst, flush=True)
    # one Adam step moves the loss down on this sample (at lr 1e-4: the first
    # step moves every weight by about lr, and at 1e-3 it overshoots -- the
    # float64 reference with torch.optim.Adam goes from 0.258 to 2.34 there)
    net.step(lr=1e-4)
    net.forward(nn.to_bf16_tensor(x.reshape(-1)), n, n, n)
    loss2, _ = net.loss_and_grad(torch.from_numpy(target.reshape(-1)).cuda())
    assert float(loss2) < float(rl)
