"""Pins of the FP64 MLP reference (surrogate): gradients against central
finite differences of the loss, GELU against its definition's closed-form
special values and numerical derivative, Adam against torch.optim.Adam, and
the BF16 rounding helper against torch's bfloat16 conversion."""
import math

import numpy as np
import pytest

from oracle import mlp_ref as M


def _setup(n=7, seed=0):
    rng = np.random.default_rng(seed)
    params = M.init_params(seed) + 0.01 * rng.standard_normal(M.N_PARAMS)
    freq = rng.standard_normal((M.N_FREQ, M.N_IN))
    xt = rng.uniform(0, 2 * math.pi, (4, n))
    xt[3] = rng.uniform(4, 8, n)
    shift = [0.0, 0.0, 0.0, 6.0]
    scale = [1 / (2 * math.pi)] * 3 + [0.25]
    target = rng.standard_normal((3, n)) * 0.3
    return params, freq, xt, shift, scale, target


def test_gradient_matches_central_differences():
    params, freq, xt, shift, scale, target = _setup()
    out_scale = 0.7

    def loss(p):
        y, _ = M.forward(p, freq, xt, shift, scale, out_scale)
        return M.mse(y, target)[0]

    y, cache = M.forward(params, freq, xt, shift, scale, out_scale)
    L, dy = M.mse(y, target)
    g = M.backward(params, cache, dy)
    rng = np.random.default_rng(3)
    # every bias entry of the head and a spread of entries of every tensor
    offs = np.cumsum([0] + [int(np.prod(s)) for s in M.SHAPES])
    idx = []
    for t in range(len(M.SHAPES)):
        idx += list(rng.choice(np.arange(offs[t], offs[t + 1]), size=min(6, offs[t + 1] - offs[t]),
                               replace=False))
    h = 1e-6
    for i in idx:
        e = np.zeros_like(params)
        e[i] = h
        fd = (loss(params + e) - loss(params - e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-10, (i, fd, g[i])


def test_gelu_definition():
    z = np.array([0.0, 1.0, -1.0, 3.0, -3.0])
    # closed-form values of the tanh form
    c = math.sqrt(2 / math.pi)
    ref = [0.5 * x * (1 + math.tanh(c * (x + 0.044715 * x ** 3))) for x in z]
    np.testing.assert_allclose(M.gelu(z), ref, rtol=1e-15)
    assert M.gelu(np.array([0.0]))[0] == 0.0
    # derivative against a central difference
    zz = np.linspace(-6, 6, 101)
    h = 1e-6
    np.testing.assert_allclose(M.gelu_prime(zz), (M.gelu(zz + h) - M.gelu(zz - h)) / (2 * h),
                               rtol=1e-7, atol=1e-9)
    # the tanh form is within 1e-3 of the exact (erf) GELU
    import scipy.special as sp
    exact = 0.5 * zz * (1 + sp.erf(zz / math.sqrt(2)))
    assert np.abs(M.gelu(zz) - exact).max() < 1e-3


def test_adam_matches_torch():
    import torch
    rng = np.random.default_rng(5)
    p0 = rng.standard_normal(50)
    p = torch.tensor(p0.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    mine, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for step in range(1, 6):
        g = rng.standard_normal(50)
        opt.zero_grad()
        p.grad = torch.tensor(g)
        opt.step()
        mine, m, v = M.adam(mine, g, m, v, step, lr=3e-3)
        np.testing.assert_allclose(mine, p.detach().numpy(), rtol=1e-14, atol=1e-15)


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(1)
    a = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-8, 8, 10000),
                        [0.0, -0.0, 1.0, 65504.0, 1e-40]]).astype(np.float32)
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(M.round_to_bf16(a), ref)


def test_parameter_count():
    assert M.N_PARAMS == 128 * 256 + 256 + 3 * (256 * 256 + 256) + 256 * 3 + 3


def _torch_network(params, freq, shift, scale, out_scale):
    """The surrogate written a second time with torch modules (FP64): Linear
    layers (weight stored [out][in]), the tanh-form GELU of torch, cos/sin
    features of 2 pi B v.  Shares nothing with mlp_ref but the flat layout."""
    import torch
    import torch.nn.functional as F
    p = torch.tensor(np.asarray(params, np.float64), dtype=torch.float64, requires_grad=True)
    B = torch.tensor(np.asarray(freq, np.float64))
    sh = torch.tensor(np.asarray(shift, np.float64))
    sc = torch.tensor(np.asarray(scale, np.float64))
    widths = [(128, 256), (256, 256), (256, 256), (256, 256)]

    def run(xt):
        v = (torch.tensor(xt).T - sh) * sc                       # (n, 4)
        ph = 2.0 * math.pi * (v @ B.T)                            # (n, 64)
        h = torch.cat([torch.cos(ph), torch.sin(ph)], dim=1)      # (n, 128)
        off = 0
        for fin, fout in widths:
            W = p[off:off + fin * fout].view(fin, fout)
            off += fin * fout
            b = p[off:off + fout]
            off += fout
            h = F.gelu(F.linear(h, W.T.contiguous(), b), approximate="tanh")
        Wh = p[off:off + 256 * 3].view(256, 3)
        bh = p[off + 768:off + 771]
        assert off + 771 == p.numel()
        return out_scale * F.linear(h, Wh.T.contiguous(), bh).T   # (3, n)
    return p, run


def test_forward_and_backward_match_independent_torch_network():
    # pins features (frequency layout, 2 pi, cos-then-sin order, shift and
    # scale), the layer stack, the GELU form, the head and out_scale, which a
    # finite-difference check of backward against forward cannot see
    import torch
    params, freq, xt, shift, scale, target = _setup(n=33, seed=4)
    out_scale = 0.35
    y, cache = M.forward(params, freq, xt, shift, scale, out_scale)
    p, run = _torch_network(params, freq, shift, scale, out_scale)
    yt = run(xt)
    np.testing.assert_allclose(y, yt.detach().numpy(), rtol=1e-12, atol=1e-14)
    # backward of sum(ddx * dx) against autograd
    ddx = np.random.default_rng(9).standard_normal(y.shape)
    g = M.backward(params, cache, ddx)
    (yt * torch.tensor(ddx)).sum().backward()
    gt = p.grad.numpy()
    np.testing.assert_allclose(g, gt, rtol=1e-10, atol=1e-13)
    # and the feature map alone: the first 64 features are cosines of
    # 2 pi B (xt - shift) * scale, the last 64 sines
    f = M.features(xt, freq, shift, scale)
    v = (xt - np.array(shift)[:, None]) * np.array(scale)[:, None]
    k, s = 5, 7
    ph = 2 * math.pi * sum(freq[k, a] * v[a, s] for a in range(4))
    assert abs(f[s, k] - math.cos(ph)) < 1e-13 and abs(f[s, 64 + k] - math.sin(ph)) < 1e-13
