"""FP64 reference of the Fourier-feature MLP flow-map surrogate.

TEST INFRASTRUCTURE ONLY (see the package docstring): the product path never
imports this module.

The surrogate (a learned local approximation of the flow map over a window
tau; the paper's discussion cites local flow-map approximation as a way to
cut interpolation cost when flow maps are wanted for many start times,
Sec. 4) maps an input (x, y, z, t) to a displacement dx over the window:

  v      = (input - shift) * scale                     (4 values)
  gamma  = [cos(2 pi B v), sin(2 pi B v)]              (B: 64 x 4, 128 features)
  h_1    = gelu(gamma W_0 + b_0)                        (256)
  h_l    = gelu(h_{l-1} W_{l-1} + b_{l-1}),  l = 2..4  (256)
  dx     = out_scale * (h_4 W_h + b_h)                  (3)

with the tanh form of GELU, gelu(z) = z/2 (1 + tanh(sqrt(2/pi)(z + 0.044715 z^3))).
Parameters live in one flat FP32 vector in the order
W_0 (128x256, row-major [in][out]), b_0, W_1, b_1, W_2, b_2, W_3, b_3,
W_h (256x3), b_h -- 231171 values.  Loss: mean squared error over all
components.  Optimiser: Adam (Kingma & Ba) with bias correction.
"""
from __future__ import annotations

import math

import numpy as np

N_FREQ = 64
N_IN = 4
N_FEAT = 2 * N_FREQ
WIDTH = 256
N_HIDDEN = 4
N_OUT = 3

SHAPES = [(N_FEAT, WIDTH), (WIDTH,)] + [(WIDTH, WIDTH), (WIDTH,)] * (N_HIDDEN - 1) + \
         [(WIDTH, N_OUT), (N_OUT,)]
N_PARAMS = int(sum(int(np.prod(s)) for s in SHAPES))
assert N_PARAMS == 231171

_C = math.sqrt(2.0 / math.pi)


def unpack(params: np.ndarray):
    """Split the flat vector into [W0, b0, W1, b1, W2, b2, W3, b3, Wh, bh] views."""
    out, off = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(params[off:off + n].reshape(s))
        off += n
    return out


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(_C * (z + 0.044715 * z ** 3)))


def gelu_prime(z):
    u = _C * (z + 0.044715 * z ** 3)
    t = np.tanh(u)
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * _C * (1.0 + 3.0 * 0.044715 * z * z)


def features(xt: np.ndarray, freq: np.ndarray, shift, scale) -> np.ndarray:
    """Fourier features of inputs xt (4 x n) -> (n x 128)."""
    v = (xt - np.asarray(shift, dtype=np.float64)[:, None]) * np.asarray(scale, np.float64)[:, None]
    arg = 2.0 * math.pi * (freq @ v)                 # (64, n)
    return np.concatenate([np.cos(arg), np.sin(arg)], axis=0).T


def forward(params, freq, xt, shift, scale, out_scale, round_bf16=None):
    """Network output dx (3 x n) and the cache for backward.

    round_bf16: optional function applied to the features and to every hidden
    activation (used to reproduce the quantisation points of a BF16 run while
    keeping FP64 arithmetic)."""
    rb = round_bf16 or (lambda a: a)
    P = unpack(np.asarray(params, dtype=np.float64))
    h = rb(features(xt, freq, shift, scale))
    hs, zs = [h], []
    for l in range(N_HIDDEN):
        z = h @ P[2 * l] + P[2 * l + 1]
        zs.append(z)
        h = rb(gelu(z))
        hs.append(h)
    y = h @ P[2 * N_HIDDEN] + P[2 * N_HIDDEN + 1]
    return (out_scale * y).T, {"hs": hs, "zs": zs, "out_scale": out_scale}


def backward(params, cache, ddx: np.ndarray) -> np.ndarray:
    """Gradient of sum(ddx * dx) with respect to the flat parameter vector."""
    P = unpack(np.asarray(params, dtype=np.float64))
    G = [np.zeros(s) for s in SHAPES]
    dy = cache["out_scale"] * ddx.T                   # (n, 3)
    hs, zs = cache["hs"], cache["zs"]
    G[2 * N_HIDDEN] = hs[N_HIDDEN].T @ dy
    G[2 * N_HIDDEN + 1] = dy.sum(axis=0)
    dh = dy @ P[2 * N_HIDDEN].T
    for l in reversed(range(N_HIDDEN)):
        dz = dh * gelu_prime(zs[l])
        G[2 * l] = hs[l].T @ dz
        G[2 * l + 1] = dz.sum(axis=0)
        dh = dz @ P[2 * l].T
    return np.concatenate([g.ravel() for g in G])


def mse(pred: np.ndarray, target: np.ndarray):
    """Mean squared error and its gradient with respect to pred."""
    d = pred - target
    return float(np.mean(d * d)), 2.0 * d / d.size


def adam(params, grads, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grads
    v = beta2 * v + (1.0 - beta2) * grads * grads
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v


def init_params(seed: int = 0) -> np.ndarray:
    """Uniform fan-in initialisation (|w| <= 1/sqrt(fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for s in SHAPES:
        if len(s) == 2:
            parts.append(rng.uniform(-1.0, 1.0, s) / math.sqrt(s[0]))
        else:
            parts.append(np.zeros(s))
    return np.concatenate([p.ravel() for p in parts])


def round_to_bf16(a: np.ndarray) -> np.ndarray:
    """Round FP32/FP64 values to the nearest BF16 (ties to even), as FP64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    out = np.where(np.isnan(f), f, out)
    return out.astype(np.float64)
