"""GPU parity of the surrogate's MLP kernels (BF16 MFMA, FP32 accumulation)
against the FP64 reference run on the same BF16-rounded weights and at the
same BF16 rounding points.

Bars: forward output relative Frobenius error <= 1e-2; every gradient tensor
relative Frobenius error <= 2e-2 (the GPU also rounds the back-propagated
dZ to BF16); BF16 weight copies bit-exact; Adam within FP32 rounding (1e-6
relative); repeated backward passes bit-identical.
"""
import math
import sys

import numpy as np
import pytest

from oracle import mlp_ref as M

pytestmark = pytest.mark.gpu

SHIFT = [0.0, 0.0, 0.0, 6.0]
SCALE = [1 / (2 * math.pi)] * 3 + [0.25]
OUT_SCALE = 0.5


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a HIP device"
    return _t


@pytest.fixture(scope="module")
def lcs(torch):
    from paper_2209_13775_amd import lcs as _l
    return _l


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _model(seed=0):
    rng = np.random.default_rng(seed)
    params = (M.init_params(seed) + 0.02 * rng.standard_normal(M.N_PARAMS)).astype(np.float32)
    freq = np.concatenate([np.round(rng.standard_normal((M.N_FREQ, 3)) * 2.0),
                           rng.standard_normal((M.N_FREQ, 1))], axis=1).astype(np.float32)
    return params, freq


def _inputs(n, seed=1):
    rng = np.random.default_rng(seed)
    xt = np.stack([rng.uniform(0, 2 * math.pi, n) for _ in range(3)] +
                  [rng.choice(np.arange(4.0, 8.0, 0.5), n)]).astype(np.float32)
    return xt


def _oracle_params(params):
    """FP64 copy with the hidden-layer matrices rounded to BF16 as the GPU uses them."""
    p = params.astype(np.float64).copy()
    for t in range(M.N_HIDDEN):
        off = sum(int(np.prod(s)) for s in M.SHAPES[:2 * t])
        n = int(np.prod(M.SHAPES[2 * t]))
        p[off:off + n] = M.round_to_bf16(p[off:off + n])
    return p


def _fragment_order(WT):
    """An R x C matrix laid out as the BF16 weight copies are (the MFMA fragment
    order the header documents): blocks of 16 x 32, each 64 lanes x 8 c."""
    N, K = WT.shape
    n = np.arange(N)[:, None]
    k = np.arange(K)[None, :]
    idx = ((n // 16) * (K // 32) + k // 32) * 512 + ((n % 16) + 16 * ((k % 32) // 8)) * 8 + k % 8
    out = np.empty(N * K, dtype=WT.dtype)
    out[idx.ravel()] = WT.ravel()
    return out


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def test_bf16_copies_exact(lcs, torch):
    params, freq = _model()
    mlp = lcs.Mlp(params, freq, SHIFT, SCALE, OUT_SCALE)
    torch.cuda.synchronize()
    got = mlp.bf16.cpu().numpy().view(np.uint16)
    off_b = 0
    off_p = 0
    for t in range(M.N_HIDDEN):
        K, N = M.SHAPES[2 * t]
        W = params[off_p:off_p + K * N].reshape(K, N)
        want = M.round_to_bf16(W).astype(np.float32).view(np.uint32) >> 16
        np.testing.assert_array_equal(got[off_b:off_b + K * N], _fragment_order(want))
        np.testing.assert_array_equal(got[off_b + K * N:off_b + 2 * K * N], _fragment_order(want.T))
        off_b += 2 * K * N
        off_p += K * N + N


@pytest.mark.parametrize("n", [4096, 1000, 37])
def test_forward_matches_reference(lcs, torch, n):
    _say(f"case: mlp forward batch {n}")
    params, freq = _model()
    mlp = lcs.Mlp(params, freq, SHIFT, SCALE, OUT_SCALE)
    xt = _inputs(n)
    dx, _ = lcs.lcs_mlp_forward(mlp, torch.from_numpy(xt).cuda())
    lcs.lcs_sync_status()
    ref, _ = M.forward(_oracle_params(params), freq.astype(np.float64), xt.astype(np.float64),
                       SHIFT, SCALE, OUT_SCALE, round_bf16=M.round_to_bf16)
    err = _rel(dx.cpu().numpy(), ref)
    _say(f"forward rel err {err:.2e}")
    assert err <= 1e-2


@pytest.mark.parametrize("n", [6000, 300, 9000])   # 9000: over 64 bias chunks (tree reduction)
def test_backward_matches_reference(lcs, torch, n):
    _say(f"case: mlp backward batch {n}")
    params, freq = _model(3)
    mlp = lcs.Mlp(params, freq, SHIFT, SCALE, OUT_SCALE)
    xt = _inputs(n, 4)
    rng = np.random.default_rng(9)
    target = (rng.standard_normal((3, n)) * 0.3).astype(np.float32)
    dx, ws = lcs.lcs_mlp_forward(mlp, torch.from_numpy(xt).cuda(), training=True)
    ddx, loss = lcs.lcs_mse_grad(dx, torch.from_numpy(target).cuda())
    g = lcs.lcs_mlp_backward(mlp, ws, ddx)
    g2 = lcs.lcs_mlp_backward(mlp, ws, ddx)
    lcs.lcs_sync_status()
    assert torch.equal(g, g2), "backward is not deterministic"
    po = _oracle_params(params)
    y, cache = M.forward(po, freq.astype(np.float64), xt.astype(np.float64), SHIFT, SCALE,
                         OUT_SCALE, round_bf16=M.round_to_bf16)
    L, dy = M.mse(y, target.astype(np.float64))
    assert abs(loss.item() - L) <= 2e-2 * L
    np.testing.assert_allclose(ddx.cpu().numpy(), 2 * (dx.cpu().numpy() - target) / dx.numel(),
                               rtol=1e-6, atol=1e-12)
    gr = M.backward(po, cache, dy)
    gg = g.cpu().numpy().astype(np.float64)
    off = 0
    for t, s in enumerate(M.SHAPES):
        k = int(np.prod(s))
        err = _rel(gg[off:off + k], gr[off:off + k])
        _say(f"grad tensor {t} {s}: rel err {err:.2e}")
        assert err <= 2e-2, (t, err)
        off += k


def test_adam_matches_reference(lcs, torch):
    rng = np.random.default_rng(2)
    n = 5000
    p = rng.standard_normal(n).astype(np.float32)
    m = np.zeros(n, np.float32)
    v = np.zeros(n, np.float32)
    dp, dm, dv = (torch.from_numpy(a.copy()).cuda() for a in (p, m, v))
    rp, rm, rv = p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for step in range(1, 4):
        g = rng.standard_normal(n).astype(np.float32)
        lcs.lcs_adam_step(dp, torch.from_numpy(g).cuda(), dm, dv, step, lr=2e-3)
        rp, rm, rv = M.adam(rp, g.astype(np.float64), rm, rv, step, lr=2e-3)
    lcs.lcs_sync_status()
    np.testing.assert_allclose(dp.cpu().numpy(), rp, rtol=1e-6, atol=1e-7)


def test_short_training_reduces_loss(lcs, torch):
    """Fit a smooth periodic displacement field: the loss must fall 10x."""
    _say("case: short training run")
    params, freq = _model(5)
    freq[:, :3] = np.round(np.random.default_rng(7).standard_normal((M.N_FREQ, 3)) * 1.0)
    mlp = lcs.Mlp(params, freq, SHIFT, SCALE, 1.0)
    n = 8192
    xt = _inputs(n, 11)
    tgt = np.stack([0.3 * np.sin(xt[1]), 0.3 * np.cos(xt[2]) * np.sin(xt[0]),
                    0.2 * np.sin(xt[0] + xt[1])]).astype(np.float32)
    dxt, dtg = torch.from_numpy(xt).cuda(), torch.from_numpy(tgt).cuda()
    m = torch.zeros_like(mlp.params)
    v = torch.zeros_like(mlp.params)
    losses = []
    for step in range(1, 301):
        dx, ws = lcs.lcs_mlp_forward(mlp, dxt, training=True)
        ddx, loss = lcs.lcs_mse_grad(dx, dtg)
        g = lcs.lcs_mlp_backward(mlp, ws, ddx)
        lcs.lcs_adam_step(mlp.params, g, m, v, step, lr=1e-3)
        mlp.refresh()
        if step % 50 == 1 or step == 300:
            losses.append(loss.item())
    lcs.lcs_sync_status()
    _say(f"losses {losses}")
    assert losses[-1] < 0.1 * losses[0]


def _cosine_lr(step, total, lr, lr_final):
    frac = (step - 1) / max(1, total - 1)
    return lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * min(frac, 1.0)))


# 20000 samples: 157 tiles (the last ragged), 10 weight-gradient chunks (the
# last partial), so the chunk sum runs both its eight-wide loop and its tail
@pytest.mark.parametrize("n", [6000, 300, 4096, 20000])
def test_fused_train_step_matches_reference(lcs, torch, n):
    # one fused step (lcs_mlp_train): the loss and every gradient tensor
    # against the FP64 reference at the same BF16 rounding points, the update
    # against Adam applied to that gradient, the BF16 copies against the
    # rounded masters; a repeat from the same state is bit-identical
    _say(f"case: fused training step, batch {n}")
    params, freq = _model(5)
    xt = _inputs(n, 6)
    rng = np.random.default_rng(11)
    target = (rng.standard_normal((3, n)) * 0.3).astype(np.float32)
    dxt, dtg = torch.from_numpy(xt).cuda(), torch.from_numpy(target).cuda()
    outs = []
    for rep in range(2):
        mlp = lcs.Mlp(params, freq, SHIFT, SCALE, OUT_SCALE)
        m = torch.zeros_like(mlp.params)
        v = torch.zeros_like(mlp.params)
        losses = torch.empty(1, dtype=torch.float64, device="cuda")
        grads = torch.empty_like(mlp.params)
        lcs.lcs_mlp_train(mlp, dxt, dtg, n, 1, 1, 1, m, v, lr=2e-3, losses=losses, grads=grads)
        lcs.lcs_sync_status()
        outs.append((mlp.params.clone(), mlp.bf16.clone(), m.clone(), v.clone(), grads.clone(),
                     float(losses.item())))
    for a, b in zip(outs[0][:5], outs[1][:5]):
        assert torch.equal(a, b), "fused training step is not deterministic"
    p_new, bf_new, m_new, v_new, g, loss = outs[0]
    po = _oracle_params(params)
    y, cache = M.forward(po, freq.astype(np.float64), xt.astype(np.float64), SHIFT, SCALE,
                         OUT_SCALE, round_bf16=M.round_to_bf16)
    L, dy = M.mse(y, target.astype(np.float64))
    _say(f"loss {loss:.6e} reference {L:.6e}")
    assert abs(loss - L) <= 2e-2 * L
    gr = M.backward(po, cache, dy)
    gg = g.cpu().numpy().astype(np.float64)
    off = 0
    for t, s in enumerate(M.SHAPES):
        k = int(np.prod(s))
        err = _rel(gg[off:off + k], gr[off:off + k])
        _say(f"grad tensor {t} {s}: rel err {err:.2e}")
        assert err <= 2e-2, (t, err)
        off += k
    rp, rm, rv = M.adam(params.astype(np.float64), gg, np.zeros_like(gg), np.zeros_like(gg), 1,
                        lr=2e-3)
    np.testing.assert_allclose(p_new.cpu().numpy(), rp, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(m_new.cpu().numpy(), rm, rtol=1e-6, atol=1e-12)
    # 1 - beta2 rounded to FP32 (0.999f) is 1.3e-5 off 0.001 in relative terms
    np.testing.assert_allclose(v_new.cpu().numpy(), rv, rtol=5e-5, atol=1e-15)
    # BF16 copies of the updated masters, both layouts
    got = bf_new.cpu().numpy().view(np.uint16)
    pn = p_new.cpu().numpy()
    off_b = off_p = 0
    for t in range(M.N_HIDDEN):
        K, N = M.SHAPES[2 * t]
        W = pn[off_p:off_p + K * N].reshape(K, N)
        want = M.round_to_bf16(W).astype(np.float32).view(np.uint32) >> 16
        np.testing.assert_array_equal(got[off_b:off_b + K * N], _fragment_order(want))
        np.testing.assert_array_equal(got[off_b + K * N:off_b + 2 * K * N], _fragment_order(want.T))
        off_b += 2 * K * N
        off_p += K * N + N


def test_fused_train_steps_resume_and_schedule(lcs, torch):
    # five steps over three batches in one call equal five one-step calls
    # (batch order, cosine schedule and moments carried across calls), and the
    # last step is Adam at the scheduled rate on the gradient it reports
    n, batch, total = 3 * 2048, 2048, 5
    _say("case: fused training, 5 steps over 3 batches")
    params, freq = _model(7)
    xt = torch.from_numpy(_inputs(n, 8)).cuda()
    rng = np.random.default_rng(12)
    target = torch.from_numpy((rng.standard_normal((3, n)) * 0.3).astype(np.float32)).cuda()
    a = lcs.Mlp(params, freq, SHIFT, SCALE, OUT_SCALE)
    ma, va = torch.zeros_like(a.params), torch.zeros_like(a.params)
    la = torch.empty(total, dtype=torch.float64, device="cuda")
    lcs.lcs_mlp_train(a, xt, target, batch, 1, total, total, ma, va, lr=3e-3, lr_final=2e-4,
                      losses=la)
    b = lcs.Mlp(params, freq, SHIFT, SCALE, OUT_SCALE)
    mb, vb = torch.zeros_like(b.params), torch.zeros_like(b.params)
    lb = torch.empty(1, dtype=torch.float64, device="cuda")
    g = torch.empty_like(b.params)
    for step in range(1, total + 1):
        if step == total:
            p_before, m_before, v_before = b.params.clone(), mb.clone(), vb.clone()
        lcs.lcs_mlp_train(b, xt, target, batch, step, 1, total, mb, vb, lr=3e-3, lr_final=2e-4,
                          losses=lb, grads=g if step == total else None)
        assert float(lb.item()) == float(la[step - 1].item())
    lcs.lcs_sync_status()
    assert torch.equal(a.params, b.params) and torch.equal(a.bf16, b.bf16)
    assert torch.equal(ma, mb) and torch.equal(va, vb)
    lr5 = _cosine_lr(total, total, 3e-3, 2e-4)
    rp, _, _ = M.adam(p_before.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64),
                      m_before.cpu().numpy().astype(np.float64),
                      v_before.cpu().numpy().astype(np.float64), total, lr=lr5)
    np.testing.assert_allclose(b.params.cpu().numpy(), rp, rtol=1e-6, atol=1e-7)
    assert bool(torch.isfinite(la).all())
