"""GPU tests of the surrogate path: composition, check samples, RK4 fallback,
and a short training run.

* tol = 0 sends every tile to the fallback: the result must equal plain
  lcs_advect bit for bit (the fallback runs the same integrator);
* tol = inf keeps the composition untouched;
* the per-tile check error equals the largest distance between the
  composition and an independent full-grid RK4 run at the check seeds;
* the composition matches the FP64 reference network iterated over the
  windows at sampled seeds (relative error of the displacement <= 1e-2);
* after a short training run on a smooth field the hybrid FTLE is within
  1e-2 (mean absolute) of plain RK4, and the validation loss has dropped.
"""
import math
import sys

import numpy as np
import pytest

from oracle import mlp_ref as M
from paper_2209_13775_amd import inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_2209_13775_amd import lcs, surrogate
    fs = inputs.abc_frames(n=64, n_frames=33, dt_frame=0.5)
    frames = lcs.DeviceFrames(fs)
    cfg = surrogate.SurrogateConfig(tau=0.5, n_windows=8, t0=4.0, dt=0.02, sigma_x=1.0,
                                    sigma_t=0.5, speed_scale=math.sqrt(6.0))
    return torch, lcs, surrogate, fs, frames, cfg


def _seeds(n=(48, 40, 24)):
    L = 2 * math.pi
    return inputs.SeedGrid(3, n, (0.0, 0.0, 0.0), tuple(L / k for k in n), (True, True, True))


def test_forced_fallback_equals_plain_rk4(env):
    torch, lcs, sur, fs, frames, cfg = env
    g = _seeds()
    mlp = sur.new_model(cfg)
    xf, flags, n_fail, err = sur.surrogate_flowmap(mlp, frames, g, cfg, tol=0.0)
    ref, _, rflags = lcs.lcs_advect(frames, g, cfg.t0, cfg.n_windows * cfg.tau, cfg.dt)
    lcs.lcs_sync_status()
    nt = lcs.lcs_check_tile_count(g)
    assert int(n_fail.item()) == nt
    assert torch.equal(xf, ref) and torch.equal(flags, rflags)


def test_infinite_tolerance_keeps_composition(env):
    torch, lcs, sur, fs, frames, cfg = env
    g = _seeds()
    mlp = sur.new_model(cfg)
    comp = lcs.lcs_surrogate_compose(mlp, g, cfg.t0, cfg.tau, cfg.n_windows)
    xf, flags, n_fail, err = sur.surrogate_flowmap(mlp, frames, g, cfg, tol=float("inf"))
    lcs.lcs_sync_status()
    assert int(n_fail.item()) == 0
    assert torch.equal(xf, comp)


def test_check_error_matches_independent_rk4(env):
    torch, lcs, sur, fs, frames, cfg = env
    g = _seeds()
    mlp = sur.new_model(cfg)
    T = cfg.n_windows * cfg.tau
    comp = lcs.lcs_surrogate_compose(mlp, g, cfg.t0, cfg.tau, cfg.n_windows)
    err, fail, n_fail = lcs.lcs_surrogate_check(frames, g, cfg.t0, T, cfg.dt, comp, 0.5)
    ref, _, _ = lcs.lcs_advect(frames, g, cfg.t0, T, cfg.dt)
    lcs.lcs_sync_status()
    c = comp.cpu().numpy().astype(np.float64)
    r = ref.cpu().numpy().astype(np.float64)
    ct = [(g.n[a] + (16, 16, 8)[a] - 1) // (16, 16, 8)[a] for a in range(3)]
    want = np.zeros(ct[0] * ct[1] * ct[2])
    for tz in range(ct[2]):
        for ty in range(ct[1]):
            for tx in range(ct[0]):
                t = tx + ct[0] * (ty + ct[1] * tz)
                for q in range(0, 2048, 100):
                    i, j, k = tx * 16 + q % 16, ty * 16 + (q // 16) % 16, tz * 8 + q // 256
                    if i >= g.n[0] or j >= g.n[1] or k >= g.n[2]:
                        continue
                    s = i + g.n[0] * (j + g.n[1] * k)
                    want[t] = max(want[t], np.linalg.norm(c[:, s] - r[:, s]))
    np.testing.assert_allclose(err.cpu().numpy(), want, rtol=1e-5, atol=1e-6)
    np.testing.assert_array_equal(fail.cpu().numpy(), (want > 0.5).astype(np.uint8))
    assert int(n_fail.item()) == int((want > 0.5).sum())


def test_composition_matches_reference_network(env):
    torch, lcs, sur, fs, frames, cfg = env
    g = _seeds((20, 16, 8))
    mlp = sur.new_model(cfg)
    comp = lcs.lcs_surrogate_compose(mlp, g, cfg.t0, cfg.tau, cfg.n_windows)
    lcs.lcs_sync_status()
    params = mlp.params.cpu().numpy().astype(np.float64)
    for t in range(M.N_HIDDEN):
        off = sum(int(np.prod(s)) for s in M.SHAPES[:2 * t])
        n = int(np.prod(M.SHAPES[2 * t]))
        params[off:off + n] = M.round_to_bf16(params[off:off + n])
    d = mlp.desc
    idx = np.arange(0, g.count, 37)
    c = g.coords_of(idx).astype(np.float64)
    x = np.stack([g.origin[a] + c[a] * g.spacing[a] for a in range(3)])
    x0 = x.copy()
    for k in range(cfg.n_windows):
        xt = np.concatenate([x, np.full((1, x.shape[1]), cfg.t0 + k * cfg.tau)])
        dx, _ = M.forward(params, mlp.freq.cpu().numpy().astype(np.float64), xt,
                          list(d.in_shift), list(d.in_scale), d.out_scale, round_bf16=M.round_to_bf16)
        x = x + dx
    got = comp.cpu().numpy()[:, idx].astype(np.float64)
    rel = np.linalg.norm(got - x) / np.linalg.norm(x - x0)
    _say(f"composition vs reference: relative error {rel:.2e}")
    assert rel <= 1e-2


def test_training_and_hybrid_ftle(env):
    torch, lcs, sur, fs, frames, cfg = env
    _say("case: short surrogate training on the ABC field")
    mlp = sur.new_model(cfg)
    xt, dx, fl = sur.training_data(frames, cfg, 1 << 19, seed=1)
    vxt, vdx, _ = sur.training_data(frames, cfg, 1 << 16, seed=2)
    assert not bool(fl.any())
    before = sur.evaluate(mlp, vxt, vdx)
    log = sur.train(mlp, xt, dx, epochs=6, batch=16384, lr=3e-3, val=(vxt, vdx))
    rms = float(np.sqrt(before))
    _say(f"val MSE {before:.3e} -> {log.val_loss:.3e} in {log.seconds:.1f} s ({log.steps} steps)")
    assert log.val_loss < 0.05 * before
    g = _seeds((64, 64, 32))
    T = cfg.n_windows * cfg.tau
    ref, _, rfl = lcs.lcs_advect(frames, g, cfg.t0, T, cfg.dt)
    _, rsig, rsfl = lcs.lcs_cg_ftle(g, ref, T, flags=rfl)
    for tol in [1e-3, 1e-2]:
        xf, flags, n_fail, err = sur.surrogate_flowmap(mlp, frames, g, cfg, tol=tol)
        _, sig, sfl = lcs.lcs_cg_ftle(g, xf, T, flags=flags)
        lcs.lcs_sync_status()
        e = (sig - rsig).abs()
        nt = lcs.lcs_check_tile_count(g)
        _say(f"tol {tol}: fallback {int(n_fail.item())}/{nt} tiles, FTLE err mean "
             f"{e.mean().item():.2e} max {e.max().item():.2e}")
        assert e.mean().item() <= 1e-2
