"""GPU tests of the surrogate path: composition, check samples, RK4 fallback,
and a short training run.

* tol = 0 sends every tile to the fallback: the result must equal plain
  lcs_advect bit for bit (whole-grid and tile-by-tile branches: the fallback
  runs the same integrator);
* tol = inf keeps the composition untouched;
* a tolerance between the smallest and largest tile errors re-advects only
  the failing tiles (bit-identical to lcs_advect there) and keeps the
  composition elsewhere;
* the per-tile check error equals, within the position bar, the largest
  distance between the composition and the FP64 oracle's RK4 at the check
  seeds;
* the composition matches the FP64 reference network iterated over the
  windows at sampled seeds (relative error of the displacement <= 1e-2);
* training on the smooth ABC field: the validation loss drops 1000-fold, the
  composition alone comes within 2e-2 (mean FTLE) of plain RK4, a loose
  tolerance accepts part of the tiles and improves on the composition, and
  the 1e-3 tolerance rejects every tile (plain RK4 bit for bit).
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


def _check_seed_index(g):
    """Natural indices of the check seeds (local index 0, 100, 200, ... of each
    aligned 16 x 16 x 8 tile) and the tile each belongs to."""
    ct = [(g.n[a] + (16, 16, 8)[a] - 1) // (16, 16, 8)[a] for a in range(3)]
    idx, tile = [], []
    for tz in range(ct[2]):
        for ty in range(ct[1]):
            for tx in range(ct[0]):
                for q in range(0, 2048, 100):
                    i, j, k = tx * 16 + q % 16, ty * 16 + (q // 16) % 16, tz * 8 + q // 256
                    if i < g.n[0] and j < g.n[1] and k < g.n[2]:
                        idx.append(i + g.n[0] * (j + g.n[1] * k))
                        tile.append(tx + ct[0] * (ty + ct[1] * tz))
    return np.array(idx), np.array(tile), ct[0] * ct[1] * ct[2]


def _tile_of_seed(g):
    c = g.coords_of(np.arange(g.count))
    ct0, ct1 = (g.n[0] + 15) // 16, (g.n[1] + 15) // 16
    return c[0] // 16 + ct0 * (c[1] // 16 + ct1 * (c[2] // 8))


@pytest.mark.parametrize("whole_fraction", [0.25, 1.0])
def test_all_tiles_fail_equals_plain_rk4(env, whole_fraction):
    # tol = 0 fails every tile; the whole-grid branch (re-bundled RK4) and the
    # tile-by-tile branch must both reproduce lcs_advect bit for bit
    torch, lcs, sur, fs, frames, cfg = env
    _say(f"case: every tile fails, whole_grid_fraction {whole_fraction}")
    g = _seeds()
    mlp = sur.new_model(cfg)
    xf, flags, nf, whole, err = lcs.lcs_surrogate_flowmap(
        mlp, frames, g, cfg.t0, cfg.tau, cfg.n_windows, 0.0, cfg.dt,
        whole_grid_fraction=whole_fraction)
    ref, _, rflags = lcs.lcs_advect(frames, g, cfg.t0, cfg.n_windows * cfg.tau, cfg.dt)
    lcs.lcs_sync_status()
    assert nf == lcs.lcs_check_tile_count(g)
    assert whole == (whole_fraction < 1.0)
    assert torch.equal(xf, ref) and torch.equal(flags, rflags)


def test_infinite_tolerance_keeps_composition(env):
    torch, lcs, sur, fs, frames, cfg = env
    g = _seeds()
    mlp = sur.new_model(cfg)
    comp = lcs.lcs_surrogate_compose(mlp, g, cfg.t0, cfg.tau, cfg.n_windows)
    xf, flags, nf, whole, err = lcs.lcs_surrogate_flowmap(
        mlp, frames, g, cfg.t0, cfg.tau, cfg.n_windows, float("inf"), cfg.dt)
    lcs.lcs_sync_status()
    assert nf == 0 and not whole
    assert torch.equal(xf, comp) and not bool(flags.any())


@pytest.mark.parametrize("n", [(48, 40, 24), (37, 21, 11)])
def test_mixed_accept_and_fallback(env, n):
    # a tolerance between the smallest and largest tile errors: the failing
    # tiles (some of them ragged at the grid's upper faces) are re-advected by
    # the tile kernel and must equal lcs_advect bit for bit, the accepted ones
    # must keep the composition bit for bit
    torch, lcs, sur, fs, frames, cfg = env
    g = _seeds(n)
    _say(f"case: mixed accept / fallback on seeds {n}")
    mlp = sur.new_model(cfg)
    T = cfg.n_windows * cfg.tau
    comp = lcs.lcs_surrogate_compose(mlp, g, cfg.t0, cfg.tau, cfg.n_windows)
    err0, _, _ = lcs.lcs_surrogate_check(frames, g, cfg.t0, T, cfg.dt, comp, float("inf"))
    e = np.sort(err0.cpu().numpy())
    tol = float(0.5 * (e[len(e) // 2 - 1] + e[len(e) // 2]))
    xf, flags, nf, whole, err = lcs.lcs_surrogate_flowmap(
        mlp, frames, g, cfg.t0, cfg.tau, cfg.n_windows, tol, cfg.dt, whole_grid_fraction=1.0)
    ref, _, rflags = lcs.lcs_advect(frames, g, cfg.t0, T, cfg.dt)
    lcs.lcs_sync_status()
    nt = lcs.lcs_check_tile_count(g)
    fail = err.cpu().numpy() > tol
    _say(f"  tol {tol:.3e}: {nf}/{nt} tiles re-advected")
    assert 0 < nf < nt and nf == int(fail.sum()) and not whole
    np.testing.assert_array_equal(err.cpu().numpy(), err0.cpu().numpy())
    bad = fail[_tile_of_seed(g)]
    x, r, c = xf.cpu().numpy(), ref.cpu().numpy(), comp.cpu().numpy()
    np.testing.assert_array_equal(x[:, bad], r[:, bad])
    np.testing.assert_array_equal(x[:, ~bad], c[:, ~bad])
    fl = flags.cpu().numpy()
    np.testing.assert_array_equal(fl[bad], rflags.cpu().numpy()[bad])
    assert not fl[~bad].any()
    # the whole-grid branch on the same tolerance re-advects every seed
    xw, _, nfw, wholew, _ = lcs.lcs_surrogate_flowmap(
        mlp, frames, g, cfg.t0, cfg.tau, cfg.n_windows, tol, cfg.dt, whole_grid_fraction=0.0)
    lcs.lcs_sync_status()
    assert wholew and nfw == nf and torch.equal(xw, ref)


def test_check_error_matches_oracle_rk4(orc, env):
    # the per-tile error of the check samples against the FP64 oracle's RK4 at
    # the same check seeds: the two differ by no more than the position bar
    # (1e-5 of the domain length), and the failing set is the same wherever a
    # tile's error is not within that bar of the tolerance
    torch, lcs, sur, fs, frames, cfg = env
    g = _seeds()
    _say("case: check samples against the oracle")
    mlp = sur.new_model(cfg)
    T = cfg.n_windows * cfg.tau
    comp = lcs.lcs_surrogate_compose(mlp, g, cfg.t0, cfg.tau, cfg.n_windows)
    idx, tile, nt = _check_seed_index(g)
    vel = orc.Velocity(fs)
    rx, _, rfl = orc.advect_seeds(vel, g, cfg.t0, T, cfg.dt, idx=idx)
    assert not rfl.any()
    c = comp.cpu().numpy().astype(np.float64)[:, idx]
    d = np.linalg.norm(c - rx, axis=0)
    want = np.zeros(nt)
    np.maximum.at(want, tile, d)
    tol = float(np.median(want))
    err, fail, n_fail = lcs.lcs_surrogate_check(frames, g, cfg.t0, T, cfg.dt, comp, tol)
    lcs.lcs_sync_status()
    bar = 1e-5 * 2 * math.pi
    got = err.cpu().numpy().astype(np.float64)
    _say(f"  max |tile err - oracle tile err| = {np.abs(got - want).max():.2e}")
    assert np.abs(got - want).max() <= bar
    clear = np.abs(want - tol) > bar
    np.testing.assert_array_equal(fail.cpu().numpy()[clear], (want > tol)[clear].astype(np.uint8))
    assert int(n_fail.item()) == int(fail.cpu().numpy().sum())


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


def test_training_gain_and_fallback_frontier(env):
    # what training buys on the smooth ABC field, measured against plain RK4
    # over the same interval (the reference the check samples use):
    #  * the validation loss drops by three orders of magnitude;
    #  * the composition alone reaches a mean FTLE error within 2e-2 of RK4;
    #  * at a tolerance of 1e-1 part of the tiles are accepted and the rest
    #    re-advected, and the hybrid's FTLE error is below the composition's;
    #  * at the 1e-3 tolerance every tile falls back (the network's per-window
    #    error compounds over 8 windows to well above 1e-3), and the result
    #    is plain RK4 bit for bit.
    torch, lcs, sur, fs, frames, cfg = env
    _say("case: surrogate training on the ABC field, then the accept / fallback frontier")
    mlp = sur.new_model(cfg)
    xt, dx, fl = sur.training_data(frames, cfg, 1 << 20, seed=1)
    vxt, vdx, _ = sur.training_data(frames, cfg, 1 << 16, seed=2)
    assert not bool(fl.any())
    before = sur.evaluate(mlp, vxt, vdx)
    log = sur.train(mlp, xt, dx, epochs=16, batch=16384, lr=3e-3, val=(vxt, vdx))
    _say(f"val MSE {before:.3e} -> {log.val_loss:.3e} in {log.seconds:.2f} s ({log.steps} steps)")
    assert log.val_loss < 1e-3 * before
    g = _seeds((64, 64, 32))
    T = cfg.n_windows * cfg.tau
    nt = lcs.lcs_check_tile_count(g)
    ref, _, rfl = lcs.lcs_advect(frames, g, cfg.t0, T, cfg.dt)
    _, rsig, _ = lcs.lcs_cg_ftle(g, ref, T, flags=rfl)
    res = {}
    for tol in [float("inf"), 1e-1, 1e-3]:
        xf, flags, n_fail, err = sur.surrogate_flowmap(mlp, frames, g, cfg, tol=tol,
                                                       full_fallback_fraction=1.0)
        _, sig, _ = lcs.lcs_cg_ftle(g, xf, T, flags=flags)
        lcs.lcs_sync_status()
        e = (sig - rsig).abs()
        res[tol] = (n_fail, float(e.mean().item()), xf)
        _say(f"tol {tol}: fallback {n_fail}/{nt} tiles, median tile error "
             f"{float(err.median().item()):.3e}, FTLE err mean {e.mean().item():.2e} "
             f"max {e.max().item():.2e}")
    assert res[float("inf")][0] == 0 and res[float("inf")][1] <= 2e-2
    assert 0 < res[1e-1][0] < nt and res[1e-1][1] < res[float("inf")][1]
    assert res[1e-3][0] == nt and torch.equal(res[1e-3][2], ref)
