"""GPU tests of lcs_advect_batched: many t0 windows in one persistent,
graph-replayed launch.

Bar: every window's xf / cell / flags are bit-identical to lcs_advect on that
window (the per-tracer arithmetic does not depend on scheduling), and the
windows match the FP64 oracle to the parity bar of the single-window tests.
Graph replays (with eager work in between) reproduce the eager result.
"""
import math
import sys

import numpy as np
import pytest

from paper_2209_13775_amd import inputs
from tests import parity

pytestmark = pytest.mark.gpu


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


def _per_window(lcs, frames, g, windows, dt):
    outs = []
    for t0, T in windows:
        xf, cell, flags = lcs.lcs_advect(frames, g, t0, T, dt)
        outs.append((xf, cell, flags))
    return outs


def _assert_same(torch, batched, single):
    xf, cell, flags = batched
    for w, (sx, sc, sf) in enumerate(single):
        assert torch.equal(xf[w], sx), f"window {w}: xf differs"
        assert torch.equal(cell[w], sc), f"window {w}: cell differs"
        assert torch.equal(flags[w], sf), f"window {w}: flags differ"


def test_batched_equals_per_window_2d(lcs, torch):
    _say("case: batched double gyre, 12 windows, ragged seeds")
    fs = inputs.double_gyre_frames(nx=129, ny=65, n_frames=41, dt_frame=0.5)
    g = inputs.linspace_seeds(2, (100, 37), (0.0, 0.0), (2.0, 1.0))
    windows = inputs.t0_windows(12, t0_range=(0.0, 5.0), T_choices=(2.5, 5.0, 7.5), seed=3)
    frames = lcs.DeviceFrames(fs)
    plan = lcs.Plan()
    b = lcs.lcs_advect_batched(plan, frames, g, windows, 0.05)
    single = _per_window(lcs, frames, g, windows, 0.05)
    lcs.lcs_sync_status()
    _assert_same(torch, b, single)
    assert plan.stats() == {"graph_launches": 1, "graph_captures": 1}


def test_batched_backward_3d(lcs, torch):
    _say("case: batched ABC 24^3 backward, 5 windows")
    fs = inputs.abc_frames(n=24, n_frames=17, dt_frame=0.5)
    L = 2 * math.pi
    g = inputs.periodic_seeds(3, (20, 13, 9), (L, L, L))
    windows = [(8.0, -2.0), (7.5, -4.0), (6.0, -1.0), (8.0, -3.0), (5.0, -5.0)]
    frames = lcs.DeviceFrames(fs)
    plan = lcs.Plan()
    b = lcs.lcs_advect_batched(plan, frames, g, windows, -0.02)
    single = _per_window(lcs, frames, g, windows, -0.02)
    lcs.lcs_sync_status()
    _assert_same(torch, b, single)


def test_graph_replay_with_eager_work_between(lcs, torch):
    _say("case: graph replays")
    fs = inputs.double_gyre_frames(nx=101, ny=51, n_frames=21)
    g = inputs.linspace_seeds(2, (64, 32), (0.0, 0.0), (2.0, 1.0))
    windows = inputs.t0_windows(8, t0_range=(0.0, 8.0), T_choices=(5.0, 10.0), seed=1)
    frames = lcs.DeviceFrames(fs)
    plan = lcs.Plan()
    single = _per_window(lcs, frames, g, windows, 0.05)
    xf = torch.empty((8, 2, g.count), dtype=torch.float32, device="cuda")
    cell = torch.empty((8, g.count), dtype=torch.int64, device="cuda")
    flags = torch.empty((8, g.count), dtype=torch.uint8, device="cuda")
    for rep in range(4):
        xf.fill_(float("nan"))
        cell.fill_(-7)
        flags.fill_(255)
        lcs.lcs_advect_batched(plan, frames, g, windows, 0.05, xf, cell, flags)
        # eager work on the same stream between replays
        lcs.lcs_advect(frames, g, 1.0, 3.0, 0.05)
        lcs.lcs_sync_status()
        _assert_same(torch, (xf, cell, flags), single)
    st = plan.stats()
    assert st["graph_captures"] == 1 and st["graph_launches"] == 4
    # different windows -> a new capture
    w2 = [(t0 + 0.5, T) for t0, T in windows]
    lcs.lcs_advect_batched(plan, frames, g, w2, 0.05, xf, cell, flags)
    single2 = _per_window(lcs, frames, g, w2, 0.05)
    lcs.lcs_sync_status()
    _assert_same(torch, (xf, cell, flags), single2)
    assert plan.stats()["graph_captures"] == 2


def test_batched_parity_with_oracle(orc, lcs, torch):
    _say("case: batched vs oracle")
    fs = inputs.double_gyre_frames(nx=101, ny=51, n_frames=21)
    g = inputs.linspace_seeds(2, (48, 24), (0.0, 0.0), (2.0, 1.0))
    windows = [(0.0, 10.0), (3.5, 5.0), (9.25, 7.5)]
    frames = lcs.DeviceFrames(fs)
    plan = lcs.Plan()
    xf, cell, flags = lcs.lcs_advect_batched(plan, frames, g, windows, 0.05)
    lcs.lcs_sync_status()
    vel = orc.Velocity(fs)
    for w, (t0, T) in enumerate(windows):
        rx, rc, rf, rm = orc.advect_seeds(vel, g, t0, T, 0.05, margin=True)
        gx = xf[w].cpu().numpy()
        gf = flags[w].cpu().numpy()
        unamb = rm > 2e-5
        np.testing.assert_array_equal(gf[unamb], rf[unamb])
        st = parity.position_stats(gx, rx, 2e-5, gf == rf)
        parity.assert_positions(st, 2e-5, f"batched window {w}")
        np.testing.assert_array_equal(cell[w].cpu().numpy(),
                                      orc.cell_index(vel, gx.astype(np.float64)))


def test_batched_full_size_64_windows(orc, lcs, torch):
    """Double gyre 1025x513 x 101 FP32 frames (t = 0.25 f), 64 windows drawn
    with default_rng(0), 1024x512 seeds each, dt = 0.05 -- the batched
    benchmark launch -- against per-window launches and (sampled) the oracle."""
    _say("case: batched full size, 64 windows x 1024x512 seeds")
    fs = inputs.double_gyre_frames(nx=1025, ny=513, n_frames=101, dt_frame=0.25,
                                   dtype=np.float32)
    g = inputs.linspace_seeds(2, (1024, 512), (0.0, 0.0), (2.0, 1.0))
    windows = inputs.t0_windows(64, seed=0)
    frames = lcs.DeviceFrames(fs)
    plan = lcs.Plan()
    xf, cell, flags = lcs.lcs_advect_batched(plan, frames, g, windows, 0.05)
    lcs.lcs_sync_status()
    for w in range(0, 64, 9):
        sx, sc, sf = lcs.lcs_advect(frames, g, windows[w][0], windows[w][1], 0.05)
        lcs.lcs_sync_status()
        assert torch.equal(xf[w], sx) and torch.equal(cell[w], sc) and torch.equal(flags[w], sf)
    vel = orc.Velocity(fs)
    idx = parity.sample_seeds(g, 64, seed=5)
    it = torch.from_numpy(idx).cuda()
    for w in range(0, 64, 7):
        rx, rc, rf, rm = orc.advect_seeds(vel, g, windows[w][0], windows[w][1], 0.05, idx=idx,
                                          margin=True)
        gx = xf[w][:, it].cpu().numpy()
        gf = flags[w][it].cpu().numpy()
        unamb = rm > 2e-5
        np.testing.assert_array_equal(gf[unamb], rf[unamb])
        st = parity.position_stats(gx, rx, 2e-5, gf == rf)
        parity.assert_positions(st, 2e-5, f"full batched window {w}")
