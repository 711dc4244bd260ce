"""lcs_advect_sorted (tracers re-bundled by position between segments) must be
bit-identical to lcs_advect: the per-tracer arithmetic is the same and the
state crosses segments exactly (two-float positions, global step index)."""
import math
import sys

import numpy as np
import pytest

from paper_2209_13775_amd import inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lcs():
    import torch
    assert torch.cuda.is_available()
    from paper_2209_13775_amd import lcs as _l
    return _l


def _same(a, b):
    return all(bool((x == y).all()) for x, y in zip(a, b))


@pytest.mark.parametrize("seg", [1, 7, 50, 1000])
def test_sorted_equals_plain_2d_with_exits_and_nan(lcs, seg):
    _say(f"case: sorted 2D, segment {seg}")
    fs = inputs.double_gyre_frames(nx=101, ny=51, n_frames=21)
    fs.u[0][5, 20, 40] = np.nan
    g = inputs.linspace_seeds(2, (150, 71), (0.0, 0.0), (2.0, 1.0))
    frames = lcs.DeviceFrames(fs)
    a = lcs.lcs_advect(frames, g, 0.0, 10.0, 0.05)
    b = lcs.lcs_advect_sorted(frames, g, 0.0, 10.0, 0.05, segment_steps=seg)
    lcs.lcs_sync_status()
    assert int((a[2] != 0).sum()) > 0
    assert _same(a, b)


@pytest.mark.parametrize("seg", [13, 100])
def test_sorted_equals_plain_3d_backward(lcs, seg):
    _say(f"case: sorted 3D backward, segment {seg}")
    fs = inputs.abc_frames(n=32, n_frames=17, dt_frame=0.5)
    L = 2 * math.pi
    g = inputs.periodic_seeds(3, (45, 38, 29), (L, L, L))
    frames = lcs.DeviceFrames(fs)
    a = lcs.lcs_advect(frames, g, 8.0, -6.0, -0.02)
    b = lcs.lcs_advect_sorted(frames, g, 8.0, -6.0, -0.02, segment_steps=seg)
    lcs.lcs_sync_status()
    assert _same(a, b)


def test_sorted_equals_plain_full_size_abc(lcs):
    _say("case: sorted ABC 128^3, 256^3 seeds, T=8")
    fs = inputs.abc_frames(n=128, n_frames=33, dt_frame=0.5)
    L = 2 * math.pi
    g = inputs.periodic_seeds(3, (256, 256, 256), (L, L, L))
    frames = lcs.DeviceFrames(fs)
    a = lcs.lcs_advect(frames, g, 0.0, 8.0, 0.02)
    b = lcs.lcs_advect_sorted(frames, g, 0.0, 8.0, 0.02, segment_steps=50)
    lcs.lcs_sync_status()
    assert _same(a, b)


def test_sorted_equals_plain_with_coarse_bins(lcs):
    # 8193 x 2049 nodes need 14 + 12 Morton bits for one-cell bins, more than
    # the 24 the sort allows, so its bins are two cells wide here
    _say("case: sorted 2D on 8193 x 2049 nodes (two-cell sort bins)")
    fs = inputs.double_gyre_frames(nx=8193, ny=2049, n_frames=3, dt_frame=5.0)
    g = inputs.linspace_seeds(2, (300, 150), (0.0, 0.0), (2.0, 1.0))
    frames = lcs.DeviceFrames(fs)
    a = lcs.lcs_advect(frames, g, 0.0, 10.0, 0.05)
    b = lcs.lcs_advect_sorted(frames, g, 0.0, 10.0, 0.05, segment_steps=37)
    lcs.lcs_sync_status()
    assert _same(a, b)


def test_sorted_equals_plain_with_crowded_bins(lcs):
    # 3 x 3 nodes: four sort bins for 90,000 tracers (~22,500 per bin, the
    # slot ranks the histogram hands out run that high), half of them leaving
    # the closed box and frozen on its edge
    _say("case: sorted 2D, 90,000 tracers in four one-cell bins")
    fs = inputs.uniform_frames(np.array([0.31, -0.17]), dim=2, n=3, lo=0.0, hi=1.0)
    g = inputs.linspace_seeds(2, (300, 300), (0.005, 0.005), (0.995, 0.995))
    frames = lcs.DeviceFrames(fs)
    a = lcs.lcs_advect(frames, g, 0.0, 2.0, 0.05)
    b = lcs.lcs_advect_sorted(frames, g, 0.0, 2.0, 0.05, segment_steps=10)
    lcs.lcs_sync_status()
    assert _same(a, b)
    n_out = int((a[2] != 0).sum())
    assert 0 < n_out < g.count


def test_tuned_equals_plain_and_cache_round_trip(lcs, tmp_path):
    # the autotuner times every candidate once, keeps the fastest, writes it to
    # the cache; a second plan reads the cache and runs the choice without
    # timing; every run gives lcs_advect's bits
    _say("case: autotuned advection and its cache")
    import torch
    fs = inputs.abc_frames(n=32, n_frames=17, dt_frame=0.5)
    L = 2 * math.pi
    g = inputs.periodic_seeds(3, (45, 38, 29), (L, L, L))
    frames = lcs.DeviceFrames(fs)
    a = lcs.lcs_advect(frames, g, 0.0, 6.0, 0.02)
    ws = torch.empty(lcs.lcs_advect_sorted_workspace_bytes(frames, g), dtype=torch.uint8,
                     device="cuda")
    cache = str(tmp_path / "tune.jsonl")
    p1 = lcs.Plan(autotune_cache=cache)
    x1, c1, f1, seg1, ms1 = lcs.lcs_advect_tuned(p1, frames, g, 0.0, 6.0, 0.02, workspace=ws,
                                                 candidates=[0, 100, 25])
    lcs.lcs_sync_status()
    assert ms1 is not None and set(ms1) == {0, 100, 25} and all(v > 0 for v in ms1.values())
    assert seg1 == min(ms1, key=ms1.get)
    assert _same(a, (x1, c1, f1))
    # same plan, same workload: no timing
    x2, c2, f2, seg2, ms2 = lcs.lcs_advect_tuned(p1, frames, g, 0.0, 6.0, 0.02, workspace=ws,
                                                 candidates=[0, 100, 25])
    lcs.lcs_sync_status()
    assert ms2 is None and seg2 == seg1 and _same(a, (x2, c2, f2))
    p1.close()
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and f'"segment_steps": {seg1}' in lines[0]
    p2 = lcs.Plan(autotune_cache=cache)
    x3, c3, f3, seg3, ms3 = lcs.lcs_advect_tuned(p2, frames, g, 0.0, 6.0, 0.02, workspace=ws)
    lcs.lcs_sync_status()
    assert ms3 is None and seg3 == seg1 and _same(a, (x3, c3, f3))
    # without a workspace only the single launch can run
    x4, c4, f4, seg4, _ = lcs.lcs_advect_tuned(p2, frames, g, 0.0, 4.0, 0.02,
                                               candidates=[100, 0])
    lcs.lcs_sync_status()
    assert seg4 == 0
    p2.close()
    b = lcs.lcs_advect(frames, g, 0.0, 4.0, 0.02)
    lcs.lcs_sync_status()
    assert _same(b, (x4, c4, f4))


def _tpair_case(name):
    """(frames, seeds, t0, T, dt) of the time-paired re-bundling cases."""
    L = 2 * math.pi
    if name == "closed_box_exits_nan":
        fs = inputs.sample_field(inputs.abc_velocity, 3, (33, 33, 33), (0.0,) * 3, (L / 32,) * 3,
                                 (False,) * 3, 0.0, 0.5, 9).astype(np.float32)
        fs.u[0][4, 10, 12, 14] = np.nan
        g = inputs.linspace_seeds(3, (40, 36, 30), (0.3,) * 3, (L - 0.3,) * 3)
        return fs, g, 0.5, 3.0, 0.02
    if name == "mixed_periodic":
        fs = inputs.sample_field(inputs.abc_velocity, 3, (32, 33, 32), (0.0,) * 3, (L / 32,) * 3,
                                 (True, False, True), 0.0, 0.5, 9).astype(np.float32)
        g = inputs.SeedGrid(3, (40, 30, 36), (0.0, 0.3, 0.0), (L / 40, (L - 0.6) / 29, L / 36),
                            (True, False, True))
        return fs, g, 0.0, 3.5, 0.02
    if name == "periodic_backward":
        fs = inputs.abc_frames(n=32, n_frames=17, dt_frame=0.5)
        return fs, inputs.periodic_seeds(3, (45, 38, 29), (L, L, L)), 8.0, -6.0, -0.02
    # a 9^3 closed box: the region can cover the whole grid
    fs = inputs.uniform_frames(np.array([0.37, -0.21, 0.13]), dim=3, n=9, lo=0.0, hi=1.0)
    g = inputs.linspace_seeds(3, (20, 18, 16), (0.013, 0.011, 0.017), (0.987, 0.989, 0.983))
    return fs, g, 0.0, 3.0, 0.05


@pytest.mark.parametrize("seg", [13, 100])
@pytest.mark.parametrize("case", ["closed_box_exits_nan", "mixed_periodic", "periodic_backward",
                                  "small_box"])
def test_sorted_tpair_equals_plain(lcs, case, seg):
    """Re-bundled 3D segments on time-paired frames (closed walls with exits
    and a NaN node, mixed periodic and closed axes, backward time, a grid
    smaller than a workgroup's spread): the same bits as the single launch."""
    _say(f"case: sorted 3D on time-paired frames, {case}, segment {seg}")
    fs, g, t0, T, dt = _tpair_case(case)
    frames = lcs.DeviceFrames.interleaved(fs, "tpair")
    a = lcs.lcs_advect(frames, g, t0, T, dt)
    b = lcs.lcs_advect_sorted(frames, g, t0, T, dt, segment_steps=seg)
    lcs.lcs_sync_status()
    if case in ("closed_box_exits_nan", "small_box"):
        assert int((a[2] != 0).sum()) > 0
    if case == "closed_box_exits_nan":
        assert int((a[2] == 2).sum()) > 0           # the NaN node was sampled
    assert _same(a, b)
