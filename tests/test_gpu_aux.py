"""GPU parity of the auxiliary-point gradient (lcs_advect_aux + lcs_cg_aux)
against the FP64 oracle, through the C ABI.

Bars: auxiliary positions mean and p99 within 1e-5 of the domain length;
flags bit-exact where unambiguous; C bit-exact when the oracle differences
the GPU's own (exact two-float) positions; FTLE within 1e-3 on clean seeds;
with delta equal to the seed spacing the auxiliary C matches the seed-grid C
at interior seeds.
"""
import math
import sys

import numpy as np
import pytest

from paper_2209_13775_amd import inputs
from tests import parity

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    return _t


@pytest.fixture(scope="module")
def lcs(torch):
    from paper_2209_13775_amd import lcs as _l
    return _l


def _flat(x):
    """[dim][2dim][Ns] -> (dim, 2dim*Ns), the oracle's auxiliary layout."""
    d = x.shape[0]
    return x.reshape(d, -1)


def _check(orc, lcs, fs, g, delta, t0, T, dt, what):
    frames = lcs.DeviceFrames(fs)
    hi, lo, fl = lcs.lcs_advect_aux(frames, g, delta, t0, T, dt)
    Cg, sg = lcs.lcs_cg_aux(g, delta, hi, lo, fl)
    _, sig = lcs.lcs_ftle(g.dim, Cg, T)
    lcs.lcs_sync_status()
    xg = _flat(_np(hi)).astype(np.float64) + _flat(_np(lo)).astype(np.float64)
    fg = _np(fl).reshape(-1)
    vel = orc.Velocity(fs)
    xo, fo, mo, Co, so = orc.advect_aux(vel, g, delta, t0, T, dt)
    L = parity.domain_length(fs)
    unamb = mo > parity.POS_TOL_FRAC * L
    np.testing.assert_array_equal(fg[unamb], fo[unamb])
    st = parity.position_stats(xg, xo, parity.POS_TOL_FRAC * L, mask=(fg == fo))
    parity.assert_positions(st, parity.POS_TOL_FRAC * L, what)
    # identical positions: bit-exact C and stencil flags
    Cx, sx = orc.cg_aux(g.dim, delta, xg, fg)
    np.testing.assert_array_equal(_np(Cg), Cx)
    np.testing.assert_array_equal(_np(sg), sx)
    _, osig = orc.ftle(g.dim, Co, T)
    clean = (_np(sg) == 0) & (so == 0)
    err = np.abs(_np(sig)[clean] - osig[clean])
    _say(f"{what}: FTLE max err {err.max():.2e} over {clean.sum()} seeds")
    assert err.max() <= parity.FTLE_TOL
    return _np(Cg), _np(sg)


def test_double_gyre_aux(orc, lcs):
    fs = inputs.double_gyre_frames()
    g = inputs.linspace_seeds(2, (256, 128), (0.0, 0.0), (2.0, 1.0))
    _say("case: aux points, double gyre 256x128 seeds, delta 1e-3")
    _check(orc, lcs, fs, g, [1e-3, 1e-3], 0.0, 10.0, 0.05, "aux double gyre")


def test_abc_aux_periodic(orc, lcs):
    fs = inputs.abc_frames(n=32, n_frames=9, dt_frame=0.5)
    L = 2 * math.pi
    g = inputs.periodic_seeds(3, (36, 30, 24), (L, L, L))
    _say("case: aux points, ABC 32^3, seeds 36x30x24")
    _check(orc, lcs, fs, g, [2e-3, 3e-3, 1e-3], 0.5, 3.0, 0.02, "aux ABC")


def test_aux_outside_start_and_exits(orc, lcs):
    c = np.array([0.37, -0.21])
    fs = inputs.uniform_frames(c, dim=2, n=9, lo=0.0, hi=1.0)
    g = inputs.linspace_seeds(2, (48, 40), (0.0, 0.0), (1.0, 1.0))   # seeds on the walls
    _say("case: aux points leaving the box")
    Cg, sg = _check(orc, lcs, fs, g, [0.02, 0.02], 0.0, 1.0, 0.05, "aux exits")
    assert (sg != 0).sum() > 100


def test_delta_equal_spacing_matches_grid(lcs, torch):
    fs = inputs.double_gyre_frames(nx=101, ny=51, n_frames=11)
    g = inputs.linspace_seeds(2, (97, 49), (0.05, 0.05), (1.95, 0.95))
    frames = lcs.DeviceFrames(fs)
    delta = [g.spacing[0], g.spacing[1]]
    hi, lo, fl = lcs.lcs_advect_aux(frames, g, delta, 0.0, 6.0, 0.05)
    Ca, sa = lcs.lcs_cg_aux(g, delta, hi, lo, fl)
    xf, _, flags = lcs.lcs_advect(frames, g, 0.0, 6.0, 0.05)
    Cg, sg = lcs.lcs_cg_tensor(g, xf, flags)
    lcs.lcs_sync_status()
    c = g.coords_of(np.arange(g.count))
    inner = (c[0] > 0) & (c[0] < g.n[0] - 1) & (c[1] > 0) & (c[1] < g.n[1] - 1)
    ok = inner & (_np(sa) == 0) & (_np(sg) == 0)
    Ca, Cg = _np(Ca), _np(Cg)
    rel = np.abs(Ca[:, ok] - Cg[:, ok]).max(axis=0) / np.abs(Cg[:, ok]).max(axis=0)
    _say(f"delta = h: max relative C difference {rel.max():.2e}")
    assert rel.max() <= 1e-3


@pytest.mark.parametrize("seg", [1, 7, 100])
def test_aux_sorted_equals_aux(lcs, torch, seg):
    """Re-bundled auxiliary tracers give lcs_advect_aux's outputs bit for bit:
    2D with exits and points starting outside, 3D periodic on time-paired
    frames."""
    c = np.array([0.37, -0.21])
    fs = inputs.uniform_frames(c, dim=2, n=9, lo=0.0, hi=1.0)
    g = inputs.linspace_seeds(2, (48, 40), (0.0, 0.0), (1.0, 1.0))
    frames = lcs.DeviceFrames(fs)
    a = lcs.lcs_advect_aux(frames, g, [0.02, 0.02], 0.0, 1.0, 0.05)
    b = lcs.lcs_advect_aux_sorted(frames, g, [0.02, 0.02], 0.0, 1.0, 0.05, segment_steps=seg)
    lcs.lcs_sync_status()
    assert int((a[2] != 0).sum()) > 100
    for u, v in zip(a, b):
        assert torch.equal(u, v)
    fs3 = inputs.abc_frames(n=32, n_frames=9, dt_frame=0.5)
    L = 2 * math.pi
    g3 = inputs.periodic_seeds(3, (24, 20, 18), (L, L, L))
    fr3 = lcs.DeviceFrames.interleaved(fs3, "tpair")
    d3 = [1e-3, 2e-3, 1.5e-3]
    a = lcs.lcs_advect_aux(fr3, g3, d3, 0.5, 3.0, 0.02)
    b = lcs.lcs_advect_aux_sorted(fr3, g3, d3, 0.5, 3.0, 0.02, segment_steps=seg)
    lcs.lcs_sync_status()
    for u, v in zip(a, b):
        assert torch.equal(u, v)
