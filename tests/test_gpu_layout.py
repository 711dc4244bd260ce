"""GPU tests of the interleaved frame layouts (LCS_LAYOUT_XYZ, LCS_LAYOUT_XYZW,
LCS_LAYOUT_TPAIR):
lcs_frames_interleave copies values exactly, and the advection entry points
reading interleaved frames meet the same oracle parity bars as with
structure-of-arrays frames (positions 1e-5 L mean and p99, FTLE 1e-3, flags
and cell index bit-exact where unambiguous); within one layout the
re-bundled, batched and single-launch paths stay bit-identical."""
import math
import sys

import numpy as np
import pytest

from paper_2209_13775_amd import inputs
from tests import parity
from tests.test_gpu_parity import compare_full

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


def _gpu(lcs, frames, g, t0, T, dt):
    xf, cell, flags = lcs.lcs_advect(frames, g, t0, T, dt)
    C, sfl = lcs.lcs_cg_tensor(g, xf, flags)
    lam, sig = lcs.lcs_ftle(g.dim, C, T)
    lcs.lcs_sync_status()
    return dict(xf=_np(xf), cell=_np(cell), flags=_np(flags), C=_np(C), sflags=_np(sfl),
                lam=_np(lam), ftle=_np(sig))


def _orc(orc, fs, g, t0, T, dt):
    vel = orc.Velocity(fs)
    xf, cell, flags, margin = orc.advect_seeds(vel, g, t0, T, dt, margin=True)
    C, sfl = orc.cg_tensor(g, xf, flags)
    lam, sig = orc.ftle(g.dim, C, T)
    return dict(vel=vel, xf=xf, cell=cell, flags=flags, margin=margin, C=C, sflags=sfl, lam=lam,
                ftle=sig)


@pytest.mark.parametrize("dim,layout", [(2, "xyz"), (3, "xyz"), (3, "xyzw")])
def test_interleave_copies_exactly(lcs, torch, dim, layout):
    fs = inputs.random_frames(dim, (9, 7, 5)[:dim], 6, seed=dim).astype(np.float32)
    soa = lcs.DeviceFrames(fs)
    il = lcs.lcs_frames_interleave(soa, layout, f_first=1, f_count=4)
    lcs.lcs_sync_status()
    got = _np(il.u[0])
    S = 4 if layout == "xyzw" else dim
    assert got.shape == (4, int(np.prod((9, 7, 5)[:dim])), S)
    for c in range(dim):
        want = np.asarray(fs.u[c])[1:5].reshape(4, -1)
        np.testing.assert_array_equal(got[..., c], want)
    if S == 4:
        assert (got[..., 3] == 0).all()
    assert il.desc.n_frames == 4 and il.desc.t_first == fs.t_first + fs.dt_frame
    assert il.desc.layout == (lcs.LCS_LAYOUT_XYZW if S == 4 else lcs.LCS_LAYOUT_XYZ)


@pytest.mark.parametrize("periodic,n_frames,f_first,f_count",
                         [(True, 6, 1, 4), (False, 6, 1, 4), (True, 24, 2, 21)])
def test_tpair_records_exact(lcs, torch, periodic, n_frames, f_first, f_count):
    """Time-paired records: frames p and p+1 of each node side by side, one
    extra node per x row repeating node 0 (3 pairs; and 20 pairs, which the
    staging kernel takes as runs of 8, 8 and 4)."""
    fs = inputs.random_frames(3, (9, 7, 5), n_frames, seed=4,
                              periodic=(True, True, True) if periodic else None).astype(np.float32)
    soa = lcs.DeviceFrames(fs)
    il = lcs.lcs_frames_interleave(soa, "tpair", f_first=f_first, f_count=f_count)
    lcs.lcs_sync_status()
    pairs = f_count - 1
    got = _np(il.u[0]).reshape(pairs, 5, 7, 10, 6)
    u = [np.asarray(c)[f_first:f_first + f_count] for c in fs.u]   # (f_count, 5, 7, 9) per component
    for p in range(pairs):
        for c in range(3):
            np.testing.assert_array_equal(got[p, :, :, :9, c], u[c][p])
            np.testing.assert_array_equal(got[p, :, :, :9, 3 + c], u[c][p + 1])
            np.testing.assert_array_equal(got[p, :, :, 9, c], u[c][p][:, :, 0])
            np.testing.assert_array_equal(got[p, :, :, 9, 3 + c], u[c][p + 1][:, :, 0])
    assert il.desc.layout == lcs.LCS_LAYOUT_TPAIR and il.desc.n_frames == f_count
    assert il.desc.t_first == fs.t_first + f_first * fs.dt_frame
    want = lcs.lib().lcs_frames_interleave_floats(soa.ref, lcs.LCS_LAYOUT_TPAIR, f_count)
    assert want == il.u[0].numel()


@pytest.mark.parametrize("periodic,n_frames,f_first,f_count",
                         [(True, 6, 1, 4), (False, 24, 2, 21)])
def test_tpair_records_exact_2d(lcs, torch, periodic, n_frames, f_first, f_count):
    """2D time-paired records: (u, v) of frame p then of frame p+1 per node,
    16 bytes, one extra node per x row repeating node 0."""
    fs = inputs.random_frames(2, (9, 7), n_frames, seed=6,
                              periodic=(True, True) if periodic else None).astype(np.float32)
    soa = lcs.DeviceFrames(fs)
    il = lcs.lcs_frames_interleave(soa, "tpair", f_first=f_first, f_count=f_count)
    lcs.lcs_sync_status()
    pairs = f_count - 1
    got = _np(il.u[0]).reshape(pairs, 7, 10, 4)
    u = [np.asarray(c)[f_first:f_first + f_count] for c in fs.u]   # (f_count, 7, 9) per component
    for p in range(pairs):
        for c in range(2):
            np.testing.assert_array_equal(got[p, :, :9, c], u[c][p])
            np.testing.assert_array_equal(got[p, :, :9, 2 + c], u[c][p + 1])
            np.testing.assert_array_equal(got[p, :, 9, c], u[c][p][:, 0])
            np.testing.assert_array_equal(got[p, :, 9, 2 + c], u[c][p + 1][:, 0])
    assert il.desc.layout == lcs.LCS_LAYOUT_TPAIR and il.desc.n_frames == f_count
    want = lcs.lib().lcs_frames_interleave_floats(soa.ref, lcs.LCS_LAYOUT_TPAIR, f_count)
    assert want == il.u[0].numel()


@pytest.mark.parametrize("layout", ["xyz", "tpair"])
def test_double_gyre_interleaved(orc, lcs, layout):
    fs = inputs.double_gyre_frames()
    g = inputs.linspace_seeds(2, (256, 128), (0.0, 0.0), (2.0, 1.0))
    _say(f"case: double gyre, {layout} frames")
    frames = lcs.DeviceFrames.interleaved(fs, layout)
    compare_full(orc, fs, g, _gpu(lcs, frames, g, 0.0, 10.0, 0.05), _orc(orc, fs, g, 0.0, 10.0, 0.05),
                 f"double gyre {layout}")


@pytest.mark.parametrize("layout", ["xyz", "tpair"])
def test_periodic_2d_interleaved_wrap(orc, lcs, layout):
    fs = inputs.taylor_green_frames(n=48, n_frames=9)
    L = 2 * math.pi
    g = inputs.periodic_seeds(2, (96, 80), (L, L))
    _say(f"case: periodic Taylor-Green, {layout} frames")
    frames = lcs.DeviceFrames.interleaved(fs, layout)
    compare_full(orc, fs, g, _gpu(lcs, frames, g, 0.0, 3.5, 0.05), _orc(orc, fs, g, 0.0, 3.5, 0.05),
                 f"taylor-green {layout}")


@pytest.mark.parametrize("layout", ["xyz", "xyzw", "tpair"])
def test_abc_small_interleaved(orc, lcs, layout):
    fs = inputs.abc_frames(n=32, n_frames=9, dt_frame=0.5)
    L = 2 * math.pi
    g = inputs.periodic_seeds(3, (40, 36, 28), (L, L, L))
    _say(f"case: ABC 32^3, {layout} frames")
    frames = lcs.DeviceFrames.interleaved(fs, layout)
    compare_full(orc, fs, g, _gpu(lcs, frames, g, 0.5, 3.0, 0.02), _orc(orc, fs, g, 0.5, 3.0, 0.02),
                 f"abc {layout}")


@pytest.mark.parametrize("layout3", ["xyzw", "tpair"])
def test_exits_and_nan_interleaved(orc, lcs, layout3):
    c = np.array([0.37, -0.21, 0.13])
    fs = inputs.uniform_frames(c, dim=3, n=9, lo=0.0, hi=1.0)
    g = inputs.linspace_seeds(3, (20, 18, 16), (0.013, 0.011, 0.017), (0.987, 0.989, 0.983))
    frames = lcs.DeviceFrames.interleaved(fs, layout3)
    ref = _orc(orc, fs, g, 0.0, 3.0, 0.05)
    assert (ref["flags"] == 1).sum() > 500
    compare_full(orc, fs, g, _gpu(lcs, frames, g, 0.0, 3.0, 0.05), ref, f"uniform {layout3}")
    fs2 = inputs.double_gyre_frames(nx=51, ny=26, n_frames=11)
    fs2.u[1][3, 12, 20] = np.nan
    g2 = inputs.linspace_seeds(2, (64, 32), (0.02, 0.02), (1.98, 0.98))
    ref2 = _orc(orc, fs2, g2, 0.0, 8.0, 0.05)
    assert (ref2["flags"] == 2).sum() > 0
    layout2 = "xyz" if layout3 == "xyzw" else "tpair"
    frames2 = lcs.DeviceFrames.interleaved(fs2, layout2)
    compare_full(orc, fs2, g2, _gpu(lcs, frames2, g2, 0.0, 8.0, 0.05), ref2, f"NaN {layout2}")


@pytest.mark.parametrize("layout", ["xyz", "xyzw", "tpair"])
def test_abc_full_size_interleaved_sampled(orc, lcs, torch, layout):
    """The benchmark launch (ABC 128^3, 256^3 seeds, T = 8, re-bundled segments
    of 50) on interleaved frames, checked at sampled seeds; the single-launch
    path on the same frames gives the same bits."""
    fs = inputs.abc_frames(n=128, n_frames=33, dt_frame=0.5)
    L = 2 * math.pi
    g = inputs.periodic_seeds(3, (256, 256, 256), (L, L, L))
    _say(f"case: ABC full size, {layout} frames, re-bundled")
    frames = lcs.DeviceFrames.interleaved(fs, layout)
    xf, cell, flags = lcs.lcs_advect_sorted(frames, g, 0.0, 8.0, 0.02, 50)
    xt, ct, ft = lcs.lcs_advect(frames, g, 0.0, 8.0, 0.02)
    lam, sig, sfl = lcs.lcs_cg_ftle(g, xf, 8.0, flags=flags)
    lcs.lcs_sync_status()
    assert torch.equal(xf, xt) and torch.equal(cell, ct) and torch.equal(flags, ft)
    idx = parity.sample_seeds(g, 300, seed=7)
    it = torch.from_numpy(idx).to(xf.device)
    gx, gcell, gflags, gsig = _np(xf[:, it]), _np(cell[it]), _np(flags[it]), _np(sig[it])
    del xf, cell, flags, lam, sig, sfl, xt, ct, ft, frames
    torch.cuda.empty_cache()
    vel = orc.Velocity(fs.astype(np.float32))
    ref = parity.oracle_sampled_ftle(orc, vel, g, idx, 0.0, 8.0, 0.02)
    assert not gflags.any() and not ref["flags"].any()
    tol = parity.POS_TOL_FRAC * L
    st = parity.position_stats(gx, ref["xf"], tol)
    parity.assert_positions(st, tol, f"abc full {layout} (sampled)")
    np.testing.assert_array_equal(gcell, orc.cell_index(vel, gx.astype(np.float64)))
    err = np.abs(gsig - ref["ftle"])
    _say(f"abc full {layout}: FTLE max err {err.max():.3e}")
    assert err.max() <= parity.FTLE_TOL


@pytest.mark.parametrize("layout", ["xyz", "tpair"])
def test_batched_interleaved_equals_per_window(lcs, torch, layout):
    fs = inputs.double_gyre_frames(nx=101, ny=51, n_frames=41, dt_frame=0.25)
    g = inputs.linspace_seeds(2, (96, 48), (0.0, 0.0), (2.0, 1.0))
    frames = lcs.DeviceFrames.interleaved(fs, layout)
    windows = [(0.5, 4.0), (2.0, 1.5), (1.0, 6.5)]
    plan = lcs.Plan()
    xb, cb, fb = lcs.lcs_advect_batched(plan, frames, g, windows, 0.05)
    for k, (t0, T) in enumerate(windows):
        x, c, f = lcs.lcs_advect(frames, g, t0, T, 0.05)
        lcs.lcs_sync_status()
        assert torch.equal(xb[k], x) and torch.equal(cb[k], c) and torch.equal(fb[k], f)
    plan.close()


def test_layouts_give_identical_bits(lcs, torch):
    """The interpolation arithmetic is written out (explicit FMAs, no
    contraction), so every frame layout gives the same bits, single-launch and
    re-bundled alike."""
    fs = inputs.abc_frames(n=32, n_frames=9, dt_frame=0.5)
    L = 2 * math.pi
    g = inputs.periodic_seeds(3, (48, 40, 36), (L, L, L))
    outs = []
    for layout in ("soa", "xyz", "xyzw", "tpair"):
        fr = lcs.DeviceFrames(fs) if layout == "soa" else lcs.DeviceFrames.interleaved(fs, layout)
        a = lcs.lcs_advect(fr, g, 0.5, 3.0, 0.02)
        b = lcs.lcs_advect_sorted(fr, g, 0.5, 3.0, 0.02, 20)
        c = lcs.lcs_advect_ab_sorted(fr, g, 0.5, 3.0, 0.02, order=4, segment_steps=20)
        lcs.lcs_sync_status()
        for u, v in zip(a, b):
            assert torch.equal(u, v), layout
        outs.append((a[0], c[0]))
    for k in (1, 2, 3):
        assert torch.equal(outs[0][0], outs[k][0]) and torch.equal(outs[0][1], outs[k][1])
    fs2 = inputs.double_gyre_frames(nx=51, ny=26, n_frames=11)
    g2 = inputs.linspace_seeds(2, (97, 45), (0.0, 0.0), (2.0, 1.0))
    outs2 = []
    for layout in ("soa", "xyz", "tpair"):
        fr = lcs.DeviceFrames(fs2) if layout == "soa" else lcs.DeviceFrames.interleaved(fs2, layout)
        a = lcs.lcs_advect(fr, g2, 0.5, 7.0, 0.05)
        b = lcs.lcs_advect_sorted(fr, g2, 0.5, 7.0, 0.05, 20)
        c = lcs.lcs_advect_ab_sorted(fr, g2, 0.5, 7.0, 0.05, order=3, segment_steps=20)
        lcs.lcs_sync_status()
        for u, v in zip(a, b):
            assert torch.equal(u, v), layout
        outs2.append((a[0], c[0]))
    for k in (1, 2):
        assert torch.equal(outs2[0][0], outs2[k][0]) and torch.equal(outs2[0][1], outs2[k][1])


def test_tpair_equals_soa_in_every_entry_point(lcs, torch):
    """Points, batched windows, auxiliary points, snapshots and early FTLE read
    time-paired frames through the same step loop: the same bits as with
    structure-of-arrays frames, on a closed box where tracers leave."""
    L = 2 * math.pi
    fs = inputs.sample_field(inputs.abc_velocity, 3, (33, 33, 33), (0.0,) * 3, (L / 32,) * 3,
                             (False,) * 3, 0.0, 0.5, 9).astype(np.float32)
    g = inputs.linspace_seeds(3, (22, 20, 18), (0.3,) * 3, (L - 0.3,) * 3)
    t0, dt, N = 0.5, 0.02, 150
    soa = lcs.DeviceFrames(fs)
    tp = lcs.lcs_frames_interleave(soa, "tpair")
    rng = np.random.default_rng(5)
    x0 = torch.from_numpy(rng.uniform(0.2, L - 0.2, size=(3, 777)).astype(np.float32)).cuda()
    tt = torch.from_numpy(rng.uniform(0.0, 1.0, size=777)).cuda()
    windows = [(0.5, 2.0), (1.0, 1.5), (0.0, 3.0)]
    out = {}
    for name, fr in (("soa", soa), ("tpair", tp)):
        plan = lcs.Plan()
        r = {"points": lcs.lcs_advect_points(fr, x0, tt, 2.5, dt),
             "batched": lcs.lcs_advect_batched(plan, fr, g, windows, dt),
             "aux": lcs.lcs_advect_aux(fr, g, [1e-3, 1e-3, 1e-3], t0, 2.0, dt),
             "snap": lcs.lcs_advect_snapshots(fr, g, t0, dt, [40, N])}
        r["early"] = lcs.lcs_ftle_early(fr, g, t0, dt, N, r["snap"][0][1], r["snap"][2])
        lcs.lcs_sync_status()
        plan.close()
        out[name] = r
    for key in out["soa"]:
        for u, v in zip(out["soa"][key], out["tpair"][key]):
            assert torch.equal(u, v), key
    assert int((out["soa"]["snap"][1][1] != 0).sum()) > 0      # some tracers left the box
