"""GPU parity of the Adams-Bashforth flow map (lcs_advect_ab, orders 2-4 with
RK4 start-up) against the FP64 oracle, through the C ABI.  Same bars as the
RK4 path (positions 1e-5 L mean and p99, FTLE 1e-3 on clean stencils, flags
and cell index bit-exact where unambiguous)."""
import math
import sys

import numpy as np
import pytest

from paper_2209_13775_amd import inputs
from tests import parity
from tests.test_gpu_parity import compare_full

pytestmark = pytest.mark.gpu

AB = {2: [3 / 2, -1 / 2], 3: [23 / 12, -16 / 12, 5 / 12], 4: [55 / 24, -59 / 24, 37 / 24, -9 / 24]}


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


def run_gpu(lcs, fs, g, t0, T, dt, order):
    frames = lcs.DeviceFrames(fs)
    xf, cell, flags = lcs.lcs_advect_ab(frames, g, t0, T, dt, order=order)
    C, sfl = lcs.lcs_cg_tensor(g, xf, flags)
    lam, sig = lcs.lcs_ftle(g.dim, C, T)
    lcs.lcs_sync_status()
    return dict(xf=_np(xf), cell=_np(cell), flags=_np(flags), C=_np(C), sflags=_np(sfl),
                lam=_np(lam), ftle=_np(sig))


def run_oracle(orc, fs, g, t0, T, dt, order):
    vel = orc.Velocity(fs)
    xf, cell, flags, margin = orc.advect_seeds_ab(vel, g, t0, T, dt, order=order, margin=True)
    C, sfl = orc.cg_tensor(g, xf, flags)
    lam, sig = orc.ftle(g.dim, C, T)
    return dict(vel=vel, xf=xf, cell=cell, flags=flags, margin=margin, C=C, sflags=sfl, lam=lam,
                ftle=sig)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_double_gyre_full_size(orc, lcs, order):
    _say(f"case: AB{order} double gyre 201x101, seeds 256x128, T=10")
    fs = inputs.double_gyre_frames()
    g = inputs.linspace_seeds(2, (256, 128), (0.0, 0.0), (2.0, 1.0))
    gpu = run_gpu(lcs, fs, g, 0.0, 10.0, 0.05, order)
    ref = run_oracle(orc, fs, g, 0.0, 10.0, 0.05, order)
    compare_full(orc, fs, g, gpu, ref, f"AB{order} double gyre")


def test_abc_small_backward(orc, lcs):
    _say("case: AB4 ABC 32^3, seeds 40x36x28, backward")
    fs = inputs.abc_frames(n=32, n_frames=9, dt_frame=0.5)
    L = 2 * math.pi
    g = inputs.periodic_seeds(3, (40, 36, 28), (L, L, L))
    gpu = run_gpu(lcs, fs, g, 4.0, -3.0, -0.02, 4)
    ref = run_oracle(orc, fs, g, 4.0, -3.0, -0.02, 4)
    compare_full(orc, fs, g, gpu, ref, "AB4 ABC backward")


def test_abc_full_size_sampled(orc, lcs, torch):
    """The benchmark field and seeds (ABC 128^3, 256^3 seeds, T = 8, dt = 0.02)
    with AB4, checked at sampled seeds."""
    _say("case: AB4 ABC 128^3 full size (sampled)")
    fs = inputs.abc_frames(n=128, n_frames=33, dt_frame=0.5)
    L = 2 * math.pi
    g = inputs.periodic_seeds(3, (256, 256, 256), (L, L, L))
    frames = lcs.DeviceFrames(fs)
    xf, cell, flags = lcs.lcs_advect_ab(frames, g, 0.0, 8.0, 0.02, order=4)
    lam, sig, sfl = lcs.lcs_cg_ftle(g, xf, 8.0, flags=flags)
    lcs.lcs_sync_status()
    idx = parity.sample_seeds(g, 256, seed=3)
    it = torch.from_numpy(idx).to(xf.device)
    gx, gcell, gflags, gsig = _np(xf[:, it]), _np(cell[it]), _np(flags[it]), _np(sig[it])
    del xf, cell, flags, lam, sig, sfl, frames
    torch.cuda.empty_cache()
    vel = orc.Velocity(fs.astype(np.float32))
    c, im, ip = parity.neighbour_indices(g, idx)
    allidx = np.unique(np.concatenate([idx] + im + ip))
    xo, co, fo = orc.advect_seeds_ab(vel, g, 0.0, 8.0, 0.02, order=4, idx=allidx)
    pos = {int(k): p for p, k in enumerate(allidx)}
    Cm = np.empty((6, idx.size))
    for q, s in enumerate(idx):
        Cm[:, q] = orc.cg_point(g, c[:, q], xo[:, pos[int(s)]],
                                [xo[:, pos[int(im[b][q])]] for b in range(3)],
                                [xo[:, pos[int(ip[b][q])]] for b in range(3)])
    _, osig = orc.ftle(3, Cm, 8.0)
    sel = np.array([pos[int(s)] for s in idx])
    assert not gflags.any() and not fo.any()
    tol = parity.POS_TOL_FRAC * L
    st = parity.position_stats(gx, xo[:, sel], tol)
    parity.assert_positions(st, tol, "AB4 abc full size (sampled)")
    np.testing.assert_array_equal(gcell, orc.cell_index(vel, gx.astype(np.float64)))
    err = np.abs(gsig - osig)
    _say(f"AB4 abc full: FTLE max err {err.max():.3e}")
    assert err.max() <= parity.FTLE_TOL


def test_uniform_stream_exit_flags(orc, lcs):
    c = np.array([0.37, -0.21])
    fs = inputs.uniform_frames(c, dim=2, n=9, lo=0.0, hi=1.0)
    g = inputs.linspace_seeds(2, (40, 40), (0.013, 0.011), (0.987, 0.989))
    for order in (2, 4):
        gpu = run_gpu(lcs, fs, g, 0.0, 4.0, 0.05, order)
        ref = run_oracle(orc, fs, g, 0.0, 4.0, 0.05, order)
        assert (ref["flags"] == 1).sum() > 100
        compare_full(orc, fs, g, gpu, ref, f"AB{order} uniform exit")


def test_nonfinite_frame_value(orc, lcs):
    fs = inputs.double_gyre_frames(nx=51, ny=26, n_frames=11)
    fs.u[1][3, 12, 20] = np.nan
    g = inputs.linspace_seeds(2, (64, 32), (0.02, 0.02), (1.98, 0.98))
    gpu = run_gpu(lcs, fs, g, 0.0, 8.0, 0.05, 4)
    ref = run_oracle(orc, fs, g, 0.0, 8.0, 0.05, 4)
    assert (ref["flags"] == 2).sum() > 0
    compare_full(orc, fs, g, gpu, ref, "AB4 NaN node")


def test_short_runs_match_rk4(lcs, torch):
    """Fewer steps than the order: the start-up RK4 steps alone."""
    fs = inputs.double_gyre_frames(nx=51, ny=26, n_frames=11)
    g = inputs.linspace_seeds(2, (64, 32), (0.02, 0.02), (1.98, 0.98))
    frames = lcs.DeviceFrames(fs)
    for order in (2, 3, 4):
        for N in range(1, order):
            a, _, fa = lcs.lcs_advect_ab(frames, g, 0.0, 0.05 * N, 0.05, order=order)
            b, _, fb = lcs.lcs_advect(frames, g, 0.0, 0.05 * N, 0.05)
            lcs.lcs_sync_status()
            assert torch.equal(fa, fb)
            assert (a - b).abs().max().item() <= 1e-6


def test_linear_saddle_recurrence(lcs):
    lam, dt, T = 0.5, 0.05, 2.0
    N = int(round(T / dt))
    fs = inputs.saddle_frames(lam=lam, dim=2)
    g = inputs.linspace_seeds(2, (33, 29), (-0.5, -0.5), (0.5, 0.5))

    def growth(z, order):
        y = [1.0]
        R = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
        for n in range(N):
            y.append(y[-1] * R if n < order - 1 else
                     y[-1] + z * sum(AB[order][j] * y[-1 - j] for j in range(order)))
        return y[-1]

    for order in (2, 3, 4):
        gpu = run_gpu(lcs, fs, g, 0.0, T, dt, order)
        gx, gy = growth(lam * dt, order), growth(-lam * dt, order)
        np.testing.assert_allclose(gpu["ftle"], math.log(max(abs(gx), abs(gy))) / T, atol=1e-5)


@pytest.mark.parametrize("order,seg", [(2, 7), (3, 50), (4, 1), (4, 33)])
def test_rebundled_equals_single_launch_2d(lcs, torch, order, seg):
    """Re-bundled AB (history carried with the tracer through the sorts) is
    bit-identical to the single-launch AB, with exits and a NaN node."""
    fs = inputs.double_gyre_frames(nx=51, ny=26, n_frames=11)
    fs.u[0][4, 10, 30] = np.nan
    g = inputs.linspace_seeds(2, (97, 45), (0.0, 0.0), (2.0, 1.0))
    frames = lcs.DeviceFrames(fs)
    a = lcs.lcs_advect_ab(frames, g, 0.5, 7.0, 0.05, order=order)
    b = lcs.lcs_advect_ab_sorted(frames, g, 0.5, 7.0, 0.05, order=order, segment_steps=seg)
    lcs.lcs_sync_status()
    assert (a[2] == 2).sum().item() > 0
    for u, v in zip(a, b):
        assert torch.equal(u, v)


def test_rebundled_equals_single_launch_abc_full(lcs, torch):
    fs = inputs.abc_frames(n=128, n_frames=33, dt_frame=0.5)
    L = 2 * math.pi
    g = inputs.periodic_seeds(3, (256, 256, 256), (L, L, L))
    frames = lcs.DeviceFrames(fs)
    a = lcs.lcs_advect_ab(frames, g, 8.0, -8.0, -0.02, order=4, want_cell=False)
    b = lcs.lcs_advect_ab_sorted(frames, g, 8.0, -8.0, -0.02, order=4, segment_steps=50,
                                 want_cell=False)
    lcs.lcs_sync_status()
    assert torch.equal(a[0], b[0]) and torch.equal(a[2], b[2])
