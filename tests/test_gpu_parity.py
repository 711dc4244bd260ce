"""GPU parity: the HIP path (called through the C ABI) against the FP64 oracle.

Tolerances (written here, derived in the parity helper module):
  positions  mean and p99 of |x_gpu - x_oracle| <= 1e-5 x domain length
  FTLE       |sigma_gpu - sigma_oracle| <= 1e-3 on seeds with clean stencils
  flags, cell index   bit-exact (cell recomputed from the GPU's positions:
             all tracers; against the oracle's own run: unambiguous tracers)
  C from identical positions: bit-exact; lambda_max from identical C: 1e-12
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


def _np(t):
    return t.detach().cpu().numpy()


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_gpu(lcs, fs, g, t0, T, dt, frames=None):
    frames = frames or lcs.DeviceFrames(fs)
    xf, cell, flags = lcs.lcs_advect(frames, g, t0, T, dt)
    C, sfl = lcs.lcs_cg_tensor(g, xf, flags)
    lam, sig = lcs.lcs_ftle(g.dim, C, T)
    lcs.lcs_sync_status()
    return dict(xf=_np(xf), cell=_np(cell), flags=_np(flags), C=_np(C), sflags=_np(sfl),
                lam=_np(lam), ftle=_np(sig))


def run_oracle(orc, fs, g, t0, T, dt):
    vel = orc.Velocity(fs)
    xf, cell, flags, margin = orc.advect_seeds(vel, g, t0, T, dt, margin=True)
    C, sfl = orc.cg_tensor(g, xf, flags)
    lam, sig = orc.ftle(g.dim, C, T)
    return dict(vel=vel, xf=xf, cell=cell, flags=flags, margin=margin, C=C, sflags=sfl, lam=lam,
                ftle=sig)


def compare_full(orc, fs, g, gpu, ref, what, pos_tol=None):
    L = parity.domain_length(fs)
    tol = pos_tol if pos_tol is not None else parity.POS_TOL_FRAC * L
    amb_tol = parity.POS_TOL_FRAC * L
    # flags: bit-exact on unambiguous tracers
    unamb = ref["margin"] > amb_tol
    bad_flags = np.nonzero((gpu["flags"] != ref["flags"]) & unamb)[0]
    assert bad_flags.size == 0, f"{what}: flags differ at {bad_flags[:10]}"
    # positions, over tracers whose flags agree
    agree = gpu["flags"] == ref["flags"]
    st = parity.position_stats(gpu["xf"], ref["xf"], tol, agree)
    parity.assert_positions(st, tol, what)
    # cell index recomputed by the oracle from the GPU's positions: all tracers
    cell_from_gpu = orc.cell_index(ref["vel"], gpu["xf"].astype(np.float64))
    np.testing.assert_array_equal(gpu["cell"], cell_from_gpu)
    # against the oracle's own run: unambiguous tracers
    ok = agree & unamb & ~parity.near_cell_face(fs, ref["xf"], amb_tol)
    diff = np.nonzero((gpu["cell"] != ref["cell"]) & ok)[0]
    assert diff.size == 0, f"{what}: cell index differs at {diff[:10]}"
    # FTLE on clean stencils
    clean = (gpu["sflags"] == 0) & (ref["sflags"] == 0)
    np.testing.assert_array_equal(gpu["sflags"][unamb_stencil(g, unamb)],
                                  ref["sflags"][unamb_stencil(g, unamb)])
    err = np.abs(gpu["ftle"][clean] - ref["ftle"][clean])
    emax = float(err.max()) if err.size else 0.0
    _say(f"{what}: FTLE max err {emax:.3e} over {clean.sum()} seeds; "
         f"ambiguous for flags: {(~unamb).sum()}")
    assert emax <= parity.FTLE_TOL


def unamb_stencil(g, unamb):
    """Seeds whose whole difference stencil consists of unambiguous tracers."""
    idx = np.arange(g.count)
    _, im, ip = parity.neighbour_indices(g, idx)
    ok = unamb.copy()
    for b in range(g.dim):
        ok &= unamb[im[b]] & unamb[ip[b]]
    return ok


def test_double_gyre_full_size(orc, lcs):
    """2D double gyre 201x101 FP64-sampled frames, 256x128 seeds, T=10, dt=0.05."""
    _say("case: double gyre 201x101, seeds 256x128, T=10")
    fs = inputs.double_gyre_frames()
    g = inputs.linspace_seeds(2, (256, 128), (0.0, 0.0), (2.0, 1.0))
    gpu = run_gpu(lcs, fs, g, 0.0, 10.0, 0.05)
    ref = run_oracle(orc, fs, g, 0.0, 10.0, 0.05)
    compare_full(orc, fs, g, gpu, ref, "double gyre")


@pytest.mark.parametrize("n", [(37, 23), (2, 2), (65, 3)])
def test_double_gyre_ragged(orc, lcs, n):
    _say(f"case: double gyre ragged seeds {n}")
    fs = inputs.double_gyre_frames(nx=51, ny=26, n_frames=11)
    g = inputs.linspace_seeds(2, n, (0.05, 0.05), (1.95, 0.95))
    gpu = run_gpu(lcs, fs, g, 1.0, 6.0, 0.05)
    ref = run_oracle(orc, fs, g, 1.0, 6.0, 0.05)
    compare_full(orc, fs, g, gpu, ref, f"double gyre {n}")


def test_double_gyre_backward(orc, lcs):
    _say("case: double gyre backward T=-7")
    fs = inputs.double_gyre_frames(nx=101, ny=51, n_frames=21)
    g = inputs.linspace_seeds(2, (70, 33), (0.0, 0.0), (2.0, 1.0))
    gpu = run_gpu(lcs, fs, g, 15.0, -7.0, -0.05)
    ref = run_oracle(orc, fs, g, 15.0, -7.0, -0.05)
    compare_full(orc, fs, g, gpu, ref, "double gyre backward")


def test_taylor_green_periodic_2d(orc, lcs):
    _say("case: periodic Taylor-Green 2D")
    fs = inputs.taylor_green_frames(n=48, n_frames=9, dt_frame=0.5)
    L = 2 * math.pi
    g = inputs.periodic_seeds(2, (90, 41), (L, L))
    gpu = run_gpu(lcs, fs, g, 0.5, 3.0, 0.02)
    ref = run_oracle(orc, fs, g, 0.5, 3.0, 0.02)
    compare_full(orc, fs, g, gpu, ref, "taylor-green")
    assert np.abs(gpu["xf"]).max() > L     # positions are unwrapped


@pytest.mark.parametrize("n_seed", [(13, 11, 9), (24, 24, 24)])
def test_abc_small_3d(orc, lcs, n_seed):
    _say(f"case: ABC 24^3 grid seeds {n_seed}")
    fs = inputs.abc_frames(n=24, n_frames=9, dt_frame=0.5)
    L = 2 * math.pi
    g = inputs.periodic_seeds(3, n_seed, (L, L, L))
    gpu = run_gpu(lcs, fs, g, 0.25, 2.0, 0.02)
    ref = run_oracle(orc, fs, g, 0.25, 2.0, 0.02)
    compare_full(orc, fs, g, gpu, ref, f"abc {n_seed}")


def test_abc_full_size_sampled(orc, lcs, torch):
    """ABC 128^3, 33 frames, 256^3 seeds, T=8, dt=0.02 -- the benchmark launch;
    the oracle checks a deterministic sample of seeds and their stencils."""
    _say("case: ABC 128^3 full size, 256^3 seeds, T=8 (sampled)")
    fs = inputs.abc_frames(n=128, n_frames=33, dt_frame=0.5)
    L = 2 * math.pi
    g = inputs.periodic_seeds(3, (256, 256, 256), (L, L, L))
    frames = lcs.DeviceFrames(fs)
    xf, cell, flags = lcs.lcs_advect(frames, g, 0.0, 8.0, 0.02)
    lam, sig, sfl = lcs.lcs_cg_ftle(g, xf, 8.0, flags=flags)
    lcs.lcs_sync_status()
    idx = parity.sample_seeds(g, 384, seed=2)
    it = torch.from_numpy(idx).to(xf.device)
    gx = _np(xf[:, it])
    gcell, gflags, gsig = _np(cell[it]), _np(flags[it]), _np(sig[it])
    del xf, cell, flags, lam, sig, sfl, frames
    torch.cuda.empty_cache()
    vel = orc.Velocity(fs.astype(np.float32))
    ref = parity.oracle_sampled_ftle(orc, vel, g, idx, 0.0, 8.0, 0.02)
    assert not gflags.any() and not ref["flags"].any()
    tol = parity.POS_TOL_FRAC * L
    err = np.abs(gsig - ref["ftle"])
    _say(f"abc full: FTLE max err {err.max():.3e}, FTLE mean {ref['ftle'].mean():.3f} "
         f"max {ref['ftle'].max():.3f}")
    st = parity.position_stats(gx, ref["xf"], tol)
    parity.assert_positions(st, tol, "abc full size (sampled)")
    np.testing.assert_array_equal(gcell, orc.cell_index(vel, gx.astype(np.float64)))
    assert err.max() <= parity.FTLE_TOL


def test_uniform_stream_exit_flags(orc, lcs, torch):
    _say("case: uniform stream exit")
    c = np.array([0.37, -0.21])
    fs = inputs.uniform_frames(c, dim=2, n=9, lo=0.0, hi=1.0)
    g = inputs.linspace_seeds(2, (40, 40), (0.013, 0.011), (0.987, 0.989))
    gpu = run_gpu(lcs, fs, g, 0.0, 4.0, 0.05)
    ref = run_oracle(orc, fs, g, 0.0, 4.0, 0.05)
    assert (ref["flags"] == 1).sum() > 100
    compare_full(orc, fs, g, gpu, ref, "uniform exit")


def test_nonfinite_frame_value(orc, lcs):
    _say("case: NaN in a frame node")
    fs = inputs.double_gyre_frames(nx=51, ny=26, n_frames=11)
    fs.u[1][3, 12, 20] = np.nan
    g = inputs.linspace_seeds(2, (64, 32), (0.02, 0.02), (1.98, 0.98))
    gpu = run_gpu(lcs, fs, g, 0.0, 6.0, 0.05)
    ref = run_oracle(orc, fs, g, 0.0, 6.0, 0.05)
    assert (ref["flags"] == 2).sum() > 0
    compare_full(orc, fs, g, gpu, ref, "nan frame")


def test_points_with_own_t0_and_time_out(orc, lcs, torch):
    _say("case: advect_points with per-point t0")
    fs = inputs.double_gyre_frames(nx=101, ny=51, n_frames=21)
    rng = np.random.default_rng(12)
    m = 3001
    x0 = np.stack([rng.uniform(0.01, 1.99, m), rng.uniform(0.01, 0.99, m)]).astype(np.float32)
    t0 = rng.uniform(0.0, 20.0, m)      # some intervals leave the frame span
    t0[:5] = [0.0, 15.0, 15.0000001, 20.0, 14.99]
    frames = lcs.DeviceFrames(fs)
    dx = torch.from_numpy(x0).cuda()
    dt0 = torch.from_numpy(t0).cuda()
    xf, cell, flags = lcs.lcs_advect_points(frames, dx, dt0, 5.0, 0.05)
    lcs.lcs_sync_status()
    vel = orc.Velocity(fs)
    rx, rcell, rflags, rmargin = orc.advect_points(vel, x0.astype(np.float64), t0, 5.0, 0.05,
                                                   margin=True)
    gpu = dict(xf=_np(xf), cell=_np(cell), flags=_np(flags))
    assert (rflags == 8).sum() > 100
    unamb = rmargin > 2e-5
    np.testing.assert_array_equal(gpu["flags"][unamb], rflags[unamb])
    np.testing.assert_array_equal(gpu["flags"] == 8, rflags == 8)
    st = parity.position_stats(gpu["xf"], rx, 2e-5, gpu["flags"] == rflags)
    parity.assert_positions(st, 2e-5, "advect_points")
    np.testing.assert_array_equal(gpu["cell"], orc.cell_index(vel, gpu["xf"].astype(np.float64)))


def test_cg_bitexact_on_identical_positions(orc, lcs, torch):
    _say("case: C from identical positions")
    for g in [inputs.linspace_seeds(2, (131, 67), (0.0, 0.0), (2.0, 1.0)),
              inputs.SeedGrid(3, (70, 9, 5), (0.0, 0.0, 0.0), (0.1, 0.2, 0.3), (True, False, True))]:
        rng = np.random.default_rng(g.dim)
        ns = g.count
        xf = (rng.standard_normal((g.dim, ns)) * 3.0).astype(np.float32)
        flags = (rng.random(ns) < 0.01).astype(np.uint8)
        dxf = torch.from_numpy(xf).cuda()
        dfl = torch.from_numpy(flags).cuda()
        C, sfl = lcs.lcs_cg_tensor(g, dxf, dfl)
        lam, sig = lcs.lcs_ftle(g.dim, C, 2.5)
        lam2, sig2, sfl2 = lcs.lcs_cg_ftle(g, dxf, 2.5, flags=dfl)
        lcs.lcs_sync_status()
        rC, rs = orc.cg_tensor(g, xf.astype(np.float64), flags)
        np.testing.assert_array_equal(_np(C), rC)
        np.testing.assert_array_equal(_np(sfl), rs)
        rl, rsig = orc.ftle(g.dim, rC, 2.5)
        np.testing.assert_allclose(_np(lam), rl, rtol=1e-12, atol=0)
        np.testing.assert_allclose(_np(sig), rsig, rtol=0, atol=1e-12)
        # fused path equals the two-kernel path
        np.testing.assert_array_equal(_np(lam2), _np(lam))
        np.testing.assert_array_equal(_np(sig2), _np(sig))
        np.testing.assert_array_equal(_np(sfl2), _np(sfl))


def test_lambda_max_ill_conditioned(orc, lcs, torch):
    _say("case: lambda_max on ill-conditioned SPD matrices")
    rng = np.random.default_rng(77)
    mats = []
    for k in range(4096):
        Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        kind = k % 3
        if kind == 0:
            ev = np.exp(rng.uniform(-8, 16, 3))
        elif kind == 1:
            top = math.exp(rng.uniform(0, 10))
            ev = np.array([top, top * (1 + 1e-10), 1e-6])
        else:
            ev = np.full(3, math.exp(rng.uniform(-1, 1)))
        M = Q @ np.diag(ev) @ Q.T
        mats.append(0.5 * (M + M.T))
    packed = np.stack([[M[0, 0], M[0, 1], M[0, 2], M[1, 1], M[1, 2], M[2, 2]] for M in mats], axis=1)
    lam, _ = lcs.lcs_ftle(3, torch.from_numpy(np.ascontiguousarray(packed)).cuda(), 1.0)
    lcs.lcs_sync_status()
    rl, _ = orc.ftle(3, packed, 1.0)
    np.testing.assert_allclose(_np(lam), rl, rtol=1e-12)


def test_repeatable_bitwise(lcs):
    _say("case: repeated runs are bit-identical")
    fs = inputs.abc_frames(n=32, n_frames=9)
    L = 2 * math.pi
    g = inputs.periodic_seeds(3, (40, 40, 40), (L, L, L))
    frames = lcs.DeviceFrames(fs)
    a = lcs.lcs_advect(frames, g, 0.0, 2.0, 0.02)
    b = lcs.lcs_advect(frames, g, 0.0, 2.0, 0.02)
    lcs.lcs_sync_status()
    for u, v in zip(a, b):
        assert bool((u == v).all())
