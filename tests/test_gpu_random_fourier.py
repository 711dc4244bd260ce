"""GPU parity on the divergence-free random-Fourier field: 256^3 periodic grid,
65 FP32 frames (t = 0.125 f), 512x512x256 seeds, forward (T = +4) and backward
(T = -4) FTLE from t0 = 4 with dt = +-0.01 -- full size on the GPU, checked
against the FP64 oracle on a deterministic sample of seeds and their stencils;
the benchmark's launch configuration (time-paired frames, re-bundled every 100
steps) gives the same bits as the single launch at this size.
"""
import math
import sys

import numpy as np
import pytest

from paper_2209_13775_amd import inputs
from tests import parity

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def field():
    import torch
    assert torch.cuda.is_available()
    _say("generating the 256^3 x 65 random-Fourier field on the GPU")
    fs = inputs.random_fourier_frames(n=256, n_frames=65, dt_frame=0.125, device="cuda")
    torch.cuda.synchronize()
    return fs


@pytest.mark.parametrize("T", [4.0, -4.0])
def test_random_fourier_full_size_sampled(orc, field, T):
    import torch
    from paper_2209_13775_amd import lcs
    L = 2 * math.pi
    dt = 0.01 if T > 0 else -0.01
    g = inputs.SeedGrid(3, (512, 512, 256), (0.0, 0.0, 0.0), (L / 512, L / 512, L / 256),
                        (True, True, True))
    _say(f"case: random Fourier 256^3, seeds 512x512x256, t0=4, T={T}")
    frames = lcs.DeviceFrames(field, tensors=field.u)
    xf, cell, flags = lcs.lcs_advect(frames, g, 4.0, T, dt)
    # the benchmark's launch: time-paired frames, re-bundled every 100 steps --
    # the same bits as the single launch on structure-of-arrays frames
    tpair = lcs.lcs_frames_interleave(frames, "tpair")
    xs, cs, fs_ = lcs.lcs_advect_sorted(tpair, g, 4.0, T, dt, 100)
    lcs.lcs_sync_status()
    assert torch.equal(xs, xf) and torch.equal(cs, cell) and torch.equal(fs_, flags)
    del tpair, xs, cs, fs_
    lam, sig, sfl = lcs.lcs_cg_ftle(g, xf, T, flags=flags)
    lcs.lcs_sync_status()
    idx = parity.sample_seeds(g, 160, seed=11)
    it = torch.from_numpy(idx).cuda()
    gx = xf[:, it].cpu().numpy()
    gcell, gflags, gsig = cell[it].cpu().numpy(), flags[it].cpu().numpy(), sig[it].cpu().numpy()
    gsig_all = sig.cpu().numpy()
    del xf, cell, flags, lam, sig, sfl
    host = inputs.FrameSet(3, field.n, field.origin, field.spacing, field.periodic,
                           field.t_first, field.dt_frame, [u.cpu().numpy() for u in field.u])
    vel = orc.Velocity(host, keep_f32=True)
    ref = parity.oracle_sampled_ftle(orc, vel, g, idx, 4.0, T, dt)
    assert not gflags.any() and not ref["flags"].any()
    tol = parity.POS_TOL_FRAC * L
    err = np.abs(gsig - ref["ftle"])
    st = parity.position_stats(gx, ref["xf"], tol)
    _say(f"random Fourier T={T}: FTLE mean {gsig_all.mean():.3f} max {gsig_all.max():.3f}; "
         f"FTLE err max {err.max():.3e}; positions mean {st.mean:.3e} p99 {st.p99:.3e} "
         f"max {st.max:.3e} ({st.n_over}/{st.n} above {tol:.1e})")
    np.testing.assert_array_equal(gcell, orc.cell_index(vel, gx.astype(np.float64)))
    assert err.max() <= parity.FTLE_TOL
    parity.assert_positions(st, tol, f"random Fourier T={T}")
