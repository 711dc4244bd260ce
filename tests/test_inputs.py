"""Checks of the seeded synthetic inputs (not of the method)."""
import math

import numpy as np

from paper_2209_13775_amd import inputs


def test_random_fourier_properties():
    n, nf, dtf, tau, kmax = 32, 33, 0.125, 2.0, 8
    fs = inputs.random_fourier_frames(n=n, n_frames=nf, dt_frame=dtf, kmax=kmax, tau=tau, seed=1)
    u = np.stack(fs.u).astype(np.float64)            # (3, F, z, y, x)
    # RMS speed 1 over all frames
    assert abs(math.sqrt((u ** 2).sum(0).mean()) - 1.0) < 1e-6
    k = np.fft.fftfreq(n, d=1.0 / n)
    kr = np.fft.rfftfreq(n, d=1.0 / n)
    KZ, KY, KX = np.meshgrid(k, k, kr, indexing="ij")
    spec = [np.fft.rfftn(u[c], axes=(1, 2, 3)) for c in range(3)]
    # solenoidal: k . u_hat = 0 (to FP32 rounding of the stored frames)
    div = KX * spec[0] + KY * spec[1] + KZ * spec[2]
    mag = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2) * np.sqrt(sum(np.abs(s) ** 2 for s in spec))
    assert np.abs(div).max() <= 1e-5 * mag.max()
    # band limit
    K = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    e = sum(np.abs(s) ** 2 for s in spec).mean(0)
    assert e[K > kmax + 0.5].max() <= 1e-8 * e.max()
    # shell-averaged spectrum slope -5/3
    w = np.where(KX == 0, 1.0, 2.0)
    shells = np.arange(2, kmax + 1)
    E = np.array([(e * w)[(K >= s - 0.5) & (K < s + 0.5)].sum() for s in shells])
    slope = np.polyfit(np.log(shells), np.log(E), 1)[0]
    assert abs(slope + 5.0 / 3.0) < 0.25, slope
    # lag-1 time autocorrelation of the OU amplitudes ~ exp(-dt/tau)
    a = u.reshape(3, nf, -1)
    r = np.mean([np.corrcoef(a[c, :-1].ravel(), a[c, 1:].ravel())[0, 1] for c in range(3)])
    assert abs(r - math.exp(-dtf / tau)) < 0.02, r


def test_t0_windows_draw():
    w = inputs.t0_windows(64, seed=0)
    assert w.shape == (64, 2)
    assert np.all((w[:, 0] >= 0) & (w[:, 0] <= 10))
    assert set(np.unique(w[:, 1])) <= {5.0, 7.5, 10.0, 12.5, 15.0}
    assert (w[:, 0] + w[:, 1]).max() < 25.0
    assert np.array_equal(w, inputs.t0_windows(64, seed=0))


def test_double_gyre_is_divergence_free_and_walls():
    x = np.linspace(0, 2, 41)[None, :]
    y = np.linspace(0, 1, 21)[:, None]
    h = 1e-6
    for t in [0.0, 1.3, 7.7]:
        u, v = inputs.double_gyre_velocity(x, y, t)
        du = (inputs.double_gyre_velocity(x + h, y, t)[0] - inputs.double_gyre_velocity(x - h, y, t)[0]) / (2 * h)
        dv = (inputs.double_gyre_velocity(x, y + h, t)[1] - inputs.double_gyre_velocity(x, y - h, t)[1]) / (2 * h)
        assert np.abs(du + dv).max() < 1e-7
        assert np.abs(v[0]).max() < 1e-15 and np.abs(v[-1]).max() < 1e-15   # y walls
        assert np.abs(u[:, 0]).max() < 1e-15 and np.abs(u[:, -1]).max() < 1e-12  # x walls
