"""Checks of the seeded synthetic inputs (not of the method)."""
import math

import numpy as np
import pytest

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


# ---------------------------------------------------------------------------
# Unstructured meshes
# ---------------------------------------------------------------------------


def _faces(cells):
    d1 = cells.shape[1]
    f = np.concatenate([np.delete(cells, i, axis=1) for i in range(d1)], axis=0)
    f = np.sort(f, axis=1)
    _, counts = np.unique(f, axis=0, return_counts=True)
    return counts


@pytest.mark.parametrize("dim,cells,shuffle", [(2, (6, 4), False), (2, (6, 4), True),
                                               (3, (4, 3, 2), False), (3, (4, 3, 2), True)])
def test_box_mesh_is_conforming_and_fills_the_box(dim, cells, shuffle):
    from paper_2209_13775_amd import inputs as I
    hi = (2.0, 1.0, 1.5)[:dim]
    m = I.box_mesh(dim, cells, (0.0,) * dim, hi, jitter=0.2, seed=2, shuffle=shuffle)
    meas = np.abs(I._signed_measure(m.nodes, m.cells)) / (2 if dim == 2 else 6)
    assert meas.min() > 0
    assert abs(meas.sum() - np.prod(hi)) < 1e-12
    counts = _faces(m.cells)
    assert counts.max() == 2                       # every face in at most two cells
    if dim == 2:
        want_boundary = 2 * (cells[0] + cells[1])
    else:
        nx, ny, nz = cells
        want_boundary = 4 * (nx * ny + ny * nz + nx * nz)
    assert (counts == 1).sum() == want_boundary
    # the walls stay exact
    for a in range(dim):
        x = m.nodes[:, a]
        assert x.min() == 0.0 and x.max() == hi[a]


def test_box_cells_field_is_divergence_free_and_wall_tangent():
    from paper_2209_13775_amd import inputs as I
    rng = np.random.default_rng(0)
    p = rng.uniform(0.1, math.pi - 0.1, (3, 500))
    t, h = 0.7, 1e-5
    div = 0.0
    for a in range(3):
        e = np.zeros((3, 1))
        e[a] = h
        div = div + (I.box_cells_velocity(*(p + e), t)[a] - I.box_cells_velocity(*(p - e), t)[a]) / (2 * h)
    assert np.abs(div).max() < 1e-8
    for a in range(3):
        for wall in (0.0, math.pi):
            q = p.copy()
            q[a] = wall
            assert np.abs(I.box_cells_velocity(*q, t)[a]).max() < 1e-15
