"""Pins of the oracle's space-time interpolation and cell location.

The interpolant (multilinear in space inside each frame, linear in time
between the bracketing frames; Sec. 2 Interpolator and Sec. 3.2) is, as a
whole, multilinear interpolation over the product grid (t, [z,] y, x).  SciPy's
RegularGridInterpolator(method="linear") is an independent implementation of
exactly that, so it pins the oracle on random data.  Further pins: exact
reproduction of multilinear polynomials and of node values, the periodic wrap,
and the cell index against a search with numpy.searchsorted.
"""
import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

from paper_2209_13775_amd import inputs


def _rgi(fs, comp, periodic_pad=False):
    """RegularGridInterpolator over (t, [z,] y, x) for one component."""
    dim = fs.dim
    data = fs.u[comp]
    axes = []
    for a in reversed(range(dim)):          # array axes are (.., y, x)
        n = fs.n[a]
        ax = fs.origin[a] + np.arange(n) * fs.spacing[a]
        axes.append(ax)
    if periodic_pad:
        # append node 0 again at the end of every periodic axis (x = L)
        for k, a in enumerate(reversed(range(dim))):
            if fs.periodic[a]:
                ax_i = 1 + k
                first = np.take(data, [0], axis=ax_i)
                data = np.concatenate([data, first], axis=ax_i)
                axes[k] = np.append(axes[k], fs.origin[a] + fs.n[a] * fs.spacing[a])
    t = fs.t_first + np.arange(fs.n_frames) * fs.dt_frame
    return RegularGridInterpolator([t] + axes, data, method="linear", bounds_error=True)


@pytest.mark.parametrize("dim", [2, 3])
def test_matches_regular_grid_interpolator(orc, dim):
    n = (5, 4, 3)[:dim]
    fs = inputs.random_frames(dim, n, n_frames=4, seed=11 + dim,
                              origin=[-1.0, 0.5, 2.0][:dim], spacing=[0.3, 0.7, 0.25][:dim],
                              t_first=1.5, dt_frame=0.4)
    vel = orc.Velocity(fs)
    rng = np.random.default_rng(5)
    m = 4000
    lo = np.array(fs.origin[:dim])
    hi = lo + (np.array(fs.n[:dim]) - 1) * np.array(fs.spacing[:dim])
    x = lo[:, None] + rng.random((dim, m)) * (hi - lo)[:, None]
    # include the faces and the corners of the domain
    x[:, :8] = lo[:, None]
    x[:, 8:16] = hi[:, None]
    t = fs.t_first + rng.random(m) * (fs.n_frames - 1) * fs.dt_frame
    t[:5] = fs.t_first
    t[5:10] = fs.t_first + (fs.n_frames - 1) * fs.dt_frame
    got = orc.velocity_at(vel, x, t)
    pts = np.concatenate([t[:, None], x[::-1].T], axis=1)   # (t, [z,] y, x)
    for c in range(dim):
        ref = _rgi(fs, c)(pts)
        np.testing.assert_allclose(got[c], ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_periodic_wrap_matches_padded_interpolator(orc, dim):
    n = (6, 5, 4)[:dim]
    L = [2.0, 3.0, 1.5][:dim]
    fs = inputs.random_frames(dim, n, n_frames=3, seed=3, periodic=[True] * dim,
                              spacing=[L[a] / n[a] for a in range(dim)], dt_frame=0.5)
    vel = orc.Velocity(fs)
    rng = np.random.default_rng(9)
    m = 3000
    Lv = np.array(L)[:, None]
    x = (rng.random((dim, m)) * 7.0 - 3.0) * Lv          # spans several periods, negative too
    t = rng.random(m) * (fs.n_frames - 1) * fs.dt_frame
    got = orc.velocity_at(vel, x, t)
    xw = np.mod(x, Lv)
    pts = np.concatenate([t[:, None], xw[::-1].T], axis=1)
    for c in range(dim):
        ref = _rgi(fs, c, periodic_pad=True)(pts)
        np.testing.assert_allclose(got[c], ref, rtol=0, atol=1e-12)
    # a shift by a whole period is invisible
    shifted = orc.velocity_at(vel, x + 2 * Lv, t)
    np.testing.assert_allclose(shifted, got, rtol=0, atol=1e-12)


def test_multilinear_polynomials_are_reproduced(orc):
    # u = a + b x + c y + d z + e xy + f yz + g xz + h xyz, times (p + q t)
    co = np.array([0.3, -1.2, 0.7, 2.0, 0.5, -0.25, 1.5, -0.8])

    def poly(X, Y, Z, t):
        base = (co[0] + co[1] * X + co[2] * Y + co[3] * Z + co[4] * X * Y + co[5] * Y * Z
                + co[6] * X * Z + co[7] * X * Y * Z)
        return base * (1.0 + 0.3 * t), -base * (2.0 - 0.1 * t), base
    fs = inputs.sample_field(poly, 3, (4, 5, 6), (-1.0, 0.0, 0.5), (0.5, 0.25, 0.2),
                             (False,) * 3, 0.0, 0.75, 3)
    vel = orc.Velocity(fs)
    rng = np.random.default_rng(1)
    m = 2000
    lo = np.array([-1.0, 0.0, 0.5])
    hi = lo + np.array([3 * 0.5, 4 * 0.25, 5 * 0.2])
    x = lo[:, None] + rng.random((3, m)) * (hi - lo)[:, None]
    t = rng.random(m) * 1.5
    got = orc.velocity_at(vel, x, t)
    ref = poly(x[0], x[1], x[2], t)
    for c in range(3):
        np.testing.assert_allclose(got[c], ref[c], rtol=0, atol=1e-12)


def test_node_values_exact(orc):
    fs = inputs.random_frames(2, (5, 4), n_frames=3, seed=2, spacing=[0.5, 0.25], dt_frame=2.0)
    vel = orc.Velocity(fs)
    jj, ii = np.meshgrid(np.arange(4), np.arange(5), indexing="ij")
    x = np.stack([ii.ravel() * 0.5, jj.ravel() * 0.25])
    for f in range(3):
        got = orc.velocity_at(vel, x, f * 2.0)
        for c in range(2):
            assert np.array_equal(got[c], fs.u[c][f].ravel())


def test_cell_index_matches_search(orc):
    fs = inputs.random_frames(3, (7, 5, 4), n_frames=2, seed=0, origin=[0.5, -1.0, 0.0],
                              spacing=[0.2, 0.5, 1.0 / 3.0])
    vel = orc.Velocity(fs)
    rng = np.random.default_rng(4)
    lo = np.array(fs.origin)
    n = np.array(fs.n)
    h = np.array(fs.spacing)
    hi = lo + (n - 1) * h
    m = 5000
    x = lo[:, None] + rng.random((3, m)) * (hi - lo)[:, None]
    # points exactly on interior nodes belong to the higher cell, the last face to the last cell
    x[:, 0] = lo + 2 * h
    x[:, 1] = hi
    x[:, 2] = lo
    got = orc.cell_index(vel, x)
    idx = np.zeros(m, dtype=np.int64)
    stride = 1
    for a in range(3):
        nodes = lo[a] + np.arange(n[a]) * h[a]
        i = np.searchsorted(nodes, x[a], side="right") - 1
        i = np.clip(i, 0, n[a] - 2)
        idx += i * stride
        stride *= n[a]
    np.testing.assert_array_equal(got, idx)


def test_cell_index_periodic_and_nonfinite(orc):
    L = 2.0
    fs = inputs.random_frames(2, (8, 4), n_frames=2, seed=0, periodic=[True, True],
                              spacing=[L / 8, L / 4])
    vel = orc.Velocity(fs)
    x = np.array([[0.1, 0.1 + 3 * L, -0.1, -1e-20, np.nan],
                  [0.6, 0.6 - 2 * L, 1.9, 0.0, 0.2]])
    got = orc.cell_index(vel, x)
    # node spacing 0.25 (x) and 0.5 (y); -0.1 folds to 1.9 -> i=7; -1e-20 folds to node 0
    assert got[0] == 0 + 8 * 1
    assert got[1] == got[0]
    assert got[2] == 7 + 8 * 3
    assert got[3] == 0
    assert got[4] == -1
