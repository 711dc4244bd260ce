"""Pins of the oracle's unstructured-mesh path (triangles / tetrahedra).

Each check compares the oracle with something other than itself:

* point location and piecewise-linear interpolation against SciPy's Qhull
  Delaunay triangulation (``find_simplex``) and ``LinearNDInterpolator`` run on
  the very same simplices;
* point location against brute force over every cell (NumPy linear solves);
* exact reproduction of node values and of fields linear in space (the P1
  interpolant is exact for them) and linear in time (linear time blending is);
* RK4 on a linear saddle field sampled on a jittered tetrahedron mesh: the
  discrete flow map is R(lambda dt)^N per axis with R the RK4 stability
  polynomial, so positions, FTLE = (N/T) ln max R(lambda_a dt) and det C are
  known in closed form;
* a uniform stream on a mesh leaves the box at a closed-form step.
"""
import math

import numpy as np
import pytest
from scipy.interpolate import LinearNDInterpolator
from scipy.spatial import Delaunay

import oracle
from paper_2209_13775_amd import inputs as I


def _delaunay_mesh(dim, n_pts, seed):
    rng = np.random.default_rng(seed)
    pts = rng.random((n_pts, dim))
    tri = Delaunay(pts)
    # drop numerically flat simplices Qhull may keep on the hull
    cells = tri.simplices.astype(np.int32)
    meas = np.abs(I._signed_measure(pts, cells))
    assert meas.min() > 1e-10
    return I.Mesh(dim, pts, cells), tri


@pytest.mark.parametrize("dim", [2, 3])
def test_locate_and_interpolate_match_scipy(dim):
    mesh, tri = _delaunay_mesh(dim, 400 if dim == 2 else 250, seed=dim)
    rng = np.random.default_rng(10 + dim)
    vals = rng.standard_normal((2, mesh.n_nodes, dim))
    mf = I.MeshFrames(mesh, 0.0, 2.0, vals)
    mv = oracle.MeshVelocity(mf)
    q = rng.random((dim, 4000)) * 1.2 - 0.1           # some points outside the hull
    cell, lam = mv.locate(q)
    want = tri.find_simplex(q.T, tol=0.0)
    interior = np.where(cell >= 0, np.nan_to_num(lam, nan=-1.0).min(axis=0), -1.0) > 1e-9
    inside = want >= 0
    # outside the hull: both say so (no query lies within rounding of the hull)
    assert np.array_equal(cell < 0, ~inside)
    # strictly interior points: the same simplex
    assert np.array_equal(cell[interior & inside], want[interior & inside])
    assert (interior & inside).sum() > 1000
    # interpolation in space (alpha = 0, 1) and time (alpha = 0.3)
    for t, a in [(0.0, 0.0), (2.0, 1.0), (0.6, 0.3)]:
        u, found = mv.velocity_at(q, t)
        ref = (1 - a) * LinearNDInterpolator(tri, vals[0])(q.T) + a * LinearNDInterpolator(tri, vals[1])(q.T)
        assert np.array_equal(found, inside)
        np.testing.assert_allclose(u[:, found].T, ref[found], rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("dim", [2, 3])
def test_locate_matches_brute_force(dim):
    cells_ax = (5, 4) if dim == 2 else (3, 3, 2)
    mesh = I.box_mesh(dim, cells_ax, (0.0,) * dim, (1.0, 0.7, 1.3)[:dim], jitter=0.2, seed=3,
                      shuffle=True)
    mf = I.MeshFrames(mesh, 0.0, 1.0, np.zeros((2, mesh.n_nodes, dim)))
    mv = oracle.MeshVelocity(mf)
    rng = np.random.default_rng(4)
    q = rng.random((dim, 3000)) * np.array([1.0, 0.7, 1.3][:dim])[:, None]
    cell, _ = mv.locate(q)
    # brute force: barycentric coordinates from a linear solve in every cell
    v = mesh.nodes[mesh.cells]                         # (nc, dim+1, dim)
    E = np.transpose(v[:, 1:, :] - v[:, :1, :], (0, 2, 1))   # columns v_i - v_0
    Einv = np.linalg.inv(E)
    D = q[None, :, :] - v[:, 0, :, None]               # (nc, dim, m)
    mu = np.einsum("cab,cbp->cap", Einv, D)
    lam = np.concatenate([1.0 - mu.sum(axis=1, keepdims=True), mu], axis=1)
    mins = lam.min(axis=1)                             # (nc, m)
    best = mins.argmax(axis=0)
    srt = np.sort(mins, axis=0)
    clear = (srt[-1] - srt[-2]) > 1e-9                 # no tie between two cells
    assert np.all(cell >= 0)
    assert np.array_equal(cell[clear], best[clear])
    assert clear.mean() > 0.95


@pytest.mark.parametrize("dim", [2, 3])
def test_nodes_and_linear_fields_reproduced(dim):
    cells_ax = (8, 6) if dim == 2 else (4, 4, 3)
    mesh = I.box_mesh(dim, cells_ax, (-1.0,) * dim, (1.0,) * dim, jitter=0.2, seed=5, shuffle=True)
    rng = np.random.default_rng(6)
    A = rng.standard_normal((dim, dim))
    b = rng.standard_normal(dim)
    c = rng.standard_normal(dim)

    def fn(*xt):
        x, t = np.stack(xt[:-1]), xt[-1]
        return tuple(b[k] + A[k] @ x + c[k] * t for k in range(dim))

    mf = I.mesh_sample(fn, mesh, 3, 0.0, 0.5)
    mv = oracle.MeshVelocity(mf)
    u, found = mv.velocity_at(mesh.nodes.T, 0.25)
    assert found.all()
    np.testing.assert_allclose(u, 0.5 * (mf.u[0] + mf.u[1]).T, rtol=1e-13, atol=1e-13)
    q = rng.uniform(-1, 1, (dim, 2000))
    for t in (0.0, 0.3, 0.75, 1.0):
        u, found = mv.velocity_at(q, t)
        assert found.all()
        np.testing.assert_allclose(u, np.stack(fn(*q, t)), rtol=1e-12, atol=1e-12)


def _R(z):
    return 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24


def test_rk4_closed_form_on_tet_mesh():
    lam = np.array([0.5, -0.3, -0.2])
    mesh = I.box_mesh(3, (6, 6, 6), (-3.0,) * 3, (3.0,) * 3, jitter=0.2, seed=7, shuffle=True)
    mf = I.mesh_sample(lambda x, y, z, t: (lam[0] * x, lam[1] * y, lam[2] * z), mesh, 2, 0.0, 10.0)
    mv = oracle.MeshVelocity(mf)
    g = I.linspace_seeds(3, (9, 8, 7), (-0.5, -0.5, -0.5), (0.5, 0.5, 0.5))
    T, dt = 2.0, 0.05
    N = int(round(T / dt))
    xf, cell, flags, mg, lm = mv.advect_seeds(g, 0.0, T, dt)
    assert not flags.any() and (cell >= 0).all()
    x0 = oracle.seed_points(g)
    want = x0 * (_R(lam * dt) ** N)[:, None]
    np.testing.assert_allclose(xf, want, rtol=1e-12, atol=1e-14)
    Cm, sfl = oracle.cg_tensor(g, xf, flags)
    lmax, sig = oracle.ftle(3, Cm, T)
    np.testing.assert_allclose(sig, (N / T) * math.log(_R(lam * dt).max()), rtol=1e-11)
    det = Cm[0] * (Cm[3] * Cm[5] - Cm[4] ** 2) - Cm[1] * (Cm[1] * Cm[5] - Cm[4] * Cm[2]) \
        + Cm[2] * (Cm[1] * Cm[4] - Cm[3] * Cm[2])
    np.testing.assert_allclose(det, np.prod(_R(lam * dt)) ** (2 * N), rtol=1e-10)


def test_linear_in_time_uniform_field_exact():
    a = np.array([0.3, -0.2])
    b = np.array([0.05, 0.1])
    mesh = I.box_mesh(2, (10, 10), (-5.0, -5.0), (5.0, 5.0), jitter=0.2, seed=8)
    mf = I.mesh_sample(lambda x, y, t: (a[0] + b[0] * t + 0 * x, a[1] + b[1] * t + 0 * y), mesh,
                       6, 0.0, 1.0)
    mv = oracle.MeshVelocity(mf)
    rng = np.random.default_rng(9)
    x0 = rng.uniform(-1, 1, (2, 200))
    t0, T, dt = 0.7, 3.2, 0.1
    xf, cell, flags, _, _ = mv.advect_points(x0, t0, T, dt)
    assert not flags.any()
    want = x0 + (a * T + b * ((t0 + T) ** 2 - t0 ** 2) / 2)[:, None]
    np.testing.assert_allclose(xf, want, rtol=1e-12, atol=1e-12)
    # a start time whose interval leaves the frame span is flagged, not advected
    xf2, _, fl2, _, _ = mv.advect_points(x0[:, :3], 4.0, 2.0, 0.1)
    assert (fl2 == oracle.FLAG_TIME_OUT).all() and np.array_equal(xf2, x0[:, :3])


def test_uniform_stream_exit_step():
    c = np.array([0.37, -0.11, 0.23])
    mesh = I.box_mesh(3, (5, 5, 5), (0.0,) * 3, (1.0,) * 3, jitter=0.2, seed=11, shuffle=True)
    mf = I.mesh_sample(lambda x, y, z, t: (c[0] + 0 * x, c[1] + 0 * y, c[2] + 0 * z), mesh,
                       2, 0.0, 100.0)
    mv = oracle.MeshVelocity(mf)
    rng = np.random.default_rng(12)
    dt, T = 0.05, 5.0
    N = int(round(T / dt))
    x0 = rng.uniform(0.05, 0.95, (3, 400))
    n = np.arange(N + 1)
    path = x0[:, :, None] + (n * dt)[None, None, :] * c[:, None, None]     # (3, m, N+1)
    dist = np.minimum(path, 1.0 - path).min(axis=0)                       # (m, N+1)
    keep = np.abs(dist).min(axis=1) > 1e-3                               # no step near a wall
    x0 = x0[:, keep]
    path, dist = path[:, keep], dist[keep]
    xf, cell, flags, mg, _ = mv.advect_points(x0, 0.0, T, dt)
    outside = dist < 0
    exits = outside.any(axis=1)
    first = np.where(exits, outside.argmax(axis=1), N + 1)
    assert exits.sum() > 50
    np.testing.assert_array_equal(flags, np.where(exits, oracle.FLAG_OUT, 0))
    want = path[:, np.arange(x0.shape[1]), np.minimum(first - 1, N)]
    np.testing.assert_allclose(xf, want, rtol=0, atol=1e-12)


def test_seed_outside_mesh_flagged():
    mesh = I.box_mesh(2, (4, 4), (0.0, 0.0), (1.0, 1.0), jitter=0.1, seed=13)
    mf = I.mesh_sample(lambda x, y, t: (0 * x + 0.1, 0 * y), mesh, 2, 0.0, 10.0)
    mv = oracle.MeshVelocity(mf)
    g = I.linspace_seeds(2, (7, 3), (-0.5, 0.2), (1.5, 0.8))
    xf, cell, flags, _, _ = mv.advect_seeds(g, 0.0, 1.0, 0.1)
    x0 = oracle.seed_points(g)
    out0 = (x0[0] < 0) | (x0[0] > 1)
    assert np.array_equal(flags[out0], np.full(out0.sum(), oracle.FLAG_OUT, np.uint8))
    assert np.array_equal(xf[:, out0], x0[:, out0]) and (cell[out0] == -1).all()
