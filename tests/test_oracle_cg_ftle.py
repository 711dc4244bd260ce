"""Pins of the oracle's flow-map gradient, Cauchy-Green tensor (Eq. 1),
largest eigenvalue and FTLE.

* A linear map F(x) = A x + b has grad F = A exactly, including at the
  one-sided edges, so C = A^T A (formed here with numpy.matmul).
* On periodic seed axes a translation F(x) = x + c has grad F = I everywhere;
  without the period shift at the seam the difference would be ~ -L/(2h).
* A smooth periodic displacement has a central-difference error bounded by
  max|F'''| h^2/6.
* lambda_max against LAPACK (numpy.linalg.eigvalsh) on random SPD matrices,
  including near-degenerate and ill-conditioned ones.
* End to end on the linear saddle: FTLE = (N/T) ln R(lam dt) and
  det C = (R(lam dt) R(-lam dt))^(2N) in closed form.
"""
import math

import numpy as np
import pytest

from paper_2209_13775_amd import inputs


def _grid_coords(g):
    idx = np.arange(g.count)
    return g.coords_of(idx)


def _positions(g):
    ijk = _grid_coords(g).astype(np.float64)
    return np.stack([g.origin[a] + ijk[a] * g.spacing[a] for a in range(g.dim)])


def _pack(M):
    d = M.shape[0]
    return np.array([M[r, s] for r in range(d) for s in range(r, d)])


@pytest.mark.parametrize("dim", [2, 3])
def test_linear_map_gradient_exact(orc, dim):
    rng = np.random.default_rng(dim)
    A = rng.standard_normal((dim, dim))
    b = rng.standard_normal(dim)
    g = inputs.linspace_seeds(dim, (7, 5, 4)[:dim], (-1.0, 0.0, 2.0)[:dim], (1.0, 3.0, 2.5)[:dim])
    x0 = _positions(g)
    xf = A @ x0 + b[:, None]
    Cm, sfl = orc.cg_tensor(g, xf)
    ref = _pack(A.T @ A)
    np.testing.assert_allclose(Cm, np.repeat(ref[:, None], g.count, axis=1), rtol=1e-12, atol=1e-12)
    assert not sfl.any()


@pytest.mark.parametrize("dim", [2, 3])
def test_periodic_translation_seam(orc, dim):
    L = (2 * math.pi, 2 * math.pi, 2 * math.pi)[:dim]
    g = inputs.periodic_seeds(dim, (8, 6, 5)[:dim], L)
    c = np.array([0.3, -5.1, 9.7])[:dim]
    xf = _positions(g) + c[:, None]
    Cm, _ = orc.cg_tensor(g, xf)
    np.testing.assert_allclose(Cm, np.repeat(_pack(np.eye(dim))[:, None], g.count, axis=1),
                               rtol=0, atol=1e-12)
    lam, sig = orc.ftle(dim, Cm, 1.0)
    np.testing.assert_allclose(sig, 0.0, atol=1e-12)


def test_periodic_smooth_displacement_error_bound(orc):
    L = 2 * math.pi
    n = 64
    g = inputs.periodic_seeds(2, (n, 3), (L, L))
    x0 = _positions(g)
    eps = 0.1
    xf = x0.copy()
    xf[0] = x0[0] + eps * np.sin(x0[0])
    Cm, _ = orc.cg_tensor(g, xf)
    h = L / n
    dFdx = 1.0 + eps * np.cos(x0[0])
    # C_xx = (dF_x/dx)^2; central-difference error <= eps*h^2/6 in dF/dx
    err = np.abs(np.sqrt(Cm[0]) - dFdx)
    assert err.max() <= eps * h * h / 6 * 1.01
    # the seam columns (i = 0 and i = n-1) are included
    ijk = _grid_coords(g)
    assert err[ijk[0] == 0].max() <= eps * h * h / 6 * 1.01


def test_stencil_flags_mark_neighbours(orc):
    g = inputs.SeedGrid(2, (6, 5, 1), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (True, False, False))
    xf = _positions(g)
    flags = np.zeros(g.count, dtype=np.uint8)
    bad = [g.index_of(np.array([[0], [2]]))[0], g.index_of(np.array([[3], [4]]))[0]]
    flags[bad[0]] = 1
    flags[bad[1]] = 2
    _, sfl = orc.cg_tensor(g, xf, flags)
    ijk = _grid_coords(g)
    expect = np.zeros(g.count, dtype=np.uint8)
    for s in range(g.count):
        i, j = ijk[0][s], ijk[1][s]
        for bi, bj in [(0, 2), (3, 4)]:
            di = min((i - bi) % 6, (bi - i) % 6)      # periodic in x
            dj = abs(j - bj)
            if di + dj <= 1:
                expect[s] = 4
    np.testing.assert_array_equal(sfl, expect)


def test_cg_point_matches_grid(orc):
    g = inputs.SeedGrid(3, (5, 4, 6), (0.0, 0.0, 0.0), (0.5, 0.5, 0.5), (True, False, True))
    rng = np.random.default_rng(0)
    xf = _positions(g) + 0.05 * rng.standard_normal((3, g.count))
    Cm, _ = orc.cg_tensor(g, xf)
    ijk = _grid_coords(g)
    for s in [0, 7, 33, g.count - 1, 61]:
        c = ijk[:, s]
        xm, xp = [], []
        for b in range(3):
            nb = g.n[b]
            per = g.periodic[b]
            lo = (c[b] - 1) % nb if per else max(c[b] - 1, 0)
            hi = (c[b] + 1) % nb if per else min(c[b] + 1, nb - 1)
            cm = c.copy(); cm[b] = lo
            cp = c.copy(); cp[b] = hi
            xm.append(xf[:, g.index_of(cm[:, None])[0]])
            xp.append(xf[:, g.index_of(cp[:, None])[0]])
        got = orc.cg_point(g, c, xf[:, s], xm, xp)
        np.testing.assert_array_equal(got, Cm[:, s])


def _random_spd(rng, d, count):
    mats = []
    for k in range(count):
        Q, _ = np.linalg.qr(rng.standard_normal((d, d)))
        kind = k % 4
        if kind == 0:
            ev = np.exp(rng.uniform(-5, 5, d))
        elif kind == 1:                       # near-degenerate top pair
            top = math.exp(rng.uniform(0, 4))
            ev = np.array([top, top * (1 + 1e-12), math.exp(rng.uniform(-4, 0))][:d])
        elif kind == 2:                       # condition number 1e12
            ev = np.array([1e6, 1.0, 1e-6][:d]) * math.exp(rng.uniform(-2, 2))
        else:                                 # exactly repeated eigenvalues
            ev = np.full(d, math.exp(rng.uniform(-1, 1)))
        mats.append(Q @ np.diag(ev) @ Q.T)
    return mats


@pytest.mark.parametrize("dim", [2, 3])
def test_lambda_max_against_lapack(orc, dim):
    rng = np.random.default_rng(100 + dim)
    mats = _random_spd(rng, dim, 10000)
    packed = np.stack([_pack(0.5 * (M + M.T)) for M in mats], axis=1)
    lam, _ = orc.ftle(dim, packed, 1.0)
    ref = np.array([np.linalg.eigvalsh(0.5 * (M + M.T))[-1] for M in mats])
    np.testing.assert_allclose(lam, ref, rtol=1e-13, atol=0)


def test_ftle_definition_and_degenerate(orc):
    sigma, T = 0.37, 2.5
    big = math.exp(2 * sigma * T)
    Cm = np.array([[big, 0.0], [0.0, 0.0], [1.0 / big, 0.0]])
    lam, sig = orc.ftle(2, Cm, -T)        # backward time uses |T|
    assert abs(sig[0] - sigma) < 1e-15
    assert sig[1] == -np.inf and lam[1] == 0.0


@pytest.mark.parametrize("dim", [2, 3])
def test_saddle_ftle_and_det_closed_form(orc, dim):
    lam, dt, T = 0.5, 0.05, 2.0
    N = int(round(T / dt))
    R = lambda z: 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    fs = inputs.saddle_frames(lam=lam, dim=dim)
    vel = orc.Velocity(fs)
    g = inputs.linspace_seeds(dim, (9, 7, 5)[:dim], (-0.5,) * dim, (0.5,) * dim)
    xf, _, flags = orc.advect_seeds(vel, g, 0.0, T, dt)
    Cm, sfl = orc.cg_tensor(g, xf, flags)
    lmax, sig = orc.ftle(dim, Cm, T)
    expect = (N / T) * math.log(R(lam * dt))
    np.testing.assert_allclose(sig, expect, rtol=0, atol=1e-12)
    if dim == 2:
        det = Cm[0] * Cm[2] - Cm[1] ** 2
        np.testing.assert_allclose(det, (R(lam * dt) * R(-lam * dt)) ** (2 * N), rtol=1e-11)
    assert abs(expect - 0.4999999984) < 1e-10


def test_cg_is_spd_and_det_near_one_for_incompressible(orc):
    # the double gyre is divergence free, so det C = 1 (Liouville); the discrete
    # value carries interpolation and differencing errors of order h^2, so with
    # the velocity grid and the seed grid refined together the median deviation
    # must fall about 4x per halving of h
    devs = []
    for nx in [51, 101, 201]:
        fs = inputs.double_gyre_frames(nx=nx, ny=(nx + 1) // 2)
        vel = orc.Velocity(fs)
        h = 2.0 / (nx - 1)
        g = inputs.linspace_seeds(2, (int(round(1.5 / h)) + 1, int(round(0.6 / h)) + 1),
                                  (0.25, 0.2), (1.75, 0.8))
        xf, _, flags = orc.advect_seeds(vel, g, 0.0, 2.0, 0.02)
        Cm, sfl = orc.cg_tensor(g, xf, flags)
        det = Cm[0] * Cm[2] - Cm[1] ** 2
        assert not flags.any()
        # symmetric positive definite: both eigenvalues of [[a,b],[b,c]] > 0
        assert np.all(det > 0) and np.all(Cm[0] > 0)
        devs.append(np.median(np.abs(det - 1.0)))
    assert devs[0] / devs[1] > 3.0 and devs[1] / devs[2] > 3.0, devs
    assert devs[2] < 1e-3


def test_cg_is_spd_and_det_near_one_for_incompressible_3d(orc):
    # the ABC flow is divergence free (u depends on y, z only, v on x, z, w on
    # x, y), so the exact flow map preserves volume and det C = 1 (Liouville);
    # trilinear interpolation and central differences on a seed grid of the
    # node spacing break that by O(h^2), so refining the velocity grid and the
    # seeds together must shrink the median deviation about 4x per halving
    devs = []
    for n in [16, 32, 64, 128]:
        fs = inputs.abc_frames(n=n, n_frames=5, dt_frame=0.5, dtype=np.float64)
        vel = orc.Velocity(fs)
        h = 2 * math.pi / n
        m = int(round(2.0 / h)) + 1
        g = inputs.linspace_seeds(3, (m, m, m), (0.5,) * 3, (0.5 + (m - 1) * h,) * 3)
        xf, _, flags = orc.advect_seeds(vel, g, 0.0, 1.0, 0.02)
        assert not flags.any()
        Cm, _ = orc.cg_tensor(g, xf, flags)
        M = np.empty((g.count, 3, 3))
        k = 0
        for r in range(3):
            for s in range(r, 3):
                M[:, r, s] = M[:, s, r] = Cm[k]
                k += 1
        assert np.linalg.eigvalsh(M).min() > 0          # positive definite at every seed
        devs.append(np.median(np.abs(np.linalg.det(M) - 1.0)))
    for a, b in zip(devs, devs[1:]):
        assert a / b > 3.0, devs
    assert devs[-1] < 3e-3, devs
