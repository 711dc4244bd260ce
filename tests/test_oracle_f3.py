"""Pins of the oracle's eigen-decomposition of C, time-resolved flow maps and
early CG evaluation (Sec. 2 Flow Map and Cauchy-Green filters; Sec. 3.1).

* Eigenvalues and eigenvectors against LAPACK (numpy.linalg.eigh): values to
  1e-13 relative, vectors to sign where the eigengap is clear, residual
  ||C v - lambda v||, orthonormality, and the sign convention (largest
  component positive), on random, near-degenerate and ill-conditioned SPD
  matrices.
* Snapshots on the linear saddle: the position after k steps is R(z)^k x0.
* Exit steps and early FTLE on a saddle inside the closed box [-1, 1]^2: for a
  linear field the RK4 stage points of step n are x_{n-1} times (1 + z/2),
  (1 + z/2 + z^2/4), (1 + z + z^2/2 + z^3/4) and x_n = R(z) x_{n-1}, so the
  step at which a tracer leaves follows in closed form; the gradient of a
  linear map is exact and its FTLE is ln R(z)/dt whatever the evaluation
  time, so the early FTLE is known too, and its time is the earliest exit in
  the stencil.
"""
import math

import numpy as np
import pytest

import oracle as orc
from paper_2209_13775_amd import inputs


def R(z):
    return 1.0 + z + z * z / 2.0 + z ** 3 / 6.0 + z ** 4 / 24.0


def _packed(S):
    d = S.shape[-1]
    iu = np.triu_indices(d)
    return np.stack([S[:, i, j] for i, j in zip(*iu)])


@pytest.mark.parametrize("dim", [2, 3])
def test_eig_against_lapack(dim):
    rng = np.random.default_rng(dim)
    A = rng.standard_normal((3000, dim, dim))
    S = A @ np.transpose(A, (0, 2, 1))
    # near-degenerate and ill-conditioned cases
    Q, _ = np.linalg.qr(rng.standard_normal((1000, dim, dim)))
    w = np.ones((1000, dim))
    w[:500, -1] = 1.0 + 1e-9 * rng.random(500)      # two top eigenvalues nearly equal
    w[500:, 0] = 1e-12                                 # condition number 1e12
    w[500:, -1] = 1.0 + rng.random(500)
    S2 = Q @ (w[:, :, None] * np.transpose(Q, (0, 2, 1)))
    S = np.concatenate([S, 0.5 * (S2 + np.transpose(S2, (0, 2, 1)))])
    ev, V = orc.eig(dim, _packed(S))
    lw, LU = np.linalg.eigh(S)
    scale = np.abs(lw).max(axis=1)
    assert (np.abs(ev.T - lw).max(axis=1) / scale).max() <= 1e-13
    Vt = np.transpose(V, (2, 0, 1))                     # (n, k, a)
    # residual and orthonormality
    res = np.einsum("nab,nkb->nka", S, Vt) - ev.T[:, :, None] * Vt
    assert (np.abs(res).max(axis=(1, 2)) / scale).max() <= 1e-13
    gram = np.einsum("nka,nla->nkl", Vt, Vt)
    assert np.abs(gram - np.eye(dim)).max() <= 1e-13
    # sign convention
    big = np.abs(Vt).argmax(axis=2)
    assert (np.take_along_axis(Vt, big[:, :, None], axis=2) > 0).all()
    # eigenvectors agree with LAPACK's up to sign where the gap is clear
    gaps = np.diff(lw, axis=1) / scale[:, None]
    for k in range(dim):
        gap = np.full(len(S), np.inf)
        if k > 0:
            gap = np.minimum(gap, gaps[:, k - 1])
        if k < dim - 1:
            gap = np.minimum(gap, gaps[:, k])
        ok = gap > 1e-6
        dots = np.abs(np.einsum("na,na->n", Vt[:, k, :], LU[:, :, k]))
        assert np.abs(dots[ok] - 1.0).max() <= 1e-8
    # the top eigenvalue is the one the FTLE uses
    lam, _ = orc.ftle(dim, _packed(S), 1.0)
    np.testing.assert_allclose(ev[-1], lam, rtol=1e-13)


def test_snapshots_saddle_closed_form():
    lam, dt = 0.5, 0.05
    fs = inputs.saddle_frames(lam=lam, dim=2)
    vel = orc.Velocity(fs)
    g = inputs.linspace_seeds(2, (7, 6), (-0.5, -0.5), (0.5, 0.5))
    steps = [1, 3, 10, 40]
    xf, fl, done = orc.advect_seeds_snap(vel, g, 0.0, dt, steps)
    x0 = orc.seed_points(g)
    assert not fl.any() and (done == 40).all()
    for k, n in enumerate(steps):
        np.testing.assert_allclose(xf[k, 0], x0[0] * R(lam * dt) ** n, rtol=1e-13, atol=1e-16)
        np.testing.assert_allclose(xf[k, 1], x0[1] * R(-lam * dt) ** n, rtol=1e-13, atol=1e-16)


def _exit_step(x0, z, N):
    """Accepted steps before a tracer x' = (lam x) leaves [-1, 1] (closed form)."""
    x = abs(x0)
    for n in range(1, N + 1):
        pts = [x * (1 + z / 2), x * (1 + z / 2 + z * z / 4), x * (1 + z + z * z / 2 + z ** 3 / 4),
               x * R(z)]
        if max(pts) > 1.0:
            return n - 1
        x = x * R(z)
    return N


def test_exit_steps_and_early_ftle_saddle_box():
    lam, dt, T = 0.5, 0.05, 4.0
    N = int(round(T / dt))
    z = lam * dt
    fs = inputs.saddle_frames(lam=lam, dim=2, half=1.0, n=9)
    vel = orc.Velocity(fs)
    g = inputs.linspace_seeds(2, (41, 9), (-0.95, -0.6), (0.95, 0.6))
    xf, fl, done = orc.advect_seeds_snap(vel, g, 0.0, dt, [N])
    x0 = orc.seed_points(g)
    want = np.array([_exit_step(x0[0, p], z, N) for p in range(g.count)])
    np.testing.assert_array_equal(done, want)
    assert ((want < N) & (want > 0)).sum() > 100
    np.testing.assert_array_equal(fl[0] != 0, want < N)
    lamx, sig, te = orc.ftle_early(vel, g, 0.0, dt, done)
    # earliest exit among the seeds each gradient uses
    c = g.coords_of(np.arange(g.count))
    ns = done.copy()
    for b in range(2):
        for d in (-1, 1):
            cc = c.copy()
            cc[b] = np.clip(c[b] + d, 0, g.n[b] - 1)
            ns = np.minimum(ns, done[g.index_of(cc)])
    np.testing.assert_allclose(te, ns * dt, rtol=1e-15)
    ok = ns > 0
    np.testing.assert_allclose(sig[ok], math.log(R(z)) / dt, rtol=1e-10)
    assert np.isnan(sig[~ok]).all()


def test_early_equals_ordinary_without_exits():
    fs = inputs.double_gyre_frames(nx=51, ny=26, n_frames=11)
    vel = orc.Velocity(fs)
    g = inputs.linspace_seeds(2, (23, 12), (0.1, 0.1), (1.9, 0.9))
    t0, dt, N = 0.5, 0.05, 80
    xs, fl, done = orc.advect_seeds_snap(vel, g, t0, dt, [N])
    assert (done == N).all()
    Cm, _ = orc.cg_tensor(g, xs[0], fl[0])
    lam, sig = orc.ftle(2, Cm, N * dt)
    l2, s2, te = orc.ftle_early(vel, g, t0, dt, done)
    np.testing.assert_array_equal(s2, sig)
    np.testing.assert_allclose(te, N * dt)
