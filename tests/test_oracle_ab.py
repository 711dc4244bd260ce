"""Pins of the oracle's Adams-Bashforth flow map (Sec. 2 Flow Map filter:
multistep methods), orders 2-4 with RK4 start-up steps.

* Convergence on a bilinear, time-dependent field that the interpolant
  reproduces exactly, against SciPy's DOP853: observed order s for the
  s-step method.
* Linear saddle u = (lam x, -lam y): the discrete method is a linear scalar
  recurrence per axis, y_{n+1} = y_n + z sum_j b_j y_{n-j} (z = lam dt), with
  the start-up values y_m = R(z)^m y_0 of classical RK4 -- so positions and the
  FTLE follow from the recurrence alone (no field evaluation).
* A field linear in time and uniform in space is integrated exactly by every
  order >= 2 (and by RK4 during start-up).
* A run of fewer than s steps is plain RK4; a uniform stream leaves the box
  at the closed-form step.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle as orc
from paper_2209_13775_amd import inputs

AB = {2: [3 / 2, -1 / 2], 3: [23 / 12, -16 / 12, 5 / 12], 4: [55 / 24, -59 / 24, 37 / 24, -9 / 24]}


def R(z):
    return 1.0 + z + z * z / 2.0 + z ** 3 / 6.0 + z ** 4 / 24.0


def recurrence(z, order, N):
    """Growth factor y_N / y_0 of s-step AB with RK4 start-up on y' = lam y."""
    y = [1.0]
    for n in range(N):
        if n < order - 1:
            y.append(y[-1] * R(z))
        else:
            y.append(y[-1] + z * sum(AB[order][j] * y[-1 - j] for j in range(order)))
    return y[-1]


@pytest.mark.parametrize("order", [2, 3, 4])
def test_order_against_dop853(order):
    fs = inputs.bilinear_rotor_frames()
    vel = orc.Velocity(fs)
    x0 = np.array([[0.5, -0.3, 0.2, 0.0], [0.0, 0.4, -0.6, 0.7]])
    t0, T = 0.5, 4.0
    ref = np.empty_like(x0)
    for p in range(x0.shape[1]):
        sol = solve_ivp(inputs.bilinear_rotor_rhs, (t0, t0 + T), x0[:, p], method="DOP853",
                        rtol=1e-13, atol=1e-14)
        ref[:, p] = sol.y[:, -1]
    errs = []
    for dt in (0.05, 0.025, 0.0125, 0.00625):
        xf, _, flags = orc.advect_points_ab(vel, x0, t0, T, dt, order=order)
        assert not flags.any()
        errs.append(np.max(np.linalg.norm(xf - ref, axis=0)))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    for o in orders:
        assert order - 0.1 <= o <= order + 0.1, (errs, orders)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_saddle_recurrence_closed_form(order):
    lam, dt, T = 0.5, 0.05, 2.0
    N = int(round(T / dt))
    fs = inputs.saddle_frames(lam=lam, dim=2)
    vel = orc.Velocity(fs)
    g = inputs.linspace_seeds(2, (9, 9), (-0.5, -0.5), (0.5, 0.5))
    xf, cell, flags = orc.advect_seeds_ab(vel, g, 0.0, T, dt, order=order)
    x0 = orc.seed_points(g)
    assert not flags.any()
    gx, gy = recurrence(lam * dt, order, N), recurrence(-lam * dt, order, N)
    np.testing.assert_allclose(xf[0], x0[0] * gx, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(xf[1], x0[1] * gy, rtol=1e-12, atol=1e-15)
    Cm, _ = orc.cg_tensor(g, xf, flags)
    _, sig = orc.ftle(2, Cm, T)
    np.testing.assert_allclose(sig, math.log(max(abs(gx), abs(gy))) / T, rtol=1e-11)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_linear_in_time_field_exact(order):
    a = np.array([0.3, -0.2])
    b = np.array([0.05, 0.1])
    fs = inputs.sample_field(lambda X, Y, t: (a[0] + b[0] * t + 0 * X, a[1] + b[1] * t + 0 * Y),
                             2, (9, 9), (-5.0, -5.0), (1.25, 1.25), (False, False), 0.0, 8.0, 2)
    vel = orc.Velocity(fs)
    x0 = np.random.default_rng(0).uniform(-1, 1, (2, 50))
    t0, T, dt = 0.7, 3.2, 0.1
    xf, _, flags = orc.advect_points_ab(vel, x0, t0, T, dt, order=order)
    assert not flags.any()
    want = x0 + (a * T + b * ((t0 + T) ** 2 - t0 ** 2) / 2)[:, None]
    np.testing.assert_allclose(xf, want, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_short_run_is_rk4(order):
    fs = inputs.double_gyre_frames(nx=41, ny=21, n_frames=11)
    vel = orc.Velocity(fs)
    x0 = np.random.default_rng(1).uniform(0.1, 0.9, (2, 40)) * np.array([[2.0], [1.0]])
    for N in range(1, order):
        xa, _, fa = orc.advect_points_ab(vel, x0, 0.0, 0.1 * N, 0.1, order=order)
        xr, _, fr = orc.advect_points(vel, x0, 0.0, 0.1 * N, 0.1)
        np.testing.assert_array_equal(xa, xr)
        np.testing.assert_array_equal(fa, fr)
    xa, _, _ = orc.advect_points_ab(vel, x0, 0.0, 0.1 * order, 0.1, order=order)
    xr, _, _ = orc.advect_points(vel, x0, 0.0, 0.1 * order, 0.1)
    assert np.abs(xa - xr).max() > 0          # the multistep formula takes over


@pytest.mark.parametrize("order", [2, 4])
def test_uniform_stream_exit_step(order):
    c = np.array([0.37, -0.21])
    fs = inputs.uniform_frames(c, dim=2, n=9, lo=0.0, hi=1.0)
    vel = orc.Velocity(fs)
    rng = np.random.default_rng(2)
    dt, T = 0.05, 5.0
    N = int(round(T / dt))
    x0 = rng.uniform(0.05, 0.95, (2, 400))
    n = np.arange(N + 1)
    path = x0[:, :, None] + (n * dt)[None, None, :] * c[:, None, None]
    dist = np.minimum(path, 1.0 - path).min(axis=0)
    keep = np.abs(dist).min(axis=1) > 1e-3
    x0, path, dist = x0[:, keep], path[:, keep], dist[keep]
    xf, _, flags = orc.advect_points_ab(vel, x0, 0.0, T, dt, order=order)
    outside = dist < 0
    exits = outside.any(axis=1)
    first = np.where(exits, outside.argmax(axis=1), N + 1)
    assert exits.sum() > 50
    np.testing.assert_array_equal(flags, np.where(exits, orc.FLAG_OUT, 0))
    want = path[:, np.arange(x0.shape[1]), np.minimum(first - 1, N)]
    np.testing.assert_allclose(xf, want, rtol=0, atol=1e-12)
