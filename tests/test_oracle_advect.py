"""Pins of the oracle's RK4 flow map (Eq. 2; Sec. 3.1) and its exit rule.

* Linear saddle u = (lam x, -lam y): the interpolant is exact, and classical
  RK4 applied to x' = lam x multiplies x by the stability polynomial
  R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24 (z = lam dt) every step, so
  x_N = R(lam dt)^N x_0 in closed form.
* A bilinear, time-dependent field (reproduced exactly by the interpolant)
  integrated by SciPy's DOP853 at tight tolerance: the oracle's error must
  fall as dt^4 (observed order in [3.8, 4.2]).
* A uniform stream: RK4 is exact, so the step at which a tracer leaves the
  closed domain (and its frozen position) follows in closed form.
* Forward-then-backward integration returns to the seed within O(dt^4).
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from paper_2209_13775_amd import inputs


def R(z):
    return 1.0 + z + z * z / 2.0 + z ** 3 / 6.0 + z ** 4 / 24.0


@pytest.mark.parametrize("dim", [2, 3])
def test_saddle_positions_closed_form(orc, dim):
    lam, dt, T = 0.5, 0.05, 2.0
    N = int(round(T / dt))
    fs = inputs.saddle_frames(lam=lam, dim=dim)
    vel = orc.Velocity(fs)
    g = inputs.linspace_seeds(dim, (9,) * dim, (-0.5,) * dim, (0.5,) * dim)
    xf, cell, flags = orc.advect_seeds(vel, g, 0.0, T, dt)
    x0 = orc.seed_points(g)
    assert not flags.any()
    np.testing.assert_allclose(xf[0], x0[0] * R(lam * dt) ** N, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(xf[1], x0[1] * R(-lam * dt) ** N, rtol=1e-13, atol=1e-15)
    if dim == 3:
        np.testing.assert_array_equal(xf[2], x0[2])


def test_backward_saddle_closed_form(orc):
    lam, dt, T = 0.4, -0.1, -3.0
    N = 30
    fs = inputs.saddle_frames(lam=lam, t_first=-5.0, dt_frame=10.0)
    vel = orc.Velocity(fs)
    x0 = np.array([[0.3, -0.2, 0.05], [0.1, 0.4, -0.35]])
    xf, _, flags = orc.advect_points(vel, x0, 1.0, T, dt)
    assert not flags.any()
    np.testing.assert_allclose(xf[0], x0[0] * R(lam * dt) ** N, rtol=1e-13)
    np.testing.assert_allclose(xf[1], x0[1] * R(-lam * dt) ** N, rtol=1e-13)


def test_rk4_fourth_order_against_dop853(orc):
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
    dts = [0.2, 0.1, 0.05, 0.025]
    for dt in dts:
        xf, _, flags = orc.advect_points(vel, x0, t0, T, dt)
        assert not flags.any()
        errs.append(np.max(np.linalg.norm(xf - ref, axis=0)))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    for o in orders:
        assert 3.8 <= o <= 4.2, (errs, orders)
    assert errs[-1] < 1e-7


def test_uniform_stream_exit_step(orc):
    c = np.array([0.37, -0.21])
    fs = inputs.uniform_frames(c, dim=2, n=9, lo=0.0, hi=1.0)
    vel = orc.Velocity(fs)
    dt, T = 0.05, 10.0
    rng = np.random.default_rng(3)
    x0 = rng.uniform(0.1, 0.9, size=(2, 200))
    # exact positions x0 + n dt c; the first rejected step n_exit is the first
    # n whose end point x0 + (n+1) dt c lies outside [0,1]^2 (the k4 stage point
    # of a constant field is that end point, and earlier stage points lie between)
    steps = np.arange(0, 201)
    pos = x0[:, :, None] + steps[None, None, :] * dt * c[:, None, None]
    inside = np.all((pos >= 0.0) & (pos <= 1.0), axis=0)
    # keep tracers whose path never comes within 1e-3 of a wall at a step
    dist = np.min(np.minimum(np.abs(pos), np.abs(pos - 1.0)), axis=0)
    keep = np.all(dist > 1e-3, axis=1)
    x0 = x0[:, keep]
    inside = inside[keep]
    n_ok = np.argmin(inside, axis=1) - 1            # last step index still inside
    expect = x0 + n_ok[None, :] * dt * c[:, None]
    xf, cell, flags = orc.advect_points(vel, x0, 0.0, T, dt)
    np.testing.assert_allclose(xf, expect, rtol=0, atol=1e-12)
    assert np.all(flags == 1)
    # cell of the frozen position: brute force over the 8x8 cells
    h = 1.0 / 8
    i = np.clip(np.floor(expect / h).astype(np.int64), 0, 7)
    np.testing.assert_array_equal(cell, i[0] + 9 * i[1])


def test_never_exits_and_periodic_unwrapped(orc):
    c = np.array([0.8, -0.3, 0.55])
    fs = inputs.uniform_frames(c, dim=3, n=8, lo=0.0, hi=2.0, periodic=True)
    vel = orc.Velocity(fs)
    x0 = np.array([[0.1, 1.9], [0.2, 0.05], [1.7, 1.0]])
    xf, cell, flags = orc.advect_points(vel, x0, 0.0, 7.5, 0.05)
    assert not flags.any()
    np.testing.assert_allclose(xf, x0 + 7.5 * c[:, None], rtol=0, atol=1e-12)
    # cell index of the wrapped position
    w = np.mod(xf, 2.0)
    i = np.floor(w / 0.25).astype(np.int64)
    np.testing.assert_array_equal(cell, i[0] + 8 * (i[1] + 8 * i[2]))


def test_nonfinite_velocity_flags_only_tracers_that_sample_it(orc):
    c = np.array([0.5, 0.0])
    fs = inputs.uniform_frames(c, dim=2, n=11, lo=0.0, hi=1.0)
    # poison node (i=6, j=5) at x=0.6, y=0.5 in the second frame
    fs.u[0][1, 5, 6] = np.nan
    vel = orc.Velocity(fs)
    ys = np.array([0.12, 0.33, 0.43, 0.47, 0.55, 0.58, 0.66, 0.87])
    x0 = np.stack([np.full(ys.size, 0.13), ys])
    xf, _, flags = orc.advect_points(vel, x0, 0.0, 1.0, 0.01)
    # paths along y = const cross x in [0.13, 0.63]: they touch cells next to the
    # poisoned node exactly when 0.4 < y < 0.6
    expect = np.where((ys > 0.4) & (ys < 0.6), 2, 0)
    np.testing.assert_array_equal(flags, expect)
    # frozen tracers stopped before the cells next to x=0.6, i.e. x < 0.5 + dt*0.5 + tiny
    assert np.all(xf[0][flags == 2] <= 0.5 + 1e-12)


def test_forward_backward_returns(orc):
    fs = inputs.double_gyre_frames()
    vel = orc.Velocity(fs)
    rng = np.random.default_rng(7)
    x0 = np.stack([rng.uniform(0.2, 1.8, 64), rng.uniform(0.2, 0.8, 64)])
    for dt, tol in [(0.05, 2e-5), (0.025, 2e-6)]:
        xf, _, fl = orc.advect_points(vel, x0, 0.0, 5.0, dt)
        xb, _, fl2 = orc.advect_points(vel, xf, 5.0, -5.0, -dt)
        assert not fl.any() and not fl2.any()
        assert np.median(np.linalg.norm(xb - x0, axis=0)) < tol


def test_threads_do_not_change_results(orc):
    fs = inputs.double_gyre_frames(nx=51, ny=26)
    vel = orc.Velocity(fs)
    g = inputs.linspace_seeds(2, (33, 17), (0.0, 0.0), (2.0, 1.0))
    a = orc.advect_seeds(vel, g, 0.0, 5.0, 0.05, threads=1)
    b = orc.advect_seeds(vel, g, 0.0, 5.0, 0.05, threads=4)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    # a seed subset gives the same values as the full grid
    idx = np.array([0, 5, 100, 560])
    c = orc.advect_seeds(vel, g, 0.0, 5.0, 0.05, idx=idx)
    assert np.array_equal(c[0], a[0][:, idx])


def test_time_span_rule(orc):
    # no extrapolation in time: a point whose [t0, t0+T] leaves the frame span
    # is flagged TIME_OUT and left where it started
    fs = inputs.uniform_frames(np.array([0.1, 0.0]), dim=2, n=5, t_first=1.0, dt_frame=2.0)
    vel = orc.Velocity(fs)          # frames at t = 1 and t = 3
    x0 = np.array([[0.2, 0.2, 0.2, 0.2], [0.5, 0.5, 0.5, 0.5]])
    t0 = np.array([1.0, 0.5, 2.5, 3.0])
    xf, _, flags = orc.advect_points(vel, x0, t0, 0.5, 0.1)
    np.testing.assert_array_equal(flags, [0, 8, 0, 8])
    np.testing.assert_allclose(xf[0], [0.25, 0.2, 0.25, 0.2], atol=1e-14)


def test_trajectory_recording_closed_form_and_freeze(orc):
    # positions after every step on the steady linear saddle: the interpolant is
    # exact and RK4 multiplies x by R(lam dt) and y by R(-lam dt) per step, so
    # step n holds R^n x0 (the e_S(t) curves of the FP32 / FP64 comparison read
    # these positions)
    lam, dt, T = 0.5, 0.05, 2.0
    N = int(round(T / dt))
    R = lambda z: 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    vel = orc.Velocity(inputs.saddle_frames(lam=lam))
    x0 = np.array([[0.3, -0.2, 0.05], [0.1, 0.4, -0.35]])
    traj, flags = orc.advect_points_traj(vel, x0, 0.0, T, dt)
    assert traj.shape == (N, 2, 3) and not flags.any()
    n = np.arange(1, N + 1)[:, None]
    np.testing.assert_allclose(traj[:, 0], x0[0] * R(lam * dt) ** n, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(traj[:, 1], x0[1] * R(-lam * dt) ** n, rtol=1e-13, atol=1e-15)
    # a tracer that leaves: the x-growth R(lam dt)^n carries x = 2.9 past the
    # wall at 3 in the first step whose end point (or stage) is outside; from
    # then on every recorded position is the frozen one
    x1 = np.array([[2.9], [0.0]])
    traj, flags = orc.advect_points_traj(vel, x1, 0.0, T, dt)
    assert flags[0] == 1
    n_exit = next(k for k in range(1, N + 1) if 2.9 * R(lam * dt) ** k > 3.0)
    # steps before the exit step are the closed form; the exit step and all
    # later ones repeat the last accepted position (stage points of the exit
    # step may leave first, so allow it to come one step earlier)
    frozen = traj[-1, 0, 0]
    first_frozen = int(np.argmax(traj[:, 0, 0] == frozen))
    assert n_exit - 2 <= first_frozen <= n_exit - 1
    np.testing.assert_allclose(traj[:first_frozen, 0, 0],
                               2.9 * R(lam * dt) ** np.arange(1, first_frozen + 1), rtol=1e-13)
    assert np.all(traj[first_frozen:, 0, 0] == frozen)
