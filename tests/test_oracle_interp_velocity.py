"""Pins of the oracle's interpolation and Bohmian velocities (Eqs. 10-11)
against band-limited identities, the periodic-sinc formula and the closed-form
Bohmian trajectories of a free Gaussian."""

import math

import numpy as np
import pytest

from oracle import grid, icwf, interp, models, velocity

from test_oracle_propagation import free_gaussian


def test_exact_at_grid_points(rng):
    f = rng.standard_normal((3, 32)) + 1j * rng.standard_normal((3, 32))
    x, h = grid.points(-2.0, 3.0, 32)
    val, _ = interp.trig_interp(f, -2.0, h, x)
    # phases up to 2 pi * 31 * 16 / 32 ~ 100 rad round at ~1e-14
    assert np.max(np.abs(val - f.T)) < 5e-14


def test_band_limited_values_and_derivatives(rng):
    n, x_min, L = 24, -1.5, 7.0
    x, h = grid.points(x_min, x_min + L, n)
    modes = np.arange(-n // 2 + 1, n // 2)
    a = rng.standard_normal(modes.size) + 1j * rng.standard_normal(modes.size)

    def f(t):
        return np.exp(2j * np.pi * np.outer(t - x_min, modes) / L) @ a

    def df(t):
        return (np.exp(2j * np.pi * np.outer(t - x_min, modes) / L) * (2j * np.pi * modes / L)) @ a

    xq = rng.uniform(x_min - L, x_min + 2 * L, 50)          # includes points outside the box
    val, der = interp.trig_interp(f(x)[None, :], x_min, h, xq)
    assert np.max(np.abs(val[:, 0] - f(xq))) < 1e-12
    assert np.max(np.abs(der[:, 0] - df(xq))) < 1e-11


def test_nyquist_mode_is_a_cosine():
    n, x_min = 16, 0.3
    x, h = grid.points(x_min, x_min + 4.0, n)
    samples = np.cos(np.pi * (x - x_min) / h)                   # (-1)^i
    xq = np.array([0.41, 1.7, 3.05])
    val, der = interp.trig_interp(samples[None, :], x_min, h, xq)
    u = (xq - x_min) / h
    assert np.max(np.abs(val[:, 0] - np.cos(np.pi * u))) < 1e-13
    assert np.max(np.abs(der[:, 0] + np.pi / h * np.sin(np.pi * u))) < 1e-12


def test_equals_periodic_sinc(rng):
    """Trefethen's periodic sinc S(y) = sin(pi y/h) cos(pi y/L) / (n sin(pi y/L))."""
    n, x_min, L = 32, -4.0, 9.0
    x, h = grid.points(x_min, x_min + L, n)
    f = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    xq = rng.uniform(x_min, x_min + L, 20)
    y = xq[:, None] - x[None, :]
    S = np.sin(np.pi * y / h) * np.cos(np.pi * y / L) / (n * np.sin(np.pi * y / L))
    val, _ = interp.trig_interp(f[None, :], x_min, h, xq)
    assert np.max(np.abs(val[:, 0] - S @ f)) < 1e-13


def _free_setup(dt):
    zero = models.Separable(lambda r: 0.0 * r, lambda R: 0.0 * R)
    return icwf.Setup(zero, -30.0, 30.0, 256, -6.0, 6.0, 128, 1.0, 10.0, dt, 1e-8)


def test_free_gaussian_velocity_field():
    """N = 1: v(x,t) = p0/m + (x - xbar(t)) t / (4 m^2 s0^4 + t^2) in each coordinate."""
    dt = 0.05
    st_ = _free_setup(dt)
    p1 = free_gaussian(st_.r, 0.0, -2.0, 0.5, 1.0, 1.0)[None, :]
    p2 = free_gaussian(st_.R, 0.0, 1.0, -1.0, 0.5, 10.0)[None, :]
    state = icwf.init(st_, [-1.2], [1.3], p1, p2, C0=[1.0 + 0j])
    for _ in range(40):
        state = icwf.step(st_, state)
    t = state.t
    v_r, v_R, _ = velocity.velocities(state.C, state.psi1, state.psi2, st_.r_min, st_.hr,
                                      st_.R_min, st_.hR, 1.0, 10.0, state.r_traj, state.R_traj)
    xbar_r = -2.0 + 0.5 * t
    xbar_R = 1.0 - 1.0 / 10.0 * t
    ref_r = 0.5 + (state.r_traj[0] - xbar_r) * t / (4 * 1.0 * 1.0 + t * t)
    ref_R = -0.1 + (state.R_traj[0] - xbar_R) * t / (4 * 100.0 * 0.5 ** 4 + t * t)
    # roundoff of psi (~1e-12) enters through psi'/psi ~ 1/h: 1e-11 absolute
    assert v_r[0] == pytest.approx(ref_r, abs=1e-11)
    assert v_R[0] == pytest.approx(ref_R, abs=1e-11)


def _free_traj_error(dt, T=2.0, trajectories="euler"):
    st_ = _free_setup(dt)
    st_.trajectories = trajectories
    p1 = free_gaussian(st_.r, 0.0, -2.0, 0.5, 1.0, 1.0)[None, :]
    p2 = free_gaussian(st_.R, 0.0, 1.0, -1.0, 0.5, 10.0)[None, :]
    state = icwf.init(st_, [-1.2], [1.3], p1, p2, C0=[1.0 + 0j])
    for _ in range(int(round(T / dt))):
        state = icwf.step(st_, state)
    t = state.t
    sr = math.sqrt(1 + t * t / 4.0)
    sR = math.sqrt(1 + t * t / (4 * 100 * 0.5 ** 4))
    r_ex = -2.0 + 0.5 * t + (-1.2 + 2.0) * sr
    R_ex = 1.0 - 0.1 * t + (1.3 - 1.0) * sR
    return abs(state.r_traj[0] - r_ex) + abs(state.R_traj[0] - R_ex)


def test_free_gaussian_trajectory_first_order():
    """Trajectories x(t) = xbar(t) + (x0 - xbar0) s(t)/s0; explicit Euler is first order."""
    e1, e2 = _free_traj_error(0.1), _free_traj_error(0.05)
    assert e1 < 3e-2
    assert 1.8 < e1 / e2 < 2.2


def test_free_gaussian_trajectory_heun_second_order():
    """The same closed-form Bohmian paths with Heun trajectories (Euler
    predictor, trapezoid corrector with the velocity field of the new state):
    the error falls as dt^2."""
    e1, e2 = _free_traj_error(0.1, trajectories="heun"), _free_traj_error(0.05, trajectories="heun")
    assert e1 < 1e-3
    assert 3.5 < e1 / e2 < 4.5
    assert e1 < 0.1 * _free_traj_error(0.1)


def test_node_raises():
    st_ = _free_setup(0.1)
    p1 = free_gaussian(st_.r, 0.0, 0.0, 0.0, 1.0, 1.0)[None, :]
    p2 = np.zeros((1, st_.n_R), complex)
    with pytest.raises(velocity.NodeError):
        velocity.velocities(np.ones(1, complex), p1, p2, st_.r_min, st_.hr, st_.R_min, st_.hR,
                            1.0, 10.0, np.array([0.1]), np.array([0.2]))
