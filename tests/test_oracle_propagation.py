"""Pins of the oracle's grid, models and CWF propagator (Eqs. 2, 5-6) against
closed forms: free Gaussian spreading, harmonic coherent-state motion,
constant-potential phase, unitarity, and the erf/x soft-Coulomb limits."""

import math

import numpy as np
import pytest
from scipy.special import erf

from oracle import grid, models, propagate


def free_gaussian(x, t, x0, p0, s0, m):
    """Analytic free-particle Gaussian (textbook): |psi|^2 ~ N(x0 + p0 t/m, s(t)^2)."""
    tau = t / (2.0 * m * s0 * s0)
    return ((2 * math.pi * s0 * s0) ** -0.25 / np.sqrt(1 + 1j * tau)
            * np.exp(-(x - x0 - p0 * t / m) ** 2 / (4 * s0 * s0 * (1 + 1j * tau))
                     + 1j * p0 * (x - x0) - 1j * p0 * p0 * t / (2 * m)))


@pytest.mark.parametrize("m,n,box,p0", [(1.0, 512, 60.0, 0.7), (1836.0, 256, 18.0, 6.0)])
def test_free_gaussian_is_exact(m, n, box, p0):
    x, h = grid.points(-box / 2, box / 2, n)
    k = grid.wavenumbers(n, h)
    s0 = 1.0 if m == 1.0 else 0.3
    psi = free_gaussian(x, 0.0, -3.0 if m == 1.0 else -1.0, p0, s0, m)
    dt, steps = 0.05, 100
    V = np.zeros(n)
    for _ in range(steps):
        psi = propagate.strang_step(psi, V, k, m, dt)
    ref = free_gaussian(x, dt * steps, -3.0 if m == 1.0 else -1.0, p0, s0, m)
    assert np.max(np.abs(psi - ref)) < 1e-12


def test_constant_potential_is_a_phase():
    x, h = grid.points(-10, 10, 128)
    k = grid.wavenumbers(128, h)
    psi0 = free_gaussian(x, 0.0, 0.0, 0.3, 1.0, 1.0)
    a = propagate.strang_step(psi0, np.full(128, 0.37), k, 1.0, 0.1)
    b = propagate.strang_step(psi0, np.zeros(128), k, 1.0, 0.1)
    assert np.max(np.abs(a - np.exp(-0.037j) * b)) < 1e-15


def _harmonic_run(dt, T=2 * math.pi, omega=1.0, m=1.0, a=2.0):
    x, h = grid.points(-12, 12, 256)
    k = grid.wavenumbers(256, h)
    s = math.sqrt(1.0 / (2 * m * omega))
    psi = (2 * math.pi * s * s) ** -0.25 * np.exp(-(x - a) ** 2 / (4 * s * s)) + 0j
    V = 0.5 * m * omega ** 2 * x * x
    n = int(round(T / dt))
    for _ in range(n):
        psi = propagate.strang_step(psi, V, k, m, dt)
    rho = np.abs(psi) ** 2
    return h * np.sum(x * rho), h * np.sum(x * x * rho) - (h * np.sum(x * rho)) ** 2, n * dt


def test_harmonic_coherent_state_second_order():
    """Centre follows a cos(wt) with constant width 1/(2 m w); Strang error O(dt^2)."""
    errs = []
    for dt in (0.1, 0.05, 0.025):
        mean, var, t = _harmonic_run(dt, T=3.0)
        errs.append(abs(mean - 2.0 * math.cos(t)) + abs(var - 0.5))
    assert errs[-1] < 5e-4
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def test_unitarity_over_2000_steps():
    """Per-CWF norm is conserved by every split-operator step, to roundoff: each
    step's FFT pair rounds at ~log2(n) u, so 2000 steps stay below 2000*9*u ~ 2e-12."""
    model = models.ShinMetiu()
    r, hr = grid.points(-75, 75, 512)
    k = grid.wavenumbers(512, hr)
    psi = np.exp(-(r + 5.0) ** 2 / 8.0 + 0.5j * r)
    psi = psi / grid.norm(psi, hr)
    V = model.W(r, -4.0)
    for _ in range(2000):
        psi = propagate.strang_step(psi, V, k, 1.0, 0.1)
    assert abs(grid.norm(psi, hr) - 1.0) < 1e-12


def test_kinetic_matrix_plane_waves():
    """T e^{ikx} = k^2/2m e^{ikx} for every grid wavenumber; T is real symmetric."""
    n, m = 64, 3.0
    x, h = grid.points(-4, 4, n)
    T = grid.kinetic_matrix(n, h, m)
    assert np.allclose(T, T.T, atol=1e-14)
    for kk in grid.wavenumbers(n, h)[[1, 5, 31, 40]]:
        f = np.exp(1j * kk * x)
        assert np.max(np.abs(T @ f - kk * kk / (2 * m) * f)) < 1e-11 * max(1, kk * kk)


def test_erf_over_x_limits():
    a = 5.0
    assert models.erf_over_x(0.0, a) == pytest.approx(2 / (math.sqrt(math.pi) * a), rel=1e-15)
    xs = np.array([1e-3, 0.3, 2.0, 17.0, -4.0])
    ref = np.array([math.erf(abs(v) / a) / abs(v) for v in xs])
    assert np.max(np.abs(models.erf_over_x(xs, a) - ref) / ref) < 1e-15
    # series and direct form agree across the switch point
    lo, hi = models.erf_over_x(np.array([a * 1e-4 * (1 - 1e-12), a * 1e-4 * (1 + 1e-12)]), a)
    assert abs(lo - hi) / hi < 1e-14
    # Coulomb tail
    assert models.erf_over_x(60.0, 3.1) == pytest.approx(1 / 60.0, rel=1e-15)


def test_shin_metiu_mirror_and_tails():
    """Mirror r,R -> -r,-R swaps the two ions; far from every charge the
    interaction is the bare Coulomb sum."""
    sm = models.ShinMetiu(19.0, 5.0, 3.1, 4.0)
    swapped = models.ShinMetiu(19.0, 5.0, 4.0, 3.1)
    r = np.linspace(-70, 70, 41)
    R = np.linspace(-8.9, 8.9, 17)
    assert np.allclose(sm.W(r[:, None], R[None, :]), swapped.W(-r[:, None], -R[None, :]),
                       rtol=0, atol=1e-14)
    rr, RR = 70.0, 1.0
    coulomb = 1 / abs(9.5 - RR) + 1 / abs(9.5 + RR) - 1 / abs(rr - RR) - 1 / abs(rr - 9.5) - 1 / abs(rr + 9.5)
    assert sm.W(rr, RR) == pytest.approx(coulomb, abs=1e-15)
    # an electron on top of the proton feels the finite erf limit, not a singularity
    assert np.isfinite(sm.W(1.25, 1.25))


def test_cavity_model_parts():
    cav = models.Cavity(1.0, 1.0, 0.1, 0.05)
    assert cav.W(0.0, 0.0) == pytest.approx(-1.0, abs=0)
    # bilinear in (x, q) after removing the single-coordinate parts
    x, q = 3.0, -7.0
    cross = cav.W(x, q) - cav.W(x, 0.0) - cav.W(0.0, q) + cav.W(0.0, 0.0)
    assert cross == pytest.approx(0.05 * x * q, rel=1e-14)
    assert cav.W(0.0, q) - cav.W(0.0, 0.0) == pytest.approx(0.5 * 0.01 * q * q, rel=1e-14)
    assert erf(1.0) > 0  # scipy present


# --------------------------------------------------------------------------- Crank-Nicolson

@pytest.mark.parametrize("m,h,dt", [(1.0, 0.3, 0.1), (1836.0, 0.07, 0.1), (0.5, 0.1, 0.4)])
def test_crank_nicolson_plane_waves_closed_form(m, h, dt):
    """e^{i k x_j} is an eigenvector of the periodic three-point second
    difference with eigenvalue -4 sin^2(k h/2)/h^2; with a constant V0 one CN
    step multiplies it by (1 - i w dt/2) / (1 + i w dt/2),
    w = 2 sin^2(k h / 2) / (m h^2) + V0."""
    n, V0 = 64, -0.37
    x = h * np.arange(n)
    for q in (0, 1, 5, n // 2 - 1, n // 2):
        kq = 2 * math.pi * q / (n * h)
        psi = np.exp(1j * kq * x)
        w = 2 * math.sin(kq * h / 2) ** 2 / (m * h * h) + V0
        got = propagate.crank_nicolson_step(psi[None, :], np.full((1, n), V0), h, m, dt)[0]
        ref = (1 - 0.5j * w * dt) / (1 + 0.5j * w * dt) * psi
        assert np.max(np.abs(got - ref)) < 1e-13, q


def test_crank_nicolson_is_unitary_for_any_potential(rng):
    n, h, m, dt = 128, 0.2, 1.0, 0.3
    V = 3.0 * rng.standard_normal((3, n))
    psi = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
    n0 = np.sum(np.abs(psi) ** 2, axis=1)
    for _ in range(200):
        psi = propagate.crank_nicolson_step(psi, V, h, m, dt)
    assert np.max(np.abs(np.sum(np.abs(psi) ** 2, axis=1) / n0 - 1)) < 1e-12


def test_crank_nicolson_harmonic_coherent_state_converges_in_h_and_dt():
    """Centre a cos(t), width 1/(2 m w): CN with the three-point Laplacian is
    second order in h and in dt; halving both quarters the error."""
    def run(n, dt, T=3.0, a=2.0):
        x, h = grid.points(-12, 12, n)
        psi = (math.pi) ** -0.25 * np.exp(-(x - a) ** 2 / 2) + 0j
        V = 0.5 * x * x
        for _ in range(int(round(T / dt))):
            psi = propagate.crank_nicolson_step(psi[None, :], V[None, :], h, 1.0, dt)[0]
        rho = np.abs(psi) ** 2
        mean = h * np.sum(x * rho)
        return abs(mean - a * math.cos(T)) + abs(h * np.sum(x * x * rho) - mean * mean - 0.5)
    e1, e2 = run(256, 0.025), run(512, 0.0125)     # coarser pairs are not yet asymptotic
    assert e2 < 3e-3
    assert 3.5 < e1 / e2 < 4.7
