"""Pins of the oracle's matrices (Eq. 9a-9d), K (Eq. 8) and the coefficient
solve: brute force over materialised 2D basis functions, the separable-W closed
form, a finite-difference check of Eq. 8 against the full TDSE, Hermiticity and
positivity, Sherman-Morrison on a rank-one S, and RK4's order against expm."""

import numpy as np
import pytest
from scipy.linalg import expm

from oracle import coeffs, grid, matrices, models, propagate


def _random_cwfs(rng, N, n, h):
    psi = rng.standard_normal((N, n)) + 1j * rng.standard_normal((N, n))
    return psi / grid.norm(psi, h)[:, None]


@pytest.fixture(scope="module")
def tiny(rng):
    model = models.ShinMetiu()
    r, hr = grid.points(-12.0, 12.0, 16)
    R, hR = grid.points(-4.0, 4.0, 8)
    N = 5
    psi1 = _random_cwfs(rng, N, 16, hr)
    psi2 = _random_cwfs(rng, N, 8, hR)
    r_traj = rng.uniform(-10, 10, N)
    R_traj = rng.uniform(-3.5, 3.5, N)
    return model, r, hr, R, hR, psi1, psi2, r_traj, R_traj


def test_matrices_equal_brute_force_2d(tiny):
    """<Phi_b| X |Phi_a> with Phi_a(r_i, R_j) = psi1^a_i psi2^a_j materialised on the
    product grid, X = 1, W(r,R), and W(r,R) - W(r,R^a) - W(r^a,R) (ket's trajectory)."""
    model, r, hr, R, hR, psi1, psi2, r_traj, R_traj = tiny
    N = psi1.shape[0]
    Phi = psi1[:, :, None] * psi2[:, None, :]                      # (N, n_r, n_R)
    Wfull = model.W(r[:, None], R[None, :])
    S_bf = np.empty((N, N), complex)
    W_bf = np.empty((N, N), complex)
    K_bf = np.empty((N, N), complex)
    for b in range(N):
        for a in range(N):
            w = np.conj(Phi[b]) * Phi[a]
            S_bf[b, a] = hr * hR * np.sum(w)
            W_bf[b, a] = hr * hR * np.sum(w * Wfull)
            X = Wfull - model.W(r[:, None], R_traj[a]) - model.W(r_traj[a], R[None, :])
            K_bf[b, a] = hr * hR * np.sum(w * X)
    S, _, _ = matrices.overlap_matrix(psi1, psi2, hr, hR)
    Wm = matrices.two_body(psi1, psi2, Wfull, hr, hR)
    _, K = matrices.coupling(psi1, psi2, model, r, R, hr, hR, r_traj, R_traj)
    scale = np.max(np.abs(W_bf))
    assert np.max(np.abs(S - S_bf)) < 1e-14
    assert np.max(np.abs(Wm - W_bf)) < 1e-14 * scale
    assert np.max(np.abs(K - K_bf)) < 1e-13 * scale


def test_hermitian_and_psd(tiny):
    model, r, hr, R, hR, psi1, psi2, r_traj, R_traj = tiny
    S, _, _ = matrices.overlap_matrix(psi1, psi2, hr, hR)
    Wm = matrices.two_body(psi1, psi2, model.W(r[:, None], R[None, :]), hr, hR)
    assert np.max(np.abs(S - S.conj().T)) < 1e-15
    assert np.max(np.abs(Wm - Wm.conj().T)) < 1e-14
    assert np.min(np.linalg.eigvalsh(S)) > -1e-14
    assert np.max(np.abs(np.diag(S) - 1.0)) < 1e-14


def test_separable_closed_form(tiny, rng):
    """W = f(r) + g(R): K[b,a] = -(f(r^a) + g(R^a)) S[b,a] exactly."""
    _, r, hr, R, hR, psi1, psi2, r_traj, R_traj = tiny

    def f(x):
        return np.cos(0.3 * x) + 0.01 * x * x

    def g(x):
        return 0.5 * x * x - 0.2 * x

    sep = models.Separable(f, g)
    S, K = matrices.coupling(psi1, psi2, sep, r, R, hr, hR, r_traj, R_traj)
    ref = -(f(r_traj) + g(R_traj))[None, :] * S
    assert np.max(np.abs(K - ref)) < 1e-13


def test_eq8_against_tdse_finite_difference(rng):
    """K[b,a] = <phi_b|(H - i d/dt) phi_a> with d/dt taken along the Hermitian-CWF
    propagation (central difference) and H the full 2D Hamiltonian (Eqs. 1-2)."""
    model = models.ShinMetiu()
    r, hr = grid.points(-10.0, 10.0, 32)
    R, hR = grid.points(-3.0, 3.0, 16)
    m_r, m_R = 1.0, 4.0
    N = 4
    psi1 = np.exp(-(r[None, :] - rng.uniform(-3, 3, (N, 1))) ** 2 / 4 + 1j * rng.uniform(-1, 1, (N, 1)) * r)
    psi2 = np.exp(-(R[None, :] - rng.uniform(-1, 1, (N, 1))) ** 2 + 1j * rng.uniform(-1, 1, (N, 1)) * R)
    psi1 /= grid.norm(psi1, hr)[:, None]
    psi2 /= grid.norm(psi2, hR)[:, None]
    r_traj = rng.uniform(-3, 3, N)
    R_traj = rng.uniform(-1, 1, N)
    dt = 1e-4

    def prop(d):
        return propagate.propagate_cwfs(psi1, psi2, model, r, R, hr, hR, m_r, m_R, r_traj, R_traj, d)

    p1f, p2f = prop(dt)
    p1b, p2b = prop(-dt)
    Phi = psi1[:, :, None] * psi2[:, None, :]
    dPhi = (p1f[:, :, None] * p2f[:, None, :] - p1b[:, :, None] * p2b[:, None, :]) / (2 * dt)
    kr = grid.wavenumbers(r.size, hr)[:, None]
    kR = grid.wavenumbers(R.size, hR)[None, :]
    Tk = kr ** 2 / (2 * m_r) + kR ** 2 / (2 * m_R)
    Wfull = model.W(r[:, None], R[None, :])
    HPhi = np.array([np.fft.ifft2(Tk * np.fft.fft2(P)) + Wfull * P for P in Phi])
    ref = hr * hR * np.einsum("bij,aij->ba", np.conj(Phi), HPhi - 1j * dPhi)
    _, K = matrices.coupling(psi1, psi2, model, r, R, hr, hR, r_traj, R_traj)
    assert np.max(np.abs(K - ref)) < 1e-6 * np.max(np.abs(K))
    # the transposed (bra-conditioned) reading is far off
    Kt = K.T
    assert np.max(np.abs(Kt - ref)) > 1e-3 * np.max(np.abs(K))


def test_rank_one_solve_sherman_morrison(rng):
    a = rng.standard_normal(6) + 1j * rng.standard_normal(6)
    b = rng.standard_normal(6) + 1j * rng.standard_normal(6)
    eps = 1e-3
    S = np.outer(a, a.conj())
    x = coeffs.initial_coefficients(S, b, eps)
    ref = (b - a * (a.conj() @ b) / (eps + np.vdot(a, a).real)) / eps
    assert np.max(np.abs(x - ref)) < 1e-10 * np.max(np.abs(ref))


def test_rk4_fourth_order_against_expm(rng):
    N = 5
    A = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    S = A @ A.conj().T / N + np.eye(N)
    K = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    C0 = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    eps, T = 1e-8, 1.0
    exact = expm(-1j * np.linalg.solve(S + eps * np.eye(N), K) * T) @ C0
    errs = []
    for n in (20, 40):
        C = C0.copy()
        for _ in range(n):
            C, _ = coeffs.rk4_step(C, S, K, S, K, eps, T / n)
        errs.append(np.max(np.abs(C - exact)))
    assert errs[1] < 1e-5
    assert 14 < errs[0] / errs[1] < 18


def test_linear_interpolation_in_rk4():
    """Time-dependent K: scalar dC/dt = -i k(t) C with k linear in t, fed to each
    step as its two end values; exact C = exp(-i (k0 t + k1 t^2 / 2)); the
    linear interpolation is exact here, so the error is RK4's, O(dt^4)."""
    k0, k1, T = 0.7, 1.3, 2.0
    S = np.ones((1, 1))
    errs = []
    for n in (10, 20):
        dt, C = T / n, np.array([1.0 + 0j])
        for k in range(n):
            C, _ = coeffs.rk4_step(C, S, np.array([[k0 + k1 * k * dt]]), S,
                                   np.array([[k0 + k1 * (k + 1) * dt]]), 0.0, dt)
        errs.append(abs(C[0] - np.exp(-1j * (k0 * T + 0.5 * k1 * T * T))))
    # RK4's phase error per step is ~(k dt)^5/120 with k dt up to 0.33 here
    assert errs[1] < 1e-3
    assert 14 < errs[0] / errs[1] < 18


def test_singular_without_regularisation_raises():
    S = np.ones((2, 2), complex)          # two identical basis functions
    with pytest.raises(coeffs.SolveError):
        coeffs.factor(S, 0.0)
    coeffs.factor(S, 1e-8)                # regularised: fine
