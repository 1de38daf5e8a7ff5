"""Coefficient equation of motion, Eq. 8 (oracle).

i S dC/dt = K C with K = W - W1 - W2.  S is singular whenever two basis
functions coincide (at t = 0 every configured start is a product state, so S
has rank one), so the solve is Tikhonov-regularised: (S + eps I) x = y with
eps absolute on unit-norm CWFs, by Cholesky (scipy ``cho_factor``).

Integrator (reading taken; the paper does not state one): classical RK4 over
one step [t_k, t_k+1] of dC/dt = -i (S(t) + eps I)^-1 K(t) C, with S and K
linear in time between the step's end points (so the midpoint value is the
average of the two ends).
"""

import numpy as np
from scipy.linalg import cho_factor, cho_solve


class SolveError(RuntimeError):
    """S + eps I is not numerically positive definite."""


def factor(S, eps):
    """Cholesky factor of S + eps I."""
    A = S + eps * np.eye(S.shape[0])
    try:
        return cho_factor(A, lower=True, check_finite=True)
    except np.linalg.LinAlgError as exc:  # not positive definite
        raise SolveError(str(exc)) from exc


def rhs(fac, K, C):
    """dC/dt = -i (S + eps I)^-1 K C for a factor of S + eps I."""
    return -1j * cho_solve(fac, K @ C)


def rk4_step(C, S0, K0, S1, K1, eps, dt, fac0=None):
    """One RK4 step with S, K linear between (S0, K0) at t_k and (S1, K1) at t_k + dt.

    Returns (C_next, fac1) where fac1 is the factor of S1 + eps I (reusable as
    the next step's fac0 when the next step starts from the same S).
    """
    f0 = factor(S0, eps) if fac0 is None else fac0
    fm = factor(0.5 * (S0 + S1), eps)
    f1 = factor(S1, eps)
    Km = 0.5 * (K0 + K1)
    k1 = rhs(f0, K0, C)
    k2 = rhs(fm, Km, C + 0.5 * dt * k1)
    k3 = rhs(fm, Km, C + 0.5 * dt * k2)
    k4 = rhs(f1, K1, C + dt * k3)
    return C + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4), f1


def initial_coefficients(S0, b, eps):
    """C_0 = (S_0 + eps I)^-1 b, the regularised projection of Psi_0 on the basis."""
    return cho_solve(factor(S0, eps), b)
