"""Hermitian-CWF propagation (oracle; test infrastructure only).

Eqs. 5-6 with the complex potentials eta reduced to a pure time-dependent
phase and dropped (the Hermitian limit the paper takes): every electronic CWF
obeys i d/dt psi_1^a = (T_1 + W(r, R^a)) psi_1^a and every nuclear (photonic)
CWF obeys i d/dt psi_2^a = (T_2 + W(r^a, R)) psi_2^a -- independent
single-species problems, each with its own conditioning coordinate.

The paper does not state its propagator.  Reading taken: Strang split operator
with a spectral kinetic term on the periodic grid,

    psi <- exp(-i V dt/2) psi
    psi <- IFFT[ exp(-i k^2 dt / 2m) FFT psi ]
    psi <- exp(-i V dt/2) psi,

with the conditioning coordinate frozen at its value at the start of the step.
"""

import numpy as np

from . import grid


def strang_step(psi, V, k, m, dt):
    """One Strang step of i psi' = (-(1/2m) d^2/dx^2 + V) psi for each row of psi.

    psi: (..., n) complex; V: potential broadcast to psi's shape; k: wavenumbers.
    """
    half = np.exp(-0.5j * dt * V)
    out = half * psi
    out = np.fft.ifft(np.exp(-0.5j * dt * k * k / m) * np.fft.fft(out, axis=-1), axis=-1)
    return half * out


def electronic_potentials(model, r, R_traj):
    """V_1^a(r_i) = W(r_i, R^a) for every trajectory a: shape (N, n_r)."""
    return model.W(r[None, :], np.asarray(R_traj)[:, None])


def nuclear_potentials(model, R, r_traj):
    """V_2^a(R_j) = W(r^a, R_j) for every trajectory a: shape (N, n_R)."""
    return model.W(np.asarray(r_traj)[:, None], R[None, :])


def propagate_cwfs(psi1, psi2, model, r, R, hr, hR, m_r, m_R, r_traj, R_traj, dt):
    """Advance all CWFs by dt, conditioning frozen at (r_traj, R_traj) (Eqs. 5-6, eta dropped)."""
    kr = grid.wavenumbers(r.size, hr)
    kR = grid.wavenumbers(R.size, hR)
    p1 = strang_step(psi1, electronic_potentials(model, r, R_traj), kr, m_r, dt)
    p2 = strang_step(psi2, nuclear_potentials(model, R, r_traj), kR, m_R, dt)
    return p1, p2
