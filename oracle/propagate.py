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


def crank_nicolson_step(psi, V, h, m, dt):
    """One Crank-Nicolson step of the same equation on the periodic grid,
    (1 + i dt/2 H) psi_new = (1 - i dt/2 H) psi, with H = -(1/2m) D2 + V and D2
    the periodic three-point second difference (f_{i-1} - 2 f_i + f_{i+1}) / h^2:
    the Cayley transform of a Hermitian H, unitary for any dt.  The other
    standard propagator for these equations (the paper names none); dense
    solves, small grids only.

    psi: (N, n) complex; V: (N, n) real, one potential per row."""
    psi = np.atleast_2d(psi)
    V = np.broadcast_to(V, psi.shape)
    n = psi.shape[-1]
    eye = np.eye(n)
    D2 = (np.roll(eye, 1, axis=1) + np.roll(eye, -1, axis=1) - 2.0 * eye) / (h * h)
    H = -D2 / (2.0 * m) + V[:, :, None] * eye[None, :, :]
    A = eye[None] + 0.5j * dt * H
    B = eye[None] - 0.5j * dt * H
    rhs = np.einsum("aij,aj->ai", B, psi)
    return np.linalg.solve(A, rhs[:, :, None])[:, :, 0]


def electronic_potentials(model, r, R_traj):
    """V_1^a(r_i) = W(r_i, R^a) for every trajectory a: shape (N, n_r)."""
    return model.W(r[None, :], np.asarray(R_traj)[:, None])


def nuclear_potentials(model, R, r_traj):
    """V_2^a(R_j) = W(r^a, R_j) for every trajectory a: shape (N, n_R)."""
    return model.W(np.asarray(r_traj)[:, None], R[None, :])


def propagate_cwfs(psi1, psi2, model, r, R, hr, hR, m_r, m_R, r_traj, R_traj, dt, propagator="strang"):
    """Advance all CWFs by dt, conditioning frozen at (r_traj, R_traj) (Eqs. 5-6, eta dropped),
    by the split operator ("strang") or Crank-Nicolson ("cn")."""
    V1 = electronic_potentials(model, r, R_traj)
    V2 = nuclear_potentials(model, R, r_traj)
    if propagator == "cn":
        return crank_nicolson_step(psi1, V1, hr, m_r, dt), crank_nicolson_step(psi2, V2, hR, m_R, dt)
    kr = grid.wavenumbers(r.size, hr)
    kR = grid.wavenumbers(R.size, hR)
    return strang_step(psi1, V1, kr, m_r, dt), strang_step(psi2, V2, kR, m_R, dt)
