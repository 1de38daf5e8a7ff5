"""Brute-force propagation of the full 2D wavefunction (oracle; tiny grids only).

Eq. 1 with Eq. 2 (A_j = 0) on the product grid: Psi[i, j] = Psi(r_i, R_j), the
same Strang split operator as the CWF propagator but in two dimensions,

    Psi <- exp(-i W dt/2) Psi
    Psi <- IFFT2[ exp(-i (k_r^2/2m_r + k_R^2/2m_R) dt) FFT2 Psi ]
    Psi <- exp(-i W dt/2) Psi.

This is what the ICWF method avoids storing; here it pins the ICWF oracle on
grids small enough for the full wavefunction.
"""

import numpy as np

from . import grid


def propagate(Psi, Wtab, hr, hR, m_r, m_R, dt, n_steps):
    kr = grid.wavenumbers(Psi.shape[0], hr)
    kR = grid.wavenumbers(Psi.shape[1], hR)
    kin = np.exp(-1j * dt * (kr[:, None] ** 2 / (2 * m_r) + kR[None, :] ** 2 / (2 * m_R)))
    half = np.exp(-0.5j * dt * Wtab)
    for _ in range(n_steps):
        Psi = half * np.fft.ifft2(kin * np.fft.fft2(half * Psi))
    return Psi


def reduced_density_R(Psi, hr):
    """rho(R_j) = int dr |Psi(r, R_j)|^2."""
    return hr * np.sum(np.abs(Psi) ** 2, axis=0)


def reduced_density_r(Psi, hR):
    return hR * np.sum(np.abs(Psi) ** 2, axis=1)
