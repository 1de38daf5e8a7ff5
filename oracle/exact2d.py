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


def bo_projections(Psi, bo, hr):
    """chi[n, j] = <phi_n(.; R_j)|Psi(., R_j)>_r = hr sum_i phi_n(r_i; R_j) Psi(r_i, R_j)
    (real BO states bo[j, n, i]), the projection the paper's populations use."""
    return hr * np.einsum("jni,ij->nj", bo, Psi)


def observables(Psi, hr, hR, bo=None):
    """norm, rho_r, rho_R and, with BO states, P_n and D_nm of a wavefunction on
    the grid, with the same definitions as the ansatz's observables."""
    rho_r = reduced_density_r(Psi, hR)
    rho_R = reduced_density_R(Psi, hr)
    out = dict(norm=float(hr * np.sum(rho_r)), rho_r=rho_r, rho_R=rho_R)
    if bo is not None:
        dens = np.abs(bo_projections(Psi, bo, hr)) ** 2
        out["pop"] = hR * np.sum(dens, axis=1)
        out["D"] = hR * dens @ dens.T
    return out
