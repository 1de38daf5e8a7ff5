"""Observables of the ICWF ansatz (oracle).

The paper monitors the BO populations P_n(t), the reduced nuclear density
rho(R, t) = int dr |Psi|^2 and the decoherence indicator
D_nm(t) = int dR |chi^(n)(R,t)|^2 |chi^(m)(R,t)|^2 (text around the Shin-Metiu
figure), with chi^(n)(R,t) = <phi_n(.;R)|Psi(.,R,t)>_r the projection on the
n-th BO electronic state.  Their discrete formulas are not printed (the
appendix is missing); the ones below are the definitions evaluated on the
ansatz Psi = sum_a C_a psi_1^a psi_2^a (Eq. 7) with grid quadrature:

    norm      = C^H S C
    rho(R_j)  = sum_{b,a} conj(C_b psi_2^b_j) <psi_1^b|psi_1^a> C_a psi_2^a_j
    rho(r_i)  = sum_{b,a} conj(C_b psi_1^b_i) <psi_2^b|psi_2^a> C_a psi_1^a_i
    chi^(n)_j = sum_a C_a psi_2^a_j <phi_n(.;R_j)|psi_1^a>
    P_n       = hR sum_j |chi^(n)_j|^2           (not divided by the norm)
    D_nm      = hR sum_j |chi^(n)_j|^2 |chi^(m)_j|^2
"""

import numpy as np

from .matrices import overlap


def norm(C, S):
    return float(np.real(np.conj(C) @ S @ C))


def densities(C, psi1, psi2, hr, hR):
    """(rho_r[n_r], rho_R[n_R])."""
    S1 = overlap(psi1, hr)
    S2 = overlap(psi2, hR)
    u2 = C[:, None] * psi2           # C_a psi_2^a_j
    u1 = C[:, None] * psi1
    rho_R = np.real(np.sum(np.conj(u2) * (S1 @ u2), axis=0))
    rho_r = np.real(np.sum(np.conj(u1) * (S2 @ u1), axis=0))
    return rho_r, rho_R


def bo_projections(C, psi1, psi2, bo, hr):
    """chi[n, j] = sum_a C_a psi_2^a_j <phi_n(.;R_j)|psi_1^a>; bo[j, n, i] real."""
    proj = hr * np.einsum("jni,ai->nja", bo, psi1)     # <phi_n(.;R_j)|psi_1^a>
    return np.einsum("nja,a,aj->nj", proj, C, psi2)


def populations(chi, hR):
    """P_n = hR sum_j |chi^(n)_j|^2 and D_nm = hR sum_j |chi^(n)_j|^2 |chi^(m)_j|^2."""
    dens = np.abs(chi) ** 2
    P = hR * np.sum(dens, axis=1)
    D = hR * dens @ dens.T
    return P, D
