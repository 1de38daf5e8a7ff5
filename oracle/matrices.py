"""The ICWF matrices of Eq. 9a-9d and the coupling K of Eq. 8 (oracle).

Index reading.  Eq. 8 comes from inserting the ansatz (Eq. 7),
Psi = sum_a C_a psi_1^a psi_2^a, into the TDSE (Eq. 1) and projecting onto each
basis function.  Using the Hermitian-CWF equations of motion (Eqs. 5-6, eta
dropped), (H - i d/dt) acting on phi_a = psi_1^a psi_2^a leaves only
W(r,R) - W(r,R^a) - W(r^a,R) times phi_a: the kinetic terms cancel.  So the row
index is the BRA b (the conjugated function), the column is the KET a, and the
conditioning coordinate of W_1 and W_2 belongs to the ket:

    S[b,a]  = <psi_1^b|psi_1^a> <psi_2^b|psi_2^a>                     (9a)
    W[b,a]  = <psi_1^b psi_2^b| W(r,R) |psi_1^a psi_2^a>              (9b)
    W1[b,a] = <psi_1^b| W(r, R^a) |psi_1^a> <psi_2^b|psi_2^a>         (9c)
    W2[b,a] = <psi_1^b|psi_1^a> <psi_2^b| W(r^a, R) |psi_2^a>         (9d)
    K = W - W1 - W2                                                   (8)

Every integral is the grid quadrature h * sum, with the FULL interaction W.
"""

import numpy as np


def overlap(psi, h):
    """Single-species overlap O[b, a] = h sum_i conj(psi^b_i) psi^a_i."""
    return h * (np.conj(psi) @ psi.T)


def overlap_matrix(psi1, psi2, hr, hR):
    """Eq. 9a: S = S_1 * S_2 (elementwise), and the two factors."""
    S1 = overlap(psi1, hr)
    S2 = overlap(psi2, hR)
    return S1 * S2, S1, S2


def two_body(psi1, psi2, Wtab, hr, hR):
    """Eq. 9b: W[b,a] = hr hR sum_{i,j} conj(psi1^b_i) psi1^a_i W(r_i,R_j) conj(psi2^b_j) psi2^a_j.

    Wtab[i, j] = W(r_i, R_j).  Row by row over the bra b: for fixed b the
    r-sum is a product with the table, then the R-sum is a weighted dot product.
    """
    N = psi1.shape[0]
    out = np.empty((N, N), dtype=np.complex128)
    for b in range(N):
        a1 = np.conj(psi1[b])[None, :] * psi1          # (N, n_r): conj(psi1^b_i) psi1^a_i
        t = np.ascontiguousarray(a1.real) @ Wtab + 1j * (np.ascontiguousarray(a1.imag) @ Wtab)
        a2 = np.conj(psi2[b])[None, :] * psi2           # (N, n_R)
        out[b] = np.sum(a2 * t, axis=1)
    return hr * hR * out


def conditioned_1(psi1, Vcond, hr):
    """<psi_1^b| W(r, R^a) |psi_1^a> with Vcond[a, i] = W(r_i, R^a) (the r-factor of Eq. 9c)."""
    return hr * (np.conj(psi1) @ (Vcond * psi1).T)


def conditioned_2(psi2, Vcond, hR):
    """<psi_2^b| W(r^a, R) |psi_2^a> with Vcond[a, j] = W(r^a, R_j) (the R-factor of Eq. 9d)."""
    return hR * (np.conj(psi2) @ (Vcond * psi2).T)


def couplings(psi1, psi2, model, r, R, hr, hR, conditionings, Wtab=None):
    """S (Eq. 9a) and K = W - W1 - W2 (Eq. 8) at CWFs (psi1, psi2), once per conditioning.

    conditionings: list of (r_traj, R_traj) pairs.  W (Eq. 9b) does not depend
    on the trajectories and is computed once.  All terms use the full W.
    Returns (S, [K for each conditioning]).
    """
    if Wtab is None:
        Wtab = model.W(r[:, None], R[None, :])
    S, S1, S2 = overlap_matrix(psi1, psi2, hr, hR)
    Wm = two_body(psi1, psi2, Wtab, hr, hR)
    Ks = []
    for r_traj, R_traj in conditionings:
        V1 = model.W(r[None, :], np.asarray(R_traj)[:, None])   # (N, n_r): W(r_i, R^a)
        V2 = model.W(np.asarray(r_traj)[:, None], R[None, :])   # (N, n_R): W(r^a, R_j)
        W1 = conditioned_1(psi1, V1, hr) * S2
        W2 = S1 * conditioned_2(psi2, V2, hR)
        Ks.append(Wm - W1 - W2)
    return S, Ks


def coupling(psi1, psi2, model, r, R, hr, hR, r_traj, R_traj, Wtab=None):
    """(S, K) at CWFs (psi1, psi2) and one conditioning (r_traj, R_traj)."""
    S, (K,) = couplings(psi1, psi2, model, r, R, hr, hR, [(r_traj, R_traj)], Wtab)
    return S, K
