"""Bohmian velocities of the ICWF ansatz (Eqs. 10-11; oracle).

Readings taken where the printed equations are ambiguous:
* Eqs. 10-11 use the same letter for the summation index and the trajectory;
  the sum runs over all basis functions b and is evaluated at trajectory a's
  position -- the de Broglie-Bohm velocity of the full ansatz wavefunction.
* The printed equations omit the masses; the velocity is Im(grad Psi / Psi)/m
  (hbar = 1), the standard de Broglie-Bohm guidance law the paper invokes.

    Psi_a  = sum_b C_b psi_1^b(r^a) psi_2^b(R^a)
    v_r^a  = Im[ sum_b C_b psi_2^b(R^a) d_r psi_1^b(r^a) / Psi_a ] / m_r
    v_R^a  = Im[ sum_b C_b psi_1^b(r^a) d_R psi_2^b(R^a) / Psi_a ] / m_R

CWF values at off-grid positions use the trigonometric interpolant.
"""

import numpy as np

from .interp import trig_interp


class NodeError(RuntimeError):
    """|Psi| at a trajectory underflows: the velocity is undefined."""


NODE_THRESHOLD = 1e-300


def velocities(C, psi1, psi2, r_min, hr, R_min, hR, m_r, m_R, r_traj, R_traj):
    """(v_r, v_R, Psi_at_traj) for every trajectory."""
    f1, d1 = trig_interp(psi1, r_min, hr, r_traj)   # (N_traj, N_basis)
    f2, d2 = trig_interp(psi2, R_min, hR, R_traj)
    psi_at = (f1 * f2) @ C
    if np.any(np.abs(psi_at) < NODE_THRESHOLD):
        raise NodeError("trajectory at a node of the ansatz wavefunction")
    v_r = np.imag(((d1 * f2) @ C) / psi_at) / m_r
    v_R = np.imag(((f1 * d2) @ C) / psi_at) / m_R
    return v_r, v_R, psi_at
