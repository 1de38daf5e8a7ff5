"""Test helpers: run the oracle on a seeded workload and compare results.

Only tests import this module; it calls the oracle and the input generator,
never the HIP library."""

import numpy as np

from oracle import icwf as oicwf
from oracle import models


def setup_for(wl, dt=None):
    kind = "shin_metiu" if wl.model == 1 else "cavity"
    return oicwf.Setup(models.make(kind, wl.model_params), wl.r_min, wl.r_max, wl.n_r, wl.R_min, wl.R_max,
                       wl.n_R, wl.m_r, wl.m_R, wl.dt if dt is None else dt, wl.eps)


def init_for(setup, wl, C0=None):
    if C0 is None and "C0" in wl.extra:
        C0 = wl.extra["C0"]
    if C0 is not None:
        return oicwf.init(setup, wl.r0, wl.R0, wl.psi1, wl.psi2, C0=C0)
    return oicwf.init(setup, wl.r0, wl.R0, wl.psi1, wl.psi2, b0=wl.b0)


def wc_table(setup):
    """W_c(r_i, R_j): the coupling part of the model interaction, W minus its
    one-coordinate parts (Shin-Metiu: the electron-proton term; cavity: lam q x)."""
    m = setup.model
    if m.kind == "shin_metiu":
        return -models.erf_over_x(setup.r[:, None] - setup.R[None, :], m.R_f)
    return m.lam * setup.r[:, None] * setup.R[None, :]


def rel_max(a, b):
    """max |a - b| / max |b|."""
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def s_norm_diff(C1, C2, S):
    """||Phi (C1 - C2)|| = sqrt((C1-C2)^H S (C1-C2)): the difference of the two
    ansatz wavefunctions; raw C is not unique when S is near singular."""
    d = np.asarray(C1) - np.asarray(C2)
    return float(np.sqrt(abs(np.real(np.conj(d) @ S @ d))))
