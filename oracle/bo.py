"""Born-Oppenheimer electronic states on the grid (oracle).

The paper's observables (BO populations and the decoherence indicator, text
around the Shin-Metiu figure) project the wavefunction on the electronic
eigenstates phi_n(r; R) of h_e(R) = T_1 + W(r, R) at fixed R.  On the grid,
h_e(R_j) = T_spec + diag(W(r_i, R_j)), with T_spec the same spectral kinetic
operator the propagator uses.  Eigenvectors are real; each is normalised on the
grid (h sum phi^2 = 1).  The sign of each eigenvector is arbitrary and no
observable depends on it.
"""

import numpy as np
from scipy.linalg import eigh

from . import grid


def bo_states(model, r, hr, m_r, R_values, n_states):
    """phi[j, n, i] = phi_n(r_i; R_j) for the n_states lowest states, and energies[j, n]."""
    T = grid.kinetic_matrix(r.size, hr, m_r)
    R_values = np.atleast_1d(np.asarray(R_values, dtype=np.float64))
    phi = np.empty((R_values.size, n_states, r.size))
    energies = np.empty((R_values.size, n_states))
    for j, Rj in enumerate(R_values):
        h = T + np.diag(model.W(r, Rj))
        w, v = eigh(h, subset_by_index=[0, n_states - 1])
        phi[j] = (v / np.sqrt(hr)).T
        energies[j] = w
    return phi, energies
