"""The seeded input generator builds the start the recipe describes: the
electronic factor is eigenvector 1 of h_e(R_0) (checked with the oracle's own
kinetic operator and model), the CWFs are unit-norm slices of Psi_0, b0 is
their projection on Psi_0, the BO states are orthonormal eigenvectors, and the
same seed gives the same ensemble."""

import numpy as np

from oracle import grid, models
from paper_1805_11169_amd import inputs


def test_initial_electronic_state_is_eigenvector_one():
    wl = inputs.shin_metiu(8, n_r=128, n_R=64, r_box=(-40.0, 40.0), n_bo=3)
    r, hr = grid.points(wl.r_min, wl.r_max, wl.n_r)
    h = grid.kinetic_matrix(wl.n_r, hr, 1.0) + np.diag(models.ShinMetiu(*wl.model_params).W(r, -4.0))
    phi = wl.extra["phi_e"]
    e = hr * phi @ h @ phi
    assert np.max(np.abs(h @ phi - e * phi)) < 1e-10
    w = np.linalg.eigvalsh(h)
    assert abs(e - w[1]) < 1e-10


def test_cwfs_b0_and_bo_states():
    wl = inputs.shin_metiu(16, n_r=128, n_R=64, r_box=(-40.0, 40.0), n_bo=3, seed=4)
    r, hr = grid.points(wl.r_min, wl.r_max, wl.n_r)
    R, hR = grid.points(wl.R_min, wl.R_max, wl.n_R)
    assert np.allclose(grid.norm(wl.psi1, hr), 1.0, atol=1e-14)
    assert np.allclose(grid.norm(wl.psi2, hR), 1.0, atol=1e-14)
    Psi0 = np.outer(wl.extra["phi_e"], wl.extra["chi0"])
    b = hr * hR * np.einsum("ai,aj,ij->a", wl.psi1.conj(), wl.psi2.conj(), Psi0)
    assert np.max(np.abs(b - wl.b0)) < 1e-13
    G = hr * np.einsum("jni,jmi->jnm", wl.bo, wl.bo)
    assert np.max(np.abs(G - np.eye(3)[None])) < 1e-12
    # the sampled electrons sit where |phi_e|^2 lives, the protons around R_0
    assert abs(np.mean(wl.R0) + 4.0) < 3 * 0.38 / np.sqrt(16) * 2


def test_seed_reproducible_and_distinct():
    a = inputs.shin_metiu(32, n_r=64, n_R=32, r_box=(-40.0, 40.0), n_bo=0, seed=11)
    b = inputs.shin_metiu(32, n_r=64, n_R=32, r_box=(-40.0, 40.0), n_bo=0, seed=11)
    c = inputs.shin_metiu(32, n_r=64, n_R=32, r_box=(-40.0, 40.0), n_bo=0, seed=12)
    assert np.array_equal(a.r0, b.r0) and np.array_equal(a.R0, b.R0)
    assert not np.array_equal(a.R0, c.R0)


def test_cavity_start():
    wl = inputs.cavity(8, n_r=128, n_R=64, n_bo=2)
    x, hx = grid.points(wl.r_min, wl.r_max, wl.n_r)
    q, hq = grid.points(wl.R_min, wl.R_max, wl.n_R)
    h = grid.kinetic_matrix(wl.n_r, hx, 1.0) + np.diag(-1.0 / np.sqrt(x * x + 1.0))
    phi = wl.extra["phi_e"]
    e = hx * phi @ h @ phi
    assert abs(e - np.linalg.eigvalsh(h)[1]) < 1e-10
    chi = wl.extra["chi0"]
    assert abs(hq * np.sum(q * q * chi * chi) - 1.0 / (2 * 0.1)) < 1e-6
