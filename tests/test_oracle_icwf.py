"""End-to-end pins of the ICWF oracle: exact recovery of a product state under a
separable W (closed-form coherent states and Bohmian paths), equality with
brute-force 2D propagation when the basis spans the whole grid space, the 2D
propagator's own closed forms, conservation laws, completeness of the BO
populations, the decoherence indicator of a product state, and gauge /
permutation invariance of every observable."""

import math

import numpy as np
import pytest

from oracle import bo, exact2d, grid, icwf, models, observables, propagate


# --------------------------------------------------------------------------- 2D propagator pins

def test_exact2d_separable_is_tensor_product(rng):
    r, hr = grid.points(-8, 8, 32)
    R, hR = grid.points(-4, 4, 16)
    f = 0.3 * r * r
    g = 0.7 * R * R + 0.1 * R
    phi = np.exp(-(r - 1) ** 2 + 0.4j * r)
    chi = np.exp(-(R + 0.5) ** 2 * 2)
    Psi = exact2d.propagate(np.outer(phi, chi), f[:, None] + g[None, :], hr, hR, 1.0, 3.0, 0.05, 30)
    kr, kR = grid.wavenumbers(32, hr), grid.wavenumbers(16, hR)
    for _ in range(30):
        phi = propagate.strang_step(phi, f, kr, 1.0, 0.05)
        chi = propagate.strang_step(chi, g, kR, 3.0, 0.05)
    assert np.max(np.abs(Psi - np.outer(phi, chi))) < 1e-13


def _coupled_centroids(dt, kappa=0.4, T=2.0):
    r, hr = grid.points(-10, 10, 64)
    R, hR = grid.points(-10, 10, 64)
    Wtab = 0.5 * (r[:, None] ** 2 + R[None, :] ** 2) + kappa * r[:, None] * R[None, :]
    Psi = np.exp(-0.5 * (r[:, None] - 1.5) ** 2 - 0.5 * (R[None, :] + 0.5) ** 2) + 0j
    Psi = exact2d.propagate(Psi, Wtab, hr, hR, 1.0, 1.0, dt, int(round(T / dt)))
    rho = np.abs(Psi) ** 2
    nrm = hr * hR * rho.sum()
    return hr * hR * np.sum(r[:, None] * rho) / nrm, hr * hR * np.sum(R[None, :] * rho) / nrm


def test_exact2d_coupled_oscillators_follow_classical_normal_modes():
    """Quadratic H: centroids obey r'' = -r - k R, R'' = -R - k r exactly (Ehrenfest)."""
    kappa, T = 0.4, 2.0
    u0, v0 = (1.5 - 0.5) / math.sqrt(2), (1.5 + 0.5) / math.sqrt(2)
    u = u0 * math.cos(math.sqrt(1 + kappa) * T)
    v = v0 * math.cos(math.sqrt(1 - kappa) * T)
    r_ex, R_ex = (u + v) / math.sqrt(2), (u - v) / math.sqrt(2)
    errs = []
    for dt in (0.1, 0.05):
        rc, Rc = _coupled_centroids(dt, kappa, T)
        errs.append(abs(rc - r_ex) + abs(Rc - R_ex))
    assert errs[1] < 2e-3
    assert 3.5 < errs[0] / errs[1] < 4.5


def test_exact2d_observables_equal_the_ansatz_formulas(rng):
    """On Psi = sum_a C_a psi1^a psi2^a (Eq. 7 on the grid) the grid sums of
    the exact propagator's observables equal the overlap-based formulas of
    the ansatz, an independent way of writing the same integrals."""
    n_r, n_R, N, n_bo = 32, 16, 5, 3
    r, hr = grid.points(-6, 6, n_r)
    R, hR = grid.points(-3, 3, n_R)
    psi1 = rng.standard_normal((N, n_r)) + 1j * rng.standard_normal((N, n_r))
    psi2 = rng.standard_normal((N, n_R)) + 1j * rng.standard_normal((N, n_R))
    C = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    Psi = np.einsum("a,ai,aj->ij", C, psi1, psi2)
    basis = np.linalg.qr(rng.standard_normal((n_r, n_r)))[0] / np.sqrt(hr)
    bo_states = np.stack([basis[:, :n_bo].T * (1 + 0.1 * j) for j in range(n_R)])
    got = exact2d.observables(Psi, hr, hR, bo_states)
    S = (hr * np.conj(psi1) @ psi1.T) * (hR * np.conj(psi2) @ psi2.T)
    rho_r, rho_R = observables.densities(C, psi1, psi2, hr, hR)
    chi = observables.bo_projections(C, psi1, psi2, bo_states, hr)
    P, D = observables.populations(chi, hR)
    ref = dict(norm=observables.norm(C, S), rho_r=rho_r, rho_R=rho_R, pop=P, D=D)
    for key, v in ref.items():
        assert np.max(np.abs(got[key] - v)) < 1e-12 * np.max(np.abs(v)), key


def test_exact2d_populations_over_a_complete_basis_sum_to_the_norm(rng):
    n_r, n_R = 32, 16
    r, hr = grid.points(-6, 6, n_r)
    R, hR = grid.points(-3, 3, n_R)
    Psi = rng.standard_normal((n_r, n_R)) + 1j * rng.standard_normal((n_r, n_R))
    # a different orthonormal basis of the r grid at every R_j
    bo_states = np.stack([np.linalg.qr(rng.standard_normal((n_r, n_r)))[0].T / np.sqrt(hr) for _ in range(n_R)])
    got = exact2d.observables(Psi, hr, hR, bo_states)
    assert abs(np.sum(got["pop"]) - got["norm"]) < 1e-12 * got["norm"]
    assert abs(np.sum(got["rho_R"]) * hR - got["norm"]) < 1e-12 * got["norm"]


# --------------------------------------------------------------------------- product-state recovery

def _harmonic_product_run(dt, T=2.0, N=12, seed=3):
    wr, mR, wR, ar, aR = 0.5, 20.0, 0.3, 1.5, 0.4
    model = models.Separable(lambda r: 0.5 * wr ** 2 * r * r, lambda R: 0.5 * mR * wR ** 2 * R * R)
    setup = icwf.Setup(model, -16.0, 16.0, 128, -3.0, 3.0, 64, 1.0, mR, dt, 1e-8)
    sr, sR = math.sqrt(1 / (2 * wr)), math.sqrt(1 / (2 * mR * wR))

    def phi(x):
        return (2 * math.pi * sr * sr) ** -0.25 * np.exp(-(x - ar) ** 2 / (4 * sr * sr))

    def chi(x):
        return (2 * math.pi * sR * sR) ** -0.25 * np.exp(-(x - aR) ** 2 / (4 * sR * sR))

    rng = np.random.default_rng(seed)
    r0 = rng.normal(ar, sr, N)
    R0 = rng.normal(aR, sR, N)
    p1 = np.repeat(phi(setup.r)[None, :] + 0j, N, axis=0)
    p2 = np.repeat(chi(setup.R)[None, :] + 0j, N, axis=0)
    p1 /= grid.norm(p1, setup.hr)[:, None]
    p2 /= grid.norm(p2, setup.hR)[:, None]
    b = grid.inner(p1, phi(setup.r), setup.hr) * grid.inner(p2, chi(setup.R), setup.hR)
    st = icwf.init(setup, r0, R0, p1, p2, b0=b)
    st, hist = icwf.run(setup, st, int(round(T / dt)))
    t = st.t
    rho_R_ex = chi(setup.R - aR * (math.cos(wR * t) - 1)) ** 2
    rho_r_ex = phi(setup.r - ar * (math.cos(wr * t) - 1)) ** 2
    traj_r_ex = r0 + ar * (math.cos(wr * t) - 1)
    traj_R_ex = R0 + aR * (math.cos(wR * t) - 1)
    return hist[-1], rho_r_ex, rho_R_ex, traj_r_ex, traj_R_ex, setup


def test_product_state_recovery_under_separable_w():
    """W = f(r) + g(R), Psi_0 = phi chi: ICWF gives Psi(t) = A phi(t) chi(t).  The
    basis stays rank one (every CWF is phi chi times its own phase), so |A|^2 =
    C^H S C is conserved up to the O(dt^2) error of interpolating S, K linearly
    over a step; the reduced densities are the 1D coherent-state densities
    (O(dt^2)) and every trajectory moves rigidly with the classical centre
    (explicit Euler, O(dt))."""
    o1, rr1, rR1, tr1, tR1, _ = _harmonic_product_run(0.02)
    o2, rr2, rR2, tr2, tR2, _ = _harmonic_product_run(0.01)
    n1, n2 = abs(o1["norm"] - 1.0), abs(o2["norm"] - 1.0)
    assert n1 < 1e-5 and n1 / n2 > 3.5
    d1 = np.max(np.abs(o1["rho_R"] - o1["norm"] * rR1)) / np.max(rR1)
    d2 = np.max(np.abs(o2["rho_R"] - o2["norm"] * rR2)) / np.max(rR2)
    assert d1 < 3e-6 and 3.5 < d1 / d2 < 4.5
    d1 = np.max(np.abs(o1["rho_r"] - o1["norm"] * rr1)) / np.max(rr1)
    d2 = np.max(np.abs(o2["rho_r"] - o2["norm"] * rr2)) / np.max(rr2)
    assert d1 < 2e-5 and 3.5 < d1 / d2 < 4.5
    e1 = np.max(np.abs(o1["r"] - tr1)) + np.max(np.abs(o1["R"] - tR1))
    e2 = np.max(np.abs(o2["r"] - tr2)) + np.max(np.abs(o2["R"] - tR2))
    assert e1 < 2e-2
    assert 1.8 < e1 / e2 < 2.2


# --------------------------------------------------------------------------- full-span exactness

def _full_span_error(dt, T=1.0, N=96, seed=7):
    n = 8
    model = models.Table(lambda r, R: 0.5 * r * r + 0.5 * R * R + 0.3 * r * R)
    setup = icwf.Setup(model, -4.0, 4.0, n, -4.0, 4.0, n, 1.0, 1.0, dt, 1e-10)

    def Psi0(r, R):
        return np.exp(-(r - R) ** 2 / 4 - R * R / 2 - 0.3 * r) * (1 + 0.4j * r - 0.2j * R)

    P0 = Psi0(setup.r[:, None], setup.R[None, :])
    nrm = math.sqrt(setup.hr * setup.hR * np.sum(np.abs(P0) ** 2))
    P0 = P0 / nrm
    rng = np.random.default_rng(seed)
    rho = np.abs(P0) ** 2
    cells = rng.choice(n * n, size=N, p=(rho / rho.sum()).ravel())
    r0 = setup.r[cells // n] + rng.uniform(-0.5, 0.5, N) * setup.hr
    R0 = setup.R[cells % n] + rng.uniform(-0.5, 0.5, N) * setup.hR
    # Slices of a smooth Psi_0 span only a few numerical directions; generic
    # (random) factors make the N product functions span all n_r n_R directions.
    p1 = rng.standard_normal((N, n)) + 1j * rng.standard_normal((N, n))
    p2 = rng.standard_normal((N, n)) + 1j * rng.standard_normal((N, n))
    p1 /= grid.norm(p1, setup.hr)[:, None]
    p2 /= grid.norm(p2, setup.hR)[:, None]
    b = setup.hr * setup.hR * np.einsum("ai,aj,ij->a", p1.conj(), p2.conj(), P0)
    st = icwf.init(setup, r0, R0, p1, p2, b0=b)
    steps = int(round(T / dt))
    st, _ = icwf.run(setup, st, steps)
    Psi_icwf = np.einsum("a,ai,aj->ij", st.C, st.psi1, st.psi2)
    Psi_ex = exact2d.propagate(P0, setup.Wtab, setup.hr, setup.hR, 1.0, 1.0, dt / 8, 8 * steps)
    return np.max(np.abs(Psi_icwf - Psi_ex))


def test_full_span_equals_brute_force_2d():
    """With N > n_r n_R trajectories the product basis spans the grid space, so
    ICWF is the TDSE itself: agreement with 2D propagation converges as O(dt^2)."""
    e1, e2 = _full_span_error(0.05), _full_span_error(0.025)
    assert e2 < 1e-3
    assert 3.0 < e1 / e2 < 5.0


# --------------------------------------------------------------------------- invariants on a small Shin-Metiu run

@pytest.fixture(scope="module")
def small_sm():
    from paper_1805_11169_amd import inputs
    wl = inputs.shin_metiu(16, n_r=64, n_R=32, r_box=(-40.0, 40.0), n_bo=0, seed=2)
    model = models.make("shin_metiu", wl.model_params)
    setup = icwf.Setup(model, wl.r_min, wl.r_max, wl.n_r, wl.R_min, wl.R_max, wl.n_R,
                       wl.m_r, wl.m_R, wl.dt, wl.eps)
    return wl, setup


def _run_small(wl, setup, steps, psi1=None, psi2=None, b0=None, perm=None):
    p = np.arange(wl.n_traj) if perm is None else perm
    p1 = (wl.psi1 if psi1 is None else psi1)[p]
    p2 = (wl.psi2 if psi2 is None else psi2)[p]
    b = (wl.b0 if b0 is None else b0)[p]
    st = icwf.init(setup, wl.r0[p], wl.R0[p], p1, p2, b0=b)
    st, hist = icwf.run(setup, st, steps)
    return st, hist[-1]


def test_density_integrals_and_completeness(small_sm):
    """int rho(R) dR = int rho(r) dr = C^H S C, and sum over ALL BO states of P_n = norm."""
    wl, setup = small_sm
    st, o = _run_small(wl, setup, 30)
    # both sides are sums over b, a of C_b* C_a S1 S2 in a different order; the
    # regularised C carries large mutually cancelling components, so 1e-12
    assert abs(setup.hR * o["rho_R"].sum() - o["norm"]) < 1e-12
    assert abs(setup.hr * o["rho_r"].sum() - o["norm"]) < 1e-12
    phi, _ = bo.bo_states(setup.model, setup.r, setup.hr, setup.m_r, setup.R, setup.n_r)
    chi = observables.bo_projections(st.C, st.psi1, st.psi2, phi, setup.hr)
    P, D = observables.populations(chi, setup.hR)
    assert abs(P.sum() - o["norm"]) < 1e-12
    assert np.allclose(D, D.T, rtol=0, atol=1e-15)


def test_norm_conservation_improves_with_dt(small_sm):
    """d/dt (C^H S C) = 0 in continuous time; the drift shrinks with the step."""
    wl, setup = small_sm
    drifts = []
    for dt, steps in ((0.2, 20), (0.1, 40)):
        s2 = icwf.Setup(setup.model, wl.r_min, wl.r_max, wl.n_r, wl.R_min, wl.R_max, wl.n_R,
                        wl.m_r, wl.m_R, dt, wl.eps)
        st0 = icwf.init(s2, wl.r0, wl.R0, wl.psi1, wl.psi2, b0=wl.b0)
        n0 = observables.norm(st0.C, st0.S)
        st, o = icwf.run(s2, st0, steps)
        drifts.append(abs(o[-1]["norm"] - n0))
    assert drifts[1] < drifts[0]
    assert drifts[1] < 1e-4


def test_gauge_and_permutation_invariance(small_sm, rng):
    """Multiplying each CWF by a phase (and C by its inverse) or reordering the
    trajectories changes no observable beyond the roundoff floor."""
    wl, setup = small_sm
    _, ref = _run_small(wl, setup, 30)
    th = rng.uniform(0, 2 * np.pi, wl.n_traj)
    _, gauged = _run_small(wl, setup, 30, psi1=wl.psi1 * np.exp(1j * th)[:, None],
                           b0=wl.b0 * np.exp(-1j * th))
    perm = rng.permutation(wl.n_traj)
    _, permuted = _run_small(wl, setup, 30, perm=perm)
    inv = np.argsort(perm)
    for other, order in ((gauged, np.arange(wl.n_traj)), (permuted, inv)):
        assert abs(other["norm"] - ref["norm"]) < 1e-10
        assert np.max(np.abs(other["rho_R"] - ref["rho_R"])) < 1e-9 * np.max(ref["rho_R"])
        assert np.max(np.abs(other["r"][order] - ref["r"])) < 1e-9
        assert np.max(np.abs(other["R"][order] - ref["R"])) < 1e-9


def test_decoherence_of_a_product_state():
    """Psi = phi(r) chi(R) with R-independent BO states: chi^(n) = <phi_n|phi> chi,
    so P_n = |<phi_n|phi>|^2 and D_nm = P_n P_m int |chi|^4 = P_n P_m / (2 sigma sqrt(pi))."""
    r, hr = grid.points(-20, 20, 128)
    R, hR = grid.points(-6, 6, 128)
    sigma = 0.7
    chi = (2 * np.pi * sigma ** 2) ** -0.25 * np.exp(-R ** 2 / (4 * sigma ** 2)) + 0j
    phi = np.exp(-(r - 1.0) ** 2 / 3.0) * (1 + 0.5 * r) + 0j
    phi /= grid.norm(phi, hr)
    sep = models.Separable(lambda x: 0.05 * x * x, lambda y: 0.0 * y)
    states, _ = bo.bo_states(sep, r, hr, 1.0, R, 3)
    chi_n = observables.bo_projections(np.array([1.0 + 0j]), phi[None, :], chi[None, :], states, hr)
    P, D = observables.populations(chi_n, hR)
    ov = np.abs(hr * states[0] @ phi) ** 2
    assert np.max(np.abs(P - ov)) < 1e-12
    assert np.max(np.abs(D - np.outer(ov, ov) / (2 * sigma * math.sqrt(math.pi)))) < 1e-12
