"""Seeded synthetic inputs for ICWF runs.

This module only BUILDS the starting point of a run -- grids, the initial
product wavefunction, the sampled trajectories and the conditional
wavefunctions sliced from it, and the Born-Oppenheimer states used by the
population observables.  It holds none of the time-stepping arithmetic and
imports neither the HIP library nor the oracle; both of those take its arrays
as inputs.

Recipe (the paper fixes the models and the initial state in words: electron
in the first excited BO state, nuclear Gaussian / photon vacuum; its numerical
appendix is missing, so the details are the readings stated here):

* grid x_i = x_min + i h, h = (x_max - x_min)/n, periodic;
* Psi_0(r, R) = phi_e(r) chi_0(R), a product state;
* phi_e = eigenvector index 1 (0-based, ascending) of the grid electronic
  Hamiltonian h_e = T + diag(V(r)), T the spectral kinetic operator, V the
  model potential at the reference nuclear position (Shin-Metiu) or the bare
  electronic potential (cavity); sign fixed so its largest component is > 0;
* chi_0 = (2 pi sigma^2)^(-1/4) exp(-(R - R_0)^2 / (4 sigma^2)) (Shin-Metiu,
  |chi_0|^2 has standard deviation sigma) or the photon vacuum
  (omega/pi)^(1/4) exp(-omega q^2 / 2) (cavity);
* trajectories sampled from |Psi_0|^2 with numpy's PCG64 ``default_rng(seed)``:
  all R first (Gaussian), then all r (a grid cell with probability
  h |phi_e(r_i)|^2, plus a uniform offset in [-h/2, h/2));
* conditional wavefunctions are the slices of Eqs. 3-4 at t = 0,
  psi_1^a(r) = Psi_0(r, R^a) and psi_2^a(R) = Psi_0(r^a, R), normalised to one:
  psi_1^a = phi_e for every a and psi_2^a = s_a chi_0 with s_a the sign of
  phi_e at the grid point nearest r^a (the sign is a gauge choice, absorbed
  by C);
* b0[a] = <psi_1^a psi_2^a | Psi_0>, from which the library forms
  C_0 = (S_0 + eps I)^-1 b0.
"""

from dataclasses import dataclass, field
import math

import numpy as np
from scipy.linalg import eigh
from scipy.special import erf

MODEL_SHIN_METIU = 1
MODEL_CAVITY = 2


@dataclass
class Workload:
    """Everything icwf_create takes, as NumPy arrays plus the config fields."""

    name: str
    model: int
    model_params: list
    n_traj: int
    n_r: int
    n_R: int
    r_min: float
    r_max: float
    R_min: float
    R_max: float
    m_r: float
    m_R: float
    dt: float
    n_steps: int
    eps: float
    r0: np.ndarray
    R0: np.ndarray
    psi1: np.ndarray            # (N, n_r) complex128
    psi2: np.ndarray            # (N, n_R) complex128
    b0: np.ndarray              # (N,) complex128
    bo: np.ndarray = None       # (n_R, n_bo, n_r) float64 or None
    extra: dict = field(default_factory=dict)

    @property
    def n_bo(self):
        return 0 if self.bo is None else self.bo.shape[1]


# --------------------------------------------------------------------------
# grid and model potentials used to build the start (not the step)
# --------------------------------------------------------------------------

def _grid(x_min, x_max, n):
    h = (x_max - x_min) / n
    return x_min + h * np.arange(n), h


def _kinetic(n, h, m):
    """Spectral kinetic operator as a dense circulant, from its cosine series."""
    mm = np.arange(n)
    mm = np.where(mm > n // 2, mm - n, mm)          # -n/2+1 .. n/2 (Nyquist counted once)
    k = 2.0 * np.pi * mm / (n * h)
    d = np.arange(n)
    col = np.cos(2.0 * np.pi * np.outer(d, mm) / n) @ (k * k / (2.0 * m)) / n
    idx = (np.arange(n)[:, None] - np.arange(n)[None, :]) % n
    return col[idx]


def _erfx(x, a):
    ax = np.abs(x)
    small = ax < 1e-4 * a
    safe = np.where(small, a, ax)
    z = ax / a
    return np.where(small, 2.0 / (math.sqrt(math.pi) * a) * (1 - z * z / 3 + z ** 4 / 10),
                    erf(safe / a) / safe)


def shin_metiu_potential(r, R, L, R_f, R_l, R_r):
    half = 0.5 * L
    return (1.0 / abs(half - R) + 1.0 / abs(half + R) - _erfx(r - R, R_f)
            - _erfx(r - half, R_r) - _erfx(r + half, R_l))


def cavity_potential(x, q, depth, soft, omega, lam):
    return -depth / np.sqrt(x * x + soft * soft) + 0.5 * omega ** 2 * q * q + lam * q * x


def _eigvecs(T, V, n_states):
    w, v = eigh(T + np.diag(V), subset_by_index=[0, n_states - 1])
    return w, v


def bo_states(model, params, r, hr, m_r, R_values, n_bo):
    """bo[j, n, i] = phi_n(r_i; R_j), real, grid-normalised (h sum phi^2 = 1)."""
    T = _kinetic(r.size, hr, m_r)
    out = np.empty((len(R_values), n_bo, r.size))
    for j, Rj in enumerate(R_values):
        if model == MODEL_SHIN_METIU:
            V = shin_metiu_potential(r, Rj, *params[:4])
        else:
            V = cavity_potential(r, Rj, *params[:4])
        _, v = _eigvecs(T, V, n_bo)
        out[j] = (v / math.sqrt(hr)).T
    return out


# --------------------------------------------------------------------------
# the product start and its trajectory ensemble
# --------------------------------------------------------------------------

def _product_start(name, model, params, N, n_r, n_R, r_box, R_box, m_r, m_R, dt, n_steps,
                   eps, phi_V, chi0_fn, sample_R, seed, n_bo, phi_e=None, bo=None):
    r, hr = _grid(*r_box, n_r)
    R, hR = _grid(*R_box, n_R)
    if phi_e is None:
        _, v = _eigvecs(_kinetic(n_r, hr, m_r), phi_V(r), 2)
        phi = v[:, 1] / math.sqrt(hr)
    else:                       # computed elsewhere (grid-normalised eigenvector 1)
        phi = np.array(phi_e, dtype=np.float64)
    if phi[np.argmax(np.abs(phi))] < 0:
        phi = -phi
    chi = chi0_fn(R)
    chi = chi / math.sqrt(hR * np.sum(chi * chi))

    rng = np.random.default_rng(seed)
    R0 = sample_R(rng, N)
    p = hr * phi * phi
    cell = rng.choice(n_r, size=N, p=p / p.sum())
    r0 = r[cell] + rng.uniform(-0.5 * hr, 0.5 * hr, size=N)

    nearest = np.rint((r0 - r_box[0]) / hr).astype(np.int64) % n_r
    s = np.where(phi[nearest] >= 0.0, 1.0, -1.0)
    psi1 = np.repeat(phi[None, :].astype(np.complex128), N, axis=0)
    psi2 = (s[:, None] * chi[None, :]).astype(np.complex128)
    b0 = (hr * np.sum(phi * phi)) * (hR * np.sum(chi * chi)) * s + 0j
    if bo is None and n_bo:
        bo = bo_states(model, params, r, hr, m_r, R, n_bo)
    return Workload(name, model, list(params), N, n_r, n_R, r_box[0], r_box[1], R_box[0], R_box[1],
                    m_r, m_R, dt, n_steps, eps, r0, R0, psi1, psi2, b0.astype(np.complex128), bo,
                    dict(phi_e=phi, chi0=chi, seed=seed))


SHIN_METIU_PARAMS = [19.0, 5.0, 3.1, 4.0]      # L, R_f, R_l, R_r
CAVITY_PARAMS = [1.0, 1.0, 0.1, 0.05]         # depth, softening, omega, lambda


def shin_metiu(N, n_r=512, n_R=256, r_box=(-75.0, 75.0), R_box=(-9.0, 9.0), params=None,
               R_center=-4.0, sigma=0.38, m_R=1836.0, dt=0.1, n_steps=200, eps=1e-8, seed=0,
               n_bo=3, name=None, phi_e=None, bo=None):
    """Shin-Metiu PCET start: electron in BO state 1 at R_center times a proton Gaussian.
    phi_e (grid-normalised eigenvector 1 of h_e(R_center)) and bo ([n_R][n_bo][n_r])
    may be supplied precomputed; otherwise they are computed here on the host."""
    params = list(SHIN_METIU_PARAMS if params is None else params)

    def phi_V(r):
        return shin_metiu_potential(r, R_center, *params)

    def chi0(R):
        return (2 * math.pi * sigma ** 2) ** -0.25 * np.exp(-(R - R_center) ** 2 / (4 * sigma ** 2))

    def sample_R(rng, n):
        return rng.normal(R_center, sigma, size=n)

    return _product_start(name or f"shin_metiu_N{N}_{n_r}x{n_R}", MODEL_SHIN_METIU, params, N, n_r,
                          n_R, r_box, R_box, 1.0, m_R, dt, n_steps, eps, phi_V, chi0, sample_R, seed,
                          n_bo, phi_e, bo)


def cavity(N, n_r=1024, n_R=256, r_box=(-50.0, 50.0), R_box=(-20.0, 20.0), params=None, dt=0.1,
           n_steps=300, eps=1e-8, seed=0, n_bo=3, name=None, phi_e=None, bo=None):
    """Cavity start: electron in excited state 1 of its bare potential times the photon vacuum."""
    params = list(CAVITY_PARAMS if params is None else params)
    depth, soft, omega, _ = params

    def phi_V(x):
        return -depth / np.sqrt(x * x + soft * soft)

    def chi0(q):
        return (omega / math.pi) ** 0.25 * np.exp(-0.5 * omega * q * q)

    def sample_R(rng, n):
        return rng.normal(0.0, math.sqrt(1.0 / (2.0 * omega)), size=n)

    return _product_start(name or f"cavity_N{N}_{n_r}x{n_R}", MODEL_CAVITY, params, N, n_r, n_R,
                          r_box, R_box, 1.0, 1.0, dt, n_steps, eps, phi_V, chi0, sample_R, seed, n_bo,
                          phi_e, bo)


def gaussian_basis(N, n_r=128, n_R=64, r_box=(-20.0, 20.0), R_box=(-6.0, 6.0), model=MODEL_SHIN_METIU,
                   params=None, m_R=1836.0, dt=0.05, eps=1e-8, seed=0, name=None):
    """A generic (not rank-one) basis for parity checks: N random complex Gaussian
    CWFs per species (random centre, width, momentum), unit-normalised, random
    trajectory positions inside the Gaussians' support and random unit-norm C0."""
    if params is None:
        params = SHIN_METIU_PARAMS if model == MODEL_SHIN_METIU else CAVITY_PARAMS
    rng = np.random.default_rng(seed)
    r, hr = _grid(*r_box, n_r)
    R, hR = _grid(*R_box, n_R)
    Lr, LR = r_box[1] - r_box[0], R_box[1] - R_box[0]

    def gaussians(x, h, L, lo, n):
        c = lo + L * rng.uniform(0.3, 0.7, (n, 1))
        w = L * rng.uniform(0.04, 0.1, (n, 1))
        k = rng.uniform(-0.3, 0.3, (n, 1)) * np.pi / h
        g = np.exp(-(x[None, :] - c) ** 2 / (2 * w * w) + 1j * k * x[None, :])
        return g / np.sqrt(h * np.sum(np.abs(g) ** 2, axis=1, keepdims=True)), c[:, 0], w[:, 0]

    psi1, c1, w1 = gaussians(r, hr, Lr, r_box[0], N)
    psi2, c2, w2 = gaussians(R, hR, LR, R_box[0], N)
    r0 = c1 + 0.5 * w1 * rng.standard_normal(N)
    R0 = c2 + 0.5 * w2 * rng.standard_normal(N)
    C0 = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    C0 /= np.linalg.norm(C0)
    m_R_ = m_R if model == MODEL_SHIN_METIU else 1.0
    wl = Workload(name or f"gaussians_N{N}_{n_r}x{n_R}", model, list(params), N, n_r, n_R, r_box[0],
                  r_box[1], R_box[0], R_box[1], 1.0, m_R_, dt, 0, eps, r0, R0, psi1.astype(np.complex128),
                  psi2.astype(np.complex128), np.zeros(N, np.complex128), None, dict(C0=C0, seed=seed))
    return wl


# Named workloads: the parity case, the headline throughput case, the cavity
# case and the large-grid contraction stress case.
def preset(name, **kw):
    if name == "sm_n64":          # Shin-Metiu, N = 64, 512 x 256, 200 steps (parity case)
        return shin_metiu(64, **kw)
    if name == "sm_n1024":        # Shin-Metiu, N = 1024, 512 x 256, 2000 steps (throughput case)
        kw.setdefault("n_steps", 2000)
        return shin_metiu(1024, **kw)
    if name == "cavity_n2048":    # cavity, N = 2048, 1024 x 256
        return cavity(2048, **kw)
    if name == "sm_n4096_large":  # Shin-Metiu, N = 4096, 4096 x 512 (contraction stress)
        kw.setdefault("n_bo", 0)
        return shin_metiu(4096, n_r=4096, n_R=512, **kw)
    raise KeyError(name)
