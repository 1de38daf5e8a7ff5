"""Model interactions W(r, R) (oracle; test infrastructure only).

The Hamiltonian is Eq. 2: H = T_1(r) + T_2(R) + W(r, R, t); no configuration
uses a vector potential, so T_j = -(1/2 m_j) d^2/dx^2 (atomic units, hbar = 1).
W here is always the FULL interaction; the oracle never splits it.

Shin-Metiu proton-coupled electron transfer (the paper's first example): one
electron r and one proton R move on the line between two ions fixed at +-L/2.
The paper cites the model and leaves its formula to a missing appendix; the
form taken is the standard erf-softened one,

    W = 1/|L/2 - R| + 1/|L/2 + R|
        - erf(|r - R|/R_f)/|r - R|
        - erf(|r - L/2|/R_r)/|r - L/2| - erf(|r + L/2|/R_l)/|r + L/2|,

with R_r the softening of the ion at +L/2 and R_l that of the ion at -L/2.

Cavity electron-photon model (the paper's second example): a soft-Coulomb
electron x coupled to one photon displacement mode q,

    W = -1/sqrt(x^2 + a^2) * depth + omega^2 q^2 / 2 + lam q x,

with no dipole self-energy term (reading of the workload description; the
paper's own model appendix is missing).
"""

import math

import numpy as np
from scipy.special import erf

_TWO_OVER_SQRT_PI = 2.0 / math.sqrt(math.pi)


def erf_over_x(x, a):
    """g(x; a) = erf(|x|/a)/|x|, with its limit 2/(sqrt(pi) a) at x = 0.

    Below |x| < 1e-4 a the Taylor series 2/(sqrt(pi) a)(1 - z^2/3 + z^4/10),
    z = x/a, is used; its truncation error there is below 1e-20 relative.
    Coincidences r_i = R_j do occur on the configured grids, so the limit is
    needed, not only a guard.
    """
    ax = np.abs(np.asarray(x, dtype=np.float64))
    z = ax / a
    small = z < 1e-4
    safe = np.where(small, a, ax)
    exact = erf(safe / a) / safe
    series = _TWO_OVER_SQRT_PI / a * (1.0 - z * z / 3.0 + z ** 4 / 10.0)
    return np.where(small, series, exact)


class ShinMetiu:
    """Shin-Metiu model; parameters L, R_f, R_l, R_r (atomic units)."""

    kind = "shin_metiu"

    def __init__(self, L=19.0, R_f=5.0, R_l=3.1, R_r=4.0):
        self.L, self.R_f, self.R_l, self.R_r = float(L), float(R_f), float(R_l), float(R_r)

    def W(self, r, R):
        """Full W(r, R), broadcast over r and R."""
        r, R = np.broadcast_arrays(np.asarray(r, float), np.asarray(R, float))
        half = 0.5 * self.L
        ion_ion = 1.0 / np.abs(half - R) + 1.0 / np.abs(half + R)
        e_p = -erf_over_x(r - R, self.R_f)
        e_ions = -erf_over_x(r - half, self.R_r) - erf_over_x(r + half, self.R_l)
        return ion_ion + e_p + e_ions


class Cavity:
    """Cavity electron-photon model; parameters depth, softening a, omega, lam."""

    kind = "cavity"

    def __init__(self, depth=1.0, soft=1.0, omega=0.1, lam=0.05):
        self.depth, self.soft, self.omega, self.lam = float(depth), float(soft), float(omega), float(lam)

    def W(self, x, q):
        """Full W(x, q), broadcast over x and q."""
        x, q = np.broadcast_arrays(np.asarray(x, float), np.asarray(q, float))
        return (-self.depth / np.sqrt(x * x + self.soft * self.soft)
                + 0.5 * self.omega ** 2 * q * q + self.lam * q * x)


class Separable:
    """W(r, R) = f(r) + g(R) for pins (product-state recovery, closed-form K)."""

    kind = "separable"

    def __init__(self, f, g):
        self.f, self.g = f, g

    def W(self, r, R):
        r, R = np.broadcast_arrays(np.asarray(r, float), np.asarray(R, float))
        return self.f(r) + self.g(R)


class Table:
    """W given as any callable w(r, R); used for the coupled-oscillator pins."""

    kind = "callable"

    def __init__(self, w):
        self.w = w

    def W(self, r, R):
        r, R = np.broadcast_arrays(np.asarray(r, float), np.asarray(R, float))
        return self.w(r, R)


def make(kind, params):
    """Model from a kind string and its parameter list (the C-ABI's order)."""
    if kind == "shin_metiu":
        return ShinMetiu(*params[:4])
    if kind == "cavity":
        return Cavity(*params[:4])
    raise ValueError(f"unknown model {kind!r}")
