"""Periodic real-space grids (oracle; test infrastructure only).

The paper works in the position representation for both species (text around
Eq. 1) but does not state a discretisation (its numerical appendix is not part
of the text).  Reading taken: a periodic box [x_min, x_max) with n points,
spacing h = (x_max - x_min)/n, the right endpoint excluded; quadrature is
h * sum; the inner product is <f|g> = h * sum(conj(f) g).
"""

import numpy as np


def points(x_min, x_max, n):
    """Grid x_i = x_min + i h, i = 0..n-1, and h = (x_max - x_min)/n."""
    h = (x_max - x_min) / n
    return x_min + h * np.arange(n, dtype=np.float64), h


def wavenumbers(n, h):
    """Angular wavenumbers k = 2 pi fftfreq(n, h), in NumPy FFT order."""
    return 2.0 * np.pi * np.fft.fftfreq(n, d=h)


def inner(f, g, h):
    """<f|g> = h sum_i conj(f_i) g_i over the last axis."""
    return h * np.sum(np.conj(f) * g, axis=-1)


def norm(f, h):
    """sqrt(<f|f>) over the last axis."""
    return np.sqrt(np.real(inner(f, f, h)))


def kinetic_matrix(n, h, m):
    """Dense spectral kinetic operator T = F^-1 diag(k^2 / 2m) F on the grid.

    Real symmetric circulant; T[i, j] = (1/n) sum_k (k^2/2m) exp(i k (x_i - x_j)).
    Built from the definition with an explicit FFT of the identity, so that it is
    the same operator the split-operator propagator applies.
    """
    k = wavenumbers(n, h)
    eye = np.eye(n)
    T = np.fft.ifft((k ** 2 / (2.0 * m))[:, None] * np.fft.fft(eye, axis=0), axis=0)
    return np.real(T)
