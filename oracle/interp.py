"""Band-limited interpolation of grid functions at off-grid points (oracle).

Eqs. 10-11 need each CWF and its gradient at the trajectory positions, which
are not grid points.  The paper does not say how they are evaluated.  Reading
taken: the trigonometric interpolant of the grid samples (the function the
spectral kinetic operator acts on),

    f(x) = sum_{m=-n/2+1}^{n/2-1} c_m exp(2 pi i m u / n) + c_{n/2} cos(pi u),
    u = (x - x_min)/h,  c = FFT(f)/n,

with the Nyquist mode split symmetrically (a cosine), which is the convention
of the periodic sinc interpolant for even n.  The gradient is the exact
derivative of this expression.  The interpolant is periodic with the box.
"""

import numpy as np


def trig_interp(f, x_min, h, xq):
    """Values and x-derivatives of the interpolants of the rows of f at points xq.

    f: (M, n) samples of M functions; xq: (P,) points.
    Returns (val, der), each (P, M): val[p, b] = f_b(xq[p]), der[p, b] = f_b'(xq[p]).
    """
    f = np.atleast_2d(np.asarray(f))
    n = f.shape[-1]
    if n % 2:
        raise ValueError("even grid sizes only")
    c = np.fft.fft(f, axis=-1) / n                   # (M, n)
    m = np.fft.fftfreq(n, d=1.0 / n)                 # integer mode numbers, -n/2 is Nyquist
    u = (np.asarray(xq, dtype=np.float64) - x_min) / h
    phase = np.exp(2j * np.pi * np.outer(u, m) / n)  # (P, n)
    dphase = (2j * np.pi * m / (n * h))[None, :] * phase
    nyq = n // 2                                     # index of mode -n/2 in FFT order
    phase[:, nyq] = np.cos(np.pi * u)
    dphase[:, nyq] = -(np.pi / h) * np.sin(np.pi * u)
    return phase @ c.T, dphase @ c.T
