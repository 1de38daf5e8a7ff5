"""Plain FP64 CPU oracle of the interacting-conditional-wavefunction (ICWF) method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with
the HIP library (``paper_1805_11169_amd``): it takes the same seeded inputs
and computes the method again, literally, from the paper's equations.

Source: Albareda, Kelly, Rubio, "Nonadiabatic ab initio quantum dynamics
without potential energy surfaces" (arXiv:1805.11169).

* ``grid``        -- periodic grids, wavenumbers, quadrature.
* ``models``      -- the full interaction W(r, R) of the Shin-Metiu and the
                     cavity model (Eq. 2 with A_j = 0).
* ``propagate``   -- Hermitian-CWF propagation of every conditional
                     wavefunction (Eqs. 5-6 with the eta potentials reduced to
                     a dropped phase), split-operator.
* ``interp``      -- band-limited (trigonometric) interpolation of a CWF and
                     its gradient at an off-grid trajectory position.
* ``matrices``    -- the matrices of Eq. 9a-9d and K = W - W1 - W2 (Eq. 8).
* ``velocity``    -- the Bohmian velocities of Eqs. 10-11.
* ``coeffs``      -- the coefficient equation, Eq. 8, with a Tikhonov-
                     regularised Cholesky solve and RK4.
* ``observables`` -- norm, reduced densities, BO populations, decoherence.
* ``bo``          -- Born-Oppenheimer electronic states on the grid.
* ``icwf``        -- the ICWF step and run loop.
* ``exact2d``     -- brute-force propagation of the full 2D wavefunction
                     (Eq. 1), used only to pin the ICWF oracle on tiny grids.

Every function cites the equation or section of the paper it follows.  Where
the paper is silent the reading taken is stated in the docstring.

Parity pins: every function here is pinned by tests under ``tests/`` marked
``not gpu`` (closed forms, invariants, brute force on tiny grids).
"""



def _one_thread_for_scipy_blas():
    """NumPy and SciPy each bundle their own OpenBLAS; alternating calls into the
    two thread pools makes each spin against the other (a 64x64 Cholesky then
    takes ~50 ms instead of ~50 us).  The heavy products run in NumPy's pool,
    so SciPy's (used only for the small Cholesky solves) is held to one thread."""
    try:
        from threadpoolctl import ThreadpoolController
    except ImportError:  # pragma: no cover - timing only, results unaffected
        return
    for lib in ThreadpoolController().lib_controllers:
        if "scipy.libs" in lib.filepath or "scipy/.libs" in lib.filepath:
            lib.set_num_threads(1)


def blas_threads():
    """Threads of NumPy's BLAS pool (the pool the heavy oracle products use)."""
    try:
        from threadpoolctl import ThreadpoolController
        for lib in ThreadpoolController().lib_controllers:
            if "numpy" in lib.filepath and lib.user_api == "blas":
                return lib.num_threads
    except ImportError:  # pragma: no cover
        pass
    return None


import scipy.linalg  # noqa: E402  (load SciPy's BLAS before limiting it)

_one_thread_for_scipy_blas()

from . import grid, models, propagate, interp, matrices, velocity, coeffs, observables, bo, icwf, exact2d  # noqa: F401
