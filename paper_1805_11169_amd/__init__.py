"""MI355X-native ICWF hot path (interacting conditional wavefunctions, arXiv:1805.11169).

The compute path is the HIP library ``libicwf.so`` built from ``csrc/``; the
Python module ``icwf`` is a thin ctypes binding over its C ABI.  ``inputs``
builds seeded synthetic starting states.  Importing this package loads nothing;
the library is loaded on first use of ``icwf``.
"""
