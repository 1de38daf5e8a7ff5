"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point include/icwf.h declares, sizes workspaces, and rejects
invalid configurations before touching the device."""

import ctypes
import os
import re

import pytest

from paper_1805_11169_amd import icwf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_entry_points(header=None):
    """Functions declared in one header, or in every header under include/."""
    names = [header] if header else sorted(f for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h"))
    decl = r"^(?:size_t|icwf_status|void|double|const char \*)\s*(icwf_[a-z_]+)\s*\("
    found = set()
    for h in names:
        found |= set(re.findall(decl, open(os.path.join(ROOT, "include", h)).read(), flags=re.MULTILINE))
    return sorted(found)


def test_header_and_binding_agree():
    assert declared_entry_points("icwf.h") == sorted(icwf.EXPORTS)
    assert declared_entry_points("icwf_serve.h") == sorted(icwf.SERVE_EXPORTS)
    assert declared_entry_points("icwf_exact.h") == sorted(icwf.EXACT_EXPORTS)
    assert declared_entry_points("icwf_bo.h") == sorted(icwf.BO_EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(icwf.LIB_PATH):
        pytest.fail("libicwf.so is not built (python -m paper_1805_11169_amd.build)")
    L = ctypes.CDLL(icwf.LIB_PATH)
    for name in declared_entry_points():
        assert hasattr(L, name), name


def _cfg(**kw):
    base = dict(n_traj=64, n_r=512, n_R=256, r_box=(-75, 75), R_box=(-9, 9), m_r=1.0, m_R=1836.0, dt=0.1,
                model=icwf.MODEL_SHIN_METIU, model_params=[19.0, 5.0, 3.1, 4.0], eps=1e-8, n_bo=3)
    base.update(kw)
    return icwf.make_config(**base)


def test_workspace_bytes_scales_with_n_squared():
    small = icwf.workspace_bytes(_cfg(n_traj=64))
    big = icwf.workspace_bytes(_cfg(n_traj=1024))
    assert small > 0 and big > 0
    # sixteen N x N complex matrices dominate at N = 1024
    assert big > 16 * 1024 * 1024 * 16
    assert icwf.workspace_bytes(_cfg(n_traj=65)) == icwf.workspace_bytes(_cfg(n_traj=128))


def test_workspace_holds_the_explicit_inverses_only_where_they_are_used():
    def extra(n):  # seven n x n complex128 matrices in place of 256-byte-aligned single elements
        return 7 * (16 * n * n - 256)

    tri64 = icwf.workspace_bytes(_cfg(n_traj=64, solver=icwf.SOLVER_TRIANGULAR))
    assert icwf.workspace_bytes(_cfg(n_traj=64)) == tri64
    assert icwf.workspace_bytes(_cfg(n_traj=64, solver=icwf.SOLVER_INVERSE)) >= tri64 + extra(64)
    auto = icwf.workspace_bytes(_cfg(n_traj=1024))
    tri = icwf.workspace_bytes(_cfg(n_traj=1024, solver=icwf.SOLVER_TRIANGULAR))
    assert icwf.workspace_bytes(_cfg(n_traj=1024, solver=icwf.SOLVER_INVERSE)) == auto
    assert auto >= tri + extra(1024)
    # the separable form too, from 1024 padded trajectories
    sep = icwf.workspace_bytes(_cfg(n_traj=1024, precision=icwf.PREC_SEPARABLE))
    assert icwf.workspace_bytes(_cfg(n_traj=1024, precision=icwf.PREC_SEPARABLE,
                                     solver=icwf.SOLVER_INVERSE)) == sep
    assert sep >= icwf.workspace_bytes(_cfg(n_traj=1024, precision=icwf.PREC_SEPARABLE,
                                            solver=icwf.SOLVER_TRIANGULAR)) + extra(1024)
    # padded N = 192 is not a power of two: automatic falls back to the triangular solves
    assert icwf.workspace_bytes(_cfg(n_traj=150)) == icwf.workspace_bytes(_cfg(n_traj=150, solver=1))


@pytest.mark.parametrize("bad", [dict(n_traj=0), dict(n_traj=5000), dict(n_r=500), dict(n_R=8),
                                 dict(r_box=(1, 1)), dict(m_r=0.0), dict(dt=-0.1), dict(eps=-1.0),
                                 dict(model=7), dict(precision=3), dict(n_bo=-1), dict(n_bo=1000),
                                 dict(model_params=[19.0, 0.0, 3.1, 4.0]), dict(solver=3), dict(solver=-1),
                                 dict(n_traj=150, solver=icwf.SOLVER_INVERSE), dict(propagator=2),
                                 dict(n_r=4096, propagator=icwf.PROP_CRANK_NICOLSON)])
def test_invalid_configs_are_rejected_on_the_host(bad):
    cfg = _cfg(**bad)
    assert icwf.workspace_bytes(cfg) == 0
    L = icwf.lib()
    h = ctypes.c_void_p()
    one = (ctypes.c_double * 8192)()
    st = L.icwf_create(ctypes.byref(cfg), one, one, one, one, None, one, one, ctypes.c_void_p(256),
                       ctypes.c_size_t(1 << 40), None, ctypes.byref(h))
    assert st == icwf.EINVAL
    assert L.icwf_last_error(None)


def test_too_small_workspace_and_missing_inputs():
    cfg = _cfg(n_traj=4, n_r=32, n_R=32, n_bo=0)
    L = icwf.lib()
    h = ctypes.c_void_p()
    one = (ctypes.c_double * 4096)()
    need = icwf.workspace_bytes(cfg)
    st = L.icwf_create(ctypes.byref(cfg), one, one, one, one, None, one, None, ctypes.c_void_p(256),
                       ctypes.c_size_t(need - 1), None, ctypes.byref(h))
    assert st == icwf.ENOMEM
    st = L.icwf_create(ctypes.byref(cfg), one, one, one, one, None, None, None, ctypes.c_void_p(256),
                       ctypes.c_size_t(need), None, ctypes.byref(h))
    assert st == icwf.EINVAL          # neither C0 nor b0
    nan = (ctypes.c_double * 4096)(*([float("nan")] * 4096))
    st = L.icwf_create(ctypes.byref(cfg), nan, one, one, one, None, one, None, ctypes.c_void_p(256),
                       ctypes.c_size_t(need), None, ctypes.byref(h))
    assert st == icwf.ENONFINITE
    st = L.icwf_create(ctypes.byref(cfg), one, one, one, one, None, one, None, ctypes.c_void_p(257),
                       ctypes.c_size_t(need), None, ctypes.byref(h))
    assert st == icwf.EINVAL          # misaligned workspace
    assert icwf.status_string(icwf.ESOLVE) == "ICWF_ESOLVE"


def test_exact_workspace_and_invalid_configs():
    """The grid propagator's footprint is three n_r n_R complex128 arrays (the
    state, its transposed copy, the potential phase) plus tables of n_r and
    n_R entries; an invalid configuration sizes to 0 and fails creation."""
    cfg = _cfg(n_r=512, n_R=256, n_bo=0)
    ex = icwf.lib().icwf_exact_workspace_bytes(ctypes.byref(cfg))
    assert 3 * 16 * 512 * 256 <= ex < 3 * 16 * 512 * 256 + 256 * 1024
    bad = _cfg(n_r=500)
    assert icwf.lib().icwf_exact_workspace_bytes(ctypes.byref(bad)) == 0
    h = ctypes.c_void_p()
    one = (ctypes.c_double * 8)()
    st = icwf.lib().icwf_exact_create(ctypes.byref(bad), one, None, ctypes.c_void_p(256), ctypes.c_size_t(1 << 40),
                                      None, ctypes.byref(h))
    assert st == icwf.EINVAL


def test_bo_workspace_and_argument_checks():
    cfg = _cfg(n_r=512)
    one = icwf.bo_workspace_bytes(cfg, 1, 3)
    many = icwf.bo_workspace_bytes(cfg, 256, 3)
    assert 0 < one < many
    assert icwf.bo_workspace_bytes(cfg, 256, 0) == 0
    assert icwf.bo_workspace_bytes(cfg, 256, icwf.BO_MAX_STATES + 1) == 0
    assert icwf.bo_workspace_bytes(_cfg(n_r=32), 4, 9) == 0      # more than n_r / 4 states
    assert icwf.bo_workspace_bytes(cfg, 0, 3) == 0
