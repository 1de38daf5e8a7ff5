"""The allocation-free observables entry point (icwf_grid_observables_noalloc,
include/icwf_exact.h) against the handle-based one it varies
(icwf_exact_observables): the same kernels on the same wavefunction, so the
results must be bitwise equal.  Two calls in a row, the second on a smaller
grid with fewer BO states (the static scratch array keeps the first call's
contents, which the second must not see); sizes beyond the array's limit are
refused."""

import numpy as np
import pytest

from paper_1805_11169_amd import icwf, inputs

pytestmark = pytest.mark.gpu


def _start(wl, seed):
    rng = np.random.default_rng(seed)
    r = wl.r_min + (wl.r_max - wl.r_min) / wl.n_r * np.arange(wl.n_r)
    R = wl.R_min + (wl.R_max - wl.R_min) / wl.n_R * np.arange(wl.n_R)
    x = (r[:, None] - rng.uniform(-2, 2)) / 3.0
    y = (R[None, :] - rng.uniform(-1, 1)) / 1.0
    return np.exp(-0.5 * (x * x + y * y - 1.2 * x * y) + 0.7j * r[:, None]).astype(np.complex128)


def _case(n_r, n_R, n_bo, seed):
    import torch
    wl = inputs.gaussian_basis(4, n_r=n_r, n_R=n_R, seed=seed)
    hr, hR = (wl.r_max - wl.r_min) / n_r, (wl.R_max - wl.R_min) / n_R
    r = wl.r_min + hr * np.arange(n_r)
    R = wl.R_min + hR * np.arange(n_R)
    bo = inputs.bo_states(wl.model, wl.model_params, r, hr, wl.m_r, R, n_bo)
    cfg = icwf.config_from_workload(wl)
    cfg.n_bo = n_bo
    ex = icwf.ExactPropagator(cfg, _start(wl, seed), bo=bo)
    ex.step(5)
    ref = ex.observables()
    psi = ex.psi()
    ex.close()
    d_psi = torch.from_numpy(psi.view(np.float64).copy()).cuda()
    d_bo = torch.from_numpy(bo.copy()).cuda()
    n_out = 1 + n_r + n_R + n_bo + n_bo * n_bo
    d_out = torch.full((n_out,), np.nan, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    print(f"[case] no-alloc observables {n_r}x{n_R} n_bo={n_bo}", flush=True)
    st = icwf.grid_observables_noalloc(n_r, n_R, hr, hR, n_bo, d_psi.data_ptr(), d_bo.data_ptr(), d_out.data_ptr(),
                                       stream.cuda_stream)
    assert st == icwf.OK
    torch.cuda.synchronize()
    out = d_out.cpu().numpy()
    assert out[0] == ref["norm"]
    assert np.array_equal(out[1:1 + n_r], ref["rho_r"])
    assert np.array_equal(out[1 + n_r:1 + n_r + n_R], ref["rho_R"])
    po = 1 + n_r + n_R
    assert np.array_equal(out[po:po + n_bo], ref["pop"])
    assert np.array_equal(out[po + n_bo:].reshape(n_bo, n_bo), ref["D"])


def test_matches_the_handle_based_observables_on_two_calls():
    _case(256, 128, 4, 61)
    _case(64, 32, 2, 62)


def test_refuses_sizes_beyond_the_scratch_limit():
    import torch
    d = torch.zeros(1 + 64 + 64 + 17 + 17 * 17, dtype=torch.float64, device="cuda")
    st = icwf.grid_observables_noalloc(64, 64, 0.1, 0.1, 17, d.data_ptr(), d.data_ptr(), d.data_ptr(),
                                       torch.cuda.current_stream().cuda_stream)
    assert st == icwf.EINVAL
    st = icwf.grid_observables_noalloc(8192, 64, 0.1, 0.1, 0, d.data_ptr(), 0, d.data_ptr(),
                                       torch.cuda.current_stream().cuda_stream)
    assert st == icwf.EINVAL
