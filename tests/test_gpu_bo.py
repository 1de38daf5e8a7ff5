"""Born-Oppenheimer states on the GPU (include/icwf_bo.h, through the C ABI)
against the oracle's dense eigensolver of the same grid operator
h_e(R_j) = T_spec + diag(W(r_i, R_j)) (oracle/bo.py, itself pinned by
tests/test_oracle_bo.py).

Bars: energies within 1e-12 of max(1, |E|); eigenvectors (grid-normalised,
compared up to sign) within 1e-10 of the oracle's; residuals
max_i |(h_e phi - E phi)_i| within 1e-10 with h_e built by the oracle.  On
the 4096-point grid (largest kinetic energy 3.7e3 Hartree, so one rounding of
h_e phi is ~1e-12) the eigenvector bar is 1e-9 and the residual bar 1e-9."""

import numpy as np
import pytest

from oracle import bo as obo
from oracle import grid, models
from paper_1805_11169_amd import icwf, inputs, start

pytestmark = pytest.mark.gpu


def _cfg(model, n_r, r_box, params):
    return icwf.make_config(4, n_r, 32, r_box, (-9.0, 9.0), 1.0, 1836.0, 0.1, model, params)


def _compare(kind, n_r, r_box, R_values, n_states, e_bar=1e-12, v_bar=1e-10, res_bar=1e-10):
    params = inputs.SHIN_METIU_PARAMS if kind == "shin_metiu" else inputs.CAVITY_PARAMS
    model_id = inputs.MODEL_SHIN_METIU if kind == "shin_metiu" else inputs.MODEL_CAVITY
    print(f"[case] BO states {kind} n_r={n_r} values={len(R_values)} states={n_states}", flush=True)
    states, E, info = icwf.bo_states(_cfg(model_id, n_r, r_box, params), R_values, n_states)
    model = models.make(kind, params)
    r, hr = grid.points(r_box[0], r_box[1], n_r)
    ref, Eref = obo.bo_states(model, r, hr, 1.0, R_values, n_states)
    T = grid.kinetic_matrix(n_r, hr, 1.0)
    werr = verr = rerr = 0.0
    for j, Rj in enumerate(R_values):
        h = T + np.diag(model.W(r, Rj))
        for n in range(n_states):
            werr = max(werr, abs(E[j, n] - Eref[j, n]) / max(1.0, abs(Eref[j, n])))
            sgn = np.sign(np.dot(states[j, n], ref[j, n]))
            verr = max(verr, float(np.max(np.abs(states[j, n] - sgn * ref[j, n]))))
            rerr = max(rerr, float(np.max(np.abs(h @ states[j, n] - E[j, n] * states[j, n]))))
            assert abs(hr * states[j, n] @ states[j, n] - 1.0) < 1e-12
    print(f"[result] energies {werr:.2e} vectors {verr:.2e} residuals {rerr:.2e} iterations {info['iterations']} "
          f"solver residual {info['max_residual']:.2e}", flush=True)
    assert info["unconverged"] == 0
    assert werr < e_bar
    assert verr < v_bar
    assert rerr < res_bar
    return states, E


def test_shin_metiu_small_grid():
    R, _ = grid.points(-9.0, 9.0, 32)
    _compare("shin_metiu", 128, (-40.0, 40.0), R, 3)


def test_shin_metiu_parity_grid_every_nuclear_point():
    """The 512-point electronic grid at all 256 nuclear grid points: the BO
    basis of the N = 64 and N = 1024 workloads."""
    R, _ = grid.points(-9.0, 9.0, 256)
    _compare("shin_metiu", 512, (-75.0, 75.0), R, 3)


def test_cavity_grid():
    q, _ = grid.points(-20.0, 20.0, 16)
    _compare("cavity", 1024, (-50.0, 50.0), q, 3)


def test_more_states_and_ragged_count():
    R = np.array([-7.3, -2.0, 0.4, 3.3, 8.1])
    _compare("shin_metiu", 256, (-40.0, 40.0), R, 8)


def test_largest_grid():
    """4096 points on [-75, 75), four nuclear positions."""
    R = np.array([-6.0, -1.5, 2.0, 7.0])
    _compare("shin_metiu", 4096, (-75.0, 75.0), R, 3, v_bar=1e-9, res_bar=1e-9)


def test_product_start_from_gpu_states():
    """The initial state built from the GPU's electronic eigenvector and BO
    basis equals the host-built one: phi_e (eigenvector 1 at R_0) and the
    CWFs within 1e-10, b0 within 1e-12, the BO basis up to sign within 1e-10;
    ten ICWF steps from both starts give the same observables within 1e-9."""
    host = inputs.shin_metiu(64, n_bo=3, seed=0)
    gpu = start.shin_metiu(64, n_bo=3, seed=0)
    assert np.max(np.abs(gpu.extra["phi_e"] - host.extra["phi_e"])) < 1e-10
    assert np.array_equal(gpu.R0, host.R0)
    assert np.max(np.abs(gpu.r0 - host.r0)) == 0.0
    assert np.max(np.abs(gpu.psi1 - host.psi1)) < 1e-10
    assert np.max(np.abs(gpu.psi2 - host.psi2)) < 1e-12
    assert np.max(np.abs(gpu.b0 - host.b0)) < 1e-12
    sg = np.sign(np.einsum("jni,jni->jn", gpu.bo, host.bo))
    assert np.max(np.abs(gpu.bo - sg[:, :, None] * host.bo)) < 1e-10
    obs = []
    for wl in (host, gpu):
        sim = icwf.Simulation.from_workload(wl)
        sim.step(10)
        obs.append(sim.observables())
        sim.close()
    for key in ("rho_r", "rho_R", "pop", "D"):
        a, b = obs
        assert np.max(np.abs(a[key] - b[key])) < 1e-9 * np.max(np.abs(a[key])), key
    assert abs(obs[0]["norm"] - obs[1]["norm"]) < 1e-9


def test_invalid_arguments_are_refused():
    cfg = _cfg(inputs.MODEL_SHIN_METIU, 128, (-40.0, 40.0), inputs.SHIN_METIU_PARAMS)
    with pytest.raises(icwf.ICWFError) as e:
        icwf.bo_states(cfg, [0.0], icwf.BO_MAX_STATES + 1)
    assert e.value.status == icwf.EINVAL
