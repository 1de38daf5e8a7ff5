"""Library behaviour on the GPU beyond parity: graph replay equals
kernel-by-kernel launches bitwise, runs are bitwise repeatable, a checkpoint
resumes bitwise, and device-side error conditions surface as status codes."""

import numpy as np
import pytest

from paper_1805_11169_amd import icwf, inputs

from oracle_runs import rel_max, s_norm_diff

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wl():
    w = inputs.gaussian_basis(100, n_r=128, n_R=64, seed=21)
    print(f"[case] {w.name}", flush=True)
    return w


def _run(wl, steps, timing=False, precision=icwf.PREC_FP64):
    sim = icwf.Simulation.from_workload(wl, precision=precision, C0=wl.extra["C0"])
    if timing:
        sim.set_timing(True)
    sim.step(steps)
    sim.sync()
    st = sim.state()
    sim.close()
    return st


def _same(a, b):
    return all(np.array_equal(a[k], b[k]) for k in ("r", "R", "psi1", "psi2", "C"))


def test_graph_replay_equals_eager_launches(wl):
    assert _same(_run(wl, 7), _run(wl, 7, timing=True))


def test_bitwise_repeatable(wl):
    assert _same(_run(wl, 7), _run(wl, 7))
    assert _same(_run(wl, 5, precision=icwf.PREC_MIXED), _run(wl, 5, precision=icwf.PREC_MIXED))


def test_checkpoint_resume_bitwise(wl):
    full = _run(wl, 6)
    mid = _run(wl, 3)
    cfg = icwf.config_from_workload(wl)
    sim = icwf.Simulation(cfg, mid["r"], mid["R"], mid["psi1"], mid["psi2"], C0=mid["C"])
    sim.step(3)
    sim.sync()
    resumed = sim.state()
    sim.close()
    assert _same(full, resumed)


def test_kernel_times_are_recorded(wl):
    sim = icwf.Simulation.from_workload(wl, C0=wl.extra["C0"])
    sim.set_timing(True)
    sim.step(3)
    for name in ("wc_contract", "propagate", "velocity", "zgemm", "cholesky", "rk4", "assemble"):
        n, ms = sim.kernel_time(name)
        assert n == 3 and ms > 0, name
    sim.close()


def test_singular_overlap_without_regularisation_is_esolve(wl):
    """A zero CWF gives S a zero row and column; with eps = 0 its pivot is
    exactly zero and the factorisation must refuse it."""
    cfg = icwf.config_from_workload(wl, eps=0.0)
    p1 = wl.psi1.copy()
    p1[3] = 0.0
    with pytest.raises(icwf.ICWFError) as e:
        icwf.Simulation(cfg, wl.r0, wl.R0, p1, wl.psi2, C0=wl.extra["C0"])
    assert e.value.status == icwf.ESOLVE


def test_node_is_reported_and_stops_the_run(wl):
    cfg = icwf.config_from_workload(wl)
    zero2 = np.zeros_like(wl.psi2)
    sim = icwf.Simulation(cfg, wl.r0, wl.R0, wl.psi1, zero2, C0=wl.extra["C0"])
    sim.step(1)
    with pytest.raises(icwf.ICWFError) as e:
        sim.sync()
    assert e.value.status == icwf.ENODE
    with pytest.raises(icwf.ICWFError) as e:
        sim.step(1)
    assert e.value.status == icwf.ESTATE
    sim.close()


def test_observables_skip_null_arrays_and_report_box_exits(wl):
    sim = icwf.Simulation.from_workload(wl, C0=wl.extra["C0"])
    sim.step(2)
    o = sim.observables()
    assert o["step"] == 2 and abs(o["t"] - 2 * wl.dt) < 1e-15
    assert np.isfinite(o["min_abs_psi"]) and o["min_abs_psi"] > 0
    assert 0 <= o["n_out_of_box"] <= wl.n_traj
    sim.close()


def test_forked_step_graph_equals_eager_and_repeats():
    """From 1024 trajectories the step forks (factorisations on a second
    stream beside the two-body contraction); replay, eager launches and a
    second run agree bitwise."""
    w = inputs.gaussian_basis(1024, n_r=64, n_R=32, seed=22)
    print(f"[case] {w.name} forked step", flush=True)
    a = _run(w, 3)
    assert _same(a, _run(w, 3, timing=True))
    assert _same(a, _run(w, 3))


@pytest.mark.parametrize("n", [256, 2048])
def test_explicit_inverse_and_triangular_solves_agree(n):
    """The RK4 stages through (S + eps I)^-1 with one refinement step and
    through the triangular factor: at N = 256 on one stream (block inversion
    over two levels), at N = 2048 on the forked step (five levels).  The same
    observables at the FP64 bar; coefficients within 1e-9 in the S norm."""
    w = inputs.gaussian_basis(n, n_r=128, n_R=64, seed=23)
    print(f"[case] {w.name} N={n}: explicit inverse vs triangular solves, 3 steps", flush=True)
    out = {}
    for solver in (icwf.SOLVER_TRIANGULAR, icwf.SOLVER_INVERSE):
        sim = icwf.Simulation.from_workload(w, C0=w.extra["C0"], solver=solver)
        sim.step(3)
        o = sim.observables()
        st = sim.state()
        S = sim.matrices()[0]
        sim.close()
        out[solver] = (o, st, S)
    (o1, s1, S1), (o2, s2, _) = out[icwf.SOLVER_TRIANGULAR], out[icwf.SOLVER_INVERSE]
    # positions (and through them the CWFs) follow C through the velocities
    for key in ("r", "R"):
        assert np.max(np.abs(s1[key] - s2[key])) < 1e-10 * max(1.0, np.max(np.abs(s1[key]))), key
    assert rel_max(s2["psi1"], s1["psi1"]) < 1e-10
    assert abs(o1["norm"] - o2["norm"]) < 1e-10 * abs(o1["norm"])
    for key in ("rho_r", "rho_R"):
        assert rel_max(o1[key], o2[key]) < 1e-10, key
    size = np.sqrt(abs(np.conj(s1["C"]) @ S1 @ s1["C"]))
    assert s_norm_diff(s1["C"], s2["C"], S1) < 1e-9 * size


def test_forked_step_with_the_integrals_beside_the_contraction():
    """N = 1024 on a 512 x 512 grid: the dense contraction is long enough that
    the single-species integrals run on the factorisation stream beside it.
    Replay and eager launches agree bitwise; the result agrees with the
    separable form (FP64 throughout; its overlaps ahead of the fork, its
    coupling integrals after its short contraction, while the factorisation
    stream runs) at the FP64 bar, whose replays and eager launches agree
    bitwise as well."""
    w = inputs.gaussian_basis(1024, n_r=512, n_R=512, seed=24)
    print(f"[case] {w.name}: integrals on the side stream, 3 steps", flush=True)
    a = _run(w, 3)
    assert _same(a, _run(w, 3, timing=True))
    sep = _run(w, 3, precision=icwf.PREC_SEPARABLE)
    assert _same(sep, _run(w, 3, precision=icwf.PREC_SEPARABLE, timing=True))
    for key in ("r", "R"):
        assert np.max(np.abs(a[key] - sep[key])) < 1e-10 * max(1.0, np.max(np.abs(a[key]))), key
    assert rel_max(sep["psi1"], a["psi1"]) < 1e-10
    assert rel_max(sep["psi2"], a["psi2"]) < 1e-10
