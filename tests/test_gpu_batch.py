"""Fused steps of several simulations (icwf_step_batch, through the C ABI):
every kernel of the step launched once for all of them.  Each simulation's
arithmetic is that of icwf_step, so the batched results must be bitwise the
ones each simulation gets alone; a batch of unlike simulations is refused;
an error in one simulation stops only that one; the server's lanes use the
fused step and still give every request its alone result."""

import numpy as np
import pytest

from paper_1805_11169_amd import icwf, inputs

pytestmark = pytest.mark.gpu


def _family(n=5, N=64, n_r=256, n_R=128, seed=0, **kw):
    """Shin-Metiu starts of one shape with different couplings, centres and ensembles."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n):
        R_f = float(rng.uniform(4.8, 5.2))
        R_c = float(rng.uniform(-4.5, -3.5))
        out.append(inputs.shin_metiu(N, n_r=n_r, n_R=n_R, params=[19.0, R_f, 3.1, 4.0], R_center=R_c, n_bo=2,
                                     seed=100 + s, **kw))
    return out


def _state(sim):
    o = sim.observables()
    st = sim.state()
    return o, st


def _same(a, b):
    oa, sa = a
    ob, sb = b
    keys = ["norm", "rho_r", "rho_R", "pop", "D", "r", "R", "C", "step", "n_out_of_box", "min_abs_psi"]
    if not all(np.array_equal(np.asarray(oa[k]), np.asarray(ob[k])) for k in keys):
        return False
    return all(np.array_equal(sa[k], sb[k]) for k in ("psi1", "psi2", "C", "r", "R"))


def _alone(wls, steps, **kw):
    out = []
    for wl in wls:
        sim = icwf.Simulation.from_workload(wl, **kw)
        sim.step(steps)
        out.append(_state(sim))
        sim.close()
    return out


def _batched(wls, chunks, **kw):
    import torch
    stream = torch.cuda.Stream()
    sims = [icwf.Simulation.from_workload(wl, stream=stream, **kw) for wl in wls]
    for k in chunks:
        icwf.step_batch(sims, k)
    out = [_state(sim) for sim in sims]
    for sim in sims:
        sim.close()
    return out


@pytest.mark.parametrize("name,kw", [
    ("fp64", dict(precision=icwf.PREC_FP64)),
    ("mixed", dict(precision=icwf.PREC_MIXED)),
    ("separable", dict(precision=icwf.PREC_SEPARABLE)),
    ("heun", dict(trajectories=icwf.TRAJ_HEUN)),
    ("crank_nicolson", dict(propagator=icwf.PROP_CRANK_NICOLSON)),
])
def test_batched_steps_are_bitwise_the_single_ones(name, kw):
    wls = _family()
    print(f"[case] batch of {len(wls)} ({name}), 11 steps as 4 + 7", flush=True)
    alone = _alone(wls, 11, **kw)
    batched = _batched(wls, (4, 7), **kw)
    for wl, a, b in zip(wls, alone, batched):
        assert _same(a, b), wl.name


def test_ragged_trajectory_count_and_cavity():
    """N = 100 (a partial 64-tile) on the cavity model."""
    wls = [inputs.gaussian_basis(100, n_r=128, n_R=64, model=inputs.MODEL_CAVITY, r_box=(-30.0, 30.0),
                                 R_box=(-20.0, 20.0), seed=70 + s) for s in range(3)]
    print("[case] cavity batch of 3, N = 100", flush=True)
    import torch
    alone = []
    for wl in wls:
        sim = icwf.Simulation.from_workload(wl, C0=wl.extra["C0"])
        sim.step(6)
        alone.append(sim.observables())
        sim.close()
    stream = torch.cuda.Stream()
    sims = [icwf.Simulation.from_workload(wl, C0=wl.extra["C0"], stream=stream) for wl in wls]
    icwf.step_batch(sims, 6)
    got = [sim.observables() for sim in sims]
    for sim in sims:
        sim.close()
    for a, b in zip(alone, got):
        for key in ("norm", "rho_r", "rho_R", "r", "R", "C"):
            assert np.array_equal(np.asarray(a[key]), np.asarray(b[key])), key


def test_unlike_simulations_are_refused():
    import torch
    stream = torch.cuda.Stream()
    a, b = _family(2)
    c = inputs.shin_metiu(128, n_r=256, n_R=128, n_bo=2, seed=3)
    sa = icwf.Simulation.from_workload(a, stream=stream)
    sb = icwf.Simulation.from_workload(b, stream=stream)
    sc = icwf.Simulation.from_workload(c, stream=stream)
    sd = icwf.Simulation.from_workload(b)                        # another stream
    with pytest.raises(icwf.ICWFError) as e:
        icwf.step_batch([sa, sc], 1)                             # N differs
    assert e.value.status == icwf.EINVAL
    with pytest.raises(icwf.ICWFError) as e:
        icwf.step_batch([sa, sd], 1)
    assert e.value.status == icwf.EINVAL
    sa.step(1)                                                   # parities differ now
    with pytest.raises(icwf.ICWFError) as e:
        icwf.step_batch([sa, sb], 1)
    assert e.value.status == icwf.EINVAL
    with pytest.raises(icwf.ICWFError) as e:
        icwf.step_batch([sa, sa], 1)
    assert e.value.status == icwf.EINVAL
    for s in (sa, sb, sc, sd):
        s.close()


def test_a_node_stops_only_its_simulation():
    import torch
    good = _family(2)
    bad = _family(1, seed=9)[0]
    bad.psi2[:] = 0.0
    print("[case] batch with a node in one simulation", flush=True)
    alone = _alone(good, 5)
    stream = torch.cuda.Stream()
    sims = [icwf.Simulation.from_workload(wl, stream=stream) for wl in (good[0], bad, good[1])]
    icwf.step_batch(sims, 5)
    with pytest.raises(icwf.ICWFError) as e:
        sims[1].sync()
    assert e.value.status == icwf.ENODE
    got = [_state(sims[0]), _state(sims[2])]
    for s in sims:
        s.close()
    assert _same(alone[0], got[0]) and _same(alone[1], got[1])


def test_server_lanes_give_every_request_its_alone_result():
    """Eight requests of one shape and three of another through a server with
    batching on: the lanes step them with fused launches; each result is
    bitwise the alone one."""
    wls = _family(8, seed=4) + _family(3, N=128, seed=5)
    steps = [12, 9, 15, 12, 7, 20, 11, 12, 10, 13, 9]
    print("[case] server with lanes: 11 requests", flush=True)
    alone = []
    for wl, k in zip(wls, steps):
        sim = icwf.Simulation.from_workload(wl)
        sim.step(k)
        alone.append(sim.observables(check=False))
        sim.close()
    need = [icwf.workspace_bytes(icwf.config_from_workload(w)) for w in wls]
    srv = icwf.Server(2 * sum(need), max_active=11, steps_per_turn=4, turns_ahead=2, batch=True)
    ids = [srv.submit_workload(wl, k) for wl, k in zip(wls, steps)]
    got = []
    for i in ids:
        assert srv.wait(i, timeout=120.0)
        got.append(srv.result(i))
    st = srv.stats()
    srv.close()
    for wl, k, a, g in zip(wls, steps, alone, got):
        assert g["status"] == icwf.OK, (wl.name, g["message"])
        assert g["step"] == k
        for key in ("norm", "rho_r", "rho_R", "pop", "D", "r", "R", "C", "n_out_of_box"):
            assert np.array_equal(np.asarray(a[key]), np.asarray(g[key])), (wl.name, key)
    assert st["completed"] == len(wls) and st["failed"] == 0
