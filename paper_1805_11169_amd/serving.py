"""Serving mix and its measurement: a stream of independent Shin-Metiu
simulations of uneven size through the continuous-batching server
(include/icwf_serve.h).

The mix (seeded, synthetic): simulation s of n_sims draws, from
numpy's PCG64 seeded with `seed`,
  * N log-uniform over `n_choices` (powers of two: a uniform index),
  * the grid (512 x 256) or (1024 x 512) with probability 1/2 each, boxes
    [-75, 75) x [-9, 9),
  * R_f ~ U[4, 6] and R_0 ~ U[-5, -3] (the Gaussian centre and the nuclear
    position of the electronic eigenvector),
and takes its trajectory seed 1000 + s; every simulation runs n_steps steps
of dt = 0.1 from the product start of the throughput workload.

Measured:
  * capacity: all requests submitted at once (closed loop), sims/s from the
    first submission to the last result;
  * latency: Poisson arrivals at `load` x capacity (open loop), p50 / p99 of
    result time minus arrival time;
  * the baseline: the same simulations one after another through the plain
    FP64 path (icwf_create, icwf_step, icwf_observables, icwf_destroy).
"""

import time

import numpy as np

from . import icwf, inputs

GRIDS = ((512, 256), (1024, 512))


def mix(n_sims=32, n_steps=100, n_choices=(64, 128, 256, 512), seed=1):
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n_sims):
        N = int(n_choices[rng.integers(len(n_choices))])
        n_r, n_R = GRIDS[int(rng.random() < 0.5)]
        R_f = float(rng.uniform(4.0, 6.0))
        R_0 = float(rng.uniform(-5.0, -3.0))
        wl = inputs.shin_metiu(N, n_r=n_r, n_R=n_R, params=[19.0, R_f, 3.1, 4.0], R_center=R_0,
                               n_steps=n_steps, seed=1000 + s, n_bo=0,
                               name=f"serve{s}_N{N}_{n_r}x{n_R}")
        out.append(wl)
    return out


def footprints(wls, precision):
    return [icwf.workspace_bytes(icwf.config_from_workload(wl, precision)) for wl in wls]


def _collect(server, ids):
    res = []
    for i in ids:
        server.wait(i)
        res.append(server.result(i))
    return res


def run_closed(server, wls, precision):
    """Every request at t = 0; returns (sims/s, results)."""
    t0 = server.clock()
    ids = [server.submit_workload(wl, wl.n_steps, precision) for wl in wls]
    res = _collect(server, ids)
    t1 = max(r["t_done"] for r in res)
    return len(wls) / (t1 - t0), res


def run_open(server, wls, precision, rate, seed=2):
    """Poisson arrivals at `rate` sims/s; returns (latencies in s, results)."""
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=len(wls)))
    arrivals -= arrivals[0]
    start = time.perf_counter()
    ids = []
    for wl, ta in zip(wls, arrivals):
        delay = start + ta - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        ids.append(server.submit_workload(wl, wl.n_steps, precision))
    res = _collect(server, ids)
    lat = np.array([r["t_done"] - r["t_submit"] for r in res])
    return lat, res


def run_sequential(wls, precision=icwf.PREC_FP64):
    """One simulation at a time through the plain path; returns (sims/s, observables)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = []
    for wl in wls:
        sim = icwf.Simulation.from_workload(wl, precision=precision)
        sim.step(wl.n_steps)
        out.append(sim.observables(check=False))
        sim.close()
    torch.cuda.synchronize()
    return len(wls) / (time.perf_counter() - t0), out


def same_result(a, b):
    """Bitwise equality of two final-observable records."""
    keys = ("norm", "rho_r", "rho_R", "r", "R", "C", "step", "n_out_of_box")
    return all(np.array_equal(np.asarray(a[k]), np.asarray(b[k])) for k in keys)


def measure(n_sims=32, n_steps=100, n_choices=(64, 128, 256, 512), load=0.8, max_active=8,
            steps_per_turn=10, arena_fraction=0.35, log=None):
    """The serving report: capacity, p50 / p99 under load, the sequential FP64
    baseline and the alone-versus-mix check (a dict)."""
    say = log or (lambda *_: None)
    wls = mix(n_sims, n_steps, n_choices)
    prec = icwf.PREC_MIXED
    fp = footprints(wls, prec)
    arena = int(max(2 * max(fp), arena_fraction * sum(fp)))
    say(f"[serving] {n_sims} sims, {n_steps} steps, arena {arena / 1e9:.2f} GB of {sum(fp) / 1e9:.2f} GB total")

    seq_rate, seq_obs = run_sequential(wls, icwf.PREC_FP64)
    say(f"[serving] sequential FP64: {seq_rate:.2f} sims/s")
    srv = icwf.Server(arena, max_active=max_active, steps_per_turn=steps_per_turn)
    try:
        cap64, _ = run_closed(srv, wls, icwf.PREC_FP64)
        say(f"[serving] served FP64 capacity: {cap64:.2f} sims/s")
        cap, res_closed = run_closed(srv, wls, prec)
        say(f"[serving] served mixed capacity: {cap:.2f} sims/s")
        lat, res_open = run_open(srv, wls, prec, load * cap)
        say(f"[serving] open loop at {load * cap:.2f} sims/s: p50 {np.median(lat):.3f} s, "
            f"p99 {np.percentile(lat, 99):.3f} s")
        stats = srv.stats()
    finally:
        srv.close()
    # alone versus in the mix: the same mixed-precision simulation run by itself
    _, alone = run_sequential(wls[:4], prec)
    equal = all(same_result(a, m) for a, m in zip(alone, res_closed[:4])) and \
        all(same_result(a, m) for a, m in zip(alone, res_open[:4]))
    failed = sum(r["status"] != icwf.OK for r in res_closed + res_open)
    return {
        "sims": n_sims, "steps": n_steps, "n_choices": list(n_choices), "grids": [list(g) for g in GRIDS],
        "precision": "mixed", "max_active": max_active, "steps_per_turn": steps_per_turn,
        "capacity_sims_per_s": cap, "served_fp64_sims_per_s": cap64, "sequential_fp64_sims_per_s": seq_rate,
        "speedup_vs_sequential_fp64": cap / seq_rate, "arrival_rate_sims_per_s": load * cap,
        "p50_s": float(np.median(lat)), "p99_s": float(np.percentile(lat, 99)),
        "arena_bytes": arena, "footprint_total_bytes": int(sum(fp)), "arena_peak_bytes": stats["arena_peak"],
        "peak_active": stats["peak_active"], "failed": failed, "alone_equals_mix_bitwise": bool(equal),
    }
