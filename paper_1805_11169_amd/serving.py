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
Ratios are kept apart: served FP64 against sequential FP64 (what serving
gains), served FP64 with lanes of fused steps against served FP64 without
(what fusing gains), served mixed against served FP64 (what the precision
form gains).

`python -m paper_1805_11169_amd.serving --c5 [--precision P]` runs the whole
256-simulation, 500-step mix (N over 64 ... 2048, both grids) once, closed
then open loop, printing a line per 16 results.
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


def _collect(server, ids, say=None, every=16):
    """Results in completion order as they come (polling), returned in submission order."""
    res, pending, t0, last = {}, list(ids), time.perf_counter(), 0
    while pending:
        for i in list(pending):
            if server.wait(i, timeout=0.0):
                res[i] = server.result(i)
                pending.remove(i)
        if say and len(res) - last >= every:
            last = len(res)
            say(f"[serving] {len(res)}/{len(ids)} done, {time.perf_counter() - t0:.1f} s")
        if pending:
            time.sleep(0.002)
    return [res[i] for i in ids]


def run_closed(server, wls, precision, say=None):
    """Every request at t = 0; returns (sims/s, results)."""
    t0 = server.clock()
    ids = [server.submit_workload(wl, wl.n_steps, precision) for wl in wls]
    res = _collect(server, ids, say)
    t1 = max(r["t_done"] for r in res)
    return len(wls) / (t1 - t0), res


def run_open(server, wls, precision, rate, seed=2, say=None):
    """Poisson arrivals at `rate` sims/s; returns (latencies in s, results)."""
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=len(wls)))
    arrivals -= arrivals[0]
    start = time.perf_counter()
    ids = []
    for k, (wl, ta) in enumerate(zip(wls, arrivals)):
        delay = start + ta - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        ids.append(server.submit_workload(wl, wl.n_steps, precision))
        if say and (k + 1) % 16 == 0:
            say(f"[serving] {k + 1}/{len(wls)} submitted, {time.perf_counter() - start:.1f} s")
    res = _collect(server, ids, say)
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


def observable_difference(a, b):
    """Largest difference of norm and densities (relative to their maximum)."""
    d = abs(a["norm"] - b["norm"])
    for k in ("rho_r", "rho_R"):
        d = max(d, float(np.max(np.abs(np.asarray(a[k]) - np.asarray(b[k]))) / np.max(np.abs(b[k]))))
    return d


def _arena(fp, fraction):
    return int(max(2 * max(fp), fraction * sum(fp)))


def measure(n_sims=32, n_steps=100, n_choices=(64, 128, 256, 512), load=0.8, max_active=32,
            steps_per_turn=10, arena_fraction=0.35, log=None):
    """The serving report on a subset of the serving mix (a dict): sequential
    FP64; served FP64 on per-slot streams and with lanes of fused steps; served
    mixed with lanes (capacity, then Poisson arrivals at `load` x capacity for
    p50 / p99); the mixed results against their FP64 runs; alone versus in the
    mix."""
    say = log or (lambda *_: None)
    wls = mix(n_sims, n_steps, n_choices)
    fp64, mixed = icwf.PREC_FP64, icwf.PREC_MIXED
    fp = [max(a, b) for a, b in zip(footprints(wls, fp64), footprints(wls, mixed))]
    arena = _arena(fp, arena_fraction)
    say(f"[serving] {n_sims} sims, {n_steps} steps, arena {arena / 1e9:.2f} GB of {sum(fp) / 1e9:.2f} GB total")

    seq_rate, seq_obs = run_sequential(wls, fp64)
    say(f"[serving] sequential FP64: {seq_rate:.2f} sims/s")
    out = {}
    for batch in (False, True):
        srv = icwf.Server(arena, max_active=max_active, steps_per_turn=steps_per_turn, batch=batch)
        try:
            cap64, res64 = run_closed(srv, wls, fp64)
            say(f"[serving] served FP64 ({'lanes' if batch else 'streams'}): {cap64:.2f} sims/s")
            out[("fp64", batch)] = (cap64, res64)
            if batch:
                cap, res_closed = run_closed(srv, wls, mixed)
                say(f"[serving] served mixed (lanes): {cap:.2f} sims/s")
                lat, res_open = run_open(srv, wls, mixed, load * cap)
                say(f"[serving] open loop at {load * cap:.2f} sims/s: p50 {np.median(lat):.3f} s, "
                    f"p99 {np.percentile(lat, 99):.3f} s")
                stats = srv.stats()
        finally:
            srv.close()
    cap64s, res64s = out[("fp64", False)]
    cap64b, res64b = out[("fp64", True)]
    # every served result equals its alone (sequential) run; the mixed ones are within 1e-5 of their FP64 runs
    equal = all(same_result(a, m) for a, m in zip(seq_obs, res64s)) and \
        all(same_result(a, m) for a, m in zip(seq_obs, res64b))
    _, alone_mixed = run_sequential(wls[:8], mixed)
    equal = equal and all(same_result(a, m) for a, m in zip(alone_mixed, res_closed[:8])) and \
        all(same_result(a, m) for a, m in zip(alone_mixed, res_open[:8]))
    mixed_err = max(observable_difference(m, f) for m, f in zip(res_closed, seq_obs))
    failed = sum(r["status"] != icwf.OK for r in res64s + res64b + res_closed + res_open)
    return {
        "subset": f"{n_sims} of the 256-simulation mix, {n_steps} of its 500 steps, N over {list(n_choices)}",
        "sims": n_sims, "steps": n_steps, "n_choices": list(n_choices), "grids": [list(g) for g in GRIDS],
        "max_active": max_active, "steps_per_turn": steps_per_turn,
        "sequential_fp64_sims_per_s": seq_rate,
        "served_fp64_streams_sims_per_s": cap64s, "served_fp64_lanes_sims_per_s": cap64b,
        "served_mixed_lanes_sims_per_s": cap,
        "ratio_served_fp64_vs_sequential_fp64": max(cap64s, cap64b) / seq_rate,
        "ratio_fused_lanes_vs_streams_fp64": cap64b / cap64s,
        "ratio_served_mixed_vs_served_fp64": cap / cap64b,
        "mixed_vs_fp64_max_observable_difference": mixed_err,
        "arrival_rate_sims_per_s": load * cap, "p50_s": float(np.median(lat)),
        "p99_s": float(np.percentile(lat, 99)), "latency_precision": "mixed",
        "arena_bytes": arena, "footprint_total_bytes": int(sum(fp)), "arena_peak_bytes": stats["arena_peak"],
        "peak_active": stats["peak_active"], "failed": failed, "alone_equals_mix_bitwise": bool(equal),
    }


C5_CHOICES = (64, 128, 256, 512, 1024, 2048)


def c5(precision="mixed", load=0.8, max_active=32, steps_per_turn=10, arena_fraction=0.35, log=None,
       n_sims=256, n_steps=500, phase="both", capacity=None):
    """The whole serving mix: 256 simulations, N log-uniform over 64 ... 2048,
    both grids, R_f ~ U[4, 6], R_0 ~ U[-5, -3], 500 steps each; capacity
    (closed loop) then Poisson arrivals at `load` x capacity (open loop).
    phase "closed" or "open" runs one of the two (the open loop then takes
    the capacity measured by a closed run)."""
    say = log or (lambda *_: None)
    prec = {"fp64": icwf.PREC_FP64, "mixed": icwf.PREC_MIXED, "separable": icwf.PREC_SEPARABLE}[precision]
    t_in = time.perf_counter()
    wls = mix(n_sims, n_steps, C5_CHOICES)
    fp = footprints(wls, prec)
    arena = _arena(fp, arena_fraction)
    counts = {int(n): sum(wl.n_traj == n for wl in wls) for n in C5_CHOICES}
    say(f"[c5] {n_sims} sims built in {time.perf_counter() - t_in:.0f} s; N counts {counts}; arena "
        f"{arena / 1e9:.1f} GB of {sum(fp) / 1e9:.1f} GB")
    srv = icwf.Server(arena, max_active=max_active, steps_per_turn=steps_per_turn, batch=True)
    res_closed, res_open, lat, cap = [], [], None, capacity
    try:
        if phase in ("both", "closed"):
            cap, res_closed = run_closed(srv, wls, prec, say)
            say(f"[c5] capacity {cap:.4f} sims/s")
        if phase in ("both", "open"):
            lat, res_open = run_open(srv, wls, prec, load * cap, say=say)
        stats = srv.stats()
    finally:
        srv.close()
    failed = sum(r["status"] != icwf.OK for r in res_closed + res_open)
    rep = {"workload": "serving mix: 256 Shin-Metiu simulations, N log-uniform over 64..2048, grids 512x256 or "
                       "1024x512, R_f ~ U[4,6], R_0 ~ U[-5,-3], 500 steps, Poisson arrivals at 0.8 x capacity",
           "precision": precision, "phase": phase, "sims": n_sims, "steps": n_steps, "n_counts": counts,
           "capacity_sims_per_s": cap, "arena_bytes": arena, "footprint_total_bytes": int(sum(fp)),
           "arena_peak_bytes": stats["arena_peak"], "peak_active": stats["peak_active"], "max_active": max_active,
           "failed": failed}
    if res_closed:
        # per N: time from admission to result in the closed loop (the service time under full load)
        rep["closed_service_s_by_n"] = {
            int(n): float(np.median([r["t_done"] - r["t_admit"] for r, wl in zip(res_closed, wls) if wl.n_traj == n]))
            for n in C5_CHOICES if any(wl.n_traj == n for wl in wls)}
    if lat is not None:
        by_n = {}
        for n in C5_CHOICES:
            sel = [l for l, wl in zip(lat, wls) if wl.n_traj == n]
            if sel:
                by_n[int(n)] = {"p50_s": float(np.median(sel)), "p99_s": float(np.percentile(sel, 99))}
        rep.update({"arrival_rate_sims_per_s": load * cap, "p50_s": float(np.median(lat)),
                    "p99_s": float(np.percentile(lat, 99)), "latency_by_n": by_n})
    return rep


if __name__ == "__main__":
    import argparse
    import json
    import sys

    ap = argparse.ArgumentParser()
    ap.add_argument("--c5", action="store_true")
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed", "separable"])
    ap.add_argument("--sims", type=int, default=256)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--phase", default="both", choices=["both", "closed", "open"])
    ap.add_argument("--capacity", type=float, default=None, help="sims/s of a closed run (for --phase open)")
    ap.add_argument("--max-active", type=int, default=32)
    a = ap.parse_args()
    if not a.c5:
        ap.error("only --c5 runs from the command line")
    if a.phase == "open" and not a.capacity:
        ap.error("--phase open needs --capacity")
    rep = c5(a.precision, n_sims=a.sims, n_steps=a.steps, phase=a.phase, capacity=a.capacity,
             max_active=a.max_active, log=lambda m: print(m, file=sys.stderr, flush=True))
    print(json.dumps(rep), flush=True)
