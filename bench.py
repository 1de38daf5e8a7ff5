"""ICWF throughput benchmark on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64|mixed] [--no-cpu-baseline]
                    [--no-serving] [--serve-sims S] [--serve-steps T] [--no-large-propagation]

One step = one full pass of the ICWF hot path (Bohmian velocities and
trajectory update, split-operator propagation of all 2N conditional
wavefunctions, the Eq. 9 matrices including the N^2 two-body contraction,
two Tikhonov-regularised Cholesky factorisations and the RK4 coefficient
update) on the Shin-Metiu workload with N = 1024 trajectories on a 512 x 256
grid.  Inputs are seeded and synthetic and resident in HBM before timing.

Prints one JSON line: traj-steps/s over exactly K timed steps, the roofline
of the dominant kernel (the two-body contraction, timed live with HIP events
on the stream it runs on), the mixed and separable forms on the same
workload, a subset of the serving mix (served sims/s on streams and with
fused lanes, p50 / p99 time-to-result under Poisson arrivals, each ratio
against its own baseline), the GPU build of the BO basis of the large grid
against the host eigensolver, the propagation's HBM rate on the
N = 4096, 4096 x 512 workload (whose CWFs do not fit the Infinity Cache), the
step time of the exact grid propagation of the full wavefunction at
512 x 256 and 4096 x 512 (the reference ICWF converges to; skipped with
--no-large-propagation), and the FP64 oracle timed on a bounded sample on the
host cores.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6, "mixed": 157.3, "separable": 78.6}   # dense matrix-core TFLOP/s of MI355X (FP64, FP32)
HBM_PEAK_GBS = 8000.0

# HBM traffic of one two-body contraction launch on the N = 1024, 512 x 256
# Shin-Metiu workload, from two rocprofv3 --pmc passes (FETCH_SIZE, then
# WRITE_SIZE, KiB per dispatch, summed over the kernels of the stage) scaled by
# what the same counters read for a plain 1 GiB device copy (FETCH_SIZE reads
# 0.5 of the bytes copied: x2; WRITE_SIZE reads 1.0: x1).  Valid only for the
# kernel sources they were taken on (hash of the contraction's sources); after
# any change the traffic is reported as null until measured again.
TRAFFIC = {
    "sm_n1024": {
        "sources_sha256_16": "f7e36e1c54569dda",
        "fp64": 348255744.0,        # k_wc<double>: fetch 159085.2 KiB x2, write 21923.1 KiB
        "mixed": 309099520.0,       # k_wc<float> + k_wc_sep: fetch 79068.6 + 49840.5 KiB x2, write 35651.5 + 8385.3 KiB
        "separable": 162296422.4,   # k_wc_sep (K = 28): fetch 75053.6 KiB x2, write 8385.4 KiB
    },
}
TRAFFIC_SOURCES = ("paper_1805_11169_amd/csrc/k_matrices.hip", "paper_1805_11169_amd/csrc/icwf_device.hpp",
                   "paper_1805_11169_amd/csrc/icwf_plan.hpp")


def measured_traffic(workload, precision):
    import hashlib
    rec = TRAFFIC.get(workload)
    if rec is None:
        return None
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return rec.get(precision) if h.hexdigest()[:16] == rec["sources_sha256_16"] else None


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--precision", choices=["fp64", "mixed", "separable"], default="fp64")
    p.add_argument("--workload", default="sm_n1024")
    p.add_argument("--propagator", choices=["split", "cn"], default="split",
                   help="CWF propagator: split operator (default) or Crank-Nicolson")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-steps", type=int, default=2)
    p.add_argument("--no-serving", action="store_true", help="skip the serving-mix leg")
    p.add_argument("--no-other-precisions", action="store_true",
                   help="skip the mixed and separable runs beside the FP64 headline")
    p.add_argument("--exact-grid-only", action="store_true",
                   help="time only the exact grid propagation (512 x 256 and 4096 x 512) and print its JSON")
    p.add_argument("--no-large-propagation", action="store_true",
                   help="skip the propagation measurement on the N = 4096, 4096 x 512 workload")
    p.add_argument("--serve-sims", type=int, default=32)
    p.add_argument("--serve-steps", type=int, default=100)
    p.add_argument("--copy-calibration-bytes", type=int, default=0,
                   help="first run a plain device copy of this many bytes three times (the reference kernel "
                        "that scales the HBM traffic counters)")
    return p.parse_args()


def large_propagation():
    """The propagation on the working set that does not fit the 256 MB
    Infinity Cache (N = 4096, 4096 x 512: 604 MB read and written per step),
    FP64, one timed step after one untimed one."""
    from paper_1805_11169_amd import icwf, inputs
    wl = inputs.preset("sm_n4096_large", n_bo=0)
    sim = icwf.Simulation.from_workload(wl, precision=icwf.PREC_FP64, device=0)
    sim.step(1)
    sim.sync()
    sim.set_timing(True)
    sim.step(1)
    sim.sync()
    n, ms = sim.kernel_time("propagate")
    sim.set_timing(False)
    sim.close()
    _, _, prop_bytes = algorithmic_counts(wl.n_traj, wl.n_r, wl.n_R)
    gbs = prop_bytes / (ms / 1e3 / n) / 1e9
    return {"workload": wl.name, "n_traj": wl.n_traj, "n_r": wl.n_r, "n_R": wl.n_R, "bytes_per_step": prop_bytes,
            "avg_launch_ms": ms / n, "achieved_gbs": gbs, "peak_gbs": HBM_PEAK_GBS, "frac": gbs / HBM_PEAK_GBS}


def exact_grid(steps=50):
    """The grid propagation of the full wavefunction (include/icwf_exact.h)
    from the product start, per step at 512 x 256 and 4096 x 512: HIP events on
    the stream it runs on; algorithmic bytes = read + write Psi once per step."""
    import numpy as np
    import torch
    from paper_1805_11169_amd import icwf, inputs
    out = {}
    for nr, nR in ((512, 256), (4096, 512)):
        wl = inputs.shin_metiu(1, n_r=nr, n_R=nR, n_bo=0)
        psi0 = np.outer(wl.extra["phi_e"], wl.extra["chi0"]).astype(np.complex128)
        ex = icwf.ExactPropagator(icwf.config_from_workload(wl), psi0)
        ex.step(5)
        s = ex.stream
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        ex.step(steps)
        b.record(s)
        b.synchronize()
        ms = a.elapsed_time(b) / steps
        norm = ex.observables()["norm"]
        ex.close()
        nbytes = 2.0 * nr * nR * 16
        out[f"{nr}x{nR}"] = {"ms_per_step": ms, "bytes_per_step": nbytes, "achieved_gbs": nbytes / (ms / 1e3) / 1e9,
                             "peak_gbs": HBM_PEAK_GBS, "norm_after": norm}
    return out


def bo_build(n_states=3):
    """The BO basis of the large-grid workload on the GPU (include/icwf_bo.h):
    the 3 lowest states of h_e(R_j) on the 4096-point electronic grid at all 512
    nuclear grid points, wall clock of one call (upload, solve, copy-out) after
    a warm-up call; beside it the host path it replaces (the input generator's
    dense eigensolver) timed on one R value and scaled to 512."""
    import numpy as np
    from paper_1805_11169_amd import icwf, inputs
    n_r, n_R = 4096, 512
    r_box, R_box = (-75.0, 75.0), (-9.0, 9.0)
    R = R_box[0] + (R_box[1] - R_box[0]) / n_R * np.arange(n_R)
    cfg = icwf.make_config(4, n_r, n_R, r_box, R_box, 1.0, 1836.0, 0.1, inputs.MODEL_SHIN_METIU,
                           inputs.SHIN_METIU_PARAMS)
    icwf.bo_states(cfg, R[:8], n_states)
    t0 = time.perf_counter()
    _, _, info = icwf.bo_states(cfg, R, n_states)
    gpu_s = time.perf_counter() - t0
    hr = (r_box[1] - r_box[0]) / n_r
    r = r_box[0] + hr * np.arange(n_r)
    t0 = time.perf_counter()
    inputs.bo_states(inputs.MODEL_SHIN_METIU, inputs.SHIN_METIU_PARAMS, r, hr, 1.0, R[:1], n_states)
    host_one = time.perf_counter() - t0
    return {"workload": f"BO states: {n_states} lowest of h_e(R_j), Shin-Metiu, {n_r}-point electronic grid at the "
                        f"{n_R} nuclear grid points", "gpu_s": gpu_s, "iterations_max": info["iterations"],
            "max_residual": info["max_residual"], "host_dense_eigh_s_per_value": host_one,
            "host_extrapolated_s": host_one * n_R, "speedup_vs_host": host_one * n_R / gpu_s,
            "host_cores": os.cpu_count()}


def algorithmic_counts(N, nr, nR):
    """Flops / bytes the method must do per step (not what a kernel happens to do)."""
    wc = 2.0 * N * (N + 1) * nr * nR                     # Hermitian two-body contraction (Eq. 9b)
    single = 4.0 * N * (N + 1) * (nr + nR) + 16.0 * N * N * (nr + nR)   # S1, S2 and E1, E2 at two conditionings
    prop_bytes = 2.0 * N * (nr + nR) * 16                # read + write every CWF once (complex128)
    return wc, single, prop_bytes


def cpu_baseline(wl, steps, steps_one_thread=1):
    """The FP64 oracle on the host: `steps` steps with NumPy's BLAS on all its
    threads (the reported value), then `steps_one_thread` more with it held to
    one thread; also the BLAS library and the host's core count."""
    import numpy as np  # noqa: F401
    import oracle
    from oracle import icwf as oicwf
    from oracle import models
    setup = oicwf.Setup(models.make("shin_metiu", wl.model_params), wl.r_min, wl.r_max, wl.n_r, wl.R_min,
                        wl.R_max, wl.n_R, wl.m_r, wl.m_R, wl.dt, wl.eps)
    st = oicwf.init(setup, wl.r0, wl.R0, wl.psi1, wl.psi2, b0=wl.b0)
    t0 = time.perf_counter()
    for _ in range(steps):
        st = oicwf.step(setup, st)
    dt = time.perf_counter() - t0
    blas = None
    one = None
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        blas = [f"{i.get('internal_api')} {i.get('version')} ({i.get('architecture')}, {i.get('num_threads')} threads)"
                for i in threadpool_info() if i.get("user_api") == "blas" and "numpy" in i.get("filepath", "")]
        if steps_one_thread:
            with threadpool_limits(limits=1, user_api="blas"):
                t1 = time.perf_counter()
                for _ in range(steps_one_thread):
                    st = oicwf.step(setup, st)
                d1 = time.perf_counter() - t1
            one = {"value": wl.n_traj * steps_one_thread / d1, "cores": 1,
                   "sample": f"{steps_one_thread} further oracle step(s), {d1:.1f} s"}
    except ImportError:  # pragma: no cover - threadpoolctl ships with the image
        pass
    return {"value": wl.n_traj * steps / dt, "unit": "traj-steps/s", "cores": oracle.blas_threads() or os.cpu_count(),
            "kind": "oracle",
            "sample": f"{steps} oracle steps of the same workload (N={wl.n_traj}, {wl.n_r}x{wl.n_R}) from t=0, "
                      f"{dt:.1f} s on the host",
            "one_thread": one, "blas": blas, "host_cpu_count": os.cpu_count()}


def other_precision(wl, precision, steps, warmup, fp64_ms):
    """The same workload through another precision form of the library (graph
    replays, wall clock over `steps` steps), beside the headline FP64 run."""
    import torch
    from paper_1805_11169_amd import icwf
    prec = {"mixed": icwf.PREC_MIXED, "separable": icwf.PREC_SEPARABLE}[precision]
    sim = icwf.Simulation.from_workload(wl, precision=prec, device=0)
    sim.step(warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    rank = sim.contraction_rank()
    sim.close()
    return {"precision": precision, "ms_per_step": ms, "traj_steps_per_s": wl.n_traj / (ms / 1e3),
            "speedup_vs_fp64": fp64_ms / ms, "contraction_rank": rank, "steps": steps, "warmup": warmup,
            "timing": "graph replays, wall clock"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the sharding over GPUs is a design, "
              "not a measured path", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1805_11169_amd import icwf, inputs

    if args.exact_grid_only:
        print(json.dumps({"exact_grid": exact_grid()}), flush=True)
        return
    if args.copy_calibration_bytes:
        n = args.copy_calibration_bytes // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    wl = inputs.preset(args.workload, n_bo=0)
    prec = {"fp64": icwf.PREC_FP64, "mixed": icwf.PREC_MIXED, "separable": icwf.PREC_SEPARABLE}[args.precision]
    N, nr, nR = wl.n_traj, wl.n_r, wl.n_R
    prop = icwf.PROP_CRANK_NICOLSON if args.propagator == "cn" else icwf.PROP_SPLIT
    sim = icwf.Simulation.from_workload(wl, precision=prec, device=0, propagator=prop)
    stream = sim.stream

    sim.step(args.warmup)
    sim.sync()
    # graph replays first (the step as a user runs it), then the same number of
    # steps kernel by kernel with an event pair around each kernel: the
    # headline value is the slower of the two wall clocks
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    sim.sync()
    torch.cuda.synchronize()
    elapsed_graph = time.perf_counter() - t0
    sim.set_timing(True)          # kernel-by-kernel launches with an event pair around each kernel
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    sim.sync()
    torch.cuda.synchronize()
    elapsed = max(time.perf_counter() - t0, elapsed_graph)

    kt = {}
    for name in ("wc_contract", "zgemm", "velocity", "propagate", "assemble", "cholesky", "inverse", "rk4"):
        n, ms = sim.kernel_time(name)
        kt[name] = (n, ms)
    sim.set_timing(False)
    obs = sim.observables()
    rank = sim.contraction_rank()
    # observables on demand (norm, both densities): launches, copy-out and sync
    torch.cuda.synchronize()
    t_obs = time.perf_counter()
    for _ in range(5):
        sim.observables(check=False)
    obs_ms = (time.perf_counter() - t_obs) / 5 * 1e3
    sim.close()
    del stream

    wc_flops, single_flops, prop_bytes = algorithmic_counts(N, nr, nR)
    if args.precision == "separable":
        # the contraction through K products: N(N+1)/2 pairs x (n_r + n_R) x K complex x real multiply-adds
        wc_flops = 2.0 * N * (N + 1) * (nr + nR) * rank
    n_wc, ms_wc = kt["wc_contract"]
    wc_avg_s = ms_wc / 1e3 / n_wc
    achieved = wc_flops / wc_avg_s / 1e12
    n_zg, ms_zg = kt["zgemm"]
    # S/H build: the contraction plus the single-species integrals.  From 1024
    # padded trajectories the step runs the integrals on the second stream
    # beside the contraction where that stream has room: FP64 without the
    # explicit inverses of S + eps I (used for a power-of-two padded count), or
    # a dense contraction with n_r n_R >= 256 Np.  The build then spans the
    # longer of the two; otherwise they run one after the other.
    Np = (N + 63) // 64 * 64
    dense = args.precision != "separable"
    sinv = Np >= 1024 and (Np & (Np - 1)) == 0
    roomy = dense and nr * nR >= 256 * Np
    concurrent = Np >= 1024 and ((args.precision == "fp64" and not sinv) or roomy)
    build_ms = max(ms_wc, ms_zg) if concurrent else ms_wc + ms_zg
    build_tflops = (wc_flops + single_flops) / (build_ms / 1e3 / n_wc) / 1e12
    build_tflops_summed = (wc_flops + single_flops) / ((ms_wc + ms_zg) / 1e3 / n_wc) / 1e12
    n_pr, ms_pr = kt["propagate"]
    prop_gbs = prop_bytes / (ms_pr / 1e3 / n_pr) / 1e9

    value = N * args.steps / elapsed
    line = {
        "metric": "ICWF traj-steps/s at N=1024",
        "value": value,
        "unit": "traj-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-contraction/f64" if prec == icwf.PREC_MIXED else "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "hamiltonian": {1: "shin_metiu", 2: "cavity"}[wl.model], "n_traj": N,
                   "n_r": nr, "n_R": nR,
                   "dt": wl.dt, "precision": args.precision, "propagator": args.propagator, "contraction_rank": rank,
                   "timing": "kernel-by-kernel with HIP events"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK[args.precision], "unit": "TFLOP/s",
                     "frac": achieved / PEAK[args.precision],
                     "traffic": measured_traffic(args.workload, args.precision),
                     "kernel": "wc_contract", "flops_per_launch": wc_flops, "avg_launch_ms": wc_avg_s * 1e3},
        "sh_build_tflops": build_tflops,
        "sh_build_tflops_summed_kernel_time": build_tflops_summed,
        "propagation": {"achieved_gbs": prop_gbs, "peak_gbs": HBM_PEAK_GBS, "frac": prop_gbs / HBM_PEAK_GBS,
                        "avg_launch_ms": ms_pr / n_pr},
        "kernel_ms_per_step": {k: (ms / n_wc if n else None) for k, (n, ms) in kt.items()},
        "observables_ms": obs_ms,
        "final_norm": obs["norm"],
        "ms_per_step_graph_replay": elapsed_graph / args.steps * 1e3,
    }
    if args.precision == "fp64" and not args.no_other_precisions:
        fp64_ms = elapsed_graph / args.steps * 1e3
        line["mixed"] = other_precision(wl, "mixed", args.steps, args.warmup, fp64_ms)
        line["separable"] = other_precision(wl, "separable", args.steps, args.warmup, fp64_ms)
    if not args.no_large_propagation and args.workload != "sm_n4096_large":
        line["propagation_4096x512"] = large_propagation()
    if not args.no_large_propagation and args.workload != "sm_n4096_large":
        line["exact_grid"] = exact_grid()
        line["bo_states_4096x512"] = bo_build()
    if not args.no_serving:
        from paper_1805_11169_amd import serving
        line["serving"] = serving.measure(n_sims=args.serve_sims, n_steps=args.serve_steps,
                                          log=lambda m: print(m, file=sys.stderr, flush=True))
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
