"""Convergence of ICWF observables with the number of trajectories N, against
the exact grid propagation of the same initial state (include/icwf_exact.h).

The paper judges the method by how its BO populations, reduced nuclear
density and decoherence indicator follow the exact ones as the number of
conditional wavefunctions grows (text around the Shin-Metiu figures).  Here
both run on the GPU from the Shin-Metiu product start of the throughput
workload (512 x 256, dt = 0.1, three BO states): the exact wavefunction from
Psi_0 = phi_e(r) chi_0(R) on the grid, ICWF with N trajectories sampled from
|Psi_0|^2 (seed `seed`), FP64, Tikhonov eps, dt and the trajectory
integrator (Euler or Heun) as given.

Reported per N, as the maximum over the checkpoints (every `every` steps):
  * pop: max_n |P_n - P_n^exact|,
  * rho_R: max_j |rho(R_j) - rho^exact(R_j)| / max_j rho^exact(R_j),
  * D: max_nm |D_nm - D_nm^exact| / max_nm D_nm^exact,
  * norm: |C^H S C - 1| (the exact norm is 1 to rounding),
with the wall time per step of each propagation and the populations at the
last checkpoint.  Used as
    python -m paper_1805_11169_amd.convergence [--steps S] [--every K] [--n 16,64,256,1024] [--heun]
it prints one JSON line.
"""

import argparse
import json
import time

import numpy as np

from . import icwf, inputs


def _errors(got, ref):
    return dict(pop=float(np.max(np.abs(got["pop"] - ref["pop"]))),
                rho_R=float(np.max(np.abs(got["rho_R"] - ref["rho_R"])) / np.max(ref["rho_R"])),
                D=float(np.max(np.abs(got["D"] - ref["D"])) / np.max(np.abs(ref["D"]))),
                norm=float(abs(got["norm"] - 1.0)))


def run(ns=(16, 32, 64, 128, 256, 512, 1024), steps=2000, every=200, seed=0, n_bo=3, eps=1e-8, dt=0.1, log=print,
        trajectories=icwf.TRAJ_EULER):
    import torch
    base = inputs.shin_metiu(ns[0], n_bo=n_bo, seed=seed, dt=dt, eps=eps)
    psi0 = np.outer(base.extra["phi_e"], base.extra["chi0"]).astype(np.complex128)
    cfg = icwf.config_from_workload(base)
    checkpoints = list(range(every, steps + 1, every))

    ex = icwf.ExactPropagator(cfg, psi0, bo=base.bo)
    exact, t_exact = [], 0.0
    for _ in checkpoints:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ex.step(every)
        torch.cuda.synchronize()
        t_exact += time.perf_counter() - t0
        exact.append(ex.observables())
    ex.close()
    log(f"[exact] {steps} steps, {1e3 * t_exact / steps:.3f} ms/step, final P = {exact[-1]['pop']}")

    rows = []
    for N in ns:
        wl = inputs.shin_metiu(N, n_bo=n_bo, seed=seed, dt=dt, eps=eps)
        sim = icwf.Simulation.from_workload(wl, trajectories=trajectories)
        worst = dict(pop=0.0, rho_R=0.0, D=0.0, norm=0.0)
        status, t_icwf, done, last = "ok", 0.0, 0, None
        try:
            for ref in exact:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                sim.step(every)
                sim.sync()
                t_icwf += time.perf_counter() - t0
                done += every
                last = sim.observables()
                e = _errors(last, ref)
                worst = {k: max(worst[k], e[k]) for k in worst}
        except icwf.ICWFError as err:
            status = f"stopped after {done} steps: {err}"
        finally:
            sim.close()
        row = dict(N=N, status=status, steps=done, ms_per_step=1e3 * t_icwf / max(done, 1), **worst,
                   final_pop=None if last is None else last["pop"].tolist())
        log(f"[icwf] N={N}: " + ", ".join(f"{k} {v:.3g}" if isinstance(v, float) else f"{k} {v}"
                                          for k, v in row.items() if k not in ("N", "final_pop")))
        rows.append(row)
    return dict(workload=base.name.replace(f"_N{ns[0]}", ""), steps=steps, every=every, dt=base.dt, eps=eps, seed=seed,
                trajectories="heun" if trajectories == icwf.TRAJ_HEUN else "euler",
                exact_ms_per_step=1e3 * t_exact / steps, exact_final=dict(pop=exact[-1]["pop"].tolist(),
                                                                          norm=exact[-1]["norm"]),
                icwf=rows)


def main():
    p = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    p.add_argument("--steps", type=int, default=2000)
    p.add_argument("--every", type=int, default=200)
    p.add_argument("--n", default="16,32,64,128,256,512,1024")
    p.add_argument("--seed", type=int, default=0)
    p.add_argument("--eps", type=float, default=1e-8, help="Tikhonov eps of the coefficient equation")
    p.add_argument("--dt", type=float, default=0.1)
    p.add_argument("--heun", action="store_true", help="Heun (predictor-corrector) trajectories")
    a = p.parse_args()
    res = run(tuple(int(x) for x in a.n.split(",")), a.steps, a.every, a.seed, eps=a.eps, dt=a.dt,
              log=lambda m: print(m, flush=True), trajectories=icwf.TRAJ_HEUN if a.heun else icwf.TRAJ_EULER)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
