"""The coefficient solve of Eq. 8 at N = 4096, the largest trajectory count of
the contraction stress workload, against the oracle.

At this N the library factors 4096 x 4096 matrices, forms the explicit
inverse of S + eps I through six levels of block recursion (automatic solver)
and runs the look-back triangular solves over 64 blocks of 64 rows
(triangular solver).  The grid is small (64 x 32, random complex Gaussian
CWFs, seed 41) so that the oracle's three steps finish in minutes; they are
stored in tests/golden/ by tests/golden/gen_gaussians_n4096.py, which calls
only the oracle and the input generator.

Bars after each of three steps: norm, reduced densities and trajectory
positions within 1e-10 (relative to the largest entry, positions to
max(1, max |x|)); the ansatz wavefunction Psi(r_i, R_j) = sum_a C_a psi_1^a
psi_2^a (Eq. 7) within 1e-9 in the grid L2 norm relative to its own norm: the
difference of the two C vectors as the wavefunction sees it (raw C of a near
singular S is not unique), the same bar as the N = 1024 case's S-norm."""

import os

import numpy as np
import pytest

from paper_1805_11169_amd import icwf, inputs

from oracle_runs import rel_max

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "gaussians_N4096_64x32_3steps.npz")
STEPS = 3


@pytest.fixture(scope="module")
def golden():
    return np.load(GOLDEN)


@pytest.mark.parametrize("solver", [icwf.SOLVER_AUTO, icwf.SOLVER_TRIANGULAR])
def test_n4096_three_steps_against_the_oracle(golden, solver):
    wl = inputs.gaussian_basis(4096, n_r=64, n_R=32, seed=41)
    print(f"[case] {wl.name} solver={solver}: {STEPS} steps against the stored oracle run", flush=True)
    hr = (wl.r_max - wl.r_min) / wl.n_r
    hR = (wl.R_max - wl.R_min) / wl.n_R
    sim = icwf.Simulation.from_workload(wl, C0=wl.extra["C0"], solver=solver)
    try:
        for k in range(1, STEPS + 1):
            sim.step(1)
            o = sim.observables()
            st = sim.state()
            psi = np.einsum("a,ai,aj->ij", st["C"], st["psi1"], st["psi2"])
            ref_psi = golden[f"Psi_{k}"]
            dpsi = np.sqrt(hr * hR * np.sum(np.abs(psi - ref_psi) ** 2))
            npsi = np.sqrt(hr * hR * np.sum(np.abs(ref_psi) ** 2))
            errs = dict(norm=abs(o["norm"] - float(golden[f"norm_{k}"])),
                        rho_r=rel_max(o["rho_r"], golden[f"rho_r_{k}"]),
                        rho_R=rel_max(o["rho_R"], golden[f"rho_R_{k}"]),
                        r=float(np.max(np.abs(o["r"] - golden[f"r_{k}"]))) / max(1.0, np.max(np.abs(golden[f"r_{k}"]))),
                        R=float(np.max(np.abs(o["R"] - golden[f"R_{k}"]))) / max(1.0, np.max(np.abs(golden[f"R_{k}"]))),
                        psi=dpsi / npsi)
            print(f"[step {k}]", {key: f"{v:.2e}" for key, v in errs.items()}, flush=True)
            for key in ("norm", "rho_r", "rho_R", "r", "R"):
                assert errs[key] < 1e-10, (k, key)
            assert errs["psi"] < 1e-9, k
    finally:
        sim.close()
