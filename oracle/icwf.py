"""The ICWF step and run loop (oracle; test infrastructure only).

State: N electronic CWFs psi_1^a (N, n_r), N nuclear/photonic CWFs psi_2^a
(N, n_R), coefficients C (N,), trajectory positions (r^a, R^a) -- the ansatz of
Eq. 7 with its trajectory ensemble.

One step t_k -> t_k+1 = t_k + dt (the paper gives no integrator; reading taken):

  (a) velocities v_k from (C_k, psi_k, x_k)                        Eqs. 10-11
  (b) x_k+1 = x_k + dt v_k  (explicit Euler; no wrapping or clamping)
  (c) psi_k+1 = Strang step of every CWF, conditioning frozen at x_k  Eqs. 5-6
  (d) S_k+1 and K^-_k+1 = K(psi_k+1, x_k); K_k+1 = K(psi_k+1, x_k+1)    Eqs. 8-9
  (e) RK4 for C over the step with (S_k, K_k) at t_k and (S_k+1, K^-_k+1) at
      t_k+1, linear in between; K_k+1 is kept as the next step's start value.

K^- uses the conditioning of the step just taken (the CWFs moved under it);
K_k+1 uses the new positions, which condition the next step.

Heun trajectories (Setup.trajectories = "heun"; the paper fixes the velocity
field of Eqs. 10-11, not how it is integrated): (b) gives only the predictor
x~ = x_k + dt v_k; after (c)-(e) the velocity field of the new state
(C_k+1, psi_k+1) is evaluated at x~, and the trajectories take the trapezoid
x_k+1 = x_k + dt/2 (v_k + v(x~, t_k+1)).  The CWF propagation keeps the
conditioning frozen at x_k, K^- is unchanged, and K_k+1 is formed at the
corrected positions.
"""

from dataclasses import dataclass, field

import numpy as np

from . import coeffs, grid, matrices, observables, propagate, velocity


@dataclass
class Setup:
    """Grids, masses, model and numerical parameters of one ICWF run."""

    model: object
    r_min: float
    r_max: float
    n_r: int
    R_min: float
    R_max: float
    n_R: int
    m_r: float
    m_R: float
    dt: float
    eps: float = 1e-8
    propagator: str = "strang"     # or "cn" (Crank-Nicolson, oracle.propagate)
    trajectories: str = "euler"    # or "heun" (predictor x_k + dt v_k, trapezoid corrector)

    def __post_init__(self):
        self.r, self.hr = grid.points(self.r_min, self.r_max, self.n_r)
        self.R, self.hR = grid.points(self.R_min, self.R_max, self.n_R)
        self.Wtab = self.model.W(self.r[:, None], self.R[None, :])


@dataclass
class State:
    psi1: np.ndarray
    psi2: np.ndarray
    C: np.ndarray
    r_traj: np.ndarray
    R_traj: np.ndarray
    S: np.ndarray = None
    K: np.ndarray = None
    fac: object = None
    t: float = 0.0
    step: int = 0
    n_out_of_box: int = 0
    min_abs_psi: float = field(default=np.inf)


def _couplings(setup, psi1, psi2, conds):
    return matrices.couplings(psi1, psi2, setup.model, setup.r, setup.R, setup.hr, setup.hR,
                              conds, setup.Wtab)


def init(setup, r0, R0, psi1, psi2, C0=None, b0=None):
    """Initial state.  If C0 is None, C_0 = (S_0 + eps I)^-1 b0 (regularised projection)."""
    psi1 = np.array(psi1, dtype=np.complex128)
    psi2 = np.array(psi2, dtype=np.complex128)
    r0 = np.array(r0, dtype=np.float64)
    R0 = np.array(R0, dtype=np.float64)
    S, (K,) = _couplings(setup, psi1, psi2, [(r0, R0)])
    fac = coeffs.factor(S, setup.eps)
    if C0 is None:
        C = coeffs.cho_solve(fac, np.asarray(b0, dtype=np.complex128))
    else:
        C = np.array(C0, dtype=np.complex128)
    return State(psi1, psi2, C, r0, R0, S, K, fac)


def _velocities(setup, C, psi1, psi2, r_traj, R_traj):
    return velocity.velocities(C, psi1, psi2, setup.r_min, setup.hr, setup.R_min, setup.hR,
                               setup.m_r, setup.m_R, r_traj, R_traj)


def step(setup, st):
    """Advance the state by one step (a)-(e) above; returns the new State."""
    v_r, v_R, psi_at = _velocities(setup, st.C, st.psi1, st.psi2, st.r_traj, st.R_traj)
    r_new = st.r_traj + setup.dt * v_r
    R_new = st.R_traj + setup.dt * v_R
    p1, p2 = propagate.propagate_cwfs(st.psi1, st.psi2, setup.model, setup.r, setup.R,
                                      setup.hr, setup.hR, setup.m_r, setup.m_R,
                                      st.r_traj, st.R_traj, setup.dt, setup.propagator)
    min_psi = float(np.min(np.abs(psi_at)))
    if setup.trajectories == "heun":
        S1, (Kminus,) = _couplings(setup, p1, p2, [(st.r_traj, st.R_traj)])
        C_new, fac1 = coeffs.rk4_step(st.C, st.S, st.K, S1, Kminus, setup.eps, setup.dt, st.fac)
        w_r, w_R, psi_pred = _velocities(setup, C_new, p1, p2, r_new, R_new)
        r_new = st.r_traj + 0.5 * setup.dt * (v_r + w_r)
        R_new = st.R_traj + 0.5 * setup.dt * (v_R + w_R)
        _, (Knew,) = _couplings(setup, p1, p2, [(r_new, R_new)])
        min_psi = min(min_psi, float(np.min(np.abs(psi_pred))))
    else:
        S1, (Kminus, Knew) = _couplings(setup, p1, p2, [(st.r_traj, st.R_traj), (r_new, R_new)])
        C_new, fac1 = coeffs.rk4_step(st.C, st.S, st.K, S1, Kminus, setup.eps, setup.dt, st.fac)
    out = ((r_new < setup.r_min) | (r_new >= setup.r_max)
           | (R_new < setup.R_min) | (R_new >= setup.R_max))
    return State(p1, p2, C_new, r_new, R_new, S1, Knew, fac1, st.t + setup.dt, st.step + 1,
                 int(np.count_nonzero(out)), min_psi)


def observe(setup, st, bo=None):
    """Observables of the current state (dict of arrays)."""
    rho_r, rho_R = observables.densities(st.C, st.psi1, st.psi2, setup.hr, setup.hR)
    obs = dict(t=st.t, step=st.step, norm=observables.norm(st.C, st.S), rho_r=rho_r, rho_R=rho_R,
               r=st.r_traj.copy(), R=st.R_traj.copy(), C=st.C.copy(),
               n_out_of_box=st.n_out_of_box, min_abs_psi=st.min_abs_psi)
    if bo is not None:
        chi = observables.bo_projections(st.C, st.psi1, st.psi2, bo, setup.hr)
        obs["pop"], obs["D"] = observables.populations(chi, setup.hR)
    return obs


def run(setup, st, n_steps, n_obs=0, bo=None):
    """Take n_steps steps; observe every n_obs steps (0: only at the end).  Returns (state, [obs])."""
    history = []
    for k in range(n_steps):
        st = step(setup, st)
        if n_obs and (st.step % n_obs == 0):
            history.append(observe(setup, st, bo))
    if not n_obs or st.step % n_obs:
        history.append(observe(setup, st, bo))
    return st, history
