/*
 * icwf.h -- C ABI of the MI355X (gfx950) interacting-conditional-wavefunction
 * (ICWF) library.
 *
 * Method: Albareda, Kelly, Rubio, "Nonadiabatic ab initio quantum dynamics
 * without potential energy surfaces" (arXiv:1805.11169).  The full
 * wavefunction of two species (electron r, nucleus or photon mode R) is the
 * ansatz of Eq. 7,
 *
 *     Psi(r, R, t) = sum_a C_a(t) psi_1^a(r, t) psi_2^a(R, t),
 *
 * over N trajectories (r^a, R^a).  One step of the library advances every
 * piece of it:
 *   - the Bohmian velocities of the ansatz at each trajectory (Eqs. 10-11)
 *     and the trajectory positions;
 *   - every conditional wavefunction under its own conditioned potential
 *     (Eqs. 5-6, Hermitian limit: the eta potentials reduce to a dropped
 *     phase), split-operator on a periodic grid;
 *   - the matrices S, W, W1, W2 of Eq. 9 at the new wavefunctions;
 *   - the coefficients C through i S dC/dt = (W - W1 - W2) C (Eq. 8),
 *     Tikhonov-regularised (S + eps I) and integrated with RK4.
 * Observables are those the paper monitors: reduced densities, BO
 * populations P_n and the decoherence indicator D_nm.
 *
 * Units: atomic units, hbar = 1.  Grids: x_i = x_min + i h, h = (x_max -
 * x_min)/n, periodic, the right end excluded.  Complex arrays are
 * interleaved (re, im) doubles.  Matrices are row-major with the row the bra
 * (conjugated) index and the column the ket index.
 *
 * Ownership: every host array passed in is read during the call and never
 * retained.  Device memory is the caller's: one workspace of at least
 * icwf_workspace_bytes() bytes, which the handle carves and owns until
 * icwf_destroy (which does not free it).  Work is enqueued on the caller's
 * HIP stream.  One handle is one simulation; handles are not thread-safe, and
 * two handles may share a stream.
 *
 * Errors: every call returns an icwf_status (0 = ok, < 0 = error) and, where
 * there is a handle, records a message for icwf_last_error().  After
 * ICWF_ENONFINITE, ICWF_ENODE or ICWF_ESOLVE the simulation is frozen at the
 * step where the condition was detected and further steps are refused.
 */
#ifndef ICWF_H
#define ICWF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct icwf_sim icwf_sim;

typedef enum {
    ICWF_OK = 0,
    ICWF_EINVAL = -1,     /* invalid configuration or argument                       */
    ICWF_ENOMEM = -2,     /* workspace smaller than icwf_workspace_bytes()          */
    ICWF_EDEVICE = -3,    /* a HIP call failed                                       */
    ICWF_ENONFINITE = -4, /* a non-finite value in the inputs or the state           */
    ICWF_ENODE = -5,      /* |Psi| < 1e-300 at a trajectory: velocity undefined      */
    ICWF_ESOLVE = -6,     /* S + eps I not numerically positive definite             */
    ICWF_ESTATE = -7,     /* call not valid in the handle's state (e.g. after error) */
    ICWF_ETIMEDOUT = -8   /* a bounded wait ended before its condition held          */
} icwf_status;

typedef enum {
    ICWF_MODEL_SHIN_METIU = 1, /* params: L, R_f, R_l, R_r (erf-softened Coulomb)     */
    ICWF_MODEL_CAVITY = 2      /* params: depth, softening, omega, lambda             */
} icwf_model;

typedef enum {
    ICWF_PREC_FP64 = 0,  /* every step in FP64                                        */
    ICWF_PREC_MIXED = 1, /* Eq. 9b's two-body contraction in FP32 on the matrix cores,
                            accumulated in FP32 inside each R tile and in FP64 across
                            tiles; everything else FP64                              */
    ICWF_PREC_SEPARABLE = 2 /* FP64 throughout, Eq. 9b's two-body sum taken through a
                            sum of products W_c(r_i, R_j) = sum_k u_k(r_i) v_k(R_j)
                            of at most 64 terms, found at creation by cross
                            approximation of the W_c table until its residual is
                            below 4 FP64 roundings of max |W_c| (exact rank 1 for
                            the cavity coupling); creation fails with ICWF_EINVAL
                            when no such sum exists                                 */
} icwf_precision;

/* How the RK4 stages solve (S + eps I) x = r (Eq. 8).  Both factor S + eps I
 * by Cholesky at every step; they differ in what the stages apply. */
typedef enum {
    ICWF_SOLVER_AUTO = 0,       /* explicit inverses from 1024 padded
                                   trajectories (a power of two), else
                                   triangular solves                             */
    ICWF_SOLVER_TRIANGULAR = 1, /* forward and backward substitution with the factor */
    ICWF_SOLVER_INVERSE = 2     /* (S + eps I)^-1 = L^-H L^-1 formed per step, each
                                   stage x0 = A^-1 r plus one refinement step
                                   x0 + A^-1 (r - A x0); needs the padded N (the
                                   next multiple of 64) to be a power of two,
                                   else ICWF_EINVAL; 7 more N x N complex
                                   matrices of workspace                       */
} icwf_solver;

/* How every CWF advances over a step (Eqs. 5-6, conditioning frozen at the
 * step start). */
typedef enum {
    ICWF_PROP_SPLIT = 0,          /* Strang split operator with the spectral kinetic
                                     energy (the default; the paper gives no scheme)  */
    ICWF_PROP_CRANK_NICOLSON = 1  /* (1 + i dt/2 H) psi' = (1 - i dt/2 H) psi with the
                                     periodic three-point Laplacian, solved per CWF by
                                     cyclic reduction; n_r, n_R <= 2048, else
                                     ICWF_EINVAL                                       */
} icwf_propagator;

/* How the trajectories follow the Bohmian velocity field of Eqs. 10-11 over a
 * step (the paper fixes the field, not the integrator). */
typedef enum {
    ICWF_TRAJ_EULER = 0,  /* x_k+1 = x_k + dt v(x_k, t_k) (the default)                      */
    ICWF_TRAJ_HEUN = 1    /* predictor x~ = x_k + dt v(x_k, t_k); after the CWFs and C have
                             advanced, x_k+1 = x_k + dt/2 (v(x_k, t_k) + v(x~, t_k+1)), the
                             field of the new state evaluated at x~; the CWF propagation
                             stays conditioned on x_k; K_k+1 at the corrected positions   */
} icwf_trajectories;

typedef struct {
    int32_t n_traj;          /* N: trajectories = basis size of Eq. 7 (the paper's M)   */
    int32_t n_r, n_R;        /* grid points: powers of two, 32 <= n <= 4096             */
    double r_min, r_max;     /* periodic box of species 1 (electron)                    */
    double R_min, R_max;     /* periodic box of species 2 (nucleus / photon mode)       */
    double m_r, m_R;         /* masses m_1, m_2 of Eq. 2                                */
    double dt;               /* time step > 0                                           */
    int32_t model;           /* icwf_model                                              */
    double model_params[8];  /* model parameters, see icwf_model                        */
    double tikhonov_eps;     /* eps >= 0 of (S + eps I); S_aa = 1 for unit-norm CWFs    */
    int32_t precision;       /* icwf_precision                                          */
    int32_t n_bo;            /* BO states used by the populations (0: none)             */
    int32_t solver;          /* icwf_solver (0: automatic)                              */
    int32_t propagator;      /* icwf_propagator (0: split operator)                     */
    int32_t trajectories;    /* icwf_trajectories (0: explicit Euler)                   */
} icwf_config;

/* Observables at the current step (text around the Shin-Metiu figure of the
 * paper).  Every array is caller-allocated host memory; a NULL array is
 * skipped.  P_n is not divided by the norm. */
typedef struct {
    double t;                 /* out: time                                               */
    int64_t step;             /* out: steps taken                                        */
    double norm;              /* out: C^H S C                                            */
    double *rho_r;            /* [n_r]: int dR |Psi(r_i, R)|^2                           */
    double *rho_R;            /* [n_R]: int dr |Psi(r, R_j)|^2                           */
    double *pop;              /* [n_bo]: P_n = int dR |chi^(n)(R)|^2                     */
    double *D;                /* [n_bo * n_bo]: D_nm = int dR |chi^(n)|^2 |chi^(m)|^2     */
    double *r, *R;            /* [N]: trajectory positions                               */
    double *C;                /* [N][2]: coefficients                                    */
    int32_t n_out_of_box;     /* out: trajectories outside their box after the last step */
    double min_abs_psi;       /* out: min_a |Psi(r^a, R^a)| at the last velocity step    */
} icwf_obs;

/* Bytes of device workspace icwf_create needs for this configuration
 * (0 if the configuration is invalid).  This is the admission footprint. */
size_t icwf_workspace_bytes(const icwf_config *cfg);

/* Create a simulation (the start of Eq. 7's evolution).
 *   r0, R0       [N] host: trajectory positions at t = 0.
 *   psi1_0       [N][n_r][2] host: electronic CWFs psi_1^a (Eq. 3 slices).
 *   psi2_0       [N][n_R][2] host: nuclear/photonic CWFs psi_2^a (Eq. 4 slices).
 *   C0           [N][2] host coefficients, or NULL: then C0 = (S_0 + eps I)^-1 b0.
 *   b0           [N][2] host: <psi_1^a psi_2^a | Psi_0>, used when C0 == NULL.
 *   bo_states    [n_R][n_bo][n_r] host, real, grid-normalised BO states
 *                phi_n(r_i; R_j), or NULL when n_bo == 0.
 *   workspace    device memory of ws_bytes >= icwf_workspace_bytes(cfg) bytes,
 *                256-byte aligned.
 *   hip_stream   hipStream_t the work is enqueued on (NULL: the null stream).
 * Computes S_0, K_0 and the Cholesky factor of S_0 + eps I on the device and
 * returns after they are done.  Errors: EINVAL, ENOMEM, ENONFINITE (inputs),
 * ESOLVE (S_0 + eps I not positive definite), EDEVICE. */
icwf_status icwf_create(const icwf_config *cfg, const double *r0, const double *R0,
                        const double *psi1_0, const double *psi2_0, const double *C0,
                        const double *b0, const double *bo_states, void *workspace,
                        size_t ws_bytes, void *hip_stream, icwf_sim **out);

/* Enqueue n_steps steps (velocities, trajectory update, CWF propagation,
 * Eq. 9 matrices, RK4 of Eq. 8) on the handle's stream; returns without
 * waiting.  Errors raised on the device (ENODE, ESOLVE, ENONFINITE) are
 * reported by the next call that synchronises (icwf_sync, icwf_observables);
 * the device stops advancing the state as soon as one is raised. */
icwf_status icwf_step(icwf_sim *sim, int32_t n_steps);

/* Enqueue n_steps steps of n_sims simulations at once: every kernel of the
 * step is one launch for all of them (grid dimension z runs over the
 * simulations, each kernel finds its simulation's buffers and model
 * parameters in that simulation's workspace).  Each simulation's arithmetic,
 * launch shapes and summation orders are those of icwf_step, so its result is
 * bitwise the one icwf_step gives it; what the batch saves is launches (the
 * small simulations of a serving mix are launch-bound).  Conditions (else
 * ICWF_EINVAL, state untouched): 1 <= n_sims <= 64, distinct handles on one
 * stream, at the same step parity, each one that steps on a single stream
 * without the explicit inverses (padded N < 1024) and without per-kernel
 * timing, and all alike in N, grids, boxes, masses, dt, eps, model kind,
 * precision (and contraction rank in blocks of 16), propagator, trajectory
 * integrator and n_bo; model parameters may differ.  A handle stopped by an
 * earlier error is ICWF_ESTATE.  Errors raised on the device stop only the
 * simulation that raised them (reported by its next synchronising call).
 * The handles of sims[] are caller-owned; the first one's workspace holds the
 * batch's offset table. */
icwf_status icwf_step_batch(icwf_sim *const *sims, int32_t n_sims, int32_t n_steps);

/* Wait for the handle's work and return its device status. */
icwf_status icwf_sync(icwf_sim *sim);

/* Synchronise, compute the observables on the device, copy them into the
 * caller's arrays. */
icwf_status icwf_observables(icwf_sim *sim, icwf_obs *out);

/* Synchronise and copy the state out (checkpoint): r, R [N]; psi1 [N][n_r][2];
 * psi2 [N][n_R][2]; C [N][2].  Any pointer may be NULL.  Passing them back to
 * icwf_create (with C0) resumes the run. */
icwf_status icwf_get_state(icwf_sim *sim, double *r, double *R, double *psi1, double *psi2,
                           double *C);

/* Synchronise and copy the current step's matrices (Eq. 9 at the current
 * CWFs and positions): S [N][N][2] (Eq. 9a), K [N][N][2] = W - W1 - W2 (Eq. 8),
 * Wc [N][N][2] = the two-body contraction of Eq. 9b with only the coupling part
 * W_c of the interaction (W = V_1(r) + V_2(R) + W_c(r, R)).  NULL skips. */
icwf_status icwf_get_matrices(icwf_sim *sim, double *S, double *K, double *Wc);

/* Synchronise and evaluate Eqs. 10-11 at the current state without stepping:
 * v_r, v_R [N]; psi_at [N][2] = Psi(r^a, R^a).  NULL skips. */
icwf_status icwf_velocities(icwf_sim *sim, double *v_r, double *v_R, double *psi_at);

/* Per-kernel timing with HIP events on the handle's stream.  enable != 0
 * makes icwf_step launch kernel by kernel (no graph replay) and record an
 * event pair around every launch of the named kernels; 0 turns it off and
 * clears the records. */
icwf_status icwf_set_timing(icwf_sim *sim, int32_t enable);

/* Synchronise and report, for the kernel called `name` ("wc_contract",
 * "propagate", "velocity", "zgemm", "cholesky", "rk4", "assemble"), the
 * number of timed launches and their summed duration in milliseconds. */
icwf_status icwf_kernel_time(icwf_sim *sim, const char *name, int64_t *launches,
                             double *total_ms);

/* Number of terms K of the sum of products W_c = sum_k u_k v_k the handle's
 * two-body contraction uses (Eq. 9b): the rank-K FP64 part of
 * ICWF_PREC_MIXED, the whole contraction of ICWF_PREC_SEPARABLE, 0 for
 * ICWF_PREC_FP64.  *rank: caller-owned host int32.  ICWF_EINVAL on NULL. */
icwf_status icwf_contraction_rank(const icwf_sim *sim, int32_t *rank);

/* Release the handle (not the workspace).  NULL is ignored. */
void icwf_destroy(icwf_sim *sim);

/* Last error message of a handle (never NULL), or of the last failed create
 * when sim == NULL. */
const char *icwf_last_error(const icwf_sim *sim);

/* Name of a status code. */
const char *icwf_status_string(int32_t status);

#ifdef __cplusplus
}
#endif

#endif /* ICWF_H */
