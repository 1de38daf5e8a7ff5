/* Exact (grid) propagation of the full two-dimensional wavefunction.
 *
 * Eq. 1 with the Hamiltonian of Eq. 2 (no vector potentials) on the product
 * grid r_i x R_j: the many-body wavefunction the ICWF ansatz of Eq. 7
 * approximates, propagated by the Strang split operator
 *     Psi <- e^{-i W dt/2} F^-1 [ e^{-i (k_r^2/2m_r + k_R^2/2m_R) dt} F [ e^{-i W dt/2} Psi ] ]
 * (F the two-dimensional discrete Fourier transform, W the full interaction of
 * the model, one-coordinate parts included).  It stores n_r n_R values where
 * the ansatz stores N (n_r + n_R), and serves as the reference that ICWF
 * results converge to as N grows.
 *
 * The configuration is the icwf_config of icwf.h; n_traj, tikhonov_eps,
 * precision and solver are ignored (n_traj must still be valid).  Grids,
 * boxes, masses, dt, model, model_params and n_bo are used as there.
 */
#ifndef ICWF_EXACT_H
#define ICWF_EXACT_H

#include <stddef.h>
#include <stdint.h>

#include "icwf.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct icwf_exact icwf_exact;

/* Bytes of device workspace icwf_exact_create needs (0 if the configuration
 * is invalid): the state, one scratch copy and the potential phase table
 * (three n_r n_R complex128 arrays), the kinetic phase (one factor per
 * coordinate) and the BO states. */
size_t icwf_exact_workspace_bytes(const icwf_config *cfg);

/* Create a grid propagation from Psi_0.
 *   psi0        [n_r][n_R][2] host: Psi_0(r_i, R_j), interleaved complex,
 *               row-major with R fastest (not renormalised).
 *   bo_states   [n_R][n_bo][n_r] host, real BO states phi_n(r_i; R_j), or NULL
 *               when n_bo == 0 (the same layout as icwf_create).
 *   workspace   device memory of ws_bytes >= icwf_exact_workspace_bytes(cfg),
 *               256-byte aligned; owned by the caller, untouched after destroy.
 *   hip_stream  hipStream_t the work is enqueued on (NULL: the null stream).
 * Errors: ICWF_EINVAL (configuration, NULL or short arguments; the message is
 * in icwf_last_error(NULL)), ICWF_ENONFINITE (non-finite input or a model
 * singular on the grid), ICWF_EDEVICE. */
icwf_status icwf_exact_create(const icwf_config *cfg, const double *psi0, const double *bo_states, void *workspace,
                              size_t ws_bytes, void *hip_stream, icwf_exact **out);

/* Enqueue n_steps >= 0 steps of dt (2 n_steps + 1 kernels: the half-step
 * phases of consecutive steps meet in one pass); does not wait. */
icwf_status icwf_exact_step(icwf_exact *ex, int64_t n_steps);

/* Wait for the enqueued work, then the observables of Psi at the current
 * step into out (the icwf_obs of icwf.h): t, step, norm = hr hR sum |Psi|^2,
 * rho_r, rho_R, and with n_bo > 0 pop and D, with the same definitions as the
 * ansatz's (chi^(n)(R_j) = hr sum_i phi_n(r_i; R_j) Psi(r_i, R_j)).  The
 * trajectory fields (r, R, C) are ignored; n_out_of_box and min_abs_psi are
 * set to 0. */
icwf_status icwf_exact_observables(icwf_exact *ex, icwf_obs *out);

/* Wait, then copy Psi ([n_r][n_R][2] host) out. */
icwf_status icwf_exact_get_psi(icwf_exact *ex, double *psi);

/* Wait for the enqueued work and release the handle (NULL is a no-op). */
void icwf_exact_destroy(icwf_exact *ex);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * observables of icwf_exact_observables for a wavefunction the caller holds
 * on the device, with no handle and no workspace.  The intermediate BO
 * projections and partial sums live in a static device array of the library
 * (2 MiB, held on every GPU the library runs on until the process ends);
 * the call allocates nothing and does not synchronise.
 *   n_r, n_R     powers of two in [32, 4096]; h_r, h_R > 0 the grid spacings.
 *   n_bo         0 .. 16 BO states (the array's limit; more is ICWF_EINVAL).
 *   psi          device [n_r][n_R][2]: Psi(r_i, R_j), R fastest.
 *   bo_states    device [n_R][n_bo][n_r] real, or NULL when n_bo == 0.
 *   out          device [1 + n_r + n_R + n_bo + n_bo^2] doubles: norm,
 *                rho_r, rho_R, pop, D (the definitions of
 *                icwf_exact_observables), written when the stream reaches the
 *                work.
 *   hip_stream   the stream the kernels are enqueued on.
 * Every call on one GPU shares that GPU's array: calls whose work overlaps on
 * the device (other streams or threads) race and must be ordered by the
 * caller.  Errors: ICWF_EINVAL (sizes beyond the limits, NULL pointers; the
 * message is in icwf_last_error(NULL)), ICWF_EDEVICE. */
icwf_status icwf_grid_observables_noalloc(int32_t n_r, int32_t n_R, double h_r, double h_R, int32_t n_bo,
                                          const double *psi, const double *bo_states, double *out, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* ICWF_EXACT_H */
