/* Born-Oppenheimer electronic states on the grid, computed on the GPU.
 *
 * The paper's observables project the ansatz of Eq. 7 on the electronic
 * eigenstates phi_n(r; R) of the clamped-nucleus Hamiltonian
 * h_e(R) = T_1 + W(r, R) (the BO populations P_n and the decoherence
 * indicator D_nm, text around the Shin-Metiu figure), and its initial state is
 * the electron in the first excited BO state times a nuclear wavepacket.  This
 * call finds, for every value R_j of a list, the n_states lowest eigenpairs of
 * the grid operator
 *
 *     h_e(R_j) = T_spec + diag(W(r_i, R_j)),
 *
 * T_spec = F^-1 diag(k^2 / 2 m_r) F the same spectral kinetic operator the
 * propagation uses (periodic grid r_i = r_min + i h, k = 2 pi fftfreq(n_r, h)),
 * W the full model interaction (one-coordinate parts included).  Eigenvectors
 * are real, grid-normalised (h sum_i phi_n(r_i)^2 = 1), with the sign that
 * makes their largest-magnitude entry positive.
 *
 * Method (one work-group per R_j, one launch for the whole list): block
 * locally optimal preconditioned conjugate gradients (LOBPCG; Knyazev, SIAM J.
 * Sci. Comput. 23, 2001) on a block of n_states + guard vectors, h_e applied
 * through FFTs in LDS, the preconditioner (T_spec + c)^-1 with
 * c = max(1, max W - min W) over the grid, Rayleigh-Ritz on the orthonormalised
 * span of the block, its preconditioned residuals and the previous directions
 * (cyclic Jacobi on the small projected matrix), until every wanted residual
 * norm ||h_e phi - E phi|| is at most `tol`.
 */
#ifndef ICWF_BO_H
#define ICWF_BO_H

#include <stddef.h>
#include <stdint.h>

#include "icwf.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Most states per R value (the block, with its guard vectors, has at most
 * 12 columns). */
#define ICWF_BO_MAX_STATES 8

typedef struct {
    double tol;            /* in: residual norm bar (<= 0: 1e-11 * max(1, ||h_e|| bound))  */
    int32_t max_iter;      /* in: iteration cap (<= 0: 2000)                                 */
    int32_t iterations;    /* out: most iterations any R_j took                              */
    double max_residual;   /* out: largest final residual norm of a wanted state            */
    int32_t unconverged;   /* out: R values that hit the cap above the bar                   */
} icwf_bo_info;

/* Bytes of device workspace icwf_bo_states needs (0 if the arguments are
 * invalid).  cfg supplies n_r, the r box, m_r, the model and its parameters
 * (the other fields must still be valid). */
size_t icwf_bo_workspace_bytes(const icwf_config *cfg, int32_t n_values, int32_t n_states);

/* The n_states lowest eigenpairs of h_e(R_j) for j = 0 .. n_values - 1.
 *   R_values   [n_values] host: the clamped coordinate of species 2.
 *   states     [n_values][n_states][n_r] host out: phi_n(r_i; R_j), the layout
 *              icwf_create takes for its BO states (NULL skips).
 *   energies   [n_values][n_states] host out, ascending per R_j (NULL skips).
 *   workspace  device memory of ws_bytes >= icwf_bo_workspace_bytes(...),
 *              256-byte aligned, the caller's.
 *   hip_stream the stream the work runs on (NULL: the null stream); the call
 *              waits for it before returning.
 *   info       in/out (may be NULL: defaults, no report).
 * Errors: ICWF_EINVAL (arguments; n_states in [1, ICWF_BO_MAX_STATES] and at
 * most n_r / 4), ICWF_ENOMEM (workspace too small), ICWF_ENONFINITE (the model
 * is singular on the grid), ICWF_ESOLVE (some R_j did not reach the residual
 * bar within max_iter; the states are still written), ICWF_EDEVICE.  The
 * message is in icwf_last_error(NULL). */
icwf_status icwf_bo_states(const icwf_config *cfg, const double *R_values, int32_t n_values, int32_t n_states,
                           double *states, double *energies, void *workspace, size_t ws_bytes, void *hip_stream,
                           icwf_bo_info *info);

#ifdef __cplusplus
}
#endif

#endif /* ICWF_BO_H */
