/*
 * icwf_serve.h -- continuous batching of independent ICWF simulations on one
 * GPU (the serving form of the library in include/icwf.h).
 *
 * Each request is one complete simulation of the method (Eqs. 5-11 of
 * Albareda, Kelly, Rubio, arXiv:1805.11169): its own configuration (N, grids,
 * model parameters, precision), its own initial state and a number of steps.
 * Requests arrive while others run.  A scheduler thread owned by the server
 *   - admits requests in arrival order as soon as a slot and enough of the
 *     caller's device arena are free (the footprint is icwf_workspace_bytes of
 *     the request's configuration), so memory, not a fixed batch, bounds how
 *     many simulations are resident;
 *   - keeps every admitted simulation's CWFs, trajectories, coefficients and
 *     matrices resident in its block of the arena until it finishes;
 *   - advances every admitted simulation in turns of about equal device
 *     time: steps_per_turn steps for the costliest resident simulation, and
 *     for a cheaper one proportionally more (by an estimate of its step's
 *     cost from its configuration), each step a replay of the simulation's
 *     captured HIP graph on the slot's
 *     own stream (default priority), keeping up to turns_ahead turns queued,
 *     so the work of different simulations overlaps on the device; with
 *     batching on, small simulations of one shape instead share a lane and
 *     each of their turns is one fused icwf_step_batch over the lane's
 *     simulations at the same step parity;
 *   - when a simulation's last step is done, computes its observables,
 *     releases its arena block and slot, and admits the next request.
 * A simulation's arithmetic does not depend on what else runs: its kernels,
 * launch shapes and summation orders are those of icwf_step, so its result
 * is bitwise the one it has when run alone.
 *
 * Ownership: the arena is caller-owned device memory, 256-byte aligned, and
 * must outlive the server.  Host arrays passed to icwf_server_submit are
 * copied before it returns.  Results stay with the server until
 * icwf_server_result copies them out.  All calls are thread-safe.
 */
#ifndef ICWF_SERVE_H
#define ICWF_SERVE_H

#include "icwf.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct icwf_server icwf_server;

typedef struct {
    int32_t max_active;      /* slots: simulations resident and stepping at once, 1..64        */
    int32_t steps_per_turn;  /* steps per scheduling turn of the costliest resident simulation
                                (cheaper ones take proportionally more), >= 1                  */
    int32_t turns_ahead;     /* turns kept queued on a slot's stream, 1..4                      */
    int32_t device;          /* HIP device the arena lives on                                   */
    int32_t batch;           /* 0: every simulation on its own slot stream; 1: simulations of one
                                shape (icwf_step_batch's conditions, padded N < 1024) share a lane
                                stream and advance together through icwf_step_batch, one
                                launch per kernel for the whole lane (the simulations' own
                                arithmetic is unchanged)                                       */
} icwf_server_config;

/* Timing and outcome of one request; times in seconds on the server's clock
 * (icwf_server_clock). */
typedef struct {
    int64_t id;
    int32_t status;          /* icwf_status of the simulation: OK or the error that stopped it   */
    int32_t slot;            /* slot it ran in (-1 if it was never admitted)                    */
    int64_t steps;           /* steps it took                                                   */
    double t_submit;         /* request arrival                                                 */
    double t_admit;          /* admission (arena block and slot granted, simulation created)    */
    double t_done;           /* result ready                                                    */
    size_t workspace_bytes;  /* arena bytes it held                                             */
    char message[192];       /* error message when status != OK, else ""                        */
} icwf_request_info;

typedef struct {
    int64_t submitted, admitted, completed, failed;
    int32_t active, pending;
    size_t arena_bytes;      /* usable arena                                                    */
    size_t arena_in_use;     /* bytes held by resident simulations now                          */
    size_t arena_peak;       /* largest arena_in_use so far                                     */
    int32_t peak_active;     /* most simulations resident at once so far                        */
} icwf_server_stats;

/* Start a server over arena[0, arena_bytes).  Errors: EINVAL (bad config,
 * NULL or unaligned arena), EDEVICE. */
icwf_status icwf_server_create(const icwf_server_config *cfg, void *arena, size_t arena_bytes,
                               icwf_server **out);

/* Queue one simulation: the arguments of icwf_create (host arrays, copied
 * here) and the number of steps.  Returns its id in *id.  Errors: EINVAL
 * (invalid configuration, n_steps < 0), ENOMEM (its footprint exceeds the
 * whole arena: it could never be admitted), ENONFINITE, ESTATE (server
 * stopping). */
icwf_status icwf_server_submit(icwf_server *srv, const icwf_config *cfg, const double *r0,
                               const double *R0, const double *psi1_0, const double *psi2_0,
                               const double *C0, const double *b0, const double *bo_states,
                               int32_t n_steps, int64_t *id);

/* Wait until request id has its result, at most timeout_s seconds (< 0: no
 * limit).  Returns OK when the result is ready (whatever the simulation's own
 * status), ESTATE for an unknown id, ETIMEDOUT when the time ran out. */
icwf_status icwf_server_wait(icwf_server *srv, int64_t id, double timeout_s);

/* Copy a finished request's final observables into out (caller arrays sized
 * for its configuration; NULL arrays skipped) and its info; then forget the
 * request.  Returns the simulation's own status (OK, or the error that
 * stopped it), or ESTATE if id is unknown or not finished. */
icwf_status icwf_server_result(icwf_server *srv, int64_t id, icwf_obs *out, icwf_request_info *info);

/* Counters of the server. */
icwf_status icwf_server_get_stats(icwf_server *srv, icwf_server_stats *out);

/* Seconds since the server started (the clock of icwf_request_info). */
double icwf_server_clock(const icwf_server *srv);

/* Stop admitting, finish the admitted simulations, drop the pending ones,
 * join the scheduler thread and release the streams.  NULL is ignored. */
void icwf_server_destroy(icwf_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* ICWF_SERVE_H */
