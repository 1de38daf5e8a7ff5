// Internal plan of one ICWF simulation: sizes, device buffers carved from the
// caller's workspace, and the host-side launchers of every kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/icwf.h"
#include "icwf_device.hpp"

namespace icwf {

struct Dims {
    int N, nr, nR, n_bo, prec;
    int lr_rank;                          // rank of the FP64 part of the mixed contraction
    int fp32_residual;                    // mixed form: the residual left to FP32 is not negligible
    int sinv;                             // RK4 stages through explicit inverses of S + eps I
    int propagator;                       // 0 split operator, 1 Crank-Nicolson
    int traj;                             // 0 explicit Euler trajectories, 1 Heun
    int wc_grid;                          // work-groups of the persistent two-body contraction
    int prop_grid[2];                     // work-groups of the persistent propagation, per species
    double r_min, hr, R_min, hR, m_r, m_R, dt, eps;
    ModelParams mp;
    // batched launches (icwf_step_batch): `batch` simulations of the same shape
    // per launch, the k-th at this one's addresses plus zoff[k] bytes (device
    // table); mpd this simulation's device copy of mp (each kernel reads its
    // own simulation's copy).  One simulation: batch = 1, zoff = nullptr.
    int batch = 1;
    const long long *zoff = nullptr;
    const ModelParams *mpd = nullptr;
};

// Trajectory count padded to the tile size every kernel assumes.  Padding
// rows hold zero CWFs and zero coefficients, so they add nothing to any sum,
// and S + eps I is eps I on them.
constexpr int kPad = 64;
inline int padded(int N) { return (N + kPad - 1) / kPad * kPad; }
constexpr int kCholNb = 64;      // Cholesky panel width
constexpr int kLowRankMax = 64;  // most terms of a sum-of-products W_c (mixed and separable forms)
constexpr int kWcReserve = 64;   // CU slots the persistent contraction leaves to the other stream
constexpr int kWcSplitMax = 512; // most tiles the contraction splits at the end of its queue
constexpr int kWcParts = 4;      // units per split tile (FP64 step at N = 1024: 6.32 ms with 2, 6.27 with 4)
// Tiles the split applies to for Np padded trajectories: the last round of
// the persistent contraction, at most all tiles.
inline int wc_split_tiles(int Np) {
    const int t = Np / 16;
    const int tiles = t * (t + 1) / 2;
    return tiles < kWcSplitMax ? tiles : kWcSplitMax;
}
// The contraction's tiles come from one queue per XCD (each XCD's L2 then
// holds the psi1 rows of its own compact group of tiles); each queue splits
// at most ceil(split tiles / queues) of its tiles.
constexpr int kWcQueues = 8;
inline int wc_split_per_queue(int nsplit) { return (nsplit + kWcQueues - 1) / kWcQueues; }
inline int wc_split_slots(int Np) { return kWcQueues * wc_split_per_queue(wc_split_tiles(Np)); }
// Order of the 16 x 16 pair tiles (triangle index ta (ta + 1) / 2 + tb,
// tb <= ta) in which the queues hand them out: blocks of 8 x 8 tiles, so that
// consecutive tiles share their rows.
std::vector<int32_t> wc_tile_order(int Np);

struct Bufs {
    double2 *psi1, *psi2;                 // [N][nr], [N][nR] CWFs (Eq. 7)
    double *r, *R, *r_new, *R_new;        // trajectory positions at t_k and t_k+1
    double2 *C, *Cacc, *Cstage;           // coefficients and RK4 stage vectors
    double2 *y;                           // forward-substitution result of an RK stage
    double2 *rhs;                         // K v of an RK stage
    double2 *vphase_r, *vphase_R;         // exp(-i V_1(r_i) dt/2), exp(-i V_2(R_j) dt/2)
    double2 *kin_r, *kin_R;               // exp(-i k^2 dt / 2m) / n, FFT order
    double2 *tw_r, *tw_R;                 // exp(-2 pi i k / n)
    double *wc64;                         // [nr][nR] W_c(r_i, R_j)
    float *wc32;                          // [nr][nR] FP32 residual of the rank-K split (mixed form)
    double *lr_u, *lr_v;                  // [kLowRankMax][nr], [kLowRankMax][nR] rank-K factors
    float2 *psi1_f32;                     // [Np][nr] FP32 copy of psi1 (mixed form only)
    double *sinc_r, *dsinc_r;             // [N][nr] periodic sinc and derivative at r^a
    double *sinc_R, *dsinc_R;             // [N][nR]
    double2 *vpart;                       // [Np/32][Np][3] velocity partial sums
    double *v_r, *v_R;                    // [N] velocities
    double2 *psi_at;                      // [N] Psi(r^a, R^a)
    double2 *cphase;                      // [2][Np] e^{-i V_2(R^a) dt/2}, e^{-i V_1(r^a) dt/2}: the
                                          // constant part of each CWF's conditioned potential (zero rows
                                          // past N)
    double2 *G1a, *G1b;                   // [N][nr] W_c(r_i, R^a) psi_1^a_i at x_k, x_k+1
    double2 *G2a, *G2b;                   // [N][nR] W_c(r^a, R_j) psi_2^a_j at x_k, x_k+1
    double2 *S1, *S2;                     // [N][N] single-species overlaps
    double2 *E1a, *E1b, *E2a, *E2b;       // [N][N] W_c-conditioned single-species integrals
    double2 *Wc;                          // [N][N] two-body contraction (W_c part of Eq. 9b)
    double2 *Smat[2], *Kmat[2];           // S_k, K_k (current / next by step parity)
    double2 *Kminus, *Kmid;               // K(psi_k+1, x_k) and the midpoint K
    double2 *L[2], *Lmid;                 // Cholesky factors of S + eps I (lower)
    double2 *Linv[2], *Linvmid;           // [Np][64] inverses of their 64 x 64 diagonal blocks
    double2 *Finv[2], *Finvmid;           // [Np][Np] L^-1 of L[0], L[1], Lmid (lower part; sinv only)
    double2 *Hinv[2], *Hinvmid;           // [Np][Np] L^-H, the conjugate transposes (upper part; sinv only)
    double2 *Tinv[2];                     // [Np][Np] scratch of the block inversion (sinv only)
    double2 *zvec;                        // [Np] L^-1 v of an RK stage (sinv only)
    double2 *chol_diag;                   // [2][64][64] factored diagonal blocks in flight
    double2 *xsol;                        // [Np] back-substitution result of an RK stage
    int32_t *solve_sync;                  // [130] block flags and tickets of the stage solves
    double *bo;                           // [nR][n_bo][nr] BO states
    double2 *obs_psi;                     // [nr][nR] Psi on the grid (observables)
    double2 *obs_chi;                     // [n_bo][nR]
    double *obs_part;                     // [kRhoSlices][nR] partial sums of rho_R
    double *obs_out;                      // packed observables
    int32_t *flags;                       // kNumFlags status flags
    int32_t *wc_queue;                    // [kWcQueues + wc_split_slots(Np)] unit counters of the persistent
                                          // two-body contractions (one per XCD queue), then the completion
                                          // counters of split tiles
    int32_t *wc_order;                    // [Np/16 (Np/16 + 1) / 2] tile order of the queues (wc_tile_order)
    double2 *wc_part;                     // [wc_split_slots(Np)][kWcParts][256] partial sums of split tiles
    double *scal;                         // small device scalars (min |Psi|, ...)
    ModelParams *mparams;                 // device copy of the model parameters
    long long *batch_tab;                 // [kMaxBatch] workspace offsets of a batch this simulation leads
};

// Most simulations one batched launch advances.
constexpr int kMaxBatch = 64;

// Workspace offsets (bytes) of a batch's simulations from its first one.
struct BatchTable {
    long long off[kMaxBatch];
};
// Writes the first n offsets into tab (device) in stream order.
void launch_set_table(long long *tab, const BatchTable &t, int n, hipStream_t s);

// RK4 through explicit inverses of S + eps I.  Automatic choice: from 1024
// padded trajectories, where the factorisations run on the second stream
// (the inversion then follows them there beside the FP64 or mixed
// contraction, or, in the separable form, whose contraction is the shorter
// branch, runs on the main stream after the join); each stage is then a few
// matrix-vector products instead of two chains of dependent block solves.
// Either way Np must be a power of two, so that the block inversion halves
// evenly.  solver: 0 automatic, 1 triangular, 2 inverse.
inline bool use_sinv(int Np, int precision, int solver) {
    const bool pow2 = (Np & (Np - 1)) == 0;
    if (solver == 2) return pow2;
    if (solver == 1) return false;
    return Np >= 1024 && pow2;
}

// ---- launchers (each defined next to its kernels) -------------------------------------------

// Split-operator step of every CWF of one species; species 1 = electronic
// (conditioned on R^a), 2 = nuclear (conditioned on r^a).
void launch_propagate(const Dims &d, const Bufs &b, int species, hipStream_t s);
// The same step by Crank-Nicolson (grids up to 2048 points); launch_propagate
// hands over to it when d.propagator == 1.
void launch_propagate_cn(const Dims &d, const Bufs &b, int species, hipStream_t s);

// Whether the split-operator propagation takes the short series for the
// Shin-Metiu coupling phase (a property of dt and R_f).
bool propagate_tiny_phase(const Dims &d);

// Work-groups of the persistent propagation for grid size n and N trajectories:
// as many as fit the device's ncu compute units at once, at most one per CWF group.
int propagate_grid(int n, int N, int ncu);

// Periodic-sinc tables at the positions, velocity contraction and reduction
// (v_r, v_R, psi_at, min |Psi| and the flags).  mode kVelocityOnly: at r, R,
// nothing else; kVelocityEuler: at r, R, and r_new, R_new = x + dt v plus the
// constant potential phases cphase of the CWFs conditioned on r, R (the step's
// first pass); kVelocityHeun: the field of the advanced state at the
// predictor r_new, R_new, then r = r_new = r + dt/2 (v_r + v), the same for R
// (v_r, v_R keep the first pass's values; the out-of-box count is redone).
enum VelocityMode { kVelocityOnly = 0, kVelocityEuler = 1, kVelocityHeun = 2 };
void launch_velocity(const Dims &d, const Bufs &b, VelocityMode mode, hipStream_t s);

// Conditioned kets G = W_c(., x) psi: G1a, G2a at x_k = (r, R) and, with
// `next`, G1b, G2b at x_k+1 = (r_new, R_new).
void launch_cond_kets(const Dims &d, const Bufs &b, hipStream_t s, bool next = true);
// G1b, G2b alone, at (r_new, R_new).
void launch_cond_kets_next(const Dims &d, const Bufs &b, hipStream_t s);

// Batched h * conj(X) Y^T complex products: the overlaps S1, S2 (parts &
// kSingleOverlaps: all that S needs) and the coupling integrals E1a, E2a
// and, with both_conditionings, E1b, E2b (parts & kSingleCouplings: needed by
// K only).
enum SingleParts { kSingleOverlaps = 1, kSingleCouplings = 2, kSingleAll = 3 };
void launch_single_species(const Dims &d, const Bufs &b, bool both_conditionings, hipStream_t s,
                           int parts = kSingleAll);
// E1b, E2b alone.
void launch_single_species_next(const Dims &d, const Bufs &b, hipStream_t s);

// Two-body contraction Wc (upper pair tiles), FP64 or FP32 matrix cores.
void launch_wc(const Dims &d, const Bufs &b, hipStream_t s);

// The step's matrices from the single-species and two-body blocks:
//   kAssembleS: S_next and the regularised midpoint / endpoint S + eps I;
//   kAssembleK: K_minus, K_next and the midpoint K;
//   kAssembleInitial: S_0, K_0 and S_0 + eps I (start of the run);
//   kAssembleKminus: K_minus and the midpoint K only (Heun trajectories);
//   kAssembleKnext: K_next only, at (r_new, R_new) (Heun, after the corrector).
enum AssemblePart {
    kAssembleS = 1,
    kAssembleK = 2,
    kAssembleInitial = 3,
    kAssembleKminus = 2 | 4,
    kAssembleKnext = 2 | 8
};
void launch_assemble(const Dims &d, const Bufs &b, int parity, AssemblePart part, hipStream_t s);

// In-place lower Cholesky of `count` matrices (A0, A1), each Np x Np, and the
// inverses of their 64 x 64 diagonal blocks into X0, X1 ([Np][64]).  With
// F0 non-null (d.sinv), the diagonal blocks of L^-1 go into F0, F1 as well
// and, with `inverses`, launch_factor_inverses completes them.
void launch_cholesky(const Dims &d, const Bufs &b, double2 *A0, double2 *A1, double2 *X0, double2 *X1, int count,
                     hipStream_t s, double2 *F0 = nullptr, double2 *F1 = nullptr, double2 *H0 = nullptr,
                     double2 *H1 = nullptr, bool inverses = true);
// The explicit inverses of `count` factors (A0, A1) whose diagonal blocks of
// L^-1 are in F0, F1 (launch_cholesky): L^-1 into F0, F1 ([Np][Np], by block
// recursion) and L^-H into H0, H1.
void launch_factor_inverses(const Dims &d, const Bufs &b, const double2 *A0, const double2 *A1, int count,
                            hipStream_t s, double2 *F0, double2 *F1, double2 *H0, double2 *H1);

// One RK4 step of Eq. 8 with the factors / matrices of the given parity.
void launch_rk4(const Dims &d, const Bufs &b, int parity, hipStream_t s);

// C = (L L^H)^-1 rhs with L = b.L[parity] (initial coefficients).
void launch_solve_initial(const Dims &d, const Bufs &b, int parity, double2 *rhs, hipStream_t s);

// Copy x_k+1 -> x_k (end of a step).
void launch_commit_positions(const Dims &d, const Bufs &b, hipStream_t s);

// Observables into b.obs_out (layout in icwf_api.cpp).
void launch_observables(const Dims &d, const Bufs &b, hipStream_t s);

// Observables of a wavefunction given on the grid, Psi [nr][nR] complex128:
// out = [norm, rho_r[nr], rho_R[nR], pop[n_bo], D[n_bo][n_bo]]; bo is
// [nR][n_bo][nr] (real BO states), chi [n_bo][nR] and part [kRhoSlices][nR]
// scratch.
constexpr int kRhoSlices = 32;   // row slices of the rho_R reduction (nr >= 32)
void launch_grid_observables(const double2 *Psi, int nr, int nR, double hr, double hR, int n_bo, const double *bo,
                             double2 *chi, double *part, double *out, hipStream_t s);

// One Strang step of the full two-dimensional wavefunction (Eqs. 1-2 on the
// product grid; the reference the ansatz converges to):
//   Psi <- e^{-i W dt/2} IFFT2[ e^{-i T dt} FFT2[ e^{-i W dt/2} Psi ] ].
// psi [nr][nR] in place, tmp [nR][nr] scratch, half [nr][nR] = e^{-i W dt/2};
// the kinetic phase e^{-i (k_r^2/2m_r + k_R^2/2m_R) dt} / (nr nR) is the
// product kin_r [nr] x kin_R [nR] (e^{-i k_r^2 dt/2m_r} and
// e^{-i k_R^2 dt/2m_R} / (nr nR)); tw_r [nr], tw_R [nR] = e^{-2 pi i k/n}.
// nr, nR powers of two in [32, 4096].
struct ExactBufs {
    double2 *psi, *tmp, *half, *kin_r, *kin_R, *tw_r, *tw_R;
};
// nsteps >= 0 whole steps (2 nsteps + 1 passes over the state).
void launch_exact_steps(int nr, int nR, const ExactBufs &e, int64_t nsteps, hipStream_t s);

// FP32 copy of psi1 (mixed form; the propagation keeps it current afterwards).
void launch_psi1_f32(const Dims &d, const Bufs &b, hipStream_t s);

// Fill n int32 with a value (graph-safe replacement for a memset); batched:
// the same n entries in each of `batch` workspaces (zoff as in the kernels).
void launch_fill_i32(int32_t *p, int n, int32_t v, hipStream_t s, int batch = 1, const long long *zoff = nullptr);

// Records the message icwf_last_error(NULL) returns (calls without a
// handle) and passes the status through.
icwf_status set_create_error(icwf_status st, const char *msg);

}  // namespace icwf
