// C ABI of the ICWF library (declared in include/icwf.h): validation, the
// workspace layout, the host-side tables, the per-step launch plan and its
// HIP-graph capture, and the copies in and out.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/icwf.h"
#include "../../include/icwf_exact.h"
#include "icwf_internal.hpp"
#include "icwf_plan.hpp"

using icwf::Bufs;
using icwf::Dims;

namespace {

thread_local std::string g_create_error = "";

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

// Layout of every device buffer inside the caller's workspace (256-byte
// aligned pieces).  With base == nullptr it only sizes.
struct Layout {
    size_t off = 0;
    char *base = nullptr;
    template <typename T>
    T *take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

size_t obs_len(int nr, int nR, int n_bo) { return 1 + (size_t)nr + nR + n_bo + (size_t)n_bo * n_bo; }

Bufs carve(const icwf_config &c, char *base, size_t *total) {
    Layout L;
    L.base = base;
    const size_t Np = icwf::padded(c.n_traj), nr = c.n_r, nR = c.n_R, nbo = c.n_bo;
    Bufs b{};
    b.flags = L.take<int32_t>(icwf::kNumFlags);
    b.wc_queue = L.take<int32_t>(icwf::kWcQueues + icwf::wc_split_slots((int)Np));
    b.wc_order = L.take<int32_t>((Np / 16) * (Np / 16 + 1) / 2);
    b.wc_part = L.take<double2>((size_t)icwf::wc_split_slots((int)Np) * icwf::kWcParts * 256);
    b.scal = L.take<double>(8);
    b.psi1 = L.take<double2>(Np * nr);
    b.psi2 = L.take<double2>(Np * nR);
    b.r = L.take<double>(Np);
    b.R = L.take<double>(Np);
    b.r_new = L.take<double>(Np);
    b.R_new = L.take<double>(Np);
    b.C = L.take<double2>(Np);
    b.Cacc = L.take<double2>(Np);
    b.Cstage = L.take<double2>(Np);
    b.y = L.take<double2>(Np);
    b.rhs = L.take<double2>(Np);
    b.vphase_r = L.take<double2>(nr);
    b.vphase_R = L.take<double2>(nR);
    b.kin_r = L.take<double2>(nr);
    b.kin_R = L.take<double2>(nR);
    b.tw_r = L.take<double2>(nr);
    b.tw_R = L.take<double2>(nR);
    b.wc64 = L.take<double>(nr * nR);
    b.wc32 = L.take<float>(nr * nR);
    const bool mixed = c.precision == ICWF_PREC_MIXED;
    b.psi1_f32 = L.take<float2>(mixed ? Np * nr : 1);
    b.lr_u = L.take<double>(icwf::kLowRankMax * nr);
    b.lr_v = L.take<double>(icwf::kLowRankMax * nR);
    b.sinc_r = L.take<double>(Np * nr);
    b.dsinc_r = L.take<double>(Np * nr);
    b.sinc_R = L.take<double>(Np * nR);
    b.dsinc_R = L.take<double>(Np * nR);
    b.vpart = L.take<double2>((Np / 32) * Np * 3);
    b.v_r = L.take<double>(Np);
    b.v_R = L.take<double>(Np);
    b.psi_at = L.take<double2>(Np);
    b.cphase = L.take<double2>(2 * (size_t)Np);
    b.G1a = L.take<double2>(Np * nr);
    b.G1b = L.take<double2>(Np * nr);
    b.G2a = L.take<double2>(Np * nR);
    b.G2b = L.take<double2>(Np * nR);
    double2 **mats[] = {&b.S1,      &b.S2,      &b.E1a,     &b.E1b,  &b.E2a,     &b.E2b,   &b.Wc,  &b.Smat[0],
                        &b.Smat[1], &b.Kmat[0], &b.Kmat[1], &b.Kminus, &b.Kmid, &b.L[0], &b.L[1], &b.Lmid};
    for (double2 **m : mats) *m = L.take<double2>(Np * Np);
    b.Linv[0] = L.take<double2>(Np * icwf::kCholNb);
    b.Linv[1] = L.take<double2>(Np * icwf::kCholNb);
    b.Linvmid = L.take<double2>(Np * icwf::kCholNb);
    {
        // explicit inverses for the RK4 stages (see use_sinv)
        const size_t nn = icwf::use_sinv((int)Np, c.precision, c.solver) ? Np * Np : 1;
        for (double2 **m : {&b.Finv[0], &b.Finv[1], &b.Finvmid, &b.Hinv[0], &b.Hinv[1], &b.Hinvmid, &b.Tinv[0],
                            &b.Tinv[1]})
            *m = L.take<double2>(nn);
        b.zvec = L.take<double2>(nn > 1 ? Np : 1);
    }
    b.chol_diag = L.take<double2>(2 * icwf::kCholNb * icwf::kCholNb);
    b.xsol = L.take<double2>(Np);
    b.solve_sync = L.take<int32_t>(130);
    b.bo = L.take<double>(std::max<size_t>(1, nR * nbo * nr));
    b.obs_psi = L.take<double2>(nr * nR);
    b.obs_chi = L.take<double2>(std::max<size_t>(1, nbo * nR));
    b.obs_part = L.take<double>(icwf::kRhoSlices * nR);
    b.obs_out = L.take<double>(obs_len(c.n_r, c.n_R, c.n_bo));
    b.mparams = L.take<icwf::ModelParams>(1);
    b.batch_tab = L.take<long long>(icwf::kMaxBatch);
    *total = (L.off + 255) & ~size_t(255);
    return b;
}

const char *validate(const icwf_config *c) {
    if (!c) return "config is NULL";
    if (c->n_traj < 1 || c->n_traj > 4096) return "n_traj must be in [1, 4096]";
    if (!is_pow2(c->n_r) || c->n_r < 32 || c->n_r > 4096) return "n_r must be a power of two in [32, 4096]";
    if (!is_pow2(c->n_R) || c->n_R < 32 || c->n_R > 4096) return "n_R must be a power of two in [32, 4096]";
    if (!(c->r_max > c->r_min) || !std::isfinite(c->r_min) || !std::isfinite(c->r_max)) return "bad r box";
    if (!(c->R_max > c->R_min) || !std::isfinite(c->R_min) || !std::isfinite(c->R_max)) return "bad R box";
    if (!(c->m_r > 0) || !(c->m_R > 0) || !std::isfinite(c->m_r) || !std::isfinite(c->m_R)) return "masses must be > 0";
    if (!(c->dt > 0) || !std::isfinite(c->dt)) return "dt must be > 0";
    if (!(c->tikhonov_eps >= 0) || !std::isfinite(c->tikhonov_eps)) return "tikhonov_eps must be >= 0";
    if (c->model != ICWF_MODEL_SHIN_METIU && c->model != ICWF_MODEL_CAVITY) return "unknown model";
    if (c->precision != ICWF_PREC_FP64 && c->precision != ICWF_PREC_MIXED && c->precision != ICWF_PREC_SEPARABLE)
        return "unknown precision";
    if (c->n_bo < 0 || c->n_bo > c->n_r) return "n_bo must be in [0, n_r]";
    if (c->solver < ICWF_SOLVER_AUTO || c->solver > ICWF_SOLVER_INVERSE) return "unknown solver";
    if (c->propagator != ICWF_PROP_SPLIT && c->propagator != ICWF_PROP_CRANK_NICOLSON) return "unknown propagator";
    if (c->trajectories != ICWF_TRAJ_EULER && c->trajectories != ICWF_TRAJ_HEUN) return "unknown trajectory integrator";
    if (c->propagator == ICWF_PROP_CRANK_NICOLSON && (c->n_r > 2048 || c->n_R > 2048))
        return "the Crank-Nicolson propagator takes grids of at most 2048 points";
    if (c->solver == ICWF_SOLVER_INVERSE && !icwf::use_sinv(icwf::padded(c->n_traj), c->precision, c->solver))
        return "the explicit-inverse solver needs the padded N (next multiple of 64) to be a power of two";
    for (int i = 0; i < 8; ++i)
        if (!std::isfinite(c->model_params[i])) return "model parameters must be finite";
    if (c->model == ICWF_MODEL_SHIN_METIU) {
        if (!(c->model_params[1] > 0) || !(c->model_params[2] > 0) || !(c->model_params[3] > 0))
            return "Shin-Metiu softening lengths must be > 0";
    }
    return nullptr;
}

// ---- host model (tables only; the step evaluates the model on the device) --------------------
double h_erfx(double x, double a) {
    const double ax = std::fabs(x), z = ax / a;
    if (z < 1e-4) return 2.0 / (std::sqrt(M_PI) * a) * (1.0 - z * z / 3.0 + z * z * z * z / 10.0);
    return std::erf(z) / ax;
}
double h_v1(const icwf_config &c, double r) {
    const double *p = c.model_params;
    if (c.model == ICWF_MODEL_SHIN_METIU) return -h_erfx(r - 0.5 * p[0], p[3]) - h_erfx(r + 0.5 * p[0], p[2]);
    return -p[0] / std::sqrt(r * r + p[1] * p[1]);
}
double h_v2(const icwf_config &c, double R) {
    const double *p = c.model_params;
    if (c.model == ICWF_MODEL_SHIN_METIU) return 1.0 / std::fabs(0.5 * p[0] - R) + 1.0 / std::fabs(0.5 * p[0] + R);
    return 0.5 * p[2] * p[2] * R * R;
}
double h_wc(const icwf_config &c, double r, double R) {
    const double *p = c.model_params;
    if (c.model == ICWF_MODEL_SHIN_METIU) return -h_erfx(r - R, p[1]);
    return p[3] * R * r;
}

// Adaptive cross approximation with full pivoting of an n x m row-major
// table: W = sum_k u_k v_k^T + R.  On return W holds the residual R; the
// factors are appended to U ([k][n]) and V ([k][m]).  Stops when
// max |R| <= tol max |W| or after kmax terms.  (Each step takes the largest
// remaining entry as pivot, so the residual's maximum never grows.)
int cross_approximation(std::vector<double> &W, int n, int m, double tol, int kmax, std::vector<double> &U,
                        std::vector<double> &V) {
    double wmax = 0.0;
    for (double w : W) wmax = std::max(wmax, std::fabs(w));
    int k = 0;
    for (; k < kmax; ++k) {
        size_t piv = 0;
        double best = -1.0;
        for (size_t e = 0; e < W.size(); ++e)
            if (std::fabs(W[e]) > best) {
                best = std::fabs(W[e]);
                piv = e;
            }
        if (best <= tol * wmax || best == 0.0) break;
        const int pi = (int)(piv / m), pj = (int)(piv % m);
        const double p = W[piv];
        std::vector<double> u(n), v(m);
        for (int i = 0; i < n; ++i) u[i] = W[(size_t)i * m + pj];
        for (int j = 0; j < m; ++j) v[j] = W[(size_t)pi * m + j] / p;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < m; ++j) W[(size_t)i * m + j] -= u[i] * v[j];
        U.insert(U.end(), u.begin(), u.end());
        V.insert(V.end(), v.begin(), v.end());
    }
    return k;
}

// Largest relative residual the mixed form leaves to FP32 (more terms are
// taken where they fill the FP64 part's last block of 16).
constexpr double kMixedSplitTol = 1e-4;
// Residual the separable form accepts: a few roundings of the table itself.
constexpr double kSeparableTol = 4.0 * 2.220446049250313e-16;

struct Timer {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> recs;
    int64_t launches = 0;
    double total_ms = 0.0;
};

}  // namespace

namespace icwf {
icwf_status set_create_error(icwf_status st, const char *msg) {
    g_create_error = msg ? msg : "";
    return st;
}
}  // namespace icwf

struct icwf_sim {
    icwf_config cfg{};
    Dims d{};
    Bufs b{};
    int Np = 0;
    hipStream_t stream = nullptr;
    hipStream_t capture_stream = nullptr;
    hipStream_t side_stream = nullptr;        // the S assembly and the factorisations, beside the contraction
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    std::map<int, hipGraphExec_t> batch_exec;  // steps of batches this simulation leads, by 2 x size + parity
    int parity = 0;
    int64_t step = 0;
    double t = 0.0;
    int status = ICWF_OK;        // sticky device error once seen
    bool timing = false;
    std::map<std::string, Timer> timers;
    std::vector<hipEvent_t> event_pool;
    std::string err;
};

namespace {

icwf_status fail(icwf_sim *s, icwf_status st, const std::string &msg) {
    if (s) s->err = msg;
    else g_create_error = msg;
    return st;
}

#define HIP_OK(call, sim)                                                                               \
    do {                                                                                                \
        hipError_t e_ = (call);                                                                         \
        if (e_ != hipSuccess) return fail(sim, ICWF_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

hipEvent_t get_event(icwf_sim *s) {
    if (!s->event_pool.empty()) {
        hipEvent_t e = s->event_pool.back();
        s->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

// Runs `fn` on stream st, bracketed by an event pair when timing.
template <typename F>
void timed(icwf_sim *s, const char *name, hipStream_t st, F fn) {
    if (!s->timing) {
        fn();
        return;
    }
    hipEvent_t a = get_event(s), b = get_event(s);
    (void)hipEventRecord(a, st);
    fn();
    (void)hipEventRecord(b, st);
    s->timers[name].recs.emplace_back(a, b);
}

// One step on stream st.  The two-body contraction needs neither the
// single-species integrals nor the Cholesky factorisations, which need only S:
// from kOverlapMinN padded trajectories on, the step forks, the side stream
// assembles S and factors S + eps I (in the FP64 form, where the contraction
// is the longest branch, after computing the single-species integrals
// itself) while st contracts W_c (in the separable form, whose contraction is
// short, followed by the coupling integrals); st then waits for the side
// stream, assembles K and runs the RK4 stages.  The persistent contraction leaves CU slots free for the side
// stream's latency-bound kernels.  Smaller simulations (whose contraction
// does not fill the GPU, and which a server runs many at a time) stay on one
// stream: event waits between streams would serialise other simulations'
// work queued behind them on the shared hardware queues.
constexpr int kOverlapMinN = 1024;

void enqueue_step(icwf_sim *s, const Dims &d, int parity, hipStream_t st, hipStream_t side) {
    if (s->Np < kOverlapMinN) side = st;
    const Bufs &b = s->b;
    const bool heun = d.traj == ICWF_TRAJ_HEUN;
    timed(s, "velocity", st, [&] { icwf::launch_velocity(d, b, icwf::kVelocityEuler, st); });
    timed(s, "propagate", st, [&] {
        icwf::launch_propagate(d, b, 1, st);
        icwf::launch_propagate(d, b, 2, st);
    });
    const bool fork = side != st;
    // the single-species integrals join the side stream where the contraction
    // leaves room beside the factorisations: FP64 without the explicit inverses
    // (which otherwise take that room), or a dense contraction whose cost per
    // pair, n_r n_R, is at least 256 N (the factorisations and inversions, N^3,
    // then take a small part of its time); otherwise they stay on st, ahead of
    // the fork
    const bool roomy = d.prec != ICWF_PREC_SEPARABLE && (size_t)d.nr * d.nR >= 256 * (size_t)s->Np;
    const hipStream_t ss = fork && ((d.prec == ICWF_PREC_FP64 && !d.sinv) || roomy) ? side : st;
    // the separable form's contraction is the short branch: ahead of the fork
    // only the overlaps (all that S needs), the coupling integrals (needed by
    // K only) on st after the contraction, while the factorisation stream
    // still runs
    const bool late_couplings = fork && ss == st && d.prec == ICWF_PREC_SEPARABLE;
    auto single_species = [&](hipStream_t q, int parts) {
        // with Heun trajectories the integrals at x_k+1 wait for the corrector
        timed(s, "zgemm", q, [&] {
            if (parts & icwf::kSingleCouplings) icwf::launch_cond_kets(d, b, q, !heun);
            icwf::launch_single_species(d, b, !heun, q, parts);
        });
    };
    if (ss == st) single_species(st, late_couplings ? icwf::kSingleOverlaps : icwf::kSingleAll);
    if (fork) {
        (void)hipEventRecord(s->ev_fork, st);
        (void)hipStreamWaitEvent(side, s->ev_fork, 0);
    }
    if (ss != st) single_species(ss, icwf::kSingleAll);
    // with the factorisations as the longer branch (the separable form), the
    // explicit inverses wait for the join and then take the whole GPU on st
    // instead of stretching the second stream further
    const bool late_inverses = late_couplings && d.sinv;
    timed(s, "cholesky", side, [&] {
        icwf::launch_assemble(d, b, parity, icwf::kAssembleS, side);
        if (d.sinv)
            icwf::launch_cholesky(d, b, b.Lmid, b.L[1 - parity], b.Linvmid, b.Linv[1 - parity], 2, side, b.Finvmid,
                                  b.Finv[1 - parity], b.Hinvmid, b.Hinv[1 - parity], !late_inverses);
        else
            icwf::launch_cholesky(d, b, b.Lmid, b.L[1 - parity], b.Linvmid, b.Linv[1 - parity], 2, side);
    });
    if (fork) (void)hipEventRecord(s->ev_join, side);
    timed(s, "wc_contract", st, [&] { icwf::launch_wc(d, b, st); });
    if (late_couplings) single_species(st, icwf::kSingleCouplings);
    if (fork) (void)hipStreamWaitEvent(st, s->ev_join, 0);
    if (late_inverses)
        timed(s, "inverse", st, [&] {
            icwf::launch_factor_inverses(d, b, b.Lmid, b.L[1 - parity], 2, st, b.Finvmid, b.Finv[1 - parity],
                                         b.Hinvmid, b.Hinv[1 - parity]);
        });
    timed(s, "assemble", st, [&] {
        icwf::launch_assemble(d, b, parity, heun ? icwf::kAssembleKminus : icwf::kAssembleK, st);
    });
    timed(s, "rk4", st, [&] { icwf::launch_rk4(d, b, parity, st); });
    if (heun) {
        // corrector at the advanced state, then K_k+1 at the corrected positions
        timed(s, "velocity", st, [&] { icwf::launch_velocity(d, b, icwf::kVelocityHeun, st); });
        timed(s, "zgemm", st, [&] {
            icwf::launch_cond_kets_next(d, b, st);
            icwf::launch_single_species_next(d, b, st);
        });
        timed(s, "assemble", st, [&] { icwf::launch_assemble(d, b, parity, icwf::kAssembleKnext, st); });
    }
}

icwf_status device_status(icwf_sim *s) {
    int32_t flags[icwf::kNumFlags];
    HIP_OK(hipMemcpyAsync(flags, s->b.flags, sizeof(flags), hipMemcpyDeviceToHost, s->stream), s);
    HIP_OK(hipStreamSynchronize(s->stream), s);
    if (flags[icwf::kFlagNode]) {
        s->status = ICWF_ENODE;
        return fail(s, ICWF_ENODE, "a trajectory sits at a node of the ansatz wavefunction (|Psi| < 1e-300)");
    }
    if (flags[icwf::kFlagSolve]) {
        s->status = ICWF_ESOLVE;
        return fail(s, ICWF_ESOLVE, "S + eps I is not numerically positive definite");
    }
    if (flags[icwf::kFlagHang]) {
        s->status = ICWF_EDEVICE;
        return fail(s, ICWF_EDEVICE, "a device-side wait between work-groups timed out");
    }
    if (flags[icwf::kFlagNonfinite]) {
        s->status = ICWF_ENONFINITE;
        return fail(s, ICWF_ENONFINITE, "non-finite value in the coefficients or positions");
    }
    return ICWF_OK;
}

icwf_status capture_graphs(icwf_sim *s) {
    for (int p = 0; p < 2; ++p) {
        hipGraph_t g = nullptr;
        HIP_OK(hipStreamBeginCapture(s->capture_stream, hipStreamCaptureModeThreadLocal), s);
        enqueue_step(s, s->d, p, s->capture_stream, s->side_stream);
        HIP_OK(hipStreamEndCapture(s->capture_stream, &g), s);
        HIP_OK(hipGraphInstantiate(&s->exec[p], g, nullptr, nullptr, 0), s);
        HIP_OK(hipGraphDestroy(g), s);
    }
    return ICWF_OK;
}

// The shape and parameters every launch of a batched step shares: equal keys
// give equal launch shapes, equal workspace layouts and equal host-side
// launch arguments (each simulation's model parameters are read from its own
// workspace).  False: the simulation steps alone (a forked step on a second
// stream, explicit inverses, or per-kernel timing).
bool batch_key(const icwf_sim *s, std::string *key) {
    const Dims &d = s->d;
    if (s->Np >= kOverlapMinN || d.sinv || s->timing) return false;
    auto bits = [](double x) {
        uint64_t u;
        std::memcpy(&u, &x, sizeof(u));
        return std::to_string(u);
    };
    std::string k;
    for (int v : {d.N, d.nr, d.nR, d.n_bo, d.prec, (d.lr_rank + 15) / 16, d.fp32_residual, d.propagator, d.traj,
                  d.wc_grid, d.prop_grid[0], d.prop_grid[1], (int)d.mp.kind, icwf::propagate_tiny_phase(d) ? 1 : 0})
        k += std::to_string(v) + ",";
    for (double v : {d.r_min, d.hr, d.R_min, d.hR, d.m_r, d.m_R, d.dt, d.eps}) k += bits(v) + ",";
    *key = k;
    return true;
}

// strided copy of the leading N x N block of an Np x Np complex matrix
icwf_status copy_matrix_out(icwf_sim *s, const double2 *dev, double *host) {
    const int N = s->cfg.n_traj;
    HIP_OK(hipMemcpy2DAsync(host, sizeof(double2) * N, dev, sizeof(double2) * s->Np, sizeof(double2) * N, N,
                            hipMemcpyDeviceToHost, s->stream),
           s);
    HIP_OK(hipStreamSynchronize(s->stream), s);
    return ICWF_OK;
}

}  // namespace

extern "C" {

size_t icwf_workspace_bytes(const icwf_config *cfg) {
    if (validate(cfg)) return 0;
    size_t total = 0;
    carve(*cfg, nullptr, &total);
    return total;
}

icwf_status icwf_create(const icwf_config *cfg, const double *r0, const double *R0, const double *psi1_0,
                        const double *psi2_0, const double *C0, const double *b0, const double *bo_states,
                        void *workspace, size_t ws_bytes, void *hip_stream, icwf_sim **out) {
    if (!out) return fail(nullptr, ICWF_EINVAL, "out is NULL");
    *out = nullptr;
    if (const char *m = validate(cfg)) return fail(nullptr, ICWF_EINVAL, m);
    if (!r0 || !R0 || !psi1_0 || !psi2_0) return fail(nullptr, ICWF_EINVAL, "positions and CWFs are required");
    if (!C0 && !b0) return fail(nullptr, ICWF_EINVAL, "one of C0 and b0 is required");
    if (cfg->n_bo > 0 && !bo_states) return fail(nullptr, ICWF_EINVAL, "n_bo > 0 needs bo_states");
    if (!workspace) return fail(nullptr, ICWF_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(nullptr, ICWF_EINVAL, "workspace must be 256-byte aligned");
    size_t need = 0;
    carve(*cfg, nullptr, &need);
    if (ws_bytes < need) return fail(nullptr, ICWF_ENOMEM, "workspace smaller than icwf_workspace_bytes()");

    const int N = cfg->n_traj, nr = cfg->n_r, nR = cfg->n_R, nbo = cfg->n_bo;
    const int Np = icwf::padded(N);
    auto finite = [](const double *p, size_t n) {
        for (size_t i = 0; i < n; ++i)
            if (!std::isfinite(p[i])) return false;
        return true;
    };
    if (!finite(r0, N) || !finite(R0, N) || !finite(psi1_0, 2 * (size_t)N * nr) ||
        !finite(psi2_0, 2 * (size_t)N * nR) || (C0 && !finite(C0, 2 * (size_t)N)) || (!C0 && !finite(b0, 2 * (size_t)N)) ||
        (nbo > 0 && !finite(bo_states, (size_t)nR * nbo * nr)))
        return fail(nullptr, ICWF_ENONFINITE, "non-finite input");

    icwf_sim *s = new icwf_sim();
    s->cfg = *cfg;
    s->Np = Np;
    s->stream = reinterpret_cast<hipStream_t>(hip_stream);
    size_t total = 0;
    s->b = carve(*cfg, reinterpret_cast<char *>(workspace), &total);
    Dims &d = s->d;
    d.N = N;
    d.nr = nr;
    d.nR = nR;
    d.n_bo = nbo;
    d.prec = cfg->precision;
    d.sinv = icwf::use_sinv(icwf::padded(N), cfg->precision, cfg->solver) ? 1 : 0;
    d.propagator = cfg->propagator;
    d.traj = cfg->trajectories;
    d.r_min = cfg->r_min;
    d.hr = (cfg->r_max - cfg->r_min) / nr;
    d.R_min = cfg->R_min;
    d.hR = (cfg->R_max - cfg->R_min) / nR;
    d.m_r = cfg->m_r;
    d.m_R = cfg->m_R;
    d.dt = cfg->dt;
    d.eps = cfg->tikhonov_eps;
    d.mp.kind = cfg->model;
    for (int i = 0; i < 8; ++i) d.mp.p[i] = cfg->model_params[i];
    d.mpd = s->b.mparams;

    auto cleanup_fail = [&](icwf_status st, const std::string &m) {
        g_create_error = m;
        icwf_destroy(s);
        return st;
    };
    auto hipchk = [&](hipError_t e, const char *what) -> bool {
        if (e != hipSuccess) {
            g_create_error = std::string(what) + ": " + hipGetErrorString(e);
            return false;
        }
        return true;
    };
#define CREATE_HIP(call)                                \
    do {                                                \
        if (!hipchk((call), #call)) {                   \
            std::string m_ = g_create_error;            \
            return cleanup_fail(ICWF_EDEVICE, m_);      \
        }                                               \
    } while (0)

    // ---- host tables
    std::vector<double> vr(nr), vR(nR), wc(static_cast<size_t>(nr) * nR);
    std::vector<float> wc32(static_cast<size_t>(nr) * nR);
    std::vector<double2> kin_r(nr), kin_R(nR), tw_r(nr), tw_R(nR);
    for (int i = 0; i < nr; ++i) vr[i] = h_v1(*cfg, d.r_min + i * d.hr);
    for (int j = 0; j < nR; ++j) vR[j] = h_v2(*cfg, d.R_min + j * d.hR);
    for (int i = 0; i < nr; ++i)
        for (int j = 0; j < nR; ++j) {
            const double w = h_wc(*cfg, d.r_min + i * d.hr, d.R_min + j * d.hR);
            wc[(size_t)i * nR + j] = w;
            wc32[(size_t)i * nR + j] = static_cast<float>(w);
        }
    if (!finite(vr.data(), nr) || !finite(vR.data(), nR) || !finite(wc.data(), wc.size()))
        return cleanup_fail(ICWF_ENONFINITE, "the model is singular on the grid");
    // mixed form: W_c = (rank-K part, FP64) + (residual, FP32 matrix cores)
    std::vector<double> lr_u, lr_v;
    d.lr_rank = 0;
    int ncu = 0;
    {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
            ncu = 256;
        // two contraction work-groups fit a CU; kWcReserve of those slots stay free
        d.wc_grid = std::max(2 * ncu - icwf::kWcReserve, ncu);
        d.prop_grid[0] = icwf::propagate_grid(nr, N, ncu);
        d.prop_grid[1] = icwf::propagate_grid(nR, N, ncu);
    }
    if (cfg->precision == ICWF_PREC_MIXED) {
        std::vector<double> res = wc;
        d.lr_rank = cross_approximation(res, nr, nR, kMixedSplitTol, icwf::kLowRankMax, lr_u, lr_v);
        auto maxabs = [](const std::vector<double> &v) {
            double m = 0.0;
            for (double x : v) m = std::max(m, std::fabs(x));
            return m;
        };
        const double wmax = maxabs(wc);
        double rmax = maxabs(res);
        // the FP64 part runs in blocks of 16 terms, so terms up to the next
        // multiple of 16 cost nothing: take them (down to the table's rounding),
        // which leaves a smaller residual, and so a smaller FP32 error, to the
        // matrix-core pass
        const int fill = std::min(icwf::kLowRankMax, (d.lr_rank + 15) / 16 * 16);
        if (d.lr_rank > 0 && fill > d.lr_rank && rmax > kSeparableTol * wmax) {
            d.lr_rank += cross_approximation(res, nr, nR, kSeparableTol * wmax / rmax, fill - d.lr_rank, lr_u, lr_v);
            rmax = maxabs(res);
        }
        for (size_t e = 0; e < res.size(); ++e) wc32[e] = static_cast<float>(res[e]);
        // a residual at the table's own rounding level (an exactly separable
        // coupling, such as the cavity's lambda q x) leaves the FP32 pass
        // nothing to add: the FP64 rank-K part is then the whole contraction
        d.fp32_residual = !(d.lr_rank > 0 && rmax <= kSeparableTol * wmax);
    } else if (cfg->precision == ICWF_PREC_SEPARABLE) {
        std::vector<double> res = wc;
        d.lr_rank = cross_approximation(res, nr, nR, kSeparableTol, icwf::kLowRankMax, lr_u, lr_v);
        double wmax = 0.0, rmax = 0.0;
        for (size_t e = 0; e < wc.size(); ++e) {
            wmax = std::max(wmax, std::fabs(wc[e]));
            rmax = std::max(rmax, std::fabs(res[e]));
        }
        if (rmax > kSeparableTol * wmax)
            return cleanup_fail(ICWF_EINVAL, "W_c is not a sum of at most 64 products to FP64 rounding; use the FP64 form");
        // a contraction through few products is the short branch of a forked
        // step where (n_r + n_R) K < 32 N (K in blocks of 16; N = 1024 on 512 x
        // 256, K = 28: 1.2 ms beside 1.9 ms of factorisations; N = 4096 on 4096
        // x 512, K = 41: 88 ms beside 49 ms): it then takes one work-group per
        // CU and leaves the other slots to the factorisation stream
        const size_t kp = (size_t)(d.lr_rank + 15) / 16 * 16;
        if (icwf::padded(N) >= kOverlapMinN && (size_t)(nr + nR) * kp < 32 * (size_t)icwf::padded(N))
            d.wc_grid = ncu;
    }
    auto fill_k = [&](std::vector<double2> &kin, std::vector<double2> &tw, int n, double h, double m) {
        for (int k = 0; k < n; ++k) {
            const int kk = (k <= n / 2) ? k : k - n;
            const double kw = 2.0 * M_PI * kk / (n * h);
            const double ph = -0.5 * d.dt * kw * kw / m;
            // times 1/n, the normalisation of the inverse transform (exact: n is a power of two)
            kin[k] = make_double2(std::cos(ph) / n, std::sin(ph) / n);
            const double a = -2.0 * M_PI * k / n;
            tw[k] = make_double2(std::cos(a), std::sin(a));
        }
    };
    fill_k(kin_r, tw_r, nr, d.hr, d.m_r);
    fill_k(kin_R, tw_R, nR, d.hR, d.m_R);
    // half-step phases of the one-coordinate parts V_1(r_i), V_2(R_j)
    std::vector<double2> vph_r(nr), vph_R(nR);
    for (int i = 0; i < nr; ++i) vph_r[i] = make_double2(std::cos(-0.5 * d.dt * vr[i]), std::sin(-0.5 * d.dt * vr[i]));
    for (int j = 0; j < nR; ++j) vph_R[j] = make_double2(std::cos(-0.5 * d.dt * vR[j]), std::sin(-0.5 * d.dt * vR[j]));

    // ---- padded state
    std::vector<double> rp(Np, cfg->r_min), Rp(Np, cfg->R_min);
    std::copy(r0, r0 + N, rp.begin());
    std::copy(R0, R0 + N, Rp.begin());

    hipStream_t st = s->stream;
    const Bufs &b = s->b;
    CREATE_HIP(hipMemsetAsync(workspace, 0, total, st));
    CREATE_HIP(hipMemcpyAsync(b.psi1, psi1_0, sizeof(double2) * (size_t)N * nr, hipMemcpyHostToDevice, st));
    CREATE_HIP(hipMemcpyAsync(b.psi2, psi2_0, sizeof(double2) * (size_t)N * nR, hipMemcpyHostToDevice, st));
    CREATE_HIP(hipMemcpyAsync(b.r, rp.data(), sizeof(double) * Np, hipMemcpyHostToDevice, st));
    CREATE_HIP(hipMemcpyAsync(b.R, Rp.data(), sizeof(double) * Np, hipMemcpyHostToDevice, st));
    CREATE_HIP(hipMemcpyAsync(b.r_new, rp.data(), sizeof(double) * Np, hipMemcpyHostToDevice, st));
    CREATE_HIP(hipMemcpyAsync(b.R_new, Rp.data(), sizeof(double) * Np, hipMemcpyHostToDevice, st));
    CREATE_HIP(hipMemcpyAsync(b.vphase_r, vph_r.data(), sizeof(double2) * nr, hipMemcpyHostToDevice, st));
    CREATE_HIP(hipMemcpyAsync(b.vphase_R, vph_R.data(), sizeof(double2) * nR, hipMemcpyHostToDevice, st));
    CREATE_HIP(hipMemcpyAsync(b.kin_r, kin_r.data(), sizeof(double2) * nr, hipMemcpyHostToDevice, st));
    CREATE_HIP(hipMemcpyAsync(b.kin_R, kin_R.data(), sizeof(double2) * nR, hipMemcpyHostToDevice, st));
    CREATE_HIP(hipMemcpyAsync(b.tw_r, tw_r.data(), sizeof(double2) * nr, hipMemcpyHostToDevice, st));
    CREATE_HIP(hipMemcpyAsync(b.tw_R, tw_R.data(), sizeof(double2) * nR, hipMemcpyHostToDevice, st));
    CREATE_HIP(hipMemcpyAsync(b.wc64, wc.data(), sizeof(double) * wc.size(), hipMemcpyHostToDevice, st));
    CREATE_HIP(hipMemcpyAsync(b.wc32, wc32.data(), sizeof(float) * wc32.size(), hipMemcpyHostToDevice, st));
    if (d.lr_rank > 0) {
        CREATE_HIP(hipMemcpyAsync(b.lr_u, lr_u.data(), sizeof(double) * lr_u.size(), hipMemcpyHostToDevice, st));
        CREATE_HIP(hipMemcpyAsync(b.lr_v, lr_v.data(), sizeof(double) * lr_v.size(), hipMemcpyHostToDevice, st));
    }
    if (nbo > 0)
        CREATE_HIP(hipMemcpyAsync(b.bo, bo_states, sizeof(double) * (size_t)nR * nbo * nr, hipMemcpyHostToDevice, st));
    CREATE_HIP(hipMemcpyAsync(b.mparams, &d.mp, sizeof(icwf::ModelParams), hipMemcpyHostToDevice, st));
    const std::vector<int32_t> order = icwf::wc_tile_order(Np);
    CREATE_HIP(hipMemcpyAsync(b.wc_order, order.data(), sizeof(int32_t) * order.size(), hipMemcpyHostToDevice, st));
    if (C0) CREATE_HIP(hipMemcpyAsync(b.C, C0, sizeof(double2) * N, hipMemcpyHostToDevice, st));
    else CREATE_HIP(hipMemcpyAsync(b.Cstage, b0, sizeof(double2) * N, hipMemcpyHostToDevice, st));

    // ---- initial S_0, K_0 and the factor of S_0 + eps I
    if (d.prec == ICWF_PREC_MIXED && d.fp32_residual) icwf::launch_psi1_f32(d, b, st);
    icwf::launch_cond_kets(d, b, st);
    icwf::launch_single_species(d, b, false, st);
    icwf::launch_wc(d, b, st);
    icwf::launch_assemble(d, b, 0, icwf::kAssembleInitial, st);
    if (d.sinv)
        icwf::launch_cholesky(d, b, b.L[0], b.L[0], b.Linv[0], b.Linv[0], 1, st, b.Finv[0], nullptr, b.Hinv[0], nullptr);
    else
        icwf::launch_cholesky(d, b, b.L[0], b.L[0], b.Linv[0], b.Linv[0], 1, st);
    if (!C0) icwf::launch_solve_initial(d, b, 0, b.Cstage, st);
    CREATE_HIP(hipGetLastError());
    const icwf_status ds = device_status(s);
    if (ds != ICWF_OK) {
        std::string m = s->err;
        return cleanup_fail(ds, m);
    }
    CREATE_HIP(hipStreamCreateWithFlags(&s->capture_stream, hipStreamNonBlocking));
    CREATE_HIP(hipStreamCreateWithFlags(&s->side_stream, hipStreamNonBlocking));
    CREATE_HIP(hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming));
    CREATE_HIP(hipEventCreateWithFlags(&s->ev_join, hipEventDisableTiming));
    if (capture_graphs(s) != ICWF_OK) {
        std::string m = s->err;
        return cleanup_fail(ICWF_EDEVICE, m);
    }
#undef CREATE_HIP
    *out = s;
    return ICWF_OK;
}

icwf_status icwf_step(icwf_sim *s, int32_t n_steps) {
    if (!s) return fail(nullptr, ICWF_EINVAL, "sim is NULL");
    if (n_steps < 0) return fail(s, ICWF_EINVAL, "n_steps must be >= 0");
    if (s->status != ICWF_OK) return fail(s, ICWF_ESTATE, "the simulation stopped on an earlier error");
    for (int k = 0; k < n_steps; ++k) {
        if (s->timing) {
            enqueue_step(s, s->d, s->parity, s->stream, s->side_stream);
            HIP_OK(hipGetLastError(), s);
        } else {
            HIP_OK(hipGraphLaunch(s->exec[s->parity], s->stream), s);
        }
        s->parity ^= 1;
        s->step += 1;
        s->t += s->d.dt;
    }
    return ICWF_OK;
}

icwf_status icwf_step_batch(icwf_sim *const *sims, int32_t n_sims, int32_t n_steps) {
    if (!sims || n_sims < 1 || n_sims > icwf::kMaxBatch || n_steps < 0)
        return fail(nullptr, ICWF_EINVAL, "icwf_step_batch: need 1..64 simulations and n_steps >= 0");
    icwf_sim *lead = sims[0];
    if (!lead) return fail(nullptr, ICWF_EINVAL, "icwf_step_batch: NULL simulation");
    std::string key;
    if (!batch_key(lead, &key))
        return fail(lead, ICWF_EINVAL, "icwf_step_batch: this simulation steps alone (padded N >= 1024, explicit "
                                       "inverses or per-kernel timing)");
    for (int k = 0; k < n_sims; ++k) {
        icwf_sim *s = sims[k];
        std::string kk;
        if (!s) return fail(lead, ICWF_EINVAL, "icwf_step_batch: NULL simulation");
        for (int q = 0; q < k; ++q)
            if (sims[q] == s) return fail(lead, ICWF_EINVAL, "icwf_step_batch: a simulation appears twice");
        if (s->status != ICWF_OK) return fail(s, ICWF_ESTATE, "the simulation stopped on an earlier error");
        if (!batch_key(s, &kk) || kk != key)
            return fail(lead, ICWF_EINVAL, "icwf_step_batch: the simulations differ in shape or parameters the "
                                           "launches share");
        if (s->stream != lead->stream) return fail(lead, ICWF_EINVAL, "icwf_step_batch: the simulations must share a stream");
        if (s->parity != lead->parity) return fail(lead, ICWF_EINVAL, "icwf_step_batch: the simulations are at steps of different parity");
    }
    if (n_sims == 1) return icwf_step(lead, n_steps);
    // the batch table: each simulation's workspace relative to the lead's (the
    // workspace starts with the flags), written by a kernel whose arguments
    // carry it, in stream order before the launches that read it
    icwf::BatchTable tab{};
    for (int k = 0; k < n_sims; ++k)
        tab.off[k] = reinterpret_cast<const char *>(sims[k]->b.flags) - reinterpret_cast<const char *>(lead->b.flags);
    icwf::launch_set_table(lead->b.batch_tab, tab, n_sims, lead->stream);
    Dims d = lead->d;
    d.batch = n_sims;
    d.zoff = lead->b.batch_tab;
    for (int k = 0; k < n_steps; ++k) {
        // the step of a batch of this size and parity, captured once per lead:
        // its launches depend on the lead and the size only (the members come
        // from the table written above)
        hipGraphExec_t &ex = lead->batch_exec[2 * n_sims + lead->parity];
        if (!ex) {
            hipGraph_t g = nullptr;
            HIP_OK(hipStreamBeginCapture(lead->capture_stream, hipStreamCaptureModeThreadLocal), lead);
            enqueue_step(lead, d, lead->parity, lead->capture_stream, lead->capture_stream);
            HIP_OK(hipStreamEndCapture(lead->capture_stream, &g), lead);
            const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                ex = nullptr;
                return fail(lead, ICWF_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
            }
        }
        HIP_OK(hipGraphLaunch(ex, lead->stream), lead);
        for (int q = 0; q < n_sims; ++q) {
            sims[q]->parity ^= 1;
            sims[q]->step += 1;
            sims[q]->t += sims[q]->d.dt;
        }
    }
    return ICWF_OK;
}

icwf_status icwf_sync(icwf_sim *s) {
    if (!s) return fail(nullptr, ICWF_EINVAL, "sim is NULL");
    if (s->status != ICWF_OK) return static_cast<icwf_status>(s->status);
    return device_status(s);
}

icwf_status icwf_observables(icwf_sim *s, icwf_obs *o) {
    if (!s || !o) return fail(s, ICWF_EINVAL, "NULL argument");
    icwf_status st = icwf_sync(s);
    const Dims &d = s->d;
    icwf::launch_observables(d, s->b, s->stream);
    HIP_OK(hipGetLastError(), s);
    std::vector<double> buf(obs_len(d.nr, d.nR, d.n_bo));
    HIP_OK(hipMemcpyAsync(buf.data(), s->b.obs_out, sizeof(double) * buf.size(), hipMemcpyDeviceToHost, s->stream), s);
    int32_t flags[icwf::kNumFlags];
    double scal[8];
    HIP_OK(hipMemcpyAsync(flags, s->b.flags, sizeof(flags), hipMemcpyDeviceToHost, s->stream), s);
    HIP_OK(hipMemcpyAsync(scal, s->b.scal, sizeof(scal), hipMemcpyDeviceToHost, s->stream), s);
    HIP_OK(hipStreamSynchronize(s->stream), s);
    o->t = s->t;
    o->step = s->step;
    o->norm = buf[0];
    if (o->rho_r) std::copy(buf.begin() + 1, buf.begin() + 1 + d.nr, o->rho_r);
    if (o->rho_R) std::copy(buf.begin() + 1 + d.nr, buf.begin() + 1 + d.nr + d.nR, o->rho_R);
    const size_t po = 1 + d.nr + d.nR;
    if (o->pop && d.n_bo) std::copy(buf.begin() + po, buf.begin() + po + d.n_bo, o->pop);
    if (o->D && d.n_bo) std::copy(buf.begin() + po + d.n_bo, buf.begin() + po + d.n_bo + d.n_bo * d.n_bo, o->D);
    if (o->r) HIP_OK(hipMemcpyAsync(o->r, s->b.r, sizeof(double) * d.N, hipMemcpyDeviceToHost, s->stream), s);
    if (o->R) HIP_OK(hipMemcpyAsync(o->R, s->b.R, sizeof(double) * d.N, hipMemcpyDeviceToHost, s->stream), s);
    if (o->C) HIP_OK(hipMemcpyAsync(o->C, s->b.C, sizeof(double2) * d.N, hipMemcpyDeviceToHost, s->stream), s);
    HIP_OK(hipStreamSynchronize(s->stream), s);
    o->n_out_of_box = flags[icwf::kFlagOut];
    uint64_t bits;
    std::memcpy(&bits, &scal[0], sizeof(bits));
    double mn;
    std::memcpy(&mn, &bits, sizeof(mn));
    o->min_abs_psi = (s->step == 0) ? INFINITY : mn;
    return st;
}

icwf_status icwf_get_state(icwf_sim *s, double *r, double *R, double *psi1, double *psi2, double *C) {
    if (!s) return fail(nullptr, ICWF_EINVAL, "sim is NULL");
    HIP_OK(hipStreamSynchronize(s->stream), s);
    const Dims &d = s->d;
    if (r) HIP_OK(hipMemcpyAsync(r, s->b.r, sizeof(double) * d.N, hipMemcpyDeviceToHost, s->stream), s);
    if (R) HIP_OK(hipMemcpyAsync(R, s->b.R, sizeof(double) * d.N, hipMemcpyDeviceToHost, s->stream), s);
    if (psi1) HIP_OK(hipMemcpyAsync(psi1, s->b.psi1, sizeof(double2) * (size_t)d.N * d.nr, hipMemcpyDeviceToHost, s->stream), s);
    if (psi2) HIP_OK(hipMemcpyAsync(psi2, s->b.psi2, sizeof(double2) * (size_t)d.N * d.nR, hipMemcpyDeviceToHost, s->stream), s);
    if (C) HIP_OK(hipMemcpyAsync(C, s->b.C, sizeof(double2) * d.N, hipMemcpyDeviceToHost, s->stream), s);
    HIP_OK(hipStreamSynchronize(s->stream), s);
    return static_cast<icwf_status>(s->status);
}

icwf_status icwf_get_matrices(icwf_sim *s, double *S, double *K, double *Wc) {
    if (!s) return fail(nullptr, ICWF_EINVAL, "sim is NULL");
    HIP_OK(hipStreamSynchronize(s->stream), s);
    if (S && copy_matrix_out(s, s->b.Smat[s->parity], S) != ICWF_OK) return ICWF_EDEVICE;
    if (K && copy_matrix_out(s, s->b.Kmat[s->parity], K) != ICWF_OK) return ICWF_EDEVICE;
    if (Wc) {
        if (copy_matrix_out(s, s->b.Wc, Wc) != ICWF_OK) return ICWF_EDEVICE;
        const int N = s->cfg.n_traj;
        for (int b = 0; b < N; ++b)
            for (int a = 0; a < b; ++a) {   // lower = conj(upper): only b <= a is computed
                Wc[2 * ((size_t)b * N + a)] = Wc[2 * ((size_t)a * N + b)];
                Wc[2 * ((size_t)b * N + a) + 1] = -Wc[2 * ((size_t)a * N + b) + 1];
            }
    }
    return static_cast<icwf_status>(s->status);
}

icwf_status icwf_velocities(icwf_sim *s, double *v_r, double *v_R, double *psi_at) {
    if (!s) return fail(nullptr, ICWF_EINVAL, "sim is NULL");
    if (s->status != ICWF_OK) return fail(s, ICWF_ESTATE, "the simulation stopped on an earlier error");
    icwf::launch_velocity(s->d, s->b, icwf::kVelocityOnly, s->stream);
    HIP_OK(hipGetLastError(), s);
    icwf_status st = device_status(s);
    const Dims &d = s->d;
    if (v_r) HIP_OK(hipMemcpyAsync(v_r, s->b.v_r, sizeof(double) * d.N, hipMemcpyDeviceToHost, s->stream), s);
    if (v_R) HIP_OK(hipMemcpyAsync(v_R, s->b.v_R, sizeof(double) * d.N, hipMemcpyDeviceToHost, s->stream), s);
    if (psi_at) HIP_OK(hipMemcpyAsync(psi_at, s->b.psi_at, sizeof(double2) * d.N, hipMemcpyDeviceToHost, s->stream), s);
    HIP_OK(hipStreamSynchronize(s->stream), s);
    return st;
}

icwf_status icwf_set_timing(icwf_sim *s, int32_t enable) {
    if (!s) return fail(nullptr, ICWF_EINVAL, "sim is NULL");
    HIP_OK(hipStreamSynchronize(s->stream), s);
    for (auto &kv : s->timers)
        for (auto &pr : kv.second.recs) {
            s->event_pool.push_back(pr.first);
            s->event_pool.push_back(pr.second);
        }
    s->timers.clear();
    s->timing = enable != 0;
    return ICWF_OK;
}

icwf_status icwf_contraction_rank(const icwf_sim *s, int32_t *rank) {
    if (!s || !rank) return ICWF_EINVAL;
    *rank = s->d.lr_rank;
    return ICWF_OK;
}

icwf_status icwf_kernel_time(icwf_sim *s, const char *name, int64_t *launches, double *total_ms) {
    if (!s || !name) return fail(s, ICWF_EINVAL, "NULL argument");
    HIP_OK(hipStreamSynchronize(s->stream), s);
    Timer &tm = s->timers[name];
    for (auto &pr : tm.recs) {
        float ms = 0.0f;
        HIP_OK(hipEventElapsedTime(&ms, pr.first, pr.second), s);
        tm.total_ms += ms;
        tm.launches += 1;
        s->event_pool.push_back(pr.first);
        s->event_pool.push_back(pr.second);
    }
    tm.recs.clear();
    if (launches) *launches = tm.launches;
    if (total_ms) *total_ms = tm.total_ms;
    return ICWF_OK;
}

void icwf_destroy(icwf_sim *s) {
    if (!s) return;
    if (s->stream || s->capture_stream) (void)hipStreamSynchronize(s->stream);
    for (auto &e : s->exec)
        if (e) (void)hipGraphExecDestroy(e);
    for (auto &kv : s->batch_exec) (void)hipGraphExecDestroy(kv.second);
    if (s->side_stream) (void)hipStreamSynchronize(s->side_stream);
    if (s->capture_stream) (void)hipStreamDestroy(s->capture_stream);
    if (s->side_stream) (void)hipStreamDestroy(s->side_stream);
    if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
    if (s->ev_join) (void)hipEventDestroy(s->ev_join);
    for (auto &kv : s->timers)
        for (auto &pr : kv.second.recs) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    for (auto e : s->event_pool) (void)hipEventDestroy(e);
    delete s;
}

const char *icwf_last_error(const icwf_sim *s) { return s ? s->err.c_str() : g_create_error.c_str(); }

const char *icwf_status_string(int32_t st) {
    switch (st) {
        case ICWF_OK: return "ICWF_OK";
        case ICWF_EINVAL: return "ICWF_EINVAL";
        case ICWF_ENOMEM: return "ICWF_ENOMEM";
        case ICWF_EDEVICE: return "ICWF_EDEVICE";
        case ICWF_ENONFINITE: return "ICWF_ENONFINITE";
        case ICWF_ENODE: return "ICWF_ENODE";
        case ICWF_ESOLVE: return "ICWF_ESOLVE";
        case ICWF_ESTATE: return "ICWF_ESTATE";
        case ICWF_ETIMEDOUT: return "ICWF_ETIMEDOUT";
        default: return "unknown";
    }
}

}  // extern "C"

// ---- exact grid propagation of the full wavefunction (icwf_exact.h) -----------------------------

struct icwf_exact {
    icwf_config cfg{};
    hipStream_t stream = nullptr;
    icwf::ExactBufs e{};
    double *bo = nullptr;
    double2 *chi = nullptr;
    double *part = nullptr;
    double *out = nullptr;
    double hr = 0, hR = 0;
    int64_t step = 0;
};

namespace {

icwf::ExactBufs carve_exact(const icwf_config &c, char *base, size_t *total, double **bo, double2 **chi,
                            double **part, double **out) {
    Layout L;
    L.base = base;
    const size_t nr = c.n_r, nR = c.n_R, nbo = c.n_bo;
    icwf::ExactBufs e{};
    e.psi = L.take<double2>(nr * nR);
    e.tmp = L.take<double2>(nr * nR);
    e.half = L.take<double2>(nr * nR);
    e.kin_r = L.take<double2>(nr);
    e.kin_R = L.take<double2>(nR);
    e.tw_r = L.take<double2>(nr);
    e.tw_R = L.take<double2>(nR);
    *bo = L.take<double>(std::max<size_t>(1, nR * nbo * nr));
    *chi = L.take<double2>(std::max<size_t>(1, nbo * nR));
    *part = L.take<double>(icwf::kRhoSlices * nR);
    *out = L.take<double>(obs_len(c.n_r, c.n_R, c.n_bo));
    *total = (L.off + 255) & ~size_t(255);
    return e;
}

}  // namespace

extern "C" {

size_t icwf_exact_workspace_bytes(const icwf_config *cfg) {
    if (validate(cfg)) return 0;
    size_t total = 0;
    double *bo, *part, *out;
    double2 *chi;
    carve_exact(*cfg, nullptr, &total, &bo, &chi, &part, &out);
    return total;
}

icwf_status icwf_exact_create(const icwf_config *cfg, const double *psi0, const double *bo_states, void *workspace,
                              size_t ws_bytes, void *hip_stream, icwf_exact **out) {
    if (!out) return fail(nullptr, ICWF_EINVAL, "out is NULL");
    *out = nullptr;
    if (const char *m = validate(cfg)) return fail(nullptr, ICWF_EINVAL, m);
    if (!psi0) return fail(nullptr, ICWF_EINVAL, "psi0 is required");
    if (cfg->n_bo > 0 && !bo_states) return fail(nullptr, ICWF_EINVAL, "n_bo > 0 needs bo_states");
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255))
        return fail(nullptr, ICWF_EINVAL, "workspace must be non-NULL and 256-byte aligned");
    if (ws_bytes < icwf_exact_workspace_bytes(cfg)) return fail(nullptr, ICWF_EINVAL, "workspace too small");
    const int nr = cfg->n_r, nR = cfg->n_R, nbo = cfg->n_bo;
    const size_t np = (size_t)nr * nR;
    for (size_t e = 0; e < 2 * np; ++e)
        if (!std::isfinite(psi0[e])) return fail(nullptr, ICWF_ENONFINITE, "non-finite psi0");
    if (nbo > 0)
        for (size_t e = 0; e < (size_t)nR * nbo * nr; ++e)
            if (!std::isfinite(bo_states[e])) return fail(nullptr, ICWF_ENONFINITE, "non-finite bo_states");

    const double hr = (cfg->r_max - cfg->r_min) / nr, hR = (cfg->R_max - cfg->R_min) / nR, dt = cfg->dt;
    // half-step phase of the full interaction W = V_1 + V_2 + W_c on the grid
    std::vector<double2> half(np), kin_r(nr), kin_R(nR), tw_r(nr), tw_R(nR);
    for (int i = 0; i < nr; ++i) {
        const double r = cfg->r_min + i * hr;
        for (int j = 0; j < nR; ++j) {
            const double R = cfg->R_min + j * hR;
            const double w = h_v1(*cfg, r) + h_v2(*cfg, R) + h_wc(*cfg, r, R);
            if (!std::isfinite(w)) return fail(nullptr, ICWF_ENONFINITE, "the model is singular on the grid");
            half[(size_t)i * nR + j] = make_double2(std::cos(-0.5 * dt * w), std::sin(-0.5 * dt * w));
        }
    }
    // kinetic phase of both species, a product of one factor per species; the
    // nuclear one carries 1/(n_r n_R) (the normalisation of the inverse
    // transform; exact, both are powers of two)
    const double inv = 1.0 / ((double)nr * nR);
    for (int kr = 0; kr < nr; ++kr) {
        const int mr = (kr <= nr / 2) ? kr : kr - nr;
        const double kw = 2.0 * M_PI * mr / (nr * hr), ph = -dt * kw * kw / (2.0 * cfg->m_r);
        kin_r[kr] = make_double2(std::cos(ph), std::sin(ph));
    }
    for (int kR = 0; kR < nR; ++kR) {
        const int mR = (kR <= nR / 2) ? kR : kR - nR;
        const double kw = 2.0 * M_PI * mR / (nR * hR), ph = -dt * kw * kw / (2.0 * cfg->m_R);
        kin_R[kR] = make_double2(std::cos(ph) * inv, std::sin(ph) * inv);
    }
    for (int k = 0; k < nr; ++k) tw_r[k] = make_double2(std::cos(-2.0 * M_PI * k / nr), std::sin(-2.0 * M_PI * k / nr));
    for (int k = 0; k < nR; ++k) tw_R[k] = make_double2(std::cos(-2.0 * M_PI * k / nR), std::sin(-2.0 * M_PI * k / nR));

    icwf_exact *x = new icwf_exact();
    x->cfg = *cfg;
    x->stream = reinterpret_cast<hipStream_t>(hip_stream);
    x->hr = hr;
    x->hR = hR;
    size_t total = 0;
    x->e = carve_exact(*cfg, reinterpret_cast<char *>(workspace), &total, &x->bo, &x->chi, &x->part, &x->out);
    const hipStream_t st = x->stream;
    auto copy = [&](void *dst, const void *src, size_t bytes) {
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st) == hipSuccess;
    };
    bool ok = hipMemsetAsync(workspace, 0, total, st) == hipSuccess && copy(x->e.psi, psi0, sizeof(double2) * np) &&
              copy(x->e.half, half.data(), sizeof(double2) * np) && copy(x->e.kin_r, kin_r.data(), sizeof(double2) * nr) &&
              copy(x->e.kin_R, kin_R.data(), sizeof(double2) * nR) &&
              copy(x->e.tw_r, tw_r.data(), sizeof(double2) * tw_r.size()) &&
              copy(x->e.tw_R, tw_R.data(), sizeof(double2) * tw_R.size());
    if (ok && nbo > 0) ok = copy(x->bo, bo_states, sizeof(double) * (size_t)nR * nbo * nr);
    if (ok) ok = hipStreamSynchronize(st) == hipSuccess;
    if (!ok) {
        delete x;
        return fail(nullptr, ICWF_EDEVICE, std::string("device copy failed: ") + hipGetErrorString(hipGetLastError()));
    }
    *out = x;
    return ICWF_OK;
}

icwf_status icwf_exact_step(icwf_exact *x, int64_t n_steps) {
    if (!x || n_steps < 0) return fail(nullptr, ICWF_EINVAL, "bad arguments to icwf_exact_step");
    icwf::launch_exact_steps(x->cfg.n_r, x->cfg.n_R, x->e, n_steps, x->stream);
    if (hipGetLastError() != hipSuccess) return fail(nullptr, ICWF_EDEVICE, "exact step launch failed");
    x->step += n_steps;
    return ICWF_OK;
}

icwf_status icwf_exact_observables(icwf_exact *x, icwf_obs *o) {
    if (!x || !o) return fail(nullptr, ICWF_EINVAL, "NULL argument");
    const int nr = x->cfg.n_r, nR = x->cfg.n_R, nbo = x->cfg.n_bo;
    icwf::launch_grid_observables(x->e.psi, nr, nR, x->hr, x->hR, nbo, x->bo, x->chi, x->part, x->out, x->stream);
    std::vector<double> buf(obs_len(nr, nR, nbo));
    if (hipMemcpyAsync(buf.data(), x->out, sizeof(double) * buf.size(), hipMemcpyDeviceToHost, x->stream) != hipSuccess ||
        hipStreamSynchronize(x->stream) != hipSuccess)
        return fail(nullptr, ICWF_EDEVICE, "observables copy failed");
    o->t = x->step * x->cfg.dt;
    o->step = x->step;
    o->norm = buf[0];
    if (o->rho_r) std::copy(buf.begin() + 1, buf.begin() + 1 + nr, o->rho_r);
    if (o->rho_R) std::copy(buf.begin() + 1 + nr, buf.begin() + 1 + nr + nR, o->rho_R);
    const size_t po = 1 + nr + nR;
    if (o->pop && nbo) std::copy(buf.begin() + po, buf.begin() + po + nbo, o->pop);
    if (o->D && nbo) std::copy(buf.begin() + po + nbo, buf.begin() + po + nbo + (size_t)nbo * nbo, o->D);
    o->n_out_of_box = 0;
    o->min_abs_psi = 0.0;
    return ICWF_OK;
}

icwf_status icwf_exact_get_psi(icwf_exact *x, double *psi) {
    if (!x || !psi) return fail(nullptr, ICWF_EINVAL, "NULL argument");
    const size_t np = (size_t)x->cfg.n_r * x->cfg.n_R;
    if (hipMemcpyAsync(psi, x->e.psi, sizeof(double2) * np, hipMemcpyDeviceToHost, x->stream) != hipSuccess ||
        hipStreamSynchronize(x->stream) != hipSuccess)
        return fail(nullptr, ICWF_EDEVICE, "state copy failed");
    return ICWF_OK;
}

void icwf_exact_destroy(icwf_exact *x) {
    if (!x) return;
    (void)hipStreamSynchronize(x->stream);
    delete x;
}

}  // extern "C"

// ---- observables of a grid wavefunction without any allocation (icwf_exact.h) ---------------------

namespace {

constexpr int kNoAllocMaxStates = 16;
constexpr int kNoAllocMaxPoints = 4096;
// the BO projections chi [n_bo][n_R] (complex) and the rho_R partial sums
// [kRhoSlices][n_R] of the largest case: 2 MiB
constexpr size_t kScratchDoubles =
    2 * (size_t)kNoAllocMaxStates * kNoAllocMaxPoints + (size_t)icwf::kRhoSlices * kNoAllocMaxPoints;
__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch[kMaxDevices] = {};

// The device address of this GPU's copy of `scratch` (taken once per device,
// with that device current); nullptr on failure, with the message set.
double *scratch_on_current_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        icwf::set_create_error(ICWF_EDEVICE, "no current device");
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            icwf::set_create_error(ICWF_EDEVICE, (std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)).c_str());
            return nullptr;
        }
        g_scratch[dev] = static_cast<double *>(p);
    }
    return g_scratch[dev];
}

}  // namespace

extern "C" {

icwf_status icwf_grid_observables_noalloc(int32_t n_r, int32_t n_R, double h_r, double h_R, int32_t n_bo,
                                          const double *psi, const double *bo_states, double *out, void *hip_stream) {
    auto pow2 = [](int n) { return n > 0 && (n & (n - 1)) == 0; };
    if (!pow2(n_r) || !pow2(n_R) || n_r < 32 || n_R < 32 || n_r > kNoAllocMaxPoints || n_R > kNoAllocMaxPoints)
        return icwf::set_create_error(ICWF_EINVAL, "n_r and n_R must be powers of two in [32, 4096]");
    if (!(h_r > 0) || !(h_R > 0) || !std::isfinite(h_r) || !std::isfinite(h_R))
        return icwf::set_create_error(ICWF_EINVAL, "grid spacings must be finite and > 0");
    if (n_bo < 0 || n_bo > kNoAllocMaxStates)
        return icwf::set_create_error(ICWF_EINVAL, "n_bo must be in [0, 16] (the static scratch holds 16 BO projections)");
    if (!psi || !out || (n_bo > 0 && !bo_states))
        return icwf::set_create_error(ICWF_EINVAL, "psi, out (and bo_states when n_bo > 0) are required");
    double *base = scratch_on_current_device();
    if (!base) return ICWF_EDEVICE;
    double2 *chi = reinterpret_cast<double2 *>(base);
    double *part = base + 2 * (size_t)kNoAllocMaxStates * kNoAllocMaxPoints;
    icwf::launch_grid_observables(reinterpret_cast<const double2 *>(psi), n_r, n_R, h_r, h_R, n_bo, bo_states, chi,
                                  part, out, reinterpret_cast<hipStream_t>(hip_stream));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return icwf::set_create_error(ICWF_EDEVICE, hipGetErrorString(e));
    return ICWF_OK;
}

}  // extern "C"

// ---- library-internal (icwf_internal.hpp) ----------------------------------------------------------

bool icwf_internal_batch_key(const icwf_sim *sim, std::string *key) { return sim && key && batch_key(sim, key); }

void icwf_internal_set_stream(icwf_sim *sim, hipStream_t stream) {
    if (sim) sim->stream = stream;
}
