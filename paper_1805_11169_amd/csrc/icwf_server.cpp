// Serving form of the ICWF library (declared in include/icwf_serve.h):
// a scheduler thread that admits independent simulations against a device
// arena, keeps them resident, and interleaves their graph-replayed steps on
// per-slot streams.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/icwf_serve.h"
#include "arena.hpp"
#include "icwf_internal.hpp"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    int64_t id = 0;
    icwf_config cfg{};
    int32_t n_steps = 0;
    size_t ws = 0;
    double cost = 1.0;             // estimated device time of one step (ms), for equal-time turns
    std::vector<double> r0, R0, psi1, psi2, C0, b0, bo;
    bool has_C0 = false;
    // result
    bool done = false;
    icwf_request_info info{};
    double t = 0, norm = 0, min_abs_psi = 0;
    int64_t step = 0;
    int32_t n_out = 0;
    std::vector<double> rho_r, rho_R, pop, D, r, R, C;
};

struct Slot {
    hipStream_t stream = nullptr;
    std::vector<hipEvent_t> pool;
    std::deque<std::pair<hipEvent_t, int32_t>> inflight;   // event after a turn, steps in it
    std::shared_ptr<Request> req;
    icwf_sim *sim = nullptr;
    size_t off = 0;
    int32_t enqueued = 0, completed = 0;
    int32_t status = ICWF_OK;
    int lane = -1;                 // lane it steps in (batching), or -1: its own stream
};

// Small simulations of one shape (icwf_internal_batch_key) share a lane: one
// stream, and each turn one icwf_step_batch per step parity over the members
// that are ready.
struct Lane {
    std::string key;
    hipStream_t stream = nullptr;
    int members = 0;
};

}  // namespace

struct icwf_server {
    icwf_server_config cfg{};
    char *arena = nullptr;
    icwf::Arena alloc;
    std::vector<Slot> slots;
    std::vector<Lane> lanes;
    Clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> pending;
    std::map<int64_t, std::shared_ptr<Request>> known;
    int64_t next_id = 1;
    bool stop = false;
    icwf_server_stats st{};
    std::thread th;

    explicit icwf_server(size_t bytes) : alloc(bytes) {}
    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

// Estimated device time of one step (ms): a launch-bound floor plus the
// step's flops at a sustained 40 TFLOP/s (the two-body contraction, dense or
// through its rank factors, the single-species products and velocities, two
// complex factorisations).  Only ratios between simulations matter: the
// scheduler gives every simulation turns of about the same device time.
double step_cost_ms(const icwf_config &c) {
    const double N = (double)((c.n_traj + 63) / 64 * 64), nr = c.n_r, nR = c.n_R;
    const double pairs = 0.5 * N * (N + 1.0);
    double contraction = 4.0 * pairs * nr * nR;
    if (c.precision == ICWF_PREC_MIXED) contraction *= 0.6;
    if (c.precision == ICWF_PREC_SEPARABLE) contraction = 4.0 * pairs * (nr + nR) * 32.0;
    const double rest = 28.0 * N * N * (nr + nR) + 2.0 * (8.0 / 3.0) * N * N * N;
    return 0.4 + (contraction + rest) / 4e10;
}

void set_message(Request &rq, const std::string &m) {
    std::strncpy(rq.info.message, m.c_str(), sizeof(rq.info.message) - 1);
    rq.info.message[sizeof(rq.info.message) - 1] = '\0';
}

// Mark a request finished and wake its waiters (caller holds no lock).
void complete(icwf_server *S, const std::shared_ptr<Request> &rq, bool admitted, size_t off) {
    std::lock_guard<std::mutex> lk(S->mu);
    if (admitted) {
        S->alloc.release(off);
        S->st.active -= 1;
    }
    rq->done = true;
    rq->info.t_done = S->now();
    if (rq->info.status == ICWF_OK) S->st.completed += 1;
    else S->st.failed += 1;
    // the inputs are no longer needed
    std::vector<double>().swap(rq->r0);
    std::vector<double>().swap(rq->R0);
    std::vector<double>().swap(rq->psi1);
    std::vector<double>().swap(rq->psi2);
    std::vector<double>().swap(rq->C0);
    std::vector<double>().swap(rq->b0);
    std::vector<double>().swap(rq->bo);
    S->cv_done.notify_all();
}

hipEvent_t take_event(Slot &sl) {
    hipEvent_t e = nullptr;
    if (!sl.pool.empty()) {
        e = sl.pool.back();
        sl.pool.pop_back();
        return e;
    }
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

// Observables of a finished simulation, then release it.
void finish(icwf_server *S, Slot &sl) {
    std::shared_ptr<Request> rq = sl.req;
    const icwf_config &c = rq->cfg;
    rq->rho_r.assign(c.n_r, 0.0);
    rq->rho_R.assign(c.n_R, 0.0);
    rq->pop.assign(std::max(c.n_bo, 0), 0.0);
    rq->D.assign((size_t)std::max(c.n_bo, 0) * std::max(c.n_bo, 0), 0.0);
    rq->r.assign(c.n_traj, 0.0);
    rq->R.assign(c.n_traj, 0.0);
    rq->C.assign(2 * (size_t)c.n_traj, 0.0);
    icwf_obs o{};
    o.rho_r = rq->rho_r.data();
    o.rho_R = rq->rho_R.data();
    o.pop = c.n_bo > 0 ? rq->pop.data() : nullptr;
    o.D = c.n_bo > 0 ? rq->D.data() : nullptr;
    o.r = rq->r.data();
    o.R = rq->R.data();
    o.C = rq->C.data();
    icwf_status s = icwf_observables(sl.sim, &o);
    if (sl.status != ICWF_OK && s == ICWF_OK) s = static_cast<icwf_status>(sl.status);
    rq->t = o.t;
    rq->step = o.step;
    rq->norm = o.norm;
    rq->n_out = o.n_out_of_box;
    rq->min_abs_psi = o.min_abs_psi;
    rq->info.status = s;
    rq->info.steps = o.step;
    if (s != ICWF_OK) set_message(*rq, icwf_last_error(sl.sim));
    icwf_destroy(sl.sim);
    if (sl.lane >= 0) S->lanes[sl.lane].members -= 1;
    sl.lane = -1;
    for (auto &pr : sl.inflight) sl.pool.push_back(pr.first);
    sl.inflight.clear();
    const size_t off = sl.off;
    sl.sim = nullptr;
    sl.req.reset();
    sl.status = ICWF_OK;
    complete(S, rq, true, off);
}

// Create the simulation of a request in its arena block on the slot's stream.
void admit(icwf_server *S, int idx, const std::shared_ptr<Request> &rq, size_t off) {
    Slot &sl = S->slots[idx];
    rq->info.slot = idx;
    rq->info.t_admit = S->now();
    icwf_sim *sim = nullptr;
    const icwf_status s = icwf_create(&rq->cfg, rq->r0.data(), rq->R0.data(), rq->psi1.data(), rq->psi2.data(),
                                      rq->has_C0 ? rq->C0.data() : nullptr, rq->has_C0 ? nullptr : rq->b0.data(),
                                      rq->bo.empty() ? nullptr : rq->bo.data(), S->arena + off, rq->ws, sl.stream,
                                      &sim);
    if (s != ICWF_OK) {
        rq->info.status = s;
        set_message(*rq, icwf_last_error(nullptr));
        complete(S, rq, true, off);
        return;
    }
    sl.sim = sim;
    sl.req = rq;
    sl.off = off;
    sl.enqueued = sl.completed = 0;
    sl.status = ICWF_OK;
    sl.lane = -1;
    std::string key;
    if (S->cfg.batch && icwf_internal_batch_key(sim, &key)) {
        // join the lane of its shape (a free lane is reused, else a new one opens)
        int li = -1;
        for (int i = 0; i < (int)S->lanes.size(); ++i)
            if (S->lanes[i].key == key && S->lanes[i].members > 0) li = i;
        if (li < 0)
            for (int i = 0; i < (int)S->lanes.size(); ++i)
                if (S->lanes[i].members == 0) {
                    li = i;
                    S->lanes[i].key = key;
                    break;
                }
        if (li < 0) {
            Lane ln;
            ln.key = key;
            if (hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking) == hipSuccess) {
                S->lanes.push_back(ln);
                li = (int)S->lanes.size() - 1;
            }
        }
        if (li >= 0) {
            icwf_internal_set_stream(sim, S->lanes[li].stream);
            S->lanes[li].members += 1;
            sl.lane = li;
        }
    }
}

// Retire the slot's finished turns; finish its simulation when its last step
// is done (or it failed).  True if anything moved; *gone when it finished.
bool poll(icwf_server *S, Slot &sl, bool *gone) {
    bool progress = false;
    *gone = false;
    while (!sl.inflight.empty()) {
        const hipError_t e = hipEventQuery(sl.inflight.front().first);
        if (e == hipErrorNotReady) break;
        if (e != hipSuccess) sl.status = ICWF_EDEVICE;
        sl.completed += sl.inflight.front().second;
        sl.pool.push_back(sl.inflight.front().first);
        sl.inflight.pop_front();
        progress = true;
    }
    if (sl.completed >= sl.req->n_steps || (sl.status != ICWF_OK && sl.inflight.empty())) {
        finish(S, sl);
        *gone = true;
        progress = true;
    }
    return progress;
}

// Steps of the slot's next turn: steps_per_turn for the costliest resident
// simulation, proportionally more for cheaper ones (turns of about equal
// device time, so that a small simulation is not held to the pace of the
// largest), never past its last step.
int32_t turn_steps(const icwf_server *S, const Slot &sl, double ref_cost) {
    const double scale = std::max(1.0, ref_cost / sl.req->cost);
    const double k = std::min(S->cfg.steps_per_turn * scale, 1e6);
    return std::max(1, std::min((int32_t)k, sl.req->n_steps - sl.enqueued));
}

double reference_cost(const icwf_server *S) {
    double ref = 0.0;
    for (const Slot &sl : S->slots)
        if (sl.sim) ref = std::max(ref, sl.req->cost);
    return ref;
}

// One turn of a lane: the members with room for another turn, grouped by step
// parity, each group one fused icwf_step_batch on the lane's stream.
bool advance_lane(icwf_server *S, int li, double ref_cost) {
    Lane &ln = S->lanes[li];
    bool progress = false;
    for (int par = 0; par < 2; ++par) {
        std::vector<Slot *> grp;
        int32_t k = 1 << 30;
        for (Slot &sl : S->slots)
            if (sl.sim && sl.lane == li && sl.status == ICWF_OK && (int)sl.inflight.size() < S->cfg.turns_ahead &&
                sl.enqueued < sl.req->n_steps && (sl.enqueued & 1) == par) {
                grp.push_back(&sl);
                k = std::min(k, turn_steps(S, sl, ref_cost));
            }
        if (grp.empty()) continue;
        std::vector<icwf_sim *> sims;
        for (Slot *sl : grp) sims.push_back(sl->sim);
        const icwf_status st = sims.size() == 1 ? icwf_step(sims[0], k)
                                                : icwf_step_batch(sims.data(), (int32_t)sims.size(), k);
        for (Slot *sl : grp) {
            hipEvent_t ev = st == ICWF_OK ? take_event(*sl) : nullptr;
            if (!ev || hipEventRecord(ev, ln.stream) != hipSuccess) {
                if (ev) sl->pool.push_back(ev);
                sl->status = ICWF_EDEVICE;
                continue;
            }
            sl->inflight.emplace_back(ev, k);
            sl->enqueued += k;
        }
        progress = true;
    }
    return progress;
}

// One pass over the admitted simulations; true if anything moved.
bool advance(icwf_server *S) {
    bool progress = false;
    const double ref_cost = reference_cost(S);
    for (Slot &sl : S->slots) {
        if (!sl.sim) continue;
        bool gone = false;
        progress = poll(S, sl, &gone) || progress;
        if (gone || sl.lane >= 0) continue;
        while (sl.status == ICWF_OK && (int)sl.inflight.size() < S->cfg.turns_ahead &&
               sl.enqueued < sl.req->n_steps) {
            const int32_t k = turn_steps(S, sl, ref_cost);
            hipEvent_t ev = take_event(sl);
            if (!ev || icwf_step(sl.sim, k) != ICWF_OK || hipEventRecord(ev, sl.stream) != hipSuccess) {
                if (ev) sl.pool.push_back(ev);
                sl.status = ICWF_EDEVICE;
                break;
            }
            sl.inflight.emplace_back(ev, k);
            sl.enqueued += k;
            progress = true;
        }
    }
    for (int li = 0; li < (int)S->lanes.size(); ++li)
        if (S->lanes[li].members > 0) progress = advance_lane(S, li, ref_cost) || progress;
    return progress;
}

void scheduler(icwf_server *S) {
    (void)hipSetDevice(S->cfg.device);
    std::unique_lock<std::mutex> lk(S->mu, std::defer_lock);
    for (;;) {
        bool progress = advance(S);
        lk.lock();
        // admission in arrival order: the head waits until a slot and its arena block are free
        while (!S->stop && !S->pending.empty()) {
            int idx = -1;
            for (int i = 0; i < (int)S->slots.size(); ++i)
                if (!S->slots[i].sim && !S->slots[i].req) {
                    idx = i;
                    break;
                }
            if (idx < 0) break;
            std::shared_ptr<Request> rq = S->pending.front();
            const size_t off = S->alloc.alloc(rq->ws);
            if (off == icwf::Arena::kFail) break;
            S->pending.pop_front();
            S->st.pending = (int32_t)S->pending.size();
            S->st.admitted += 1;
            S->st.active += 1;
            S->st.peak_active = std::max(S->st.peak_active, S->st.active);
            S->st.arena_in_use = S->alloc.in_use();
            S->st.arena_peak = S->alloc.peak();
            lk.unlock();
            admit(S, idx, rq, off);
            progress = true;
            lk.lock();
        }
        S->st.arena_in_use = S->alloc.in_use();
        bool any = false;
        for (const Slot &sl : S->slots) any = any || sl.sim != nullptr;
        if (S->stop && !any) break;
        if (!progress) S->cv_work.wait_for(lk, std::chrono::microseconds(200));
        lk.unlock();
    }
    // requests never admitted are dropped
    for (auto &rq : S->pending) {
        rq->info.status = ICWF_ESTATE;
        set_message(*rq, "the server stopped before the request was admitted");
        rq->done = true;
        rq->info.t_done = S->now();
    }
    S->pending.clear();
    S->st.pending = 0;
    S->cv_done.notify_all();
    lk.unlock();
}

bool all_finite(const double *p, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

}  // namespace

extern "C" {

icwf_status icwf_server_create(const icwf_server_config *cfg, void *arena, size_t arena_bytes, icwf_server **out) {
    if (!cfg || !arena || !out) return ICWF_EINVAL;
    *out = nullptr;
    if (cfg->max_active < 1 || cfg->max_active > 64 || cfg->steps_per_turn < 1 || cfg->turns_ahead < 1 ||
        cfg->turns_ahead > 4 || cfg->device < 0 || cfg->batch < 0 || cfg->batch > 1)
        return ICWF_EINVAL;
    if (reinterpret_cast<uintptr_t>(arena) % icwf::Arena::kAlign != 0 || arena_bytes < icwf::Arena::kAlign)
        return ICWF_EINVAL;
    if (hipSetDevice(cfg->device) != hipSuccess) return ICWF_EDEVICE;
    auto *S = new icwf_server(arena_bytes);
    S->cfg = *cfg;
    S->arena = reinterpret_cast<char *>(arena);
    S->t0 = Clock::now();
    S->st.arena_bytes = S->alloc.size();
    S->slots.resize(cfg->max_active);
    for (Slot &sl : S->slots)
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess) {
            for (Slot &x : S->slots)
                if (x.stream) (void)hipStreamDestroy(x.stream);
            delete S;
            return ICWF_EDEVICE;
        }
    S->th = std::thread(scheduler, S);
    *out = S;
    return ICWF_OK;
}

icwf_status icwf_server_submit(icwf_server *S, const icwf_config *cfg, const double *r0, const double *R0,
                               const double *psi1_0, const double *psi2_0, const double *C0, const double *b0,
                               const double *bo_states, int32_t n_steps, int64_t *id) {
    if (!S || !cfg || !id || !r0 || !R0 || !psi1_0 || !psi2_0 || (!C0 && !b0) || n_steps < 0) return ICWF_EINVAL;
    if (cfg->n_bo > 0 && !bo_states) return ICWF_EINVAL;
    const size_t ws = icwf_workspace_bytes(cfg);
    if (ws == 0) return ICWF_EINVAL;
    if (icwf::Arena::round_up(ws) > S->alloc.size()) return ICWF_ENOMEM;
    auto rq = std::make_shared<Request>();
    const size_t N = cfg->n_traj, nr = cfg->n_r, nR = cfg->n_R, nbo = std::max(cfg->n_bo, 0);
    rq->cfg = *cfg;
    rq->n_steps = n_steps;
    rq->ws = ws;
    rq->cost = step_cost_ms(*cfg);
    rq->r0.assign(r0, r0 + N);
    rq->R0.assign(R0, R0 + N);
    rq->psi1.assign(psi1_0, psi1_0 + 2 * N * nr);
    rq->psi2.assign(psi2_0, psi2_0 + 2 * N * nR);
    rq->has_C0 = C0 != nullptr;
    if (C0) rq->C0.assign(C0, C0 + 2 * N);
    else rq->b0.assign(b0, b0 + 2 * N);
    if (nbo > 0) rq->bo.assign(bo_states, bo_states + nR * nbo * nr);
    if (!all_finite(rq->r0.data(), N) || !all_finite(rq->R0.data(), N) || !all_finite(rq->psi1.data(), rq->psi1.size()) ||
        !all_finite(rq->psi2.data(), rq->psi2.size()) || !all_finite(rq->C0.data(), rq->C0.size()) ||
        !all_finite(rq->b0.data(), rq->b0.size()) || !all_finite(rq->bo.data(), rq->bo.size()))
        return ICWF_ENONFINITE;
    rq->info.slot = -1;
    rq->info.workspace_bytes = icwf::Arena::round_up(ws);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) return ICWF_ESTATE;
        rq->id = S->next_id++;
        rq->info.id = rq->id;
        rq->info.t_submit = S->now();
        S->known[rq->id] = rq;
        S->pending.push_back(rq);
        S->st.submitted += 1;
        S->st.pending = (int32_t)S->pending.size();
    }
    S->cv_work.notify_one();
    *id = rq->id;
    return ICWF_OK;
}

icwf_status icwf_server_wait(icwf_server *S, int64_t id, double timeout_s) {
    if (!S) return ICWF_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->known.find(id);
    if (it == S->known.end()) return ICWF_ESTATE;
    std::shared_ptr<Request> rq = it->second;
    auto ready = [&] { return rq->done; };
    if (timeout_s < 0) S->cv_done.wait(lk, ready);
    else if (!S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) return ICWF_ETIMEDOUT;
    return ICWF_OK;
}

icwf_status icwf_server_result(icwf_server *S, int64_t id, icwf_obs *o, icwf_request_info *info) {
    if (!S) return ICWF_EINVAL;
    std::shared_ptr<Request> rq;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->known.find(id);
        if (it == S->known.end() || !it->second->done) return ICWF_ESTATE;
        rq = it->second;
        S->known.erase(it);
    }
    if (info) *info = rq->info;
    if (o) {
        o->t = rq->t;
        o->step = rq->step;
        o->norm = rq->norm;
        o->n_out_of_box = rq->n_out;
        o->min_abs_psi = rq->min_abs_psi;
        auto put = [](double *dst, const std::vector<double> &v) {
            if (dst && !v.empty()) std::copy(v.begin(), v.end(), dst);
        };
        put(o->rho_r, rq->rho_r);
        put(o->rho_R, rq->rho_R);
        put(o->pop, rq->pop);
        put(o->D, rq->D);
        put(o->r, rq->r);
        put(o->R, rq->R);
        put(o->C, rq->C);
    }
    return static_cast<icwf_status>(rq->info.status);
}

icwf_status icwf_server_get_stats(icwf_server *S, icwf_server_stats *out) {
    if (!S || !out) return ICWF_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->st;
    out->arena_in_use = S->alloc.in_use();
    out->arena_peak = S->alloc.peak();
    return ICWF_OK;
}

double icwf_server_clock(const icwf_server *S) { return S ? S->now() : 0.0; }

void icwf_server_destroy(icwf_server *S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->th.joinable()) S->th.join();
    for (Slot &sl : S->slots) {
        for (auto &pr : sl.inflight) (void)hipEventDestroy(pr.first);
        for (hipEvent_t e : sl.pool) (void)hipEventDestroy(e);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    for (Lane &ln : S->lanes)
        if (ln.stream) (void)hipStreamDestroy(ln.stream);
    delete S;
}

}  // extern "C"
