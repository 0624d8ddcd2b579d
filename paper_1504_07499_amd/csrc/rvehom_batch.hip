// rvehom_batch.hip -- many RVEs at once: homogenize_batch and the serving
// loop of the C ABI (include/rvehom.h).
//
// Each RVE keeps its own device workspace and stream; the host enqueues
// iteration chunks for every active RVE round-robin, so the device always
// has work from all of them, and each RVE stops on its own device-side
// convergence flags (Algorithm of Sec. 3, arXiv:1504.07499, run per load
// case).  The server adds admission by device-memory footprint and slots,
// host workers for the RSA + voxelization setup of Sec. 2, and latency
// bookkeeping.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "rvegeom.h"
#include "rvehom.h"
#include "rvehom_internal.hpp"

namespace rvehom {

struct BatchItem {
    Solver *sv;
    const uint8_t *d_phase;
    hipStream_t stream;
    int max_iter;
    int index;
    SolverOpts opts;
    int timing;  // kernel timing mask (none in batches)
};

rve_status batch_solve(int count, const rve_t *rves, const double *k, const double *tol, const SolverOpts &o,
                       rve_result *out) {
    std::vector<BatchItem> act;
    for (int i = 0; i < count; ++i) {
        rve_s *r = rves[i];
        Solver &sv = r->sol[o.precision];
        int rc = sv.prepare(lookup_ops(o.precision, r->n), nullptr, 0);
        if (rc != RVE_OK) return (rve_status)rc;
        rc = sv.begin(r->d_phase, k + 3 * i, tol[i], o, sv.own_stream);
        if (rc != RVE_OK) return (rve_status)rc;
        act.push_back({&sv, r->d_phase, sv.own_stream, o.max_iter, i, o, 0});
    }
    rve_status worst = RVE_OK;
    int rc = drive(act, [&](BatchItem &a) {
        rve_result res{};
        int c = a.sv->collect(a.opts, a.stream, &res, nullptr, 0, nullptr);
        if (c != RVE_OK) return c;
        out[a.index] = res;
        rve_status s = worst_status(res, a.opts.lc_mask);
        if (s < 0 || (worst >= 0 && s > worst)) worst = s;
        return (int)RVE_OK;
    });
    if (rc != RVE_OK) return (rve_status)rc;
    return worst;
}

}  // namespace rvehom

using namespace rvehom;

// ---------------------------------------------------------------------------
// Serving
// ---------------------------------------------------------------------------
namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket;
    rve_geom geom;
    double k[3];
    double tol;
    Clock::time_point t_submit;
    std::vector<uint8_t> phases;  // filled by a host worker
    int setup_status = RVE_OK;
};

struct Done {
    rve_result res;
    rve_status status;
    double latency_s;
};

struct Slot {
    Request req;
    rve_s *rve = nullptr;
    hipStream_t stream = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct rve_server_s {
    size_t budget = 0;
    int max_slots = 1;
    int precision = 0;
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_setup, cv_ready, cv_done;
    std::deque<Request> setup_q;   // waiting for RSA + voxelization
    std::deque<Request> ready_q;   // waiting for admission
    std::map<uint64_t, Done> done;
    uint64_t next_ticket = 1;
    size_t submitted = 0, finished = 0;
    bool stop = false;
    std::vector<std::thread> workers;
    std::thread sched;
    std::vector<hipStream_t> streams;
    int fatal = RVE_OK;
};

static size_t footprint(int n, int precision) {
    const SolverOps *o = lookup_ops(precision, n);
    if (!o) return 0;
    return ws_layout(o).total + (size_t)n * n * n;
}

static void setup_worker(rve_server_s *s) {
    for (;;) {
        Request r;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_setup.wait(lk, [&] { return s->stop || !s->setup_q.empty(); });
            if (s->stop) return;
            r = std::move(s->setup_q.front());
            s->setup_q.pop_front();
        }
        const size_t M = (size_t)r.geom.n * r.geom.n * r.geom.n;
        r.phases.resize(M);
        int rc = rvegeom_generate(r.geom.n, r.geom.n_spheres, r.geom.volume_fraction, r.geom.layer, r.geom.seed,
                                  r.phases.data(), nullptr, nullptr);
        r.setup_status = rc == 0 ? RVE_OK : (rc == -2 ? RVE_ERR_JAMMED : RVE_ERR_ARG);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->ready_q.push_back(std::move(r));
        }
        s->cv_ready.notify_all();
    }
}

struct ServeItem {
    Solver *sv;
    const uint8_t *d_phase;
    hipStream_t stream;
    int max_iter;
    int slot;
    SolverOpts opts;
};

static void finish_request(rve_server_s *s, const Request &r, const rve_result &res, rve_status st) {
    const double lat = std::chrono::duration<double>(Clock::now() - r.t_submit).count();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->done[r.ticket] = Done{res, st, lat};
        s->finished++;
    }
    s->cv_done.notify_all();
}

static void scheduler(rve_server_s *s) {
    (void)hipSetDevice(s->device);
    std::vector<Slot> slots(s->max_slots);
    std::vector<int> free_slots;
    for (int i = s->max_slots - 1; i >= 0; --i) free_slots.push_back(i);
    std::vector<ServeItem> act;
    size_t used = 0;
    SolverOpts base;
    base.precision = s->precision;
    base.stall_window = s->precision == 0 ? 50 : 0;

    for (;;) {
        // admission: FIFO, by footprint and free slot
        std::vector<Request> admit;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            if (act.empty())
                s->cv_ready.wait(lk, [&] { return s->stop || !s->ready_q.empty(); });
            if (s->stop && act.empty()) return;
            while (!s->ready_q.empty() && !free_slots.empty()) {
                Request &r = s->ready_q.front();
                const size_t need = footprint(r.geom.n, s->precision);
                if (r.setup_status == RVE_OK && used + need > s->budget && !act.empty()) break;
                admit.push_back(std::move(r));
                s->ready_q.pop_front();
                if (admit.back().setup_status == RVE_OK) used += need;
                if (admit.size() + act.size() >= (size_t)s->max_slots) break;
            }
        }
        for (auto &r : admit) {
            if (r.setup_status != RVE_OK) {
                finish_request(s, r, rve_result{}, (rve_status)r.setup_status);
                continue;
            }
            const size_t need = footprint(r.geom.n, s->precision);
            rve_t h = nullptr;
            rve_status st = rve_create_from_phases(r.geom.n, r.phases.data(), &h);
            int rc = st;
            const int si = free_slots.back();
            if (st == RVE_OK) {
                Solver &sv = h->sol[s->precision];
                rc = sv.prepare(lookup_ops(s->precision, r.geom.n), nullptr, 0);
                if (rc == RVE_OK) rc = sv.begin(h->d_phase, r.k, r.tol, base, s->streams[si]);
            }
            if (rc != RVE_OK) {
                if (h) rve_destroy(h);
                used -= need;
                finish_request(s, r, rve_result{}, (rve_status)rc);
                continue;
            }
            free_slots.pop_back();
            r.phases.clear();
            r.phases.shrink_to_fit();
            slots[si].rve = h;
            slots[si].stream = s->streams[si];
            slots[si].bytes = need;
            slots[si].req = std::move(r);
            act.push_back({&h->sol[s->precision], h->d_phase, s->streams[si], base.max_iter, si, base});
        }
        if (act.empty()) continue;
        // one scheduling round: top up every active request, retire finished ones
        for (auto &a : act)
            if ((int)a.sv->inflight.size() < kLookahead && a.sv->issued < a.max_iter)
                if (a.sv->enqueue(a.d_phase, kChunk, a.max_iter, 0, a.stream) != RVE_OK) {
                    std::lock_guard<std::mutex> lk(s->mu);
                    s->fatal = RVE_ERR_DEVICE;
                }
        bool any = false;
        for (size_t i = 0; i < act.size();) {
            int rc = act[i].sv->poll(false, act[i].max_iter);
            if (rc == 0) {
                ++i;
                continue;
            }
            Slot &sl = slots[act[i].slot];
            rve_result res{};
            rve_status st = (rve_status)rc;
            if (rc == 1) {
                int c = act[i].sv->collect(act[i].opts, act[i].stream, &res, nullptr, 0, nullptr);
                st = c == RVE_OK ? worst_status(res, 7) : (rve_status)c;
            }
            finish_request(s, sl.req, res, st);
            rve_destroy(sl.rve);
            sl.rve = nullptr;
            used -= sl.bytes;
            free_slots.push_back(act[i].slot);
            act.erase(act.begin() + i);
            any = true;
        }
        if (!any) {
            bool all_full = true;
            for (auto &a : act)
                if ((int)a.sv->inflight.size() < kLookahead && a.sv->issued < a.max_iter) all_full = false;
            bool waiting;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                waiting = !s->ready_q.empty() && !free_slots.empty();
            }
            if (all_full && !waiting) (void)act[0].sv->poll(true, act[0].max_iter);
            if (all_full && waiting) std::this_thread::yield();
            // a blocking poll that finished a request is picked up next round
        }
    }
}

extern "C" rve_status rve_server_create(size_t hbm_budget_bytes, int max_slots, int precision, rve_server_t *out) {
    clear_error();
    if (!out || max_slots < 1 || max_slots > 256 || (precision != 0 && precision != 1) || hbm_budget_bytes == 0) {
        set_error("rve_server_create: bad arguments");
        return RVE_ERR_ARG;
    }
    rve_server_s *s = new rve_server_s();
    s->budget = hbm_budget_bytes;
    s->max_slots = max_slots;
    s->precision = precision;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        set_error("hipGetDevice failed");
        return RVE_ERR_DEVICE;
    }
    s->streams.resize(max_slots);
    for (auto &st : s->streams)
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            set_error("hipStreamCreate failed");
            return RVE_ERR_DEVICE;
        }
    const int nw = 4;
    for (int i = 0; i < nw; ++i) s->workers.emplace_back(setup_worker, s);
    s->sched = std::thread(scheduler, s);
    *out = s;
    return RVE_OK;
}

extern "C" rve_status rve_server_submit(rve_server_t s, const rve_geom *g, const double k[3], double tol,
                                        uint64_t *ticket) {
    clear_error();
    if (!s || !g || !ticket) {
        set_error("rve_server_submit: null pointer");
        return RVE_ERR_ARG;
    }
    if (!lookup_ops(s->precision, g->n) || g->n_spheres < 1 ||
        !(g->volume_fraction > 0.0 && g->volume_fraction < 1.0) || !(g->layer > 0.0 && g->layer < 1.0) ||
        !(rvegeom_radius(g->n_spheres, g->volume_fraction) < 0.5)) {
        set_error("rve_server_submit: invalid geometry");
        return RVE_ERR_ARG;
    }
    int rc = validate_k(k, tol);
    if (rc != RVE_OK) return (rve_status)rc;
    if (footprint(g->n, s->precision) > s->budget) {
        set_error("request footprint %zu exceeds the server budget %zu", footprint(g->n, s->precision), s->budget);
        return RVE_ERR_OOM;
    }
    Request r;
    r.geom = *g;
    std::memcpy(r.k, k, sizeof(r.k));
    r.tol = tol;
    r.t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        r.ticket = s->next_ticket++;
        *ticket = r.ticket;
        s->submitted++;
        s->setup_q.push_back(std::move(r));
    }
    s->cv_setup.notify_one();
    return RVE_OK;
}

extern "C" rve_status rve_server_poll(rve_server_t s, uint64_t ticket, rve_result *out, double *latency_s) {
    clear_error();
    if (!s || !out) {
        set_error("rve_server_poll: null pointer");
        return RVE_ERR_ARG;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->fatal != RVE_OK) {
        set_error("serving loop hit a device error");
        return (rve_status)s->fatal;
    }
    auto it = s->done.find(ticket);
    if (it == s->done.end()) {
        if (ticket == 0 || ticket >= s->next_ticket) {
            set_error("unknown ticket %llu", (unsigned long long)ticket);
            return RVE_ERR_ARG;
        }
        return RVE_PENDING;
    }
    *out = it->second.res;
    if (latency_s) *latency_s = it->second.latency_s;
    rve_status st = it->second.status;
    s->done.erase(it);
    return st;
}

extern "C" rve_status rve_server_drain(rve_server_t s) {
    clear_error();
    if (!s) return RVE_ERR_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->finished >= s->submitted || s->fatal != RVE_OK; });
    return (rve_status)s->fatal;
}

extern "C" void rve_server_destroy(rve_server_t s) {
    if (!s) return;
    (void)rve_server_drain(s);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_setup.notify_all();
    s->cv_ready.notify_all();
    for (auto &t : s->workers) t.join();
    if (s->sched.joinable()) s->sched.join();
    for (auto st : s->streams) (void)hipStreamDestroy(st);
    delete s;
}
