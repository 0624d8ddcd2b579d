// rvehom_batch.hip -- many RVEs at once: homogenize_batch and the serving
// loop of the C ABI (include/rvehom.h).
//
// Each RVE keeps its own device workspace and stream; the host enqueues
// iteration chunks for every active RVE round-robin, so the device always
// has work from all of them, and each RVE stops on its own device-side
// convergence flags (Algorithm of Sec. 3, arXiv:1504.07499, run per load
// case).  The server adds host workers for the RSA + voxelization setup of
// Sec. 2, admission by device-memory footprint from one device arena
// reserved at creation (no allocation per request), per-slot solvers whose
// HIP objects live as long as the server, iteration graphs shared by all
// slots, and latency bookkeeping.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
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
    int rc = drive(act, [&](BatchItem &a) {
        rve_result res{};
        int c = a.sv->collect(a.opts, a.stream, &res, nullptr, 0, nullptr);
        if (c != RVE_OK) return c;
        out[a.index] = res;
        return (int)RVE_OK;
    });
    if (rc != RVE_OK) return (rve_status)rc;
    // FP64 continuation of the load cases stopped by the FP32 floor: every
    // RVE that has some begins its FP64 solve from its FP32 field on its own
    // stream, and these solves are driven together as the FP32 ones were
    std::vector<BatchItem> ref;
    std::vector<int> masks(count, 0);
    for (int i = 0; i < count; ++i) {
        rve_s *r = rves[i];
        Solver &sv32 = r->sol[o.precision];
        const int mask = refine_mask(out[i], o);
        const SolverOps *ops64 = mask ? lookup_ops(1, r->n) : nullptr;
        if (!ops64) continue;  // nothing to continue, or no FP64 build of this grid (stays STALLED)
        Solver &sv = r->sol[1];
        rc = sv.prepare(ops64, nullptr, 0);
        if (rc != RVE_OK) return (rve_status)rc;
        const void *src[3];
        for (int lc = 0; lc < 3; ++lc) src[lc] = (const char *)sv32.ws + sv32.layout.e;
        const SolverOpts o64 = refine_opts(o, out[i], mask, src, sv32.ops);
        rc = sv.begin(r->d_phase, k + 3 * i, tol[i], o64, sv32.own_stream);
        if (rc != RVE_OK) return (rve_status)rc;
        masks[i] = mask;
        ref.push_back({&sv, r->d_phase, sv32.own_stream, o64.max_iter, i, o64, 0});
    }
    rc = drive(ref, [&](BatchItem &a) {
        rve_result r64{};
        int c = a.sv->collect(a.opts, a.stream, &r64, nullptr, 0, nullptr);
        if (c != RVE_OK) return c;
        refine_merge(out[a.index], r64, masks[a.index], nullptr, 0, nullptr);
        return (int)RVE_OK;
    });
    if (rc != RVE_OK) return (rve_status)rc;
    rve_status worst = RVE_OK;
    for (int i = 0; i < count; ++i) {
        rve_status s = worst_status(out[i], o.lc_mask);
        if (s < 0 || (worst >= 0 && s > worst)) worst = s;
    }
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

// First-fit sub-allocator over the server's one device buffer: offsets
// aligned to 256 bytes, neighbouring free blocks merged on release.
struct Arena {
    char *base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free_;  // offset -> bytes
    size_t used = 0, peak = 0;

    void reset(char *b, size_t n) {
        base = b;
        size = n;
        free_.clear();
        free_[0] = n;
        used = peak = 0;
    }
    bool alloc(size_t bytes, size_t *off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[*off + bytes] = rest;
            used += bytes;
            peak = std::max(peak, used);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        used -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// A request's device block: [phase image | workspace of its precision |
// (FP32) the FP64 workspace of its continuation].
struct Footprint {
    size_t phase, ws, ws64, total;
};

Footprint footprint_of(int n, int precision) {
    Footprint f{};
    const SolverOps *o = lookup_ops(precision, n);
    if (!o) return f;
    f.phase = align256((size_t)n * n * n);
    f.ws = align256(ws_layout(o).total);
    const SolverOps *o64 = precision == 0 ? lookup_ops(1, n) : nullptr;
    f.ws64 = o64 ? align256(ws_layout(o64).total) : 0;
    f.total = f.phase + f.ws + f.ws64;
    return f;
}

// One slot: a request resident on the device, its solvers (FP32 or FP64
// solve, and the FP64 continuation), their stream and the pinned staging of
// its phase image.  The HIP objects are created with the server.
struct ServeSlot {
    Solver sv;
    Solver sv64;
    uint8_t *h_stage = nullptr;
    bool active = false;
    bool refining = false;
    Request req;
    size_t off = 0;
    Footprint fp{};
    uint8_t *d_phase = nullptr;
    SolverOpts o{};
    SolverOpts o64{};
    rve_result res{};
    int mask = 0;
};

}  // namespace

struct rve_server_s {
    size_t budget = 0;
    int max_slots = 1;
    int precision = 0;
    int device = 0;
    size_t max_phase = 0;  // largest phase image a request may bring (pinned staging per slot)
    void *arena_mem = nullptr;
    Arena arena;
    GraphCache graphs;  // shared by every slot's solvers; outlives them
    std::vector<ServeSlot> slots;
    std::mutex mu;
    std::condition_variable cv_setup, cv_ready, cv_done;
    std::deque<Request> setup_q;  // waiting for RSA + voxelization
    std::deque<Request> ready_q;  // waiting for admission
    std::map<uint64_t, Done> done;
    uint64_t next_ticket = 1;
    size_t submitted = 0, finished = 0;
    bool stop = false;
    std::vector<std::thread> workers;
    std::thread sched;
    int fatal = RVE_OK;
    // statistics (rve_server_get_stats)
    uint64_t admitted = 0, refined = 0;
    int resident = 0, resident_peak = 0;
};

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

static void finish_request(rve_server_s *s, const Request &r, const rve_result &res, rve_status st) {
    const double lat = std::chrono::duration<double>(Clock::now() - r.t_submit).count();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->done[r.ticket] = Done{res, st, lat};
        s->finished++;
    }
    s->cv_done.notify_all();
}

static void set_fatal(rve_server_s *s, int rc) {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->fatal == RVE_OK) s->fatal = rc < 0 ? rc : RVE_ERR_DEVICE;
}

// Bring a request onto the device in slot sl: phase image through the
// pinned staging, workspace adopted from the arena block, solve begun.
static int admit_request(rve_server_s *s, ServeSlot &sl) {
    const int n = sl.req.geom.n;
    const size_t M = (size_t)n * n * n;
    char *blk = (char *)s->arena.base + sl.off;
    sl.d_phase = (uint8_t *)blk;
    std::memcpy(sl.h_stage, sl.req.phases.data(), M);
    sl.req.phases.clear();
    sl.req.phases.shrink_to_fit();
    hipStream_t st = sl.sv.own_stream;
    if (hipMemcpyAsync(sl.d_phase, sl.h_stage, M, hipMemcpyHostToDevice, st) != hipSuccess) {
        set_error("phase upload failed");
        return RVE_ERR_DEVICE;
    }
    int rc = sl.sv.prepare(lookup_ops(s->precision, n), blk + sl.fp.phase, sl.fp.ws);
    if (rc != RVE_OK) return rc;
    sl.o = SolverOpts{};
    sl.o.precision = s->precision;
    sl.o.stall_window = s->precision == 0 ? 50 : 0;
    sl.refining = false;
    sl.res = rve_result{};
    return sl.sv.begin(sl.d_phase, sl.req.k, sl.req.tol, sl.o, st);
}

// The FP32 solve of slot sl has finished with load cases at the FP32 floor:
// begin their FP64 continuation in the block's FP64 workspace.
static int begin_refine(rve_server_s *s, ServeSlot &sl) {
    const int n = sl.req.geom.n;
    char *blk = (char *)s->arena.base + sl.off;
    const void *src[3];
    for (int lc = 0; lc < 3; ++lc) src[lc] = (const char *)sl.sv.ws + sl.sv.layout.e;
    int rc = sl.sv64.prepare(lookup_ops(1, n), blk + sl.fp.phase + sl.fp.ws, sl.fp.ws64);
    if (rc != RVE_OK) return rc;
    sl.o64 = refine_opts(sl.o, sl.res, sl.mask, src, sl.sv.ops);
    sl.refining = true;
    return sl.sv64.begin(sl.d_phase, sl.req.k, sl.req.tol, sl.o64, sl.sv.own_stream);
}

static void scheduler(rve_server_s *s) {
    (void)hipSetDevice(s->device);
    std::vector<int> free_slots;
    for (int i = s->max_slots - 1; i >= 0; --i) free_slots.push_back(i);
    std::vector<int> act;  // active slot indices

    auto retire = [&](int si, rve_status st) {
        ServeSlot &sl = s->slots[si];
        finish_request(s, sl.req, sl.res, st);
        sl.active = false;
        free_slots.push_back(si);
        std::lock_guard<std::mutex> lk(s->mu);
        s->arena.release(sl.off, sl.fp.total);
        s->resident--;
    };

    for (;;) {
        // admission: FIFO, by a free slot and an arena block of the request's footprint
        std::vector<int> admitted;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            if (act.empty()) s->cv_ready.wait(lk, [&] { return s->stop || !s->ready_q.empty(); });
            if (s->stop && act.empty()) return;
            while (!s->ready_q.empty() && !free_slots.empty()) {
                Request &r = s->ready_q.front();
                if (r.setup_status != RVE_OK) {
                    Request bad = std::move(r);
                    s->ready_q.pop_front();
                    lk.unlock();
                    finish_request(s, bad, rve_result{}, (rve_status)bad.setup_status);
                    lk.lock();
                    continue;
                }
                const Footprint fp = footprint_of(r.geom.n, s->precision);
                size_t off = 0;
                if (!s->arena.alloc(fp.total, &off)) break;  // waits for a resident request to retire
                const int si = free_slots.back();
                free_slots.pop_back();
                ServeSlot &sl = s->slots[si];
                sl.req = std::move(r);
                s->ready_q.pop_front();
                sl.off = off;
                sl.fp = fp;
                sl.active = true;
                admitted.push_back(si);
                s->admitted++;
                s->resident++;
                s->resident_peak = std::max(s->resident_peak, s->resident);
            }
        }
        for (int si : admitted) {
            int rc = admit_request(s, s->slots[si]);
            if (rc != RVE_OK) {
                retire(si, (rve_status)rc);
                continue;
            }
            act.push_back(si);
        }
        if (act.empty()) continue;
        // one scheduling round: top up every active request, retire finished ones
        for (int si : act) {
            ServeSlot &sl = s->slots[si];
            Solver &sv = sl.refining ? sl.sv64 : sl.sv;
            const int mi = sl.refining ? sl.o64.max_iter : sl.o.max_iter;
            if ((int)sv.inflight.size() < kLookahead && sv.issued < mi)
                if (sv.enqueue(sl.d_phase, kChunk, mi, 0, sl.sv.own_stream) != RVE_OK) set_fatal(s, RVE_ERR_DEVICE);
        }
        bool any = false;
        for (size_t i = 0; i < act.size();) {
            const int si = act[i];
            ServeSlot &sl = s->slots[si];
            Solver &sv = sl.refining ? sl.sv64 : sl.sv;
            const SolverOpts &so = sl.refining ? sl.o64 : sl.o;
            int rc = sv.poll(false, so.max_iter);
            if (rc == 0) {
                ++i;
                continue;
            }
            any = true;
            rve_status st = (rve_status)rc;
            if (rc == 1) {
                rve_result r{};
                int c = sv.collect(so, sl.sv.own_stream, &r, nullptr, 0, nullptr);
                if (c == RVE_OK && !sl.refining) {
                    sl.res = r;
                    sl.mask = refine_mask(sl.res, sl.o);
                    if (sl.mask && lookup_ops(1, sl.req.geom.n)) {
                        c = begin_refine(s, sl);
                        if (c == RVE_OK) {
                            std::lock_guard<std::mutex> lk(s->mu);
                            s->refined++;
                            ++i;
                            continue;  // the slot stays active for its FP64 continuation
                        }
                    }
                } else if (c == RVE_OK) {
                    refine_merge(sl.res, r, sl.mask, nullptr, 0, nullptr);
                }
                st = c == RVE_OK ? worst_status(sl.res, 7) : (rve_status)c;
            }
            retire(si, st);
            act.erase(act.begin() + i);
        }
        if (!any) {
            bool all_full = true;
            for (int si : act) {
                ServeSlot &sl = s->slots[si];
                const Solver &sv = sl.refining ? sl.sv64 : sl.sv;
                const int mi = sl.refining ? sl.o64.max_iter : sl.o.max_iter;
                if ((int)sv.inflight.size() < kLookahead && sv.issued < mi) all_full = false;
            }
            bool waiting;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                waiting = !s->ready_q.empty() && !free_slots.empty();
            }
            if (all_full && !waiting && !act.empty()) {
                ServeSlot &sl = s->slots[act[0]];
                Solver &sv = sl.refining ? sl.sv64 : sl.sv;
                (void)sv.poll(true, sl.refining ? sl.o64.max_iter : sl.o.max_iter);
            }
            if (all_full && waiting) std::this_thread::yield();
            // a blocking poll that finished a request is picked up next round
        }
    }
}

static void server_free(rve_server_s *s) {
    for (auto &sl : s->slots) {
        sl.sv.release();
        sl.sv64.release();
        if (sl.h_stage) (void)hipHostFree(sl.h_stage);
        sl.h_stage = nullptr;
    }
    s->graphs.clear();
    if (s->arena_mem) (void)hipFree(s->arena_mem);
    s->arena_mem = nullptr;
    delete s;
}

extern "C" rve_status rve_server_create(size_t hbm_budget_bytes, int max_slots, int precision, rve_server_t *out) {
    clear_error();
    if (!out || max_slots < 1 || max_slots > 256 || (precision != 0 && precision != 1) || hbm_budget_bytes == 0) {
        set_error("rve_server_create: bad arguments");
        return RVE_ERR_ARG;
    }
    *out = nullptr;
    rve_server_s *s = new (std::nothrow) rve_server_s();
    if (!s) return RVE_ERR_OOM;
    s->budget = align256(hbm_budget_bytes);
    s->max_slots = max_slots;
    s->precision = precision;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        set_error("hipGetDevice failed");
        return RVE_ERR_DEVICE;
    }
    // the largest grid whose footprint fits the budget sets the staging size
    const int *sizes = nullptr;
    const int ns = supported_sizes(precision, &sizes);
    for (int i = 0; i < ns; ++i)
        if (footprint_of(sizes[i], precision).total <= s->budget)
            s->max_phase = std::max(s->max_phase, (size_t)sizes[i] * sizes[i] * sizes[i]);
    if (!s->max_phase) {
        delete s;
        set_error("rve_server_create: budget below the smallest grid's footprint");
        return RVE_ERR_ARG;
    }
    if (hipMalloc(&s->arena_mem, s->budget) != hipSuccess) {
        (void)hipGetLastError();
        s->arena_mem = nullptr;
        server_free(s);
        set_error("hipMalloc of the %zu-byte serving arena failed", (size_t)hbm_budget_bytes);
        return RVE_ERR_OOM;
    }
    s->arena.reset((char *)s->arena_mem, s->budget);
    s->graphs.cap = 64;
    s->slots = std::vector<ServeSlot>(max_slots);
    for (auto &sl : s->slots) {
        sl.sv.graphs = &s->graphs;
        sl.sv64.graphs = &s->graphs;
        int rc = sl.sv.init_objects();
        if (rc == RVE_OK) rc = sl.sv64.init_objects();
        if (rc == RVE_OK && hipHostMalloc((void **)&sl.h_stage, s->max_phase, hipHostMallocDefault) != hipSuccess) {
            sl.h_stage = nullptr;
            set_error("pinned staging of %zu bytes failed", s->max_phase);
            rc = RVE_ERR_OOM;
        }
        if (rc != RVE_OK) {
            server_free(s);
            return (rve_status)rc;
        }
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
    const Footprint fp = footprint_of(g->n, s->precision);
    if (fp.total > s->budget) {
        set_error("request footprint %zu exceeds the server budget %zu", fp.total, s->budget);
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

extern "C" rve_status rve_server_get_stats(rve_server_t s, rve_server_stats *out) {
    clear_error();
    if (!s || !out) {
        set_error("rve_server_get_stats: null pointer");
        return RVE_ERR_ARG;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    out->arena_bytes = s->budget;
    out->peak_bytes = s->arena.peak;
    out->resident_peak = s->resident_peak;
    out->admitted = s->admitted;
    out->completed = s->finished;
    out->refined = s->refined;
    out->graph_hits = s->graphs.hits;
    out->graph_misses = s->graphs.misses;
    return RVE_OK;
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
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(s->device);
    server_free(s);
    (void)hipSetDevice(cur);
}
