// rvehom_internal.hpp -- host-side objects behind the C ABI handles.
#pragma once

#include <hip/hip_runtime.h>

#include <deque>
#include <list>
#include <vector>

#include "rvehom.h"
#include "solver_ops.hpp"
#include "solver_state.hpp"

namespace rvehom {

constexpr int kHistCap = 16384;  // residual history entries kept per load case
constexpr int kChunk = 8;        // iterations between host poll points
constexpr int kLookahead = 2;    // poll points in flight before the host waits
constexpr int kPollSlots = 4;
constexpr size_t kFlagsOffset = 2048;  // poll flags inside the pinned block
constexpr size_t kTwStageOffset = 4096;  // twiddle staging inside the pinned block
constexpr size_t kPinnedBytes = 4096 + 8192;  // N <= 512 complex doubles of twiddles

struct WsLayout {
    size_t e, spec, nyq, tw, part, prm, st, hist, peq, spec2, nyq2, total;  // spec2 / nyq2: 0 if unused
};
WsLayout ws_layout(const SolverOps *o);

struct SolverOpts {
    int precision = 0;
    int max_iter = 10000;
    int eq_check = 0;
    int stall_window = 0;
    int lc_mask = 7;
    int scheme = 0;
    int timing = 0;  // bitmask of timed kernels: 1 fwd, 2 zgreen, 4 inv, 8 reduce; 16 sampled
    hipStream_t stream = nullptr;
    const double *init_field = nullptr;
    double *out_field = nullptr;
    void *workspace = nullptr;
    size_t workspace_bytes = 0;
    double alpha = 2.0;   // polarization scheme relaxation (rve_opts)
    int fp32_refine = 0;  // 0 on, -1 off (rve_opts)
    int path_flags = 0;   // PF_* measurement switches (rve_opts)
    // FP64 continuation: start from the FP32 fields on the device (per load
    // case, the base of a 9-channel FP32 field; channels 3 lc .. 3 lc + 2 are
    // taken) instead of E; the buffers hold tau already for scheme 2
    const void *dev_init[3] = {nullptr, nullptr, nullptr};
    const SolverOps *dev_init_ops = nullptr;
};

enum : int { PF_NO_GRAPHS = 1, PF_NO_FUSED = 2, PF_NO_MERGE = 4, PF_NO_CHAINS = 8, PF_ZTILE_DEFAULT = 16,
             PF_ZTILE_ALT = 32, PF_PLANE_DEFAULT = 64, PF_PLANE_ALT = 128 };

struct LaunchRec {
    int kernel;
    int iter;
    float ms;
};

// Iterations enqueued behind one poll point, and the timing events (one
// pair per timed kernel launch) that belong to that poll slot.
struct SlotInfo {
    int first_iter = 0;
    int count = 0;
    int mask = 0;
    std::vector<hipEvent_t> ev;  // 2 * kChunk * 4
};

// What a captured iteration graph depends on: the kernels (ops), the
// pointers baked into their arguments, and the launch-sequence switches.
struct GraphKey {
    const SolverOps *ops = nullptr;
    const void *ws = nullptr;
    const uint8_t *ph = nullptr;
    // al / dual: the update kernels of the scheme (the accelerated and basic
    // schemes share theirs, as do the augmented-Lagrangian and polarization)
    bool eq = false, fused = false, merge = false, al = false, dual = false;
    int lc = -1, zvar = 0, pvar = 0;
    bool operator==(const GraphKey &o) const {
        return ops == o.ops && ws == o.ws && ph == o.ph && eq == o.eq && fused == o.fused && merge == o.merge &&
               al == o.al && dual == o.dual && lc == o.lc && zvar == o.zvar && pvar == o.pvar;
    }
};

// Instantiated iteration graphs, reused across solves whose key matches
// (a server shares one cache among its slots).  An entry some solver holds
// as its current graph (refs > 0) is never evicted; any other entry has no
// launch in flight (a solve drains its stream before its solver moves on).
struct GraphCache {
    struct Entry {
        GraphKey key;
        hipGraphExec_t exec;
        int refs;
        uint64_t used;
    };
    std::list<Entry> entries;  // stable addresses: solvers hold pointers to entries
    size_t cap = 4;
    uint64_t tick = 0;
    uint64_t hits = 0, misses = 0;  // solves whose first full chunk found / captured its graph
    Entry *find(const GraphKey &k);
    Entry *put(const GraphKey &k, hipGraphExec_t x);
    void clear();
    ~GraphCache() { clear(); }
};

// Device workspace + HIP objects of one (RVE, precision).
struct Solver {
    const SolverOps *ops = nullptr;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    bool owned = false;
    bool tw_ready = false;
    WsLayout layout{};
    hipStream_t own_stream = nullptr;
    std::vector<hipEvent_t> poll_ev;
    SlotInfo slots[kPollSlots];
    hipEvent_t run_ev[2] = {nullptr, nullptr};
    void *h_pinned = nullptr;  // [DevParams | DevState | ... | flags @ kFlagsOffset]
    // per-solve driver state
    int issued = 0;
    int slot = 0;
    bool finished = false;
    std::deque<int> inflight;
    std::vector<LaunchRec> launches;
    bool eq_check = false;
    bool fused = false;  // iterations run zgreen + fused inverse/forward + reduce
    bool merge = false;  // each reduction runs inside the next iteration's z pass
    int lc_sel = -1;     // -1: all load cases; else the only load case iterated
    int zvar = 0;        // z-pass tile width: 0 default, 1 the other (autotuned)
    int pvar = 0;        // fused-pass threads per workgroup: 0 default, 1 the other (autotuned)
    bool al = false;     // augmented-Lagrangian family update (schemes 2 and 4)
    bool dual = false;   // dual scheme update (scheme 3)
    int scheme = 0;
    int path_flags = 0;  // PF_* of the current solve
    const uint8_t *d_phase_last = nullptr;
    // captured graph of kChunk iterations (kernels only; all parameters are
    // read from device memory, so one graph serves every call with the same
    // key), held from the cache
    GraphCache own_graphs;
    GraphCache *graphs = &own_graphs;
    GraphCache::Entry *gcur = nullptr;
    bool graph_counted = false;  // this solve's graph already counted as a cache hit or miss
    bool use_graphs = true;
    // timed variants: one graph per poll slot (its own events), per mask
    hipGraphExec_t tgexec[kPollSlots] = {};
    int tg_mask = 0;
    GraphKey tg_key{};

    ~Solver();
    void release();
    int init_objects();
    int prepare(const SolverOps *o, void *user_ws, size_t user_bytes);
    GraphKey graph_key(const uint8_t *d_phase) const;
    LaunchArgs args(const uint8_t *d_phase) const;
    int ensure_twiddles(hipStream_t s);
    int begin(const uint8_t *d_phase, const double k[3], double tol, const SolverOpts &o, hipStream_t s);
    int begin_elastic(const uint8_t *d_phase, const double moduli[6], double tol, const SolverOpts &o,
                      hipStream_t s);
    int start(const uint8_t *d_phase, const SolverOpts &o, hipStream_t s);
    int tune_zpass(const LaunchArgs &a, hipStream_t s);
    int tune_plane(const LaunchArgs &a, hipStream_t s, bool &ran);
    int enqueue(const uint8_t *d_phase, int count, int max_iter, int timing, hipStream_t s);
    int launch_iteration(const LaunchArgs &a, hipStream_t s, int mask, hipEvent_t *ev, bool red_in_z,
                         bool defer_red);
    int launch_batch(const LaunchArgs &a, hipStream_t s, int count, int mask, hipEvent_t *ev);
    int ensure_graph(const uint8_t *d_phase);
    int ensure_timed_graphs(const uint8_t *d_phase, int mask);
    int read_slot_times(int sl);
    void drop_graphs();
    int poll(bool wait, int max_iter);
    int collect(const SolverOpts &o, hipStream_t s, rve_result *out, double *hist, int hist_cap,
                rve_kernel_times *kt, rve_elastic_result *eout = nullptr);
};

// The inverse pass of an iteration: fused with the next forward pass or
// not, with the update of the scheme family; pvar: the fused pass at the
// other thread count per workgroup.
using InvFn = void (*)(const LaunchArgs &, hipStream_t, int);
inline InvFn inv_launcher(const SolverOps *ops, bool fused, bool al, bool dual, int pvar = 0) {
    if (fused && pvar && ops->inv_fwd_alt[0]) return ops->inv_fwd_alt[dual ? 2 : al ? 1 : 0];
    if (fused) return dual ? ops->inv_fwd_dual : al ? ops->inv_fwd_al : ops->inv_fwd;
    return dual ? ops->inv_dual : al ? ops->inv_al : ops->inv;
}

const SolverOps *lookup_ops(int precision, int n);
// the autotuner's z-tile and fused-pass choices for a grid, as made or
// imported in this process (no timing; defaults where there are none),
// unless path_flags force them
void tuned_choices(const SolverOps *ops, int path_flags, int &zvar, int &pvar);
const SolverOps *lookup_ops_el(int precision, int n);
void set_error(const char *fmt, ...);
void clear_error();
int validate_k(const double k[3], double tol);
void fill_params(DevParams &p, const double k[3], double tol, int n, const SolverOpts &o);
int check_scheme(const SolverOpts &o, const SolverOps *ops);
SolverOpts resolve_opts(const rve_opts *opts);
rve_status worst_status(const rve_result &r, int lc_mask);
rve_status solve_one(struct ::rve_s *r, const double k[3], double tol, const SolverOpts &o, rve_result *out,
                     double *hist, int hist_cap);
rve_status batch_solve(int count, const rve_t *rves, const double *k, const double *tol, const SolverOpts &o,
                       rve_result *out);
// FP64 continuation of the load cases an FP32 solve left STALLED (rve_opts
// fp32_refine); src[lc]: base of the FP32 field holding load case lc.
// refine_mask: the load cases to continue; refine_opts: the FP64 solve's
// options; refine_merge: its results into the FP32 ones.
int refine_mask(const rve_result &res, const SolverOpts &o);
SolverOpts refine_opts(const SolverOpts &o, const rve_result &res, int mask, const void *const src[3],
                       const SolverOps *ops32);
void refine_merge(rve_result &res, const rve_result &r64, int mask, double *hist, int hist_cap, const double *h64);
rve_status refine_fp64(struct ::rve_s *r, const SolverOps *ops32, const double k[3], double tol,
                       const SolverOpts &o, rve_result &res, double *hist, int hist_cap, const void *const src[3],
                       hipStream_t s);

// Drive already-begun solvers to completion, interleaving their chunks.
// finish(item) is called once per finished solver.
template <class Active, class Finish>
inline int drive(std::vector<Active> &act, Finish finish) {
    while (!act.empty()) {
        for (auto &a : act) {
            Solver &sv = *a.sv;
            if ((int)sv.inflight.size() < kLookahead && sv.issued < a.max_iter) {
                int rc = sv.enqueue(a.d_phase, kChunk, a.max_iter, a.timing, a.stream);
                if (rc != RVE_OK) return rc;
            }
        }
        bool any = false;
        for (size_t i = 0; i < act.size();) {
            int rc = act[i].sv->poll(false, act[i].max_iter);
            if (rc < 0) return rc;
            if (rc == 1) {
                rc = finish(act[i]);
                if (rc != RVE_OK) return rc;
                act.erase(act.begin() + i);
                any = true;
            } else {
                ++i;
            }
        }
        if (!any && !act.empty()) {
            // every solver is ahead by kLookahead chunks: wait for the oldest
            bool all_full = true;
            for (auto &a : act)
                if ((int)a.sv->inflight.size() < kLookahead && a.sv->issued < a.max_iter) all_full = false;
            if (all_full) {
                int rc = act[0].sv->poll(true, act[0].max_iter);
                if (rc < 0) return rc;
                if (rc == 1) {
                    rc = finish(act[0]);
                    if (rc != RVE_OK) return rc;
                    act.erase(act.begin());
                }
            }
        }
    }
    return RVE_OK;
}

}  // namespace rvehom

struct rve_s {
    int n = 0;
    int device = 0;
    uint8_t *d_phase = nullptr;
    std::vector<uint8_t> h_phase;
    std::vector<double> centers;
    double radius = 0.0;
    double layer = 0.0;
    int method = -1;
    rvehom::Solver sol[2];
    // per precision, one solver per load case: a full solve runs as three
    // concurrent single-load-case solves on their own streams
    rvehom::Solver chain[2][3];
    // per precision, the elastic case's solver (36 channels)
    rvehom::Solver el[2];
    rve_kernel_times times{};
};
