// rvehom_api.hip -- host side of the C ABI declared in include/rvehom.h:
// RVE handles, device workspaces, the iteration loop with on-device
// convergence, batched solves, the elastic case and kernel timing.
//
// Paper: arXiv:1504.07499.  The host loop runs the Algorithm of Sec. 3
// (initialise with grad Theta, iterate steps 2-7 until eps_comp < acc, then
// L_hom from <phi>) for the three unit load cases at once; the reference
// medium is the one of Sec. 5.  The elastic case (Sec. 6) runs the same loop
// over six load cases.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "rvegeom.h"
#include "rvehom.h"
#include "rvehom_internal.hpp"
#include "solver_ops.hpp"
#include "solver_state.hpp"

namespace rvehom {

static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
}

void clear_error() { g_err.clear(); }

const SolverOps *lookup_ops(int precision, int n) {
    if (precision == 0) return ops_f32(n);
    if (precision == 1) return ops_f64(n);
    return nullptr;
}

const SolverOps *lookup_ops_el(int precision, int n) {
    if (precision == 0) return ops_el_f32(n);
    if (precision == 1) return ops_el_f64(n);
    return nullptr;
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

WsLayout ws_layout(const SolverOps *o) {
    WsLayout L{};
    const size_t n = (size_t)o->n, M = n * n * n, rb = o->real_bytes;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off += align256(bytes);
        return at;
    };
    const size_t ch = (size_t)o->nc * o->nc;  // channels: nc load cases of nc components
    L.e = take(ch * M * rb);
    L.spec = take(o->spec_elems * 2 * rb);
    L.nyq = take(o->nyq_elems * 2 * rb);
    L.tw = take(n * 2 * rb);
    L.part = take(ch * o->nper * 3 * sizeof(double));
    L.prm = take(sizeof(DevParams));
    L.st = take(sizeof(DevState));
    L.hist = take((size_t)o->nc * kHistCap * sizeof(double));
    L.peq = take((size_t)o->nc * (o->eq_tiles > 0 ? o->eq_tiles : 1) * 2 * sizeof(double));
    // split planes: the parity-layout spectrum the fused pass writes
    L.spec2 = o->zgreen_par ? take(o->spec_elems * 2 * rb) : 0;
    L.nyq2 = o->zgreen_par ? take(o->nyq_elems * 2 * rb) : 0;
    L.total = off;
    return L;
}

#define HIP_CHECK(call)                                                                   \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess) {                                                           \
            set_error("%s failed: %s", #call, hipGetErrorString(e_));                     \
            return RVE_ERR_DEVICE;                                                        \
        }                                                                                 \
    } while (0)

GraphCache::Entry *GraphCache::find(const GraphKey &k) {
    for (auto &e : entries)
        if (e.key == k) {
            e.used = ++tick;
            return &e;
        }
    return nullptr;
}

GraphCache::Entry *GraphCache::put(const GraphKey &k, hipGraphExec_t x) {
    if (entries.size() >= cap) {
        // evict the least recently used entry that no solver holds (if every
        // entry is held the cache grows past cap)
        auto victim = entries.end();
        for (auto it = entries.begin(); it != entries.end(); ++it)
            if (it->refs == 0 && (victim == entries.end() || it->used < victim->used)) victim = it;
        if (victim != entries.end()) {
            (void)hipGraphExecDestroy(victim->exec);
            entries.erase(victim);
        }
    }
    entries.push_back({k, x, 0, ++tick});
    return &entries.back();
}

void GraphCache::clear() {
    for (auto &e : entries) (void)hipGraphExecDestroy(e.exec);
    entries.clear();
}

Solver::~Solver() { release(); }

void Solver::release() {
    if (owned && ws) (void)hipFree(ws);
    ws = nullptr;
    owned = false;
    ws_bytes = 0;
    tw_ready = false;
    if (own_stream) (void)hipStreamDestroy(own_stream);
    own_stream = nullptr;
    for (auto ev : poll_ev) (void)hipEventDestroy(ev);
    poll_ev.clear();
    for (auto &si : slots) {
        for (auto ev : si.ev) (void)hipEventDestroy(ev);
        si.ev.clear();
    }
    if (run_ev[0]) (void)hipEventDestroy(run_ev[0]);
    if (run_ev[1]) (void)hipEventDestroy(run_ev[1]);
    run_ev[0] = run_ev[1] = nullptr;
    if (h_pinned) (void)hipHostFree(h_pinned);
    h_pinned = nullptr;
    drop_graphs();
}

void Solver::drop_graphs() {
    if (gcur) gcur->refs--;
    gcur = nullptr;
    if (graphs == &own_graphs) own_graphs.clear();
    for (auto &g : tgexec) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
    tg_mask = 0;
}

// The HIP objects of a solver: its stream, poll and timing events and the
// pinned host block (parameters, state, poll flags, twiddle staging).
int Solver::init_objects() {
    if (!own_stream) HIP_CHECK(hipStreamCreateWithFlags(&own_stream, hipStreamNonBlocking));
    if (poll_ev.empty()) {
        poll_ev.resize(kPollSlots);
        for (auto &ev : poll_ev) HIP_CHECK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        for (auto &si : slots) {
            // kernel-timing events: nothing waits on them, so they skip the
            // system-scope release (a cache writeback that would otherwise be
            // charged to the bracketed kernel)
            si.ev.resize(2 * kChunk * 4);
            for (auto &ev : si.ev) HIP_CHECK(hipEventCreateWithFlags(&ev, hipEventDisableSystemFence));
        }
    }
    if (!run_ev[0]) {
        HIP_CHECK(hipEventCreate(&run_ev[0]));
        HIP_CHECK(hipEventCreate(&run_ev[1]));
    }
    if (!h_pinned) {
        // [DevParams | DevState | poll flags | twiddle staging] in one pinned block
        HIP_CHECK(hipHostMalloc(&h_pinned, kPinnedBytes, hipHostMallocDefault));
    }
    return RVE_OK;
}

// Allocate (or adopt) the workspace and the per-solver HIP objects.  A change
// of grid size or precision keeps the HIP objects and the graph cache (its
// keys hold the kernels) and frees only an owned workspace.
int Solver::prepare(const SolverOps *o, void *user_ws, size_t user_bytes) {
    if (ops != o) {
        if (owned && ws) (void)hipFree(ws);
        ws = nullptr;
        owned = false;
        ws_bytes = 0;
        tw_ready = false;
        ops = o;
    }
    const WsLayout L = ws_layout(o);
    if (user_ws) {
        if (user_bytes < L.total) {
            set_error("workspace of %zu bytes is smaller than the %zu bytes needed", user_bytes, L.total);
            return RVE_ERR_ARG;
        }
        if (((uintptr_t)user_ws & 255) != 0) {
            set_error("workspace must be 256-byte aligned");
            return RVE_ERR_ARG;
        }
        if (owned && ws) (void)hipFree(ws);
        // a workspace the solver does not own may have been written by
        // others since this solver's last solve (another handle, or another
        // served request's block at the same place): its twiddle table is
        // uploaded again for every solve
        tw_ready = false;
        ws = user_ws;
        owned = false;
        ws_bytes = user_bytes;
    } else if (!ws || !owned) {
        void *p = nullptr;
        if (hipMalloc(&p, L.total) != hipSuccess) {
            (void)hipGetLastError();
            set_error("hipMalloc of %zu workspace bytes failed", L.total);
            return RVE_ERR_OOM;
        }
        ws = p;
        owned = true;
        ws_bytes = L.total;
        tw_ready = false;
    }
    layout = L;
    return init_objects();
}

LaunchArgs Solver::args(const uint8_t *d_phase) const {
    char *b = (char *)ws;
    LaunchArgs a;
    a.e = b + layout.e;
    a.ph = d_phase;
    a.spec = b + layout.spec;
    a.nyq = b + layout.nyq;
    a.tw = b + layout.tw;
    a.prm = (const DevParams *)(b + layout.prm);
    a.st = (DevState *)(b + layout.st);
    a.part = (double *)(b + layout.part);
    a.hist = (double *)(b + layout.hist);
    a.peq = (double *)(b + layout.peq);
    a.spec2 = layout.spec2 ? b + layout.spec2 : nullptr;
    a.nyq2 = layout.nyq2 ? b + layout.nyq2 : nullptr;
    return a;
}

int Solver::ensure_twiddles(hipStream_t s) {
    if (tw_ready) return RVE_OK;
    const int n = ops->n;
    // exp(-2 pi i m / n) in FP64, rounded once to the working precision,
    // staged in the pinned block (rewritten only by a later solve on this
    // solver, after this one has drained) and copied in stream order
    char *stage = (char *)h_pinned + kTwStageOffset;
    const bool f32 = ops->real_bytes == sizeof(float);
    if ((size_t)n * 2 * ops->real_bytes > kPinnedBytes - kTwStageOffset) {
        set_error("twiddle table of N = %d does not fit the staging block", n);
        return RVE_ERR_ARG;
    }
    for (int m = 0; m < n; ++m) {
        const double a = 2.0 * M_PI * (double)m / (double)n;
        const double c = std::cos(a), sn = -std::sin(a);
        if (f32) {
            ((float *)stage)[2 * m] = (float)c;
            ((float *)stage)[2 * m + 1] = (float)sn;
        } else {
            ((double *)stage)[2 * m] = c;
            ((double *)stage)[2 * m + 1] = sn;
        }
    }
    char *dst = (char *)ws + layout.tw;
    HIP_CHECK(hipMemcpyAsync(dst, stage, (size_t)n * 2 * ops->real_bytes, hipMemcpyHostToDevice, s));
    tw_ready = true;
    return RVE_OK;
}

}  // namespace rvehom

using namespace rvehom;

// ---------------------------------------------------------------------------
// Handles
// ---------------------------------------------------------------------------
extern "C" const char *rve_last_error(void) { return g_err.c_str(); }

extern "C" rve_status rve_supported_n(int precision, int *out, int cap, int *count) {
    clear_error();
    if ((precision != 0 && precision != 1) || !count || (cap > 0 && !out) || cap < 0) {
        set_error("rve_supported_n: bad arguments");
        return RVE_ERR_ARG;
    }
    const int *list = nullptr;
    const int k = supported_sizes(precision, &list);
    for (int i = 0; i < k && i < cap; ++i) out[i] = list[i];
    *count = k;
    return RVE_OK;
}

static bool size_supported(int n) {
    return lookup_ops(0, n) != nullptr || lookup_ops(1, n) != nullptr;
}

static rve_status upload_rve(rve_s *r) {
    const size_t M = (size_t)r->n * r->n * r->n;
    HIP_CHECK(hipGetDevice(&r->device));
    if (hipMalloc(&r->d_phase, M) != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipMalloc of the %zu-byte phase image failed", M);
        return RVE_ERR_OOM;
    }
    HIP_CHECK(hipMemcpy(r->d_phase, r->h_phase.data(), M, hipMemcpyHostToDevice));
    return RVE_OK;
}

extern "C" rve_status rve_create_from_phases(int n, const uint8_t *phases, rve_t *out) {
    clear_error();
    if (!out || !phases || !size_supported(n)) {
        set_error("rve_create_from_phases: null pointer or unsupported grid size %d", n);
        return RVE_ERR_ARG;
    }
    *out = nullptr;
    const size_t M = (size_t)n * n * n;
    for (size_t v = 0; v < M; ++v)
        if (phases[v] > 2) {
            set_error("phase id %d at voxel %zu is not 0, 1 or 2", (int)phases[v], v);
            return RVE_ERR_ARG;
        }
    rve_s *r = new (std::nothrow) rve_s();
    if (!r) return RVE_ERR_OOM;
    r->n = n;
    r->h_phase.assign(phases, phases + M);
    rve_status st = upload_rve(r);
    if (st != RVE_OK) {
        delete r;
        return st;
    }
    *out = r;
    return RVE_OK;
}

extern "C" rve_status rve_create(const rve_geom *g, rve_t *out) {
    clear_error();
    if (!g || !out) {
        set_error("rve_create: null pointer");
        return RVE_ERR_ARG;
    }
    *out = nullptr;
    if (!size_supported(g->n) || g->n_spheres < 1 || !(g->volume_fraction > 0.0 && g->volume_fraction < 1.0) ||
        !(g->layer > 0.0 && g->layer < 1.0) || !(rvegeom_radius(g->n_spheres, g->volume_fraction) < 0.5)) {
        set_error("rve_create: invalid geometry (n=%d, spheres=%d, f=%g, l=%g)", g->n, g->n_spheres,
                  g->volume_fraction, g->layer);
        return RVE_ERR_ARG;
    }
    rve_s *r = new (std::nothrow) rve_s();
    if (!r) return RVE_ERR_OOM;
    const size_t M = (size_t)g->n * g->n * g->n;
    r->n = g->n;
    r->h_phase.resize(M);
    r->centers.resize(3 * (size_t)g->n_spheres);
    int method = 0;
    int rc = rvegeom_generate(g->n, g->n_spheres, g->volume_fraction, g->layer, g->seed, r->h_phase.data(),
                              r->centers.data(), &method);
    if (rc != 0) {
        delete r;
        set_error(rc == -2 ? "spheres could not be placed (jammed)" : "invalid geometry");
        return rc == -2 ? RVE_ERR_JAMMED : RVE_ERR_ARG;
    }
    r->radius = rvegeom_radius(g->n_spheres, g->volume_fraction);
    r->layer = g->layer;
    r->method = method;
    rve_status st = upload_rve(r);
    if (st != RVE_OK) {
        delete r;
        return st;
    }
    *out = r;
    return RVE_OK;
}

extern "C" rve_status rve_get_phases(rve_t r, uint8_t *out, size_t cap) {
    clear_error();
    if (!r || !out || cap < r->h_phase.size()) {
        set_error("rve_get_phases: null pointer or buffer too small");
        return RVE_ERR_ARG;
    }
    std::memcpy(out, r->h_phase.data(), r->h_phase.size());
    return RVE_OK;
}

extern "C" rve_status rve_get_spheres(rve_t r, double *xyzr, int cap, int *count, double *layer) {
    clear_error();
    if (!r || !count || cap < 0 || (cap > 0 && !xyzr)) {
        set_error("rve_get_spheres: bad arguments");
        return RVE_ERR_ARG;
    }
    const int ns = (int)(r->centers.size() / 3);
    const int k = std::min(ns, cap);
    for (int i = 0; i < k; ++i) {
        for (int d = 0; d < 3; ++d) xyzr[4 * i + d] = r->centers[3 * i + d];
        xyzr[4 * i + 3] = r->radius;
    }
    *count = ns;
    if (layer) *layer = r->layer;
    return RVE_OK;
}

extern "C" int rve_n(rve_t r) { return r ? r->n : 0; }

extern "C" size_t rve_workspace_size(rve_t r, int precision) {
    if (!r) return 0;
    const SolverOps *o = lookup_ops(precision, r->n);
    return o ? ws_layout(o).total : 0;
}

extern "C" void rve_destroy(rve_t r) {
    if (!r) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(r->device);
    // every solver of the handle (thermal, load-case chains, elastic) frees
    // its workspace, streams and graphs while the handle's device is current
    for (int p = 0; p < 2; ++p) {
        r->sol[p].release();
        for (auto &c : r->chain[p]) c.release();
        r->el[p].release();
    }
    if (r->d_phase) (void)hipFree(r->d_phase);
    (void)hipSetDevice(cur);
    delete r;
}

// ---------------------------------------------------------------------------
// Solve driver
// ---------------------------------------------------------------------------
namespace rvehom {

int validate_k(const double k[3], double tol) {
    if (!k) {
        set_error("k_phases is NULL");
        return RVE_ERR_ARG;
    }
    for (int p = 0; p < 3; ++p)
        if (!(k[p] > 0.0) || !std::isfinite(k[p])) {
            set_error("conductivity of phase %d must be finite and > 0 (got %g)", p, k[p]);
            return RVE_ERR_ARG;
        }
    if (!(tol >= 0.0) || !std::isfinite(tol)) {
        set_error("tol must be finite and >= 0 (got %g)", tol);
        return RVE_ERR_ARG;
    }
    return RVE_OK;
}

void fill_params(DevParams &p, const double k[3], double tol, int n, const SolverOpts &o) {
    std::memset(&p, 0, sizeof(p));
    const double kmin = std::min(k[0], std::min(k[1], k[2]));
    const double kmax = std::max(k[0], std::max(k[1], k[2]));
    // Sec. 5: L0 = -sqrt(min k * max k) I over the three given conductivities
    // (accelerated, augmented-Lagrangian and polarization schemes); the basic
    // scheme uses the arithmetic mean of the extremes, the dual scheme their
    // harmonic mean.
    const double k0 = o.scheme == 1   ? 0.5 * (kmin + kmax)
                      : o.scheme == 3 ? 2.0 * kmin * kmax / (kmin + kmax)
                                      : std::sqrt(kmin * kmax);
    const double M = (double)n * n * n;
    for (int i = 0; i < 3; ++i) {
        p.k[i] = k[i];
        // step 2: tau = (k - k0) e; dual scheme: tau = -k0^2 phi / k, which
        // the z pass turns into k0 G*(phi / k)
        p.dk[i] = o.scheme == 3 ? -k0 * k0 / k[i] : k[i] - k0;
        // step 7: e+ = e + 2 k0 / (k + k0) (c - e); basic scheme: e+ = c;
        // dual scheme: phi+ = (1 - k0 / k) phi + c + k0 E
        p.w[i] = o.scheme == 1 ? 1.0 : o.scheme == 3 ? 1.0 - k0 / k[i] : 2.0 * k0 / (k[i] + k0);
        p.gam[i] = 1.0 / (k[i] + k0);
    }
    p.k0 = k0;
    p.scheme = o.scheme;
    p.relax = o.scheme == 4 ? o.alpha : 1.0;
    // contraction bound of the scheme at contrast c = kmax / kmin: Eyre-Milton
    // (sqrt c - 1) / (sqrt c + 1), basic and dual schemes (c - 1) / (c + 1);
    // the augmented Lagrangian averages the Eyre-Milton operator with the
    // identity (Douglas-Rachford form): (1 + rho_EM) / 2; the polarization
    // scheme with relaxation alpha: |1 - alpha/2| + (alpha/2) rho_EM
    const double c = kmax / kmin;
    const double rem = (std::sqrt(c) - 1.0) / (std::sqrt(c) + 1.0);
    const double rho = (o.scheme == 1 || o.scheme == 3) ? (c - 1.0) / (c + 1.0)
                       : o.scheme == 2                 ? 0.5 * (1.0 + rem)
                       : o.scheme == 4 ? std::fabs(1.0 - 0.5 * o.alpha) + 0.5 * o.alpha * rem
                                       : rem;
    p.prog10 = 1.0 - std::pow(rho, 10.0);
    p.inv_k0M = 1.0 / (k0 * M);
    p.tol = tol;
    p.invM = 1.0 / M;
    p.max_iter = o.max_iter;
    p.stall_window = o.stall_window;
    p.hist_cap = kHistCap;
    p.eq_check = o.eq_check;
    p.lc_mask = o.lc_mask;
    p.nc = 3;
}

// The elastic case: moduli = (kappa, mu) per phase.  Reference medium: the
// Sec. 5 rule applied to each modulus, kappa0 = sqrt(min kappa max kappa),
// mu0 = sqrt(min mu max mu).  In the orthonormal basis of the kernels the
// hydrostatic channel carries 3 kappa, the deviatoric ones 2 mu.
void fill_params_el(DevParams &p, const double moduli[6], double tol, int n, const SolverOpts &o) {
    std::memset(&p, 0, sizeof(p));
    double kap[3], mu[3];
    for (int i = 0; i < 3; ++i) {
        kap[i] = moduli[2 * i];
        mu[i] = moduli[2 * i + 1];
    }
    const double kmin = std::min(kap[0], std::min(kap[1], kap[2])), kmax = std::max(kap[0], std::max(kap[1], kap[2]));
    const double mmin = std::min(mu[0], std::min(mu[1], mu[2])), mmax = std::max(mu[0], std::max(mu[1], mu[2]));
    const double kap0 = std::sqrt(kmin * kmax), mu0 = std::sqrt(mmin * mmax);
    const double lam0 = kap0 - 2.0 * mu0 / 3.0;
    const double M = (double)n * n * n;
    for (int i = 0; i < 3; ++i) {
        p.k[i] = 3.0 * kap[i];
        p.dk[i] = 3.0 * (kap[i] - kap0);
        p.w[i] = 2.0 * kap0 / (kap[i] + kap0);
        p.k_dev[i] = 2.0 * mu[i];
        p.dk_dev[i] = 2.0 * (mu[i] - mu0);
        p.w_dev[i] = 2.0 * mu0 / (mu[i] + mu0);
    }
    p.k0 = 3.0 * kap0;
    p.k0_dev = 2.0 * mu0;
    p.el_inv_mu0M = 1.0 / (mu0 * M);
    p.el_betaM = (lam0 + mu0) / (mu0 * (lam0 + 2.0 * mu0)) / M;
    // contraction bound: the larger of the two moduli's Eyre-Milton factors
    const double ck = kmax / kmin, cm = mmax / mmin;
    const double rho = std::max((std::sqrt(ck) - 1.0) / (std::sqrt(ck) + 1.0), (std::sqrt(cm) - 1.0) / (std::sqrt(cm) + 1.0));
    p.prog10 = 1.0 - std::pow(rho, 10.0);
    p.tol = tol;
    p.invM = 1.0 / M;
    p.max_iter = o.max_iter;
    p.stall_window = o.stall_window;
    p.hist_cap = kHistCap;
    p.eq_check = 0;
    p.lc_mask = 63;
    p.nc = 6;
}

SolverOpts resolve_opts(const rve_opts *opts) {
    SolverOpts o;
    o.precision = opts ? opts->precision : 0;
    o.max_iter = (opts && opts->max_iter > 0) ? opts->max_iter : 10000;
    o.eq_check = opts ? (opts->equilibrium_check != 0) : 0;
    int sw = opts ? opts->stall_window : -1;
    o.stall_window = sw < 0 ? (o.precision == 0 ? 50 : 0) : sw;
    o.lc_mask = (opts && (opts->lc_mask & 7)) ? (opts->lc_mask & 7) : 7;
    o.timing = opts ? (opts->timing & 31) : 0;
    o.stream = opts ? (hipStream_t)opts->stream : nullptr;
    o.init_field = opts ? opts->init_field : nullptr;
    o.out_field = opts ? opts->out_field : nullptr;
    o.workspace = opts ? opts->workspace : nullptr;
    o.workspace_bytes = opts ? opts->workspace_bytes : 0;
    o.scheme = opts ? opts->scheme : 0;
    o.fp32_refine = (opts && opts->fp32_refine < 0) ? -1 : 0;
    o.alpha = (opts && opts->alpha != 0.0) ? opts->alpha : 2.0;
    o.path_flags = opts ? (opts->path_flags & 255) : 0;
    return o;
}

// Enqueue init (and optional warm start) on s.
// Autotuner: the first solve of each (precision, N) in the process times,
// on this workspace and before the solve proper,
// * the z pass at its two tile widths (before the first forward pass
//   overwrites the spectrum).  The z transform of a pencil does not depend
//   on the tile width, so the choice never changes a result.
//   PF_ZTILE_DEFAULT / PF_ZTILE_ALT force the default / the other width;
// * the fused plane pass at its two thread counts per workgroup (whole
//   planes only; the field it overwrites is initialised again after).  The
//   arithmetic per voxel is the same up to the compiler's instruction
//   choice for each shape; the grouping of the FP64 partial sums differs,
//   so results agree to rounding.  PF_PLANE_DEFAULT / PF_PLANE_ALT force
//   the choice.
// Each keeps the faster, differences under 3 % keeping the default.  The
// choices are kept per (GPU architecture, precision, N) and can be exported
// and imported as text (rve_tune_export / rve_tune_import), so a later
// process on the same architecture skips the timing.
using TuneKey = std::tuple<std::string, int, int>;  // gfx arch, precision, N
static std::mutex g_tune_mu;
static std::map<TuneKey, int> g_ztune, g_ptune;

// Times fa then fb, reps launches each after one untimed launch of each
// (code load), on stream s; alt_wins = fb took under 0.97 of fa's time.
template <class FA, class FB> static int time_two(hipStream_t s, FA fa, FB fb, bool &alt_wins) {
    constexpr int reps = 6;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    int rc = RVE_OK;
    float t0 = 0.f, t1 = 0.f;
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) rc = RVE_ERR_DEVICE;
    if (rc == RVE_OK) {
        fa();
        fb();
        bool ok = hipEventRecord(ev[0], s) == hipSuccess;
        for (int i = 0; i < reps; ++i) fa();
        ok = ok && hipEventRecord(ev[1], s) == hipSuccess;
        for (int i = 0; i < reps; ++i) fb();
        ok = ok && hipEventRecord(ev[2], s) == hipSuccess;
        ok = ok && hipGetLastError() == hipSuccess && hipEventSynchronize(ev[2]) == hipSuccess &&
             hipEventElapsedTime(&t0, ev[0], ev[1]) == hipSuccess && hipEventElapsedTime(&t1, ev[1], ev[2]) == hipSuccess;
        if (!ok) {
            set_error("autotuner: timing launches failed");
            rc = RVE_ERR_DEVICE;
        }
    }
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    alt_wins = rc == RVE_OK && t1 < 0.97f * t0;
    return rc;
}

// gfx architecture name of the current device ("gfx950"), or "" on failure.
static std::string current_arch() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return std::string();
    static std::mutex mu;
    static std::map<int, std::string> cache;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return std::string();
    std::string name(prop.gcnArchName);
    name = name.substr(0, name.find(':'));  // drop feature suffixes (":sramecc+:xnack-")
    cache[dev] = name;
    return name;
}

int Solver::tune_zpass(const LaunchArgs &a, hipStream_t s) {
    zvar = 0;
    if (!ops->zgreen_alt) return RVE_OK;
    if (path_flags & (PF_ZTILE_DEFAULT | PF_ZTILE_ALT)) {
        zvar = (path_flags & PF_ZTILE_ALT) ? 1 : 0;
        return RVE_OK;
    }
    const TuneKey key{current_arch(), ops->precision, ops->n};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_ztune.find(key);
        if (it != g_ztune.end()) {
            zvar = it->second;
            return RVE_OK;
        }
    }
    bool alt = false;
    const int rc = time_two(
        s, [&] { ops->zgreen(a, s, 0, -1); }, [&] { ops->zgreen_alt(a, s, 0, -1); }, alt);
    if (rc != RVE_OK) return rc;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    zvar = g_ztune.emplace(key, alt ? 1 : 0).first->second;
    return RVE_OK;
}

// The choices the autotuner made or imported for this grid in this process,
// without timing (0 where there is none); path_flags force them.
void tuned_choices(const SolverOps *ops, int path_flags, int &zvar, int &pvar) {
    const TuneKey key{current_arch(), ops->precision, ops->n};
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto iz = g_ztune.find(key);
    auto ip = g_ptune.find(key);
    zvar = ops->zgreen_alt ? (path_flags & (PF_ZTILE_DEFAULT | PF_ZTILE_ALT) ? (path_flags & PF_ZTILE_ALT ? 1 : 0)
                                                                             : (iz != g_ztune.end() ? iz->second : 0))
                           : 0;
    pvar = ops->inv_fwd_alt[0] ? (path_flags & (PF_PLANE_DEFAULT | PF_PLANE_ALT) ? (path_flags & PF_PLANE_ALT ? 1 : 0)
                                                                                 : (ip != g_ptune.end() ? ip->second : 0))
                               : 0;
}

// ran: the timing launched the fused pass (the caller then initialises the
// field again).  Needs the state initialised (no load case frozen), so that
// every workgroup does its whole work.
int Solver::tune_plane(const LaunchArgs &a, hipStream_t s, bool &ran) {
    ran = false;
    pvar = 0;
    if (!ops->inv_fwd_alt[0]) return RVE_OK;
    if (path_flags & (PF_PLANE_DEFAULT | PF_PLANE_ALT)) {
        pvar = (path_flags & PF_PLANE_ALT) ? 1 : 0;
        return RVE_OK;
    }
    const TuneKey key{current_arch(), ops->precision, ops->n};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_ptune.find(key);
        if (it != g_ptune.end()) {
            pvar = it->second;
            return RVE_OK;
        }
    }
    bool alt = false;
    ran = true;
    const int rc = time_two(
        s, [&] { ops->inv_fwd(a, s, -1); }, [&] { ops->inv_fwd_alt[0](a, s, -1); }, alt);
    if (rc != RVE_OK) return rc;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    pvar = g_ptune.emplace(key, alt ? 1 : 0).first->second;
    return RVE_OK;
}

extern "C" size_t rve_tune_export(char *buf, size_t cap) {
    std::string text;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (int kind = 0; kind < 2; ++kind)
            for (const auto &kv : kind ? g_ptune : g_ztune) {
                char line[160];
                std::snprintf(line, sizeof line, "%s %d %d %s %d\n", std::get<0>(kv.first).c_str(),
                              std::get<1>(kv.first), std::get<2>(kv.first), kind ? "plane" : "ztile", kv.second);
                text += line;
            }
    }
    if (buf && cap > 0) {
        const size_t m = std::min(cap - 1, text.size());
        std::memcpy(buf, text.data(), m);
        buf[m] = '\0';
    }
    return text.size() + 1;
}

extern "C" rve_status rve_tune_import(const char *text) {
    clear_error();
    if (!text) {
        set_error("rve_tune_import: text is null");
        return RVE_ERR_ARG;
    }
    std::vector<std::pair<TuneKey, int>> add[2];  // ztile, plane
    const char *p = text;
    int lineno = 0;
    while (*p) {
        const char *e = std::strchr(p, '\n');
        std::string line(p, e ? (size_t)(e - p) : std::strlen(p));
        p = e ? e + 1 : p + line.size();
        ++lineno;
        if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
        char arch[64], kind[16];
        int prec = -1, n = 0, choice = -1, used = 0;
        if (std::sscanf(line.c_str(), "%63s %d %d %15s %d %n", arch, &prec, &n, kind, &choice, &used) != 5 ||
            line.find_first_not_of(" \t\r", used) != std::string::npos ||
            (std::strcmp(kind, "ztile") != 0 && std::strcmp(kind, "plane") != 0) || (prec != 0 && prec != 1) ||
            n <= 0 || (choice != 0 && choice != 1)) {
            set_error("rve_tune_import: line %d is not \"<arch> <precision 0|1> <n> <ztile|plane> <0|1>\"",
                      lineno);
            return RVE_ERR_ARG;
        }
        add[std::strcmp(kind, "plane") == 0].push_back({TuneKey{arch, prec, n}, choice});
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto &kv : add[0]) g_ztune[kv.first] = kv.second;
    for (const auto &kv : add[1]) g_ptune[kv.first] = kv.second;
    return RVE_OK;
}

int Solver::begin(const uint8_t *d_phase, const double k[3], double tol, const SolverOpts &o, hipStream_t s) {
    fill_params(*(DevParams *)h_pinned, k, tol, ops->n, o);
    return start(d_phase, o, s);
}

int Solver::begin_elastic(const uint8_t *d_phase, const double moduli[6], double tol, const SolverOpts &o,
                          hipStream_t s) {
    fill_params_el(*(DevParams *)h_pinned, moduli, tol, ops->n, o);
    return start(d_phase, o, s);
}

// Upload the parameters (already in the pinned block), initialise the field
// and the state, and enqueue the first forward pass.
int Solver::start(const uint8_t *d_phase, const SolverOpts &o, hipStream_t s) {
    d_phase_last = d_phase;
    path_flags = o.path_flags;
    use_graphs = !(o.path_flags & PF_NO_GRAPHS);
    graph_counted = false;
    int rc = ensure_twiddles(s);
    if (rc != RVE_OK) return rc;
    DevParams *hp = (DevParams *)h_pinned;
    LaunchArgs a = args(d_phase);
    HIP_CHECK(hipMemcpyAsync((void *)a.prm, hp, sizeof(DevParams), hipMemcpyHostToDevice, s));
    const size_t M = (size_t)ops->n * ops->n * ops->n;
    ops->init(a, M, s);
    HIP_CHECK(hipGetLastError());
    // the split planes' fused pass always takes the parity-layout z pass,
    // whose tile width is fixed: nothing to tune there
    const bool par_z = ops->zgreen_par && ops->inv_fwd && !o.eq_check && !(o.path_flags & PF_NO_FUSED);
    zvar = 0;
    if (!par_z) {
        rc = tune_zpass(a, s);
        if (rc != RVE_OK) return rc;
    }
    // the fused pass's thread count (whole planes; the timing overwrites the
    // field, initialised again here)
    pvar = 0;
    if (!o.eq_check && !(o.path_flags & PF_NO_FUSED)) {
        bool ran = false;
        rc = tune_plane(a, s, ran);
        if (rc != RVE_OK) return rc;
        if (ran) {
            ops->init(a, M, s);
            HIP_CHECK(hipGetLastError());
        }
    }
    if (o.dev_init_ops) {
        // continuation: each solved load case starts from its field in another
        // workspace (FP32 -> working precision)
        for (int lc = 0; lc < 3; ++lc) {
            if (!((o.lc_mask >> lc) & 1) || !o.dev_init[lc]) continue;
            const size_t off = (size_t)3 * lc * M;
            o.dev_init_ops->to_f64((double *)((char *)a.e + off * ops->real_bytes),
                                   (const char *)o.dev_init[lc] + off * o.dev_init_ops->real_bytes, 3 * M, s);
            HIP_CHECK(hipGetLastError());
        }
    }
    if (o.init_field) {
        // stage the FP64 field through the spectrum buffer region if it fits,
        // else through a temporary device buffer
        double *tmp = nullptr;
        HIP_CHECK(hipMalloc(&tmp, (size_t)ops->nc * ops->nc * M * sizeof(double)));
        HIP_CHECK(hipMemcpyAsync(tmp, o.init_field, (size_t)ops->nc * ops->nc * M * sizeof(double), hipMemcpyHostToDevice, s));
        ops->from_f64(a.e, tmp, (size_t)ops->nc * ops->nc * M, s);
        HIP_CHECK(hipGetLastError());
        HIP_CHECK(hipStreamSynchronize(s));
        HIP_CHECK(hipFree(tmp));
    }
    issued = 0;
    inflight.clear();
    finished = false;
    slot = 0;
    launches.clear();
    eq_check = o.eq_check != 0;
    scheme = o.scheme;
    al = o.scheme == 2 || o.scheme == 4;
    dual = o.scheme == 3;
    if (al && !o.dev_init_ops) {
        // the augmented-Lagrangian state: tau^0 = (k - k0) e^0 in the field buffer
        // (a continuation's fields hold tau already)
        ops->to_tau(a, M, s);
        HIP_CHECK(hipGetLastError());
    }
    fused = ops->inv_fwd != nullptr && !eq_check && !(o.path_flags & PF_NO_FUSED);
    merge = ops->nc == 3 && !eq_check && !(o.path_flags & PF_NO_MERGE);
    // a single load case: the iteration kernels run that load case's grid only
    lc_sel = -1;
    if (!eq_check && (o.lc_mask == 1 || o.lc_mask == 2 || o.lc_mask == 4)) lc_sel = o.lc_mask == 1 ? 0 : (o.lc_mask == 2 ? 1 : 2);
    if (fused) {
        // the first forward pass; every later one is fused into the inverse pass
        (ops->fwd_par ? ops->fwd_par : ops->fwd)(a, s, lc_sel);
        HIP_CHECK(hipGetLastError());
    }
    return RVE_OK;
}

// One iteration: the three passes, the reduction and (two-stage stop only)
// the equilibrium check.  Every kernel exits at once for frozen load cases.
// Kernels whose bit is set in mask are bracketed by the next two events of ev.
// red_in_z: the z pass also reduces the previous iteration's partials;
// defer_red: this iteration's reduction is left to the next z pass.
int Solver::launch_iteration(const LaunchArgs &a, hipStream_t s, int mask, hipEvent_t *ev, bool red_in_z,
                             bool defer_red) {
    int used = 0;
    // "external" records become event-record nodes when captured into a graph
    // (a plain record under capture is only an ordering marker, with no time)
    for (int kk = 0; kk < 4; ++kk) {
        if (fused && kk == 0) continue;  // the forward pass is inside the inverse one
        if (defer_red && kk == 3) continue;
        const bool timed = (mask >> kk) & 1;
        if (timed) HIP_CHECK(hipEventRecordWithFlags(ev[used], s, hipEventRecordExternal));
        switch (kk) {
        case 0: ops->fwd(a, s, lc_sel); break;
        case 1:
            (fused && ops->zgreen_par ? ops->zgreen_par : zvar ? ops->zgreen_alt : ops->zgreen)(
                a, s, red_in_z ? ops->nper : 0, lc_sel);
            break;
        case 2: inv_launcher(ops, fused, al, dual, pvar)(a, s, lc_sel); break;
        default: ops->reduce(a, ops->nper, s); break;
        }
        if (timed) {
            HIP_CHECK(hipEventRecordWithFlags(ev[used + 1], s, hipEventRecordExternal));
            used += 2;
        }
    }
    if (eq_check) {
        ops->fwd_phi(a, s);
        ops->zeq(a, s);
        launch_eq_reduce(a, ops->eq_tiles, 0, s);
    }
    return RVE_OK;
}

static int popcount4(int m) { return (m & 1) + ((m >> 1) & 1) + ((m >> 2) & 1) + ((m >> 3) & 1); }

// count consecutive iterations; with merging, every reduction but the last
// one of the batch runs inside the following z pass (the last stays a kernel
// of its own, so the batch ends with the convergence flags up to date).
// Not when the reduction itself is timed.
int Solver::launch_batch(const LaunchArgs &a, hipStream_t s, int count, int mask, hipEvent_t *ev) {
    const bool m = merge && !(mask & 8);
    const int per = 2 * popcount4(mask);
    for (int i = 0; i < count; ++i) {
        int rc = launch_iteration(a, s, mask, ev ? ev + i * per : nullptr, m && i > 0, m && i + 1 < count);
        if (rc != RVE_OK) return rc;
    }
    return RVE_OK;
}

// kernels actually launched per iteration (the forward pass is fused away)
static int live_mask(int mask, bool fused) { return fused ? (mask & ~1) : mask; }

// Capture kChunk iterations into a graph on the solver's own stream.
GraphKey Solver::graph_key(const uint8_t *d_phase) const {
    GraphKey k;
    k.ops = ops;
    k.ws = ws;
    k.ph = d_phase;
    k.eq = eq_check;
    k.fused = fused;
    k.merge = merge;
    k.al = al;
    k.dual = dual;
    k.lc = lc_sel;
    k.zvar = zvar;
    k.pvar = pvar;
    return k;
}

int Solver::ensure_graph(const uint8_t *d_phase) {
    const GraphKey key = graph_key(d_phase);
    if (gcur && gcur->key == key) {
        if (!graph_counted) graphs->hits++;
        graph_counted = true;
        return RVE_OK;
    }
    if (gcur) gcur->refs--;
    gcur = graphs->find(key);
    if (!graph_counted) (gcur ? graphs->hits : graphs->misses)++;
    graph_counted = true;
    if (!gcur) {
        LaunchArgs a = args(d_phase);
        hipGraph_t g = nullptr;
        HIP_CHECK(hipStreamBeginCapture(own_stream, hipStreamCaptureModeThreadLocal));
        (void)launch_batch(a, own_stream, kChunk, 0, nullptr);
        hipError_t cap = hipStreamEndCapture(own_stream, &g);
        if (cap != hipSuccess) {
            set_error("graph capture failed: %s", hipGetErrorString(cap));
            return RVE_ERR_DEVICE;
        }
        hipGraphExec_t x = nullptr;
        hipError_t inst = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (inst != hipSuccess) {
            set_error("graph instantiation failed: %s", hipGetErrorString(inst));
            return RVE_ERR_DEVICE;
        }
        gcur = graphs->put(key, x);
    }
    gcur->refs++;
    return RVE_OK;
}

// Timed graphs: one per poll slot, with that slot's events recorded around
// the masked kernels of every iteration (event records are graph nodes).
int Solver::ensure_timed_graphs(const uint8_t *d_phase, int mask) {
    int rc = ensure_graph(d_phase);
    if (rc != RVE_OK) return rc;
    if (tgexec[0] && tg_mask == mask && tg_key == gcur->key) return RVE_OK;
    for (auto &g : tgexec) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
    LaunchArgs a = args(d_phase);
    const int per = 2 * popcount4(mask);
    for (int sl = 0; sl < kPollSlots; ++sl) {
        hipGraph_t g = nullptr;
        HIP_CHECK(hipStreamBeginCapture(own_stream, hipStreamCaptureModeThreadLocal));
        (void)launch_batch(a, own_stream, kChunk, mask, slots[sl].ev.data());
        hipError_t cap = hipStreamEndCapture(own_stream, &g);
        if (cap != hipSuccess) {
            set_error("graph capture failed: %s", hipGetErrorString(cap));
            return RVE_ERR_DEVICE;
        }
        hipError_t inst = hipGraphInstantiate(&tgexec[sl], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (inst != hipSuccess) {
            tgexec[sl] = nullptr;
            set_error("graph instantiation failed: %s", hipGetErrorString(inst));
            return RVE_ERR_DEVICE;
        }
    }
    tg_mask = mask;
    tg_key = gcur->key;
    return RVE_OK;
}

// Enqueue up to `count` iterations (never beyond max_iter) and a poll point.
// Full chunks replay a captured graph (the timed variant of the poll slot when
// timing); partial chunks launch kernel by kernel.
int Solver::enqueue(const uint8_t *d_phase, int count, int max_iter, int timing, hipStream_t s) {
    LaunchArgs a = args(d_phase);
    SlotInfo &si = slots[slot];
    si.first_iter = issued;
    // sampled timing (bit 16): events only in the batches of poll slot 0
    si.mask = ((timing & 16) && slot != 0) ? 0 : live_mask(timing & 15, fused);
    if (use_graphs && count == kChunk && issued + kChunk <= max_iter) {
        int rc = si.mask ? ensure_timed_graphs(d_phase, si.mask) : ensure_graph(d_phase);
        if (rc != RVE_OK) return rc;
        HIP_CHECK(hipGraphLaunch(si.mask ? tgexec[slot] : gcur->exec, s));
        issued += kChunk;
        si.count = kChunk;
    } else {
        si.count = count < max_iter - issued ? count : max_iter - issued;
        if (si.count < 0) si.count = 0;
        int rc = launch_batch(a, s, si.count, si.mask, si.ev.data());
        if (rc != RVE_OK) return rc;
        issued += si.count;
    }
    HIP_CHECK(hipGetLastError());
    int *flags = (int *)((char *)h_pinned + kFlagsOffset);
    HIP_CHECK(hipMemcpyAsync(&flags[slot], &a.st->all_done, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipEventRecord(poll_ev[slot], s));
    inflight.push_back(slot);
    slot = (slot + 1) % kPollSlots;
    return RVE_OK;
}

// After the poll point of slot sl has completed: keep its kernel times.
int Solver::read_slot_times(int sl) {
    SlotInfo &si = slots[sl];
    if (!si.mask) return RVE_OK;
    const int per = 2 * popcount4(si.mask);
    for (int i = 0; i < si.count; ++i) {
        int used = 0;
        for (int kk = 0; kk < 4; ++kk) {
            if (!((si.mask >> kk) & 1)) continue;
            float ms = 0.f;
            HIP_CHECK(hipEventElapsedTime(&ms, si.ev[i * per + used], si.ev[i * per + used + 1]));
            launches.push_back({kk, si.first_iter + i, ms});
            used += 2;
        }
    }
    si.mask = 0;
    return RVE_OK;
}

// Non-blocking (wait = false) or blocking check of the oldest poll point.
// Returns 1 when the solve has finished, 0 otherwise, < 0 on error.
int Solver::poll(bool wait, int max_iter) {
    if (finished) return 1;
    if (inflight.empty()) return (issued >= max_iter) ? 1 : 0;
    const int sl = inflight.front();
    if (wait) {
        HIP_CHECK(hipEventSynchronize(poll_ev[sl]));
    } else {
        hipError_t q = hipEventQuery(poll_ev[sl]);
        if (q == hipErrorNotReady) return 0;
        if (q != hipSuccess) {
            set_error("hipEventQuery failed: %s", hipGetErrorString(q));
            return RVE_ERR_DEVICE;
        }
    }
    inflight.pop_front();
    if (int rc = read_slot_times(sl); rc != RVE_OK) return rc;
    const int *flags = (const int *)((const char *)h_pinned + kFlagsOffset);
    if (flags[sl]) finished = true;
    if (issued >= max_iter && inflight.empty()) finished = true;
    return finished ? 1 : 0;
}

// Copy results back after the stream has drained.
int Solver::collect(const SolverOpts &o, hipStream_t s, rve_result *out, double *hist, int hist_cap,
                    rve_kernel_times *kt, rve_elastic_result *eout) {
    LaunchArgs a = args(d_phase_last);
    const int nlc = ops->nc;
    if (ops->fwd_phi && scheme < 3) {
        // equilibrium error of the final field (step 1 quantity, reported at exit)
        launch_eq_request(a, s);
        ops->fwd_phi(a, s);
        ops->zeq(a, s);
        launch_eq_reduce(a, ops->eq_tiles, 1, s);
        HIP_CHECK(hipGetLastError());
    }
    DevState *hs = (DevState *)((char *)h_pinned + sizeof(DevParams));
    HIP_CHECK(hipMemcpyAsync(hs, a.st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    const size_t M = (size_t)ops->n * ops->n * ops->n;
    double *tmp = nullptr;
    if (o.out_field) {
        HIP_CHECK(hipMalloc(&tmp, (size_t)ops->nc * ops->nc * M * sizeof(double)));
        ops->to_f64(tmp, a.e, (size_t)ops->nc * ops->nc * M, s);
        HIP_CHECK(hipGetLastError());
        HIP_CHECK(hipMemcpyAsync(o.out_field, tmp, (size_t)ops->nc * ops->nc * M * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    HIP_CHECK(hipStreamSynchronize(s));
    if (tmp) HIP_CHECK(hipFree(tmp));
    if (out && nlc == 3) {
        for (int i = 0; i < 9; ++i) out->K[i] = hs->K[i];
        for (int j = 0; j < 3; ++j) {
            out->iters[j] = hs->iters[j];
            out->status[j] = hs->status[j];
            out->final_residual[j] = hs->res[j];
            out->eps_eq[j] = hs->eps_eq[j];
        }
    }
    if (eout && nlc == 6) {
        for (int i = 0; i < 36; ++i) eout->C_basis[i] = hs->K[i];
        for (int j = 0; j < 6; ++j) {
            eout->iters[j] = hs->iters[j];
            eout->status[j] = hs->status[j];
            eout->final_residual[j] = hs->res[j];
        }
    }
    if (hist && hist_cap > 0) {
        const int cap = std::min(hist_cap, kHistCap);
        for (int j = 0; j < nlc; ++j) {
            const int cnt = std::min(cap, hs->iters[j]);
            if (cnt > 0)
                HIP_CHECK(hipMemcpy(hist + (size_t)j * hist_cap, a.hist + (size_t)j * kHistCap,
                                    cnt * sizeof(double), hipMemcpyDeviceToHost));
        }
    }
    if (kt) {
        static const char *names[4] = {"fwd_plane", "zgreen", "inv_plane", "reduce"};
        std::memset(kt, 0, sizeof(*kt));
        for (int q = 0; q < 4; ++q) kt->name[q] = names[q];
        if (fused) kt->name[2] = "inv_fwd_plane";
        int maxit = 0;
        for (int j = 0; j < nlc; ++j) maxit = std::max(maxit, hs->iters[j]);
        while (!inflight.empty()) {  // stream drained: remaining slots are complete
            if (int rc = read_slot_times(inflight.front()); rc != RVE_OK) return rc;
            inflight.pop_front();
        }
        for (size_t i = 0; i < launches.size(); ++i) {
            const int kk = launches[i].kernel, it = launches[i].iter;
            if (it >= maxit) continue;  // launches after convergence exit at once
            const float ms = launches[i].ms;
            int active = 0;
            for (int j = 0; j < nlc; ++j) active += (hs->iters[j] > it) ? 1 : 0;
            kt->total_ms[kk] += ms;
            kt->launches[kk] += 1;
            const double b = (kk == 2 && fused) ? ops->bytes_fused : (kk < 3 ? ops->bytes[kk] : 0.0);
            kt->total_bytes[kk] += b * active / (double)nlc + ((kk == 0 || kk == 2) ? ops->phase_bytes : 0.0);
        }
    }
    return RVE_OK;
}

// The worst of count per-load-case statuses (those selected by mask): an
// error first, then NONFINITE, STALLED, NOT_CONVERGED, OK.
static rve_status worst_of(const int *status, int count, int mask) {
    int worst = RVE_OK;
    auto rank = [](int s) { return s < 0 ? 100 - s : s == RVE_STALLED ? 3 : s == RVE_NOT_CONVERGED ? 2 : 0; };
    for (int j = 0; j < count; ++j)
        if ((mask >> j) & 1)
            if (rank(status[j]) > rank(worst)) worst = status[j];
    return (rve_status)worst;
}

rve_status worst_status(const rve_result &r, int lc_mask) { return worst_of(r.status, 3, lc_mask); }

// Makes a handle's device current for a scope and restores the caller's
// device on every exit path.
struct DeviceScope {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceScope(int dev) {
        int cur = 0;
        err = hipGetDevice(&cur);
        if (err == hipSuccess && cur != dev) {
            err = hipSetDevice(dev);
            if (err == hipSuccess) prev = cur;
        }
    }
    ~DeviceScope() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// The three load cases of a solve are independent (Algorithm of Sec. 3 per
// E = e_j).  Where the iteration kernels can be restricted to one load case
// (whole or split planes), a full solve runs as three single-load-case solves,
// each with its own workspace, stream and iteration graph: their kernels
// overlap on the device (one's memory-bound phases beside another's compute
// and launch ramps).  The arithmetic per load case is unchanged, so the
// results equal those of the single-stream solve.
static int run_solver(Solver &sv, const uint8_t *d_phase, const SolverOpts &o, hipStream_t s);

static bool use_chains(const SolverOps *ops, const SolverOpts &o) {
    if (o.path_flags & PF_NO_CHAINS) return false;
    return ops->split > 0 && o.lc_mask == 7 && !o.eq_check && !o.init_field && !o.out_field && !o.workspace;
}

// FP32 floor -> FP64 continuation (fp32_refine).  Load cases that the FP32
// solve stopped as STALLED (the rounding floor of the FP32 transforms above
// tol, or no new residual minimum) restart in FP64 from their FP32 fields
// (src[lc]: base of the 9-channel FP32 field holding load case lc) with the
// same scheme and tol, and iterate steps 2-7 until eps_comp < tol.  Their K
// column, status, residual and eps_eq become the FP64 ones; iterations and
// residual history continue the FP32 ones.
int refine_mask(const rve_result &res, const SolverOpts &o) {
    if (o.precision != 0 || o.fp32_refine < 0) return 0;
    int mask = 0;
    for (int lc = 0; lc < 3; ++lc)
        if (((o.lc_mask >> lc) & 1) && res.status[lc] == RVE_STALLED) mask |= 1 << lc;
    return mask;
}

SolverOpts refine_opts(const SolverOpts &o, const rve_result &res, int mask, const void *const src[3],
                       const SolverOps *ops32) {
    int maxit32 = 0;
    for (int lc = 0; lc < 3; ++lc)
        if ((mask >> lc) & 1) maxit32 = std::max(maxit32, res.iters[lc]);
    SolverOpts o64 = o;
    o64.precision = 1;
    o64.lc_mask = mask;
    o64.stall_window = 0;
    o64.max_iter = std::max(1, o.max_iter - maxit32);
    o64.timing = 0;
    o64.init_field = nullptr;
    o64.out_field = nullptr;
    o64.workspace = nullptr;
    o64.workspace_bytes = 0;
    o64.path_flags = o.path_flags & ~(PF_ZTILE_DEFAULT | PF_ZTILE_ALT | PF_PLANE_DEFAULT | PF_PLANE_ALT);
    for (int lc = 0; lc < 3; ++lc) o64.dev_init[lc] = src[lc];
    o64.dev_init_ops = ops32;
    return o64;
}

void refine_merge(rve_result &res, const rve_result &r64, int mask, double *hist, int hist_cap, const double *h64) {
    res.solve_ms += r64.solve_ms;
    for (int lc = 0; lc < 3; ++lc) {
        if (!((mask >> lc) & 1)) continue;
        for (int i = 0; i < 3; ++i) res.K[3 * i + lc] = r64.K[3 * i + lc];
        const int it32 = res.iters[lc];
        for (int i = 0; i < r64.iters[lc] && hist && h64; ++i)
            if (it32 + i < hist_cap) hist[(size_t)lc * hist_cap + it32 + i] = h64[(size_t)lc * hist_cap + i];
        res.iters[lc] = it32 + r64.iters[lc];
        res.refine_iters[lc] = r64.iters[lc];
        res.status[lc] = r64.status[lc];
        res.final_residual[lc] = r64.final_residual[lc];
        res.eps_eq[lc] = r64.eps_eq[lc];
    }
}

rve_status refine_fp64(rve_s *r, const SolverOps *ops32, const double k[3], double tol, const SolverOpts &o,
                       rve_result &res, double *hist, int hist_cap, const void *const src[3], hipStream_t s) {
    const int mask = refine_mask(res, o);
    if (!mask) return RVE_OK;
    const SolverOps *ops64 = lookup_ops(1, r->n);
    if (!ops64) return RVE_OK;  // no FP64 build of this grid: the load cases stay STALLED
    Solver &sv = r->sol[1];
    int rc = sv.prepare(ops64, nullptr, 0);
    if (rc != RVE_OK) return (rve_status)rc;
    SolverOpts o64 = refine_opts(o, res, mask, src, ops32);
    rc = sv.begin(r->d_phase, k, tol, o64, s);
    if (rc != RVE_OK) return (rve_status)rc;
    rc = run_solver(sv, r->d_phase, o64, s);
    if (rc != RVE_OK) return (rve_status)rc;
    rve_result r64{};
    std::vector<double> h64(hist && hist_cap > 0 ? (size_t)3 * hist_cap : 0);
    const size_t M = (size_t)r->n * r->n * r->n;
    std::vector<double> f64(o.out_field ? 9 * M : 0);
    o64.out_field = o.out_field ? f64.data() : nullptr;
    rc = sv.collect(o64, s, &r64, h64.empty() ? nullptr : h64.data(), hist_cap, nullptr);
    if (rc != RVE_OK) return (rve_status)rc;
    float ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&ms, sv.run_ev[0], sv.run_ev[1]));
    r64.solve_ms = ms;
    refine_merge(res, r64, mask, hist, hist_cap, h64.empty() ? nullptr : h64.data());
    if (o.out_field)
        for (int lc = 0; lc < 3; ++lc)
            if ((mask >> lc) & 1)
                std::memcpy(o.out_field + 3 * lc * M, f64.data() + 3 * lc * M, 3 * M * sizeof(double));
    return RVE_OK;
}

struct ChainItem {
    Solver *sv;
    const uint8_t *d_phase;
    hipStream_t stream;
    int max_iter;
    int lc;
    SolverOpts opts;
    int timing;
};

static rve_status solve_chains(rve_s *r, const SolverOps *ops, const double k[3], double tol, const SolverOpts &o,
                               rve_result *out, double *hist, int hist_cap) {
    Solver &c0 = r->chain[o.precision][0];
    for (int lc = 0; lc < 3; ++lc) {
        int rc = r->chain[o.precision][lc].prepare(ops, nullptr, 0);
        if (rc != RVE_OK) return (rve_status)rc;
    }
    hipStream_t s = o.stream ? o.stream : c0.own_stream;
    HIP_CHECK(hipEventRecord(c0.run_ev[0], s));
    std::vector<ChainItem> act;
    for (int lc = 0; lc < 3; ++lc) {
        Solver &cs = r->chain[o.precision][lc];
        SolverOpts co = o;
        co.lc_mask = 1 << lc;
        co.stream = nullptr;
        if (cs.own_stream != s) HIP_CHECK(hipStreamWaitEvent(cs.own_stream, c0.run_ev[0], 0));
        int rc = cs.begin(r->d_phase, k, tol, co, cs.own_stream);
        if (rc != RVE_OK) return (rve_status)rc;
        act.push_back({&cs, r->d_phase, cs.own_stream, o.max_iter, lc, co, o.timing});
    }
    rve_result res{};
    rve_kernel_times kt_sum{};
    std::vector<double> hrow(hist && hist_cap > 0 ? (size_t)3 * hist_cap : 0);
    int rc = drive(act, [&](ChainItem &a) {
        rve_result rl{};
        rve_kernel_times kt{};
        int c = a.sv->collect(a.opts, a.stream, &rl, hrow.empty() ? nullptr : hrow.data(), hist_cap,
                              o.timing ? &kt : nullptr);
        if (c != RVE_OK) return c;
        const int j = a.lc;
        for (int i = 0; i < 3; ++i) res.K[3 * i + j] = rl.K[3 * i + j];  // column j = load case e_j
        res.iters[j] = rl.iters[j];
        res.status[j] = rl.status[j];
        res.final_residual[j] = rl.final_residual[j];
        res.eps_eq[j] = rl.eps_eq[j];
        if (!hrow.empty())
            std::memcpy(hist + (size_t)j * hist_cap, hrow.data() + (size_t)j * hist_cap, hist_cap * sizeof(double));
        if (o.timing) {
            for (int q = 0; q < 4; ++q) {
                kt_sum.name[q] = kt.name[q];
                kt_sum.total_ms[q] += kt.total_ms[q];
                kt_sum.launches[q] += kt.launches[q];
                kt_sum.total_bytes[q] += kt.total_bytes[q];
            }
        }
        return (int)RVE_OK;
    });
    if (rc != RVE_OK) return (rve_status)rc;
    // join: the caller's stream continues after every load case's work
    for (int lc = 0; lc < 3; ++lc) {
        Solver &cs = r->chain[o.precision][lc];
        if (cs.own_stream == s) continue;
        HIP_CHECK(hipEventRecord(cs.run_ev[1], cs.own_stream));
        HIP_CHECK(hipStreamWaitEvent(s, cs.run_ev[1], 0));
    }
    HIP_CHECK(hipEventRecord(c0.run_ev[1], s));
    HIP_CHECK(hipEventSynchronize(c0.run_ev[1]));
    float ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&ms, c0.run_ev[0], c0.run_ev[1]));
    res.solve_ms = ms;
    if (o.timing) r->times = kt_sum;
    const void *src[3];
    for (int lc = 0; lc < 3; ++lc) {
        const Solver &cs = r->chain[o.precision][lc];
        src[lc] = (const char *)cs.ws + cs.layout.e;
    }
    rc = refine_fp64(r, ops, k, tol, o, res, hist, hist_cap, src, s);
    if (rc != RVE_OK) return (rve_status)rc;
    if (out) *out = res;
    return worst_status(res, o.lc_mask);
}

// The scheme option against the other options.
int check_scheme(const SolverOpts &o, const SolverOps *ops) {
    (void)ops;
    if (o.scheme < 0 || o.scheme > 4) {
        set_error("scheme must be 0 (accelerated), 1 (basic), 2 (augmented Lagrangian), 3 (dual) or "
                  "4 (polarization)");
        return RVE_ERR_ARG;
    }
    if (o.scheme >= 2 && o.eq_check) {
        set_error("the augmented-Lagrangian, dual and polarization schemes have no equilibrium check");
        return RVE_ERR_ARG;
    }
    if (o.scheme == 3 && o.init_field) {
        set_error("the dual scheme starts from the constant flux k0 E (no start field)");
        return RVE_ERR_ARG;
    }
    if (o.scheme == 4 && !(o.alpha > 0.0 && o.alpha <= 2.0)) {
        set_error("the polarization scheme's relaxation alpha must lie in (0, 2] (got %g)", o.alpha);
        return RVE_ERR_ARG;
    }
    return RVE_OK;
}

// Iterate a begun solver to completion on stream s, bracketed by its run
// events.  Poll points every kChunk iterations, at most kLookahead chunks
// ahead of the host; launches after convergence exit at once on the device
// flags.
static int run_solver(Solver &sv, const uint8_t *d_phase, const SolverOpts &o, hipStream_t s) {
    HIP_CHECK(hipEventRecord(sv.run_ev[0], s));
    while (true) {
        if (sv.issued < o.max_iter) {
            int rc = sv.enqueue(d_phase, kChunk, o.max_iter, o.timing, s);
            if (rc != RVE_OK) return rc;
        }
        const bool must_wait = (int)sv.inflight.size() >= kLookahead || sv.issued >= o.max_iter;
        if (must_wait) {
            int rc = sv.poll(true, o.max_iter);
            if (rc < 0) return rc;
            if (rc == 1) break;
        }
    }
    HIP_CHECK(hipEventRecord(sv.run_ev[1], s));
    return RVE_OK;
}

// The elastic case on one RVE: the six load cases E = B_j in one solver.
static const double kBasis[6][3][3] = {
    {{0.57735026918962576451, 0, 0}, {0, 0.57735026918962576451, 0}, {0, 0, 0.57735026918962576451}},
    {{0.70710678118654752440, 0, 0}, {0, -0.70710678118654752440, 0}, {0, 0, 0}},
    {{0.40824829046386301637, 0, 0}, {0, 0.40824829046386301637, 0}, {0, 0, -0.81649658092772603273}},
    {{0, 0, 0}, {0, 0, 0.70710678118654752440}, {0, 0.70710678118654752440, 0}},
    {{0, 0, 0.70710678118654752440}, {0, 0, 0}, {0.70710678118654752440, 0, 0}},
    {{0, 0.70710678118654752440, 0}, {0.70710678118654752440, 0, 0}, {0, 0, 0}},
};

// C_hom in the basis (C_basis[6 k + l] = B_k : C : B_l) to the Voigt matrix
// C[6 I + J] = C_ijkl with I = (ij), J = (kl) over 11, 22, 33, 23, 13, 12.
static void basis_to_voigt(const double *Cb, double *Cv) {
    static const int vi[6] = {0, 1, 2, 1, 0, 0}, vj[6] = {0, 1, 2, 2, 2, 1};
    for (int I = 0; I < 6; ++I)
        for (int J = 0; J < 6; ++J) {
            double acc = 0.0;
            for (int k = 0; k < 6; ++k)
                for (int l = 0; l < 6; ++l)
                    acc += Cb[6 * k + l] * kBasis[k][vi[I]][vj[I]] * kBasis[l][vi[J]][vj[J]];
            Cv[6 * I + J] = acc;
        }
}

static rve_status solve_elastic(rve_s *r, const double moduli[6], double tol, const SolverOpts &o,
                                rve_elastic_result *out, double *hist, int hist_cap) {
    const SolverOps *ops = lookup_ops_el(o.precision, r->n);
    if (!ops) {
        set_error("grid size %d is not built for the elastic case in precision %d", r->n, o.precision);
        return RVE_ERR_ARG;
    }
    DeviceScope dev(r->device);
    HIP_CHECK(dev.err);
    Solver &sv = r->el[o.precision];
    int rc = sv.prepare(ops, nullptr, 0);
    if (rc != RVE_OK) return (rve_status)rc;
    hipStream_t s = o.stream ? o.stream : sv.own_stream;
    rc = sv.begin_elastic(r->d_phase, moduli, tol, o, s);
    if (rc != RVE_OK) return (rve_status)rc;
    rc = run_solver(sv, r->d_phase, o, s);
    if (rc != RVE_OK) return (rve_status)rc;
    rve_elastic_result res{};
    rc = sv.collect(o, s, nullptr, hist, hist_cap, nullptr, &res);
    if (rc != RVE_OK) return (rve_status)rc;
    float ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&ms, sv.run_ev[0], sv.run_ev[1]));
    res.solve_ms = ms;
    basis_to_voigt(res.C_basis, res.C);
    *out = res;
    return worst_of(res.status, 6, 63);
}

// One RVE, start to finish, on stream s.
rve_status solve_one(rve_s *r, const double k[3], double tol, const SolverOpts &o, rve_result *out,
                     double *hist, int hist_cap) {
    const SolverOps *ops = lookup_ops(o.precision, r->n);
    if (!ops) {
        set_error("grid size %d is not built for precision %d", r->n, o.precision);
        return RVE_ERR_ARG;
    }
    if (check_scheme(o, ops) != RVE_OK) return RVE_ERR_ARG;
    DeviceScope dev(r->device);
    HIP_CHECK(dev.err);
    if (use_chains(ops, o)) return solve_chains(r, ops, k, tol, o, out, hist, hist_cap);
    Solver &sv = r->sol[o.precision];
    int rc = sv.prepare(ops, o.workspace, o.workspace_bytes);
    if (rc != RVE_OK) return (rve_status)rc;
    hipStream_t s = o.stream ? o.stream : sv.own_stream;
    rc = sv.begin(r->d_phase, k, tol, o, s);
    if (rc != RVE_OK) return (rve_status)rc;
    rc = run_solver(sv, r->d_phase, o, s);
    if (rc != RVE_OK) return (rve_status)rc;
    rve_result res{};
    rc = sv.collect(o, s, &res, hist, hist_cap, o.timing ? &r->times : nullptr);
    if (rc != RVE_OK) return (rve_status)rc;
    float ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&ms, sv.run_ev[0], sv.run_ev[1]));
    res.solve_ms = ms;
    if (o.precision == 0 && o.fp32_refine >= 0) {
        // FP64 continuation of load cases stopped by the FP32 floor (with a
        // caller workspace the FP64 one is still the handle's own)
        const void *src[3];
        for (int lc = 0; lc < 3; ++lc) src[lc] = (const char *)sv.ws + sv.layout.e;
        rc = refine_fp64(r, ops, k, tol, o, res, hist, hist_cap, src, s);
        if (rc != RVE_OK) return (rve_status)rc;
    }
    if (out) *out = res;
    return worst_status(res, o.lc_mask);
}

}  // namespace rvehom

extern "C" rve_status homogenize(rve_t r, const double k_phases[3], double tol, const rve_opts *opts,
                                 rve_result *out, double *residual_history, int hist_cap) {
    clear_error();
    if (!r || !out) {
        set_error("homogenize: null rve or result pointer");
        return RVE_ERR_ARG;
    }
    int rc = validate_k(k_phases, tol);
    if (rc != RVE_OK) return (rve_status)rc;
    if (opts && (opts->precision != 0 && opts->precision != 1)) {
        set_error("precision must be 0 (FP32) or 1 (FP64)");
        return RVE_ERR_ARG;
    }
    if (hist_cap < 0 || (hist_cap > 0 && !residual_history)) {
        set_error("residual_history is NULL but hist_cap > 0");
        return RVE_ERR_ARG;
    }
    SolverOpts o = resolve_opts(opts);
    if (o.timing) std::memset(&r->times, 0, sizeof(r->times));
    return solve_one(r, k_phases, tol, o, out, residual_history, hist_cap);
}

extern "C" rve_status homogenize_elastic(rve_t r, const double moduli[6], double tol, const rve_opts *opts,
                                         rve_elastic_result *out, double *residual_history, int hist_cap) {
    clear_error();
    if (!r || !out || !moduli) {
        set_error("homogenize_elastic: null rve, moduli or result pointer");
        return RVE_ERR_ARG;
    }
    for (int q = 0; q < 6; ++q)
        if (!(moduli[q] > 0.0) || !std::isfinite(moduli[q])) {
            set_error("moduli must be finite and > 0 (entry %d = %g)", q, moduli[q]);
            return RVE_ERR_ARG;
        }
    if (!(tol >= 0.0) || !std::isfinite(tol)) {
        set_error("tol must be finite and >= 0 (got %g)", tol);
        return RVE_ERR_ARG;
    }
    if (opts && (opts->precision != 0 && opts->precision != 1)) {
        set_error("precision must be 0 (FP32) or 1 (FP64)");
        return RVE_ERR_ARG;
    }
    if (opts && (opts->equilibrium_check || opts->scheme != 0 || opts->workspace ||
                 ((opts->lc_mask & 63) != 0 && (opts->lc_mask & 63) != 63))) {
        set_error("homogenize_elastic: equilibrium_check, scheme, workspace and a partial lc_mask are not supported");
        return RVE_ERR_ARG;
    }
    if (hist_cap < 0 || (hist_cap > 0 && !residual_history)) {
        set_error("residual_history is NULL but hist_cap > 0");
        return RVE_ERR_ARG;
    }
    SolverOpts o = resolve_opts(opts);
    o.lc_mask = 63;
    o.timing = 0;
    return solve_elastic(r, moduli, tol, o, out, residual_history, hist_cap);
}

extern "C" rve_status rve_supported_n_elastic(int precision, int *out, int cap, int *count) {
    clear_error();
    if ((precision != 0 && precision != 1) || !count || (cap > 0 && !out) || cap < 0) {
        set_error("rve_supported_n_elastic: bad arguments");
        return RVE_ERR_ARG;
    }
    const int *list = nullptr;
    const int k = supported_sizes_el(precision, &list);
    for (int i = 0; i < k && i < cap; ++i) out[i] = list[i];
    *count = k;
    return RVE_OK;
}

extern "C" rve_status rve_get_kernel_times(rve_t r, rve_kernel_times *out) {
    clear_error();
    if (!r || !out) {
        set_error("rve_get_kernel_times: null pointer");
        return RVE_ERR_ARG;
    }
    *out = r->times;
    return RVE_OK;
}

// Several RVEs at once: one stream per RVE, chunks enqueued round-robin so the
// device works on all of them together; each finishes on its own flags.
extern "C" rve_status homogenize_batch(int count, const rve_t *rves, const double *k_phases, const double *tol,
                                       const rve_opts *opts, rve_result *out) {
    clear_error();
    if (count < 0 || (count > 0 && (!rves || !k_phases || !tol || !out))) {
        set_error("homogenize_batch: bad arguments");
        return RVE_ERR_ARG;
    }
    if (opts && (opts->init_field || opts->out_field || opts->workspace || opts->stream)) {
        set_error("homogenize_batch: init_field, out_field, workspace and stream must be NULL");
        return RVE_ERR_ARG;
    }
    SolverOpts o = resolve_opts(opts);
    o.timing = 0;
    for (int i = 0; i < count; ++i) {
        if (!rves[i]) {
            set_error("homogenize_batch: rve %d is NULL", i);
            return RVE_ERR_ARG;
        }
        int rc = validate_k(k_phases + 3 * i, tol[i]);
        if (rc != RVE_OK) return (rve_status)rc;
        if (!lookup_ops(o.precision, rves[i]->n)) {
            set_error("grid size %d is not built for precision %d", rves[i]->n, o.precision);
            return RVE_ERR_ARG;
        }
        if (check_scheme(o, lookup_ops(o.precision, rves[i]->n)) != RVE_OK) return RVE_ERR_ARG;
        for (int j = 0; j < i; ++j)
            if (rves[j] == rves[i]) {
                set_error("homogenize_batch: rve %d appears twice", i);
                return RVE_ERR_ARG;
            }
    }
    return batch_solve(count, rves, k_phases, tol, o, out);
}
