// rvehom_noalloc.hip -- homogenize_no_alloc of include/rvehom.h: the solve of
// homogenize (same kernels, same launch order, same results) with every
// device buffer it needs beyond the caller's RVE in one fixed array of
// device memory that is part of the library image, for callers that cannot
// allocate.
//
// The array `scratch` below is a device symbol: in host code its name is a
// host-side stand-in, not a device address.  The device address is taken
// once per device with hipGetSymbolAddress (each GPU holds its own copy) and
// only that address is ever passed to kernels or copies.
//
// Nothing here calls hipMalloc, hipFree, hipHostMalloc, creates a stream,
// event or graph, or allocates on the host heap: parameters, twiddles and
// state pass through stack buffers with a synchronisation of the caller's
// stream after each upload, and the iteration chunks are launched kernel by
// kernel.  Calls on one device are serialised by a host mutex; the scratch
// array keeps the last call's contents, and everything a solve reads is
// (re)initialised by that solve.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>

#include "rvehom.h"
#include "rvehom_internal.hpp"
#include "solver_ops.hpp"
#include "solver_state.hpp"

namespace rvehom {

// 64 MiB: the FP32 workspace of a 64^3 grid with the FP64 workspace of its
// continuation (57.9 MB), or the FP64 workspace alone (38.6 MB).
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu[kMaxDevices];
static std::mutex g_addr_mu;
static void *g_scratch_addr[kMaxDevices];

// The device address of this device's scratch array (looked up on the
// device's first call, with that device current).
static int scratch_address(int dev, void **out) {
    std::lock_guard<std::mutex> lk(g_addr_mu);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("hipGetSymbolAddress of the scratch array failed: %s", hipGetErrorString(e));
            return RVE_ERR_DEVICE;
        }
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return RVE_OK;
}

static size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

#define NA_CHECK(call)                                                                    \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess) {                                                           \
            set_error("%s failed: %s", #call, hipGetErrorString(e_));                     \
            return RVE_ERR_DEVICE;                                                        \
        }                                                                                 \
    } while (0)

// One solve (all load cases of o.lc_mask) in the workspace at ws, kernel by
// kernel on stream s, as Solver does it: the first forward pass, then per
// iteration the z pass (with the previous iteration's reduction merged),
// the fused inverse + forward pass (or the separate passes), and at the end
// of each chunk of kChunk iterations a reduction of its own and a poll of
// the device flags.
struct NaSolve {
    const SolverOps *ops;
    char *ws;
    WsLayout L;
    LaunchArgs a;

    void bind(const SolverOps *o, char *base, const uint8_t *d_phase) {
        ops = o;
        ws = base;
        L = ws_layout(o);
        a.e = ws + L.e;
        a.ph = d_phase;
        a.spec = ws + L.spec;
        a.nyq = ws + L.nyq;
        a.tw = ws + L.tw;
        a.prm = (const DevParams *)(ws + L.prm);
        a.st = (DevState *)(ws + L.st);
        a.part = (double *)(ws + L.part);
        a.hist = (double *)(ws + L.hist);
        a.peq = (double *)(ws + L.peq);
        a.spec2 = L.spec2 ? ws + L.spec2 : nullptr;
        a.nyq2 = L.nyq2 ? ws + L.nyq2 : nullptr;
    }

    int run(const double k[3], double tol, const SolverOpts &o, hipStream_t s, int zvar, int pvar, DevState &hs) {
        const int n = ops->n;
        const size_t M = (size_t)n * n * n;
        // twiddles exp(-2 pi i m / n) in FP64, rounded once, via the stack
        constexpr int kMaxN = 512;  // the largest grid size built
        double tw64[2 * kMaxN];
        float tw32[2 * kMaxN];
        if (n > kMaxN) {
            set_error("grid size %d above %d", n, kMaxN);
            return RVE_ERR_ARG;
        }
        for (int m = 0; m < n; ++m) {
            const double ang = 2.0 * M_PI * (double)m / (double)n;
            tw64[2 * m] = std::cos(ang);
            tw64[2 * m + 1] = -std::sin(ang);
            tw32[2 * m] = (float)tw64[2 * m];
            tw32[2 * m + 1] = (float)tw64[2 * m + 1];
        }
        const bool f32 = ops->real_bytes == sizeof(float);
        NA_CHECK(hipMemcpyAsync((void *)a.tw, f32 ? (const void *)tw32 : (const void *)tw64,
                                (size_t)n * 2 * ops->real_bytes, hipMemcpyHostToDevice, s));
        DevParams prm;
        fill_params(prm, k, tol, n, o);
        NA_CHECK(hipMemcpyAsync((void *)a.prm, &prm, sizeof(prm), hipMemcpyHostToDevice, s));
        NA_CHECK(hipStreamSynchronize(s));  // the stack buffers may go
        ops->init(a, M, s);
        if (o.dev_init_ops)
            for (int lc = 0; lc < 3; ++lc) {
                if (!((o.lc_mask >> lc) & 1) || !o.dev_init[lc]) continue;
                const size_t off = (size_t)3 * lc * M;
                o.dev_init_ops->to_f64((double *)((char *)a.e + off * ops->real_bytes),
                                       (const char *)o.dev_init[lc] + off * o.dev_init_ops->real_bytes, 3 * M, s);
            }
        const bool al = o.scheme == 2 || o.scheme == 4, dual = o.scheme == 3;
        if (al && !o.dev_init_ops) ops->to_tau(a, M, s);
        NA_CHECK(hipGetLastError());
        const bool fused = ops->inv_fwd != nullptr && !(o.path_flags & PF_NO_FUSED);
        const bool merge = ops->nc == 3 && !(o.path_flags & PF_NO_MERGE);
        auto zg = fused && ops->zgreen_par ? ops->zgreen_par : zvar ? ops->zgreen_alt : ops->zgreen;
        if (fused) (ops->fwd_par ? ops->fwd_par : ops->fwd)(a, s, -1);
        int issued = 0, flag = 0;
        while (issued < o.max_iter) {
            const int count = std::min(kChunk, o.max_iter - issued);
            for (int i = 0; i < count; ++i) {
                const bool red_in_z = merge && i > 0, defer = merge && i + 1 < count;
                if (!fused) ops->fwd(a, s, -1);
                zg(a, s, red_in_z ? ops->nper : 0, -1);
                inv_launcher(ops, fused, al, dual, pvar)(a, s, -1);
                if (!defer) ops->reduce(a, ops->nper, s);
            }
            issued += count;
            NA_CHECK(hipGetLastError());
            NA_CHECK(hipMemcpyAsync(&flag, &a.st->all_done, sizeof(int), hipMemcpyDeviceToHost, s));
            NA_CHECK(hipStreamSynchronize(s));
            if (flag) break;
        }
        // equilibrium error of the final field, reported at exit (not for
        // the dual and polarization schemes, whose buffer holds no gradient)
        if (o.scheme < 3) {
            launch_eq_request(a, s);
            ops->fwd_phi(a, s);
            ops->zeq(a, s);
            launch_eq_reduce(a, ops->eq_tiles, 1, s);
        }
        NA_CHECK(hipGetLastError());
        NA_CHECK(hipMemcpyAsync(&hs, a.st, sizeof(DevState), hipMemcpyDeviceToHost, s));
        NA_CHECK(hipStreamSynchronize(s));
        return RVE_OK;
    }

    int history(double *hist, int hist_cap, int first, const DevState &hs, int mask, hipStream_t s) {
        if (!hist || hist_cap <= 0) return RVE_OK;
        for (int lc = 0; lc < 3; ++lc) {
            if (!((mask >> lc) & 1)) continue;
            const int cnt = std::min(std::min(hs.iters[lc], kHistCap), hist_cap - first);
            if (cnt <= 0) continue;
            NA_CHECK(hipMemcpyAsync(hist + (size_t)lc * hist_cap + first, a.hist + (size_t)lc * kHistCap,
                                    cnt * sizeof(double), hipMemcpyDeviceToHost, s));
        }
        NA_CHECK(hipStreamSynchronize(s));
        return RVE_OK;
    }
};

static void to_result(const DevState &hs, int mask, rve_result &r) {
    for (int lc = 0; lc < 3; ++lc) {
        if (!((mask >> lc) & 1)) continue;
        for (int i = 0; i < 3; ++i) r.K[3 * i + lc] = hs.K[3 * i + lc];
        r.iters[lc] = hs.iters[lc];
        r.status[lc] = hs.status[lc];
        r.final_residual[lc] = hs.res[lc];
        r.eps_eq[lc] = hs.eps_eq[lc];
    }
}

}  // namespace rvehom

using namespace rvehom;

extern "C" rve_status homogenize_no_alloc(rve_t r, const double k_phases[3], double tol, const rve_opts *opts,
                                          rve_result *out, double *residual_history, int hist_cap) {
    clear_error();
    if (!r || !out) {
        set_error("homogenize_no_alloc: null rve or result pointer");
        return RVE_ERR_ARG;
    }
    int rc = validate_k(k_phases, tol);
    if (rc != RVE_OK) return (rve_status)rc;
    if (opts && (opts->precision != 0 && opts->precision != 1)) {
        set_error("precision must be 0 (FP32) or 1 (FP64)");
        return RVE_ERR_ARG;
    }
    if (opts && (opts->init_field || opts->out_field || opts->workspace || opts->timing || opts->equilibrium_check)) {
        set_error("homogenize_no_alloc: init_field, out_field, workspace, timing and equilibrium_check "
                  "are not supported");
        return RVE_ERR_ARG;
    }
    if (hist_cap < 0 || (hist_cap > 0 && !residual_history)) {
        set_error("residual_history is NULL but hist_cap > 0");
        return RVE_ERR_ARG;
    }
    SolverOpts o = resolve_opts(opts);
    const SolverOps *ops = lookup_ops(o.precision, r->n);
    if (!ops) {
        set_error("grid size %d is not built for precision %d", r->n, o.precision);
        return RVE_ERR_ARG;
    }
    if (check_scheme(o, ops) != RVE_OK) return RVE_ERR_ARG;
    const SolverOps *ops64 = (o.precision == 0 && o.fp32_refine >= 0) ? lookup_ops(1, r->n) : nullptr;
    const size_t ws0 = up256(ws_layout(ops).total);
    const size_t need = ws0 + (ops64 ? up256(ws_layout(ops64).total) : 0);
    if (need > kScratchBytes) {
        set_error("homogenize_no_alloc: N = %d needs %zu bytes of scratch (%s), above the %zu-byte maximum", r->n,
                  need, ops64 ? "FP32 workspace and its FP64 continuation" : "one workspace", kScratchBytes);
        return RVE_ERR_ARG;
    }
    if (r->device < 0 || r->device >= kMaxDevices) {
        set_error("device %d beyond the scratch table", r->device);
        return RVE_ERR_DEVICE;
    }
    int prev = 0;
    NA_CHECK(hipGetDevice(&prev));
    if (prev != r->device) NA_CHECK(hipSetDevice(r->device));
    struct Restore {
        int dev, prev;
        ~Restore() {
            if (dev != prev) (void)hipSetDevice(prev);
        }
    } restore{r->device, prev};
    void *base = nullptr;
    rc = scratch_address(r->device, &base);
    if (rc != RVE_OK) return (rve_status)rc;
    std::lock_guard<std::mutex> lk(g_scratch_mu[r->device]);
    hipStream_t s = o.stream;
    int zvar = 0, pvar = 0;
    tuned_choices(ops, o.path_flags, zvar, pvar);
    const auto t0 = std::chrono::steady_clock::now();

    NaSolve a;
    a.bind(ops, (char *)base, r->d_phase);
    DevState hs;
    rc = a.run(k_phases, tol, o, s, zvar, pvar, hs);
    if (rc != RVE_OK) return (rve_status)rc;
    rve_result res{};
    to_result(hs, 7, res);
    rc = a.history(residual_history, hist_cap, 0, hs, o.lc_mask, s);
    if (rc != RVE_OK) return (rve_status)rc;

    const int mask = ops64 ? refine_mask(res, o) : 0;
    if (mask) {
        // FP64 continuation of the load cases stopped by the FP32 floor, in the
        // second part of the scratch array
        const void *src[3];
        for (int lc = 0; lc < 3; ++lc) src[lc] = (const char *)a.a.e;
        SolverOpts o64 = refine_opts(o, res, mask, src, ops);
        NaSolve b;
        b.bind(ops64, (char *)base + ws0, r->d_phase);
        DevState h64;
        int z64 = 0, p64 = 0;
        tuned_choices(ops64, o64.path_flags, z64, p64);
        rc = b.run(k_phases, tol, o64, s, z64, p64, h64);
        if (rc != RVE_OK) return (rve_status)rc;
        rve_result r64{};
        to_result(h64, mask, r64);
        for (int lc = 0; lc < 3; ++lc) {
            if (!((mask >> lc) & 1) || !residual_history || hist_cap <= 0) continue;
            const int first = res.iters[lc], cnt = std::min(std::min(h64.iters[lc], kHistCap), hist_cap - first);
            if (cnt > 0)
                NA_CHECK(hipMemcpyAsync(residual_history + (size_t)lc * hist_cap + first,
                                        b.a.hist + (size_t)lc * kHistCap, cnt * sizeof(double),
                                        hipMemcpyDeviceToHost, s));
        }
        NA_CHECK(hipStreamSynchronize(s));
        refine_merge(res, r64, mask, nullptr, 0, nullptr);
    }
    res.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = res;
    return worst_status(res, o.lc_mask);
}
