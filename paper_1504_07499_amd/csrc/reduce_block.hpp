// reduce_block.hpp -- the fixed-order FP64 reduction of the per-block partials
// and the convergence decisions (steps 1 and 6 of the Algorithm of Sec. 3).
#pragma once

#include <hip/hip_runtime.h>

#include "solver_state.hpp"

namespace rvehom {

// Convergence decision of one load case at iteration it with residual eps:
// history, NaN, tolerance (or the equilibrium stage), stall rules, iteration
// cap; freezes the load case when it finishes.  Returns 1 when it is done.
__device__ __forceinline__ int decide_load_case(const DevParams *__restrict__ prm, DevState *__restrict__ st,
                                                double *__restrict__ hist, int lc, int it, double eps) {
    st->res[lc] = eps;
    if (it < prm->hist_cap) hist[lc * prm->hist_cap + it] = eps;
    int fin = 0, status = ST_NOT_CONVERGED;
    if (!(eps == eps) || eps > 1e300) {
        fin = 1;
        status = ST_NONFINITE;
    } else if (eps < prm->tol) {
        if (prm->eq_check) {
            // step 1, second stage: the equilibrium error decides (k_eq_reduce)
            st->eq_pending[lc] = 1;
            if (it + 1 >= prm->max_iter) fin = 1;
        } else {
            fin = 1;
            status = ST_OK;
        }
    } else {
        if (eps < st->best[lc]) {
            st->best[lc] = eps;
            st->best_it[lc] = it;
        } else if (prm->stall_window > 0 && it - st->best_it[lc] >= prm->stall_window) {
            fin = 1;
            status = ST_STALLED;
        }
        // FP32 rounding floor: within 100 tol, the last 10 iterations
        // gained less than a quarter of the least progress the scheme's
        // contraction bound allows (1 - rho^10)
        if (!fin && prm->stall_window > 0 && it >= 10 && it - 10 < prm->hist_cap && eps < 100.0 * prm->tol &&
            eps > (1.0 - 0.25 * prm->prog10) * hist[lc * prm->hist_cap + it - 10]) {
            fin = 1;
            status = ST_STALLED;
        }
        if (!fin && it + 1 >= prm->max_iter) fin = 1;
    }
    if (fin) {
        st->done[lc] = 1;
        st->status[lc] = status;
        st->iters[lc] = it + 1;
    }
    return fin;
}

// ---------------------------------------------------------------------------
// Fixed-order FP64 reduction of the partials, steps 6 / 1 convergence test,
// <phi> of the updated field (L_hom column), per-load-case freeze.
// Run by one workgroup of 256 threads (tid = its thread index): as a kernel of
// its own, or as the first workgroup of the next z pass.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void reduce_block(const double *__restrict__ part, int nper,
                                             const DevParams *__restrict__ prm, DevState *__restrict__ st,
                                             double *__restrict__ hist, int tid) {
    // per load case {sum |e - c|^2, flux x, flux y, flux z}, and per channel
    // sum e+.  Every thread adds its strided share of all nine channels
    // (loads issued together), then a fixed-order wave and block reduction.
    __shared__ double red[4][21];
    __shared__ double tot[21];
    double v[21];
#pragma unroll
    for (int q = 0; q < 21; ++q) v[q] = 0.0;
    for (int b = tid; b < nper; b += 256) {
        double r[9], f[9], m[9];
#pragma unroll
        for (int ch = 0; ch < 9; ++ch) {
            const double *pc = part + ((size_t)ch * nper + b) * 3;
            r[ch] = pc[0];
            f[ch] = pc[1];
            m[ch] = pc[2];
        }
#pragma unroll
        for (int ch = 0; ch < 9; ++ch) {
            v[4 * (ch / 3)] += r[ch];
            v[4 * (ch / 3) + 1 + ch % 3] += f[ch];
            v[12 + ch] += m[ch];
        }
    }
#pragma unroll
    for (int q = 0; q < 21; ++q)
        for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_down(v[q], o, 64);
    const int lane = tid & 63, wv = tid >> 6;
    if (lane == 0)
        for (int q = 0; q < 21; ++q) red[wv][q] = v[q];
    __syncthreads();
    if (tid < 21) tot[tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
    __syncthreads();
    if (tid != 0) return;
    const int it = st->iter;
    int all = 1;
    for (int lc = 0; lc < 3; ++lc) {
        if (st->done[lc]) continue;
        const double eps = sqrt(tot[4 * lc] * prm->invM);  // |E| = 1
        for (int c = 0; c < 3; ++c) {
            const double F = tot[4 * lc + 1 + c] * prm->invM;  // <k e+_c>
            st->K[3 * c + lc] = F;
            // mean of tau = (k - k0) e+ for the next forward pass
            st->tau_mean[3 * lc + c] = F - prm->k0 * tot[12 + 3 * lc + c] * prm->invM;
        }
        all &= decide_load_case(prm, st, hist, lc, it, eps);
    }
    st->iter = it + 1;
    st->all_done = all;
}

// The same for the elastic case (six load cases of six components): 16
// lanes per channel (576 threads) sum channel ch's partials in a fixed order
// (lane l takes blocks l, l + 16, ...; then a fixed tree over the 16 lanes),
// and thread 0 forms each load case's residual, mean stress and per-channel
// mean of tau and decides.
__device__ __forceinline__ void reduce_block_el(const double *__restrict__ part, int nper,
                                                const DevParams *__restrict__ prm, DevState *__restrict__ st,
                                                double *__restrict__ hist, int tid) {
    __shared__ double tot[36][3];
    const int ch = tid >> 4, l = tid & 15;
    double v[3] = {0.0, 0.0, 0.0};
    if (ch < 36) {
        const double *pc = part + (size_t)ch * nper * 3;
        for (int b = l; b < nper; b += 16) {
            v[0] += pc[3 * b];
            v[1] += pc[3 * b + 1];
            v[2] += pc[3 * b + 2];
        }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q)
        for (int o = 8; o > 0; o >>= 1) v[q] += __shfl_down(v[q], o, 16);
    if (ch < 36 && l == 0) {
        tot[ch][0] = v[0];
        tot[ch][1] = v[1];
        tot[ch][2] = v[2];
    }
    __syncthreads();
    if (tid != 0) return;
    const int it = st->iter;
    int all = 1;
    for (int lc = 0; lc < 6; ++lc) {
        if (st->done[lc]) continue;
        double r2 = 0.0;
        for (int c = 0; c < 6; ++c) r2 += tot[6 * lc + c][0];
        const double eps = sqrt(r2 * prm->invM);  // |E| = 1 (unit basis tensor)
        for (int c = 0; c < 6; ++c) {
            const double F = tot[6 * lc + c][1] * prm->invM;  // mean stress component c
            st->K[6 * c + lc] = F;
            const double k0c = c == 0 ? prm->k0 : prm->k0_dev;
            st->tau_mean[6 * lc + c] = F - k0c * tot[6 * lc + c][2] * prm->invM;
        }
        all &= decide_load_case(prm, st, hist, lc, it, eps);
    }
    st->iter = it + 1;
    st->all_done = all;
}

}  // namespace rvehom
