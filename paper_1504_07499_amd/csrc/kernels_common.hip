// kernels_common.hip -- precision-independent kernels (the FP64 convergence
// reductions) and the lists of grid sizes compiled into the library.
#include <hip/hip_runtime.h>

#include "reduce_block.hpp"
#include "solver_ops.hpp"
#include "solver_state.hpp"

namespace rvehom {

// Standalone form of the reduction (one workgroup of 256 threads).
__global__ __launch_bounds__(256) void k_reduce(const double *__restrict__ part, int nper,
                                                const DevParams *__restrict__ prm,
                                                DevState *__restrict__ st, double *__restrict__ hist) {
    reduce_block(part, nper, prm, st, hist, threadIdx.x);
}

// Equilibrium error of the load cases marked eq_pending: fixed-order sum of
// the k_zeq partials, eps_eq = sqrt(num) / sqrt(den).  During the solve
// (final = 0, two-stage stop of step 1) a load case finishes when
// eps_eq < tol; at the end of a solve (final = 1) the value is only stored.
__global__ __launch_bounds__(256) void k_eq_reduce(const double *__restrict__ peq, int per_lc, int final,
                                                   const DevParams *__restrict__ prm,
                                                   DevState *__restrict__ st) {
    __shared__ double red[2 * 4];
    __shared__ double tot[3][2];
    const int tid = threadIdx.x;
    for (int lc = 0; lc < 3; ++lc) {
        double v[2] = {0.0, 0.0};
        if (st->eq_pending[lc])
            for (int b = tid; b < per_lc; b += 256) {
                v[0] += peq[((size_t)lc * per_lc + b) * 2];
                v[1] += peq[((size_t)lc * per_lc + b) * 2 + 1];
            }
#pragma unroll
        for (int q = 0; q < 2; ++q)
            for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_down(v[q], o, 64);
        const int lane = tid & 63, wv = tid >> 6;
        if (lane == 0) {
            red[2 * wv] = v[0];
            red[2 * wv + 1] = v[1];
        }
        __syncthreads();
        if (tid == 0)
            for (int q = 0; q < 2; ++q) tot[lc][q] = red[q] + red[2 + q] + red[4 + q] + red[6 + q];
        __syncthreads();
    }
    if (tid != 0) return;
    int all = 1;
    for (int lc = 0; lc < 3; ++lc) {
        if (st->eq_pending[lc]) {
            const double eq = sqrt(tot[lc][0]) / sqrt(tot[lc][1]);
            st->eps_eq[lc] = eq;
            st->eq_pending[lc] = 0;
            if (!final && eq < prm->tol) {
                // converged in the iteration just reduced (iter already advanced)
                st->done[lc] = 1;
                st->status[lc] = ST_OK;
                st->iters[lc] = st->iter;
            }
        }
        all &= st->done[lc];
    }
    st->all_done = all;
}

// Mark every solved load case for a final equilibrium-error evaluation.
__global__ void k_eq_request(const DevParams *__restrict__ prm, DevState *__restrict__ st) {
    if (threadIdx.x == 0)
        for (int lc = 0; lc < 3; ++lc) st->eq_pending[lc] = (prm->lc_mask >> lc) & 1;
}

void launch_eq_reduce(const LaunchArgs &a, int per_lc, int final, hipStream_t s) {
    hipLaunchKernelGGL(k_eq_reduce, dim3(1), dim3(256), 0, s, a.peq, per_lc, final, a.prm, a.st);
}

void launch_eq_request(const LaunchArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_eq_request, dim3(1), dim3(64), 0, s, a.prm, a.st);
}

void launch_reduce(const LaunchArgs &a, int nper, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, a.part, nper, a.prm, a.st, a.hist);
}

// The elastic case's reduction (one workgroup of 576 threads).
__global__ __launch_bounds__(576) void k_reduce_el(const double *part, int nper, const DevParams *prm, DevState *st,
                                                  double *hist) {
    reduce_block_el(part, nper, prm, st, hist, threadIdx.x);
}

static const int kSizesF32[] = {8, 12, 16, 24, 32, 36, 48, 64, 72, 96, 128, 144, 192, 256, 288, 384, 512};
static const int kSizesF64[] = {8, 12, 16, 24, 32, 36, 48, 64, 72, 96, 128, 144, 192, 256, 288, 384, 512};

static const int kSizesElF32[] = {8, 12, 16, 24, 32, 48, 64, 96, 128, 256, 512};
static const int kSizesElF64[] = {8, 12, 16, 24, 32, 48, 64, 96, 128, 256, 512};

int supported_sizes_el(int precision, const int **list) {
    if (precision == 0) {
        *list = kSizesElF32;
        return (int)(sizeof(kSizesElF32) / sizeof(int));
    }
    *list = kSizesElF64;
    return (int)(sizeof(kSizesElF64) / sizeof(int));
}

int supported_sizes(int precision, const int **list) {
    if (precision == 0) {
        *list = kSizesF32;
        return (int)(sizeof(kSizesF32) / sizeof(int));
    }
    *list = kSizesF64;
    return (int)(sizeof(kSizesF64) / sizeof(int));
}

}  // namespace rvehom
