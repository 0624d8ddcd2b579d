// kernel_instances.hpp -- builds the SolverOps launcher table of one
// (T, N) from the kernel templates.  Included by the per-precision units.
#pragma once

#include "solver_kernels.hpp"
#include "solver_ops.hpp"

namespace rvehom {

constexpr size_t kLdsBytes = 160 * 1024;

// Row-parity split of the xy-plane so that N/S rows x (N/2 + 1) columns fit in LDS.
template <typename T, int N> constexpr int plane_split() {
    return ((size_t)N * (N / 2 + 1) * sizeof(Cx<T>) + 1024 <= kLdsBytes)           ? 1
           : ((size_t)(N / 2) * (N / 2 + 1) * sizeof(Cx<T>) + 1024 <= kLdsBytes) ? 2
                                                                                   : 0;
}

// z-tile width: largest W <= 16 dividing N/2 and N with 3 N W complex <= 64 KiB.
template <typename T, int N> constexpr int ztile() {
    for (int w = 16; w >= 1; --w)
        if ((N / 2) % w == 0 && N % w == 0 && (size_t)3 * N * w * sizeof(Cx<T>) <= 64 * 1024) return w;
    return 1;
}

// Threads for the plane kernels: 512 when a 256-thread block would need too
// many registers to hold one Stockham stage.
template <typename T, int N> constexpr int plane_threads() {
    constexpr int S = plane_split<T, N>();
    constexpr size_t elems = (size_t)(N / (S ? S : 1)) * (N / 2 + 1);
    return (elems * sizeof(Cx<T>) > 48 * 1024) ? 512 : 256;
}

template <typename T, int N> struct Instance {
    static constexpr int S = plane_split<T, N>();
    static constexpr int W = ztile<T, N>();
    static constexpr int NTP = plane_threads<T, N>();
    static constexpr int NTZ = 256;
    static_assert(S == 1 || S == 2, "plane does not fit in LDS");

    static void fwd(const LaunchArgs &a, hipStream_t s) {
        hipLaunchKernelGGL((k_fwd_plane<T, N, S, NTP>), dim3(9 * N * S), dim3(NTP), 0, s,
                           (const T *)a.e, a.ph, (Cx<T> *)a.spec, (Cx<T> *)a.nyq,
                           (const Cx<T> *)a.tw, a.prm, (const DevState *)a.st);
    }
    static void fwd_phi(const LaunchArgs &a, hipStream_t s) {
        hipLaunchKernelGGL((k_fwd_plane<T, N, S, NTP, true>), dim3(9 * N * S), dim3(NTP), 0, s,
                           (const T *)a.e, a.ph, (Cx<T> *)a.spec, (Cx<T> *)a.nyq,
                           (const Cx<T> *)a.tw, a.prm, (const DevState *)a.st);
    }
    static void zeq(const LaunchArgs &a, hipStream_t s) {
        hipLaunchKernelGGL((k_zeq<T, N, W, NTZ>), dim3(3 * ZTiles<N, W>::PER_LC), dim3(NTZ), 0, s,
                           (const Cx<T> *)a.spec, (const Cx<T> *)a.nyq, (const Cx<T> *)a.tw,
                           (const DevState *)a.st, a.peq);
    }
    static void zgreen(const LaunchArgs &a, hipStream_t s) {
        hipLaunchKernelGGL((k_zgreen<T, N, W, NTZ>), dim3(3 * ZTiles<N, W>::PER_LC), dim3(NTZ), 0, s,
                           (Cx<T> *)a.spec, (Cx<T> *)a.nyq, (const Cx<T> *)a.tw, a.prm,
                           (const DevState *)a.st);
    }
    static void inv(const LaunchArgs &a, hipStream_t s) {
        hipLaunchKernelGGL((k_inv_plane<T, N, S, NTP>), dim3(9 * N * S), dim3(NTP), 0, s, (T *)a.e,
                           a.ph, (const Cx<T> *)a.spec, (const Cx<T> *)a.nyq, (const Cx<T> *)a.tw,
                           a.prm, (const DevState *)a.st, a.part);
    }
    static void init(const LaunchArgs &a, size_t M, hipStream_t s) {
        hipLaunchKernelGGL((k_init<T>), dim3(1024), dim3(256), 0, s, (T *)a.e, M, a.prm, a.st);
    }
    static void from_f64(void *e, const double *src, size_t count, hipStream_t s) {
        hipLaunchKernelGGL((k_from_f64<T>), dim3(1024), dim3(256), 0, s, (T *)e, src, count);
    }
    static void to_f64(double *dst, const void *e, size_t count, hipStream_t s) {
        hipLaunchKernelGGL((k_to_f64<T>), dim3(1024), dim3(256), 0, s, dst, (const T *)e, count);
    }

    static const SolverOps *ops(int precision) {
        constexpr size_t M = (size_t)N * N * N;
        constexpr size_t H = N / 2;
        constexpr double cb = (double)sizeof(Cx<T>);
        constexpr double rb = (double)sizeof(T);
        constexpr double spec_b = 9.0 * N * N * (H + 1) * cb;  // spec + nyq
        static const SolverOps o = {
            N,
            precision,
            S,
            W,
            N * S,
            sizeof(T),
            (size_t)9 * N * N * H,
            (size_t)9 * N * N,
            {9 * N * S, 3 * ZTiles<N, W>::PER_LC, 9 * N * S},
            {NTP, NTZ, NTP},
            // P1: read e + phases once per channel, write spectrum.
            // P2: read + write spectrum.  P3: read spectrum, e, phases; write e.
            {9.0 * M * rb + 9.0 * M + spec_b, 2.0 * spec_b, spec_b + 2.0 * 9.0 * M * rb + 9.0 * M},
            ZTiles<N, W>::PER_LC,
            &fwd,
            &fwd_phi,
            &zeq,
            &zgreen,
            &inv,
            &init,
            &from_f64,
            &to_f64,
        };
        return &o;
    }
};

}  // namespace rvehom
