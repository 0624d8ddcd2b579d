// kernel_instances.hpp -- builds the SolverOps launcher table of one
// (T, N) from the kernel templates.  Included by the per-precision units.
#pragma once

#include "solver_kernels.hpp"
#include "solver_ops.hpp"

namespace rvehom {

constexpr size_t kLdsBytes = 160 * 1024;

// Row-parity split of the xy-plane so that its rows (pitch N/2 + 2 complex for
// a whole plane, N/2 + 1 for a half), the twiddle table (N complex) and the
// reduction scratch fit in LDS.
template <typename T, int N> constexpr int plane_split() {
    constexpr size_t extra = (size_t)N * sizeof(Cx<T>) + 1024;
    return ((size_t)N * (N / 2 + 2) * sizeof(Cx<T>) + extra <= kLdsBytes)           ? 1
           : ((size_t)(N / 2) * (N / 2 + 1) * sizeof(Cx<T>) + extra <= kLdsBytes) ? 2
                                                                                    : 0;
}

// z-tile width: largest even W <= 16 dividing N/2 and N with 3 N W complex in
// 64 KiB of LDS; if that leaves fewer than 8 columns (long pencils), up to
// 96 KiB is allowed so that global accesses keep >= 64-byte segments.
template <typename T, int N> constexpr int ztile_cap(size_t cap) {
    for (int w = 16; w >= 2; w -= 2)
        if ((N / 2) % w == 0 && N % w == 0 && (size_t)3 * N * w * sizeof(Cx<T>) <= cap) return w;
    return 2;
}
template <typename T, int N> constexpr int ztile() {
    // FP32 128^3: 8-column tiles (24 KiB, six workgroups per CU instead of
    // three; rows of 64 bytes, paired per XCD by ztile_of) -- measured faster
    if constexpr (sizeof(T) == 4 && N == 128) return 8;
    return ztile_cap<T, N>(64 * 1024) >= 8 ? ztile_cap<T, N>(64 * 1024) : ztile_cap<T, N>(96 * 1024);
}

// The other z-tile width the autotuner tries: half the default where that
// still divides N/2 (even, >= 2), else double it where that fits; the
// default itself if neither exists.  The z transform of a pencil does not
// depend on how many pencils a tile holds, so both give identical results.
template <typename T, int N> constexpr int ztile_alt() {
    constexpr int W = ztile<T, N>();
    if constexpr (W / 2 >= 2 && (W / 2) % 2 == 0 && (N / 2) % (W / 2) == 0) return W / 2;
    if constexpr (2 * W <= 16 && (N / 2) % (2 * W) == 0 && (size_t)3 * N * 2 * W * sizeof(Cx<T>) <= 96 * 1024)
        return 2 * W;
    return W;
}

// Five-pass form: rows per block of the x passes, columns per block of the y passes.
template <typename T, int N> constexpr int row_group() { return N >= 16 ? 16 : N; }
template <typename T, int N> constexpr int col_tile() {
    for (int w = 16; w >= 1; --w)
        if ((N / 2) % w == 0 && N % w == 0 && (size_t)N * w * sizeof(Cx<T>) <= 64 * 1024) return w;
    return 1;
}

// Threads for the plane kernels: 512 when a 256-thread block would need too
// many registers to hold one Stockham stage; 1024 for split planes (FP32
// 256^3), whose LDS leaves room for one workgroup per CU: four waves per
// SIMD instead of two, at <= 128 VGPRs without spills (measured 8 % faster
// per pass).  The whole FP64 128^3 plane, also one workgroup per CU, spills
// at 1024 threads and stays at 512 (measured 6 % slower otherwise).
template <typename T, int N> constexpr int plane_threads() {
    constexpr int S = plane_split<T, N>();
    constexpr size_t elems = (size_t)(N / (S ? S : 1)) * (N / 2 + (S == 1 ? 2 : 1));
    if constexpr (S == 2) return 1024;
    return (elems * sizeof(Cx<T>) > 48 * 1024) ? 512 : 256;
}

// The other thread count the autotuner tries for the fused pass of whole
// planes: 512 where the default is 256 (more threads per plane, for the
// small grids whose launches do not fill the GPU), 256 where it is 512 (more
// workgroups per CU where registers allow); split planes and the five-pass
// form have one shape.  Both run the same arithmetic per voxel (up to the
// compiler's instruction choice for each shape) and group the FP64 partial
// sums differently: results agree to rounding.
template <typename T, int N> constexpr int plane_threads_alt() {
    if constexpr (plane_split<T, N>() != 1) return plane_threads<T, N>();
    return plane_threads<T, N>() == 256 ? 512 : 256;
}

template <typename T, int N> struct Instance {
    static constexpr int S = plane_split<T, N>();
    static constexpr bool FIVE = (S == 0);  // plane does not fit in LDS
    static constexpr int SP = FIVE ? 1 : S;
    static constexpr int W = ztile<T, N>();
    static constexpr int W2 = ztile_alt<T, N>();
    static constexpr int NTP = plane_threads<T, N>();
    static constexpr int NTZ = 256;
    static constexpr int G = row_group<T, N>();
    static constexpr int WC = col_tile<T, N>();
    static constexpr int NTR = 256;
    static constexpr int NPER = FIVE ? N * (N / G) : N * S;

    // lc_sel < 0: all three load cases; else only load case lc_sel (plane and
    // z grids of that load case alone; the five-pass form launches all and
    // relies on the frozen-load-case early exit)
    static int pgrid(int lc_sel) { return (lc_sel < 0 ? 9 : 3) * N * SP; }
    static int ch0(int lc_sel) { return lc_sel < 0 ? 0 : 3 * lc_sel; }
    // split planes: the fused pass writes the parity layout (k_inv_plane with
    // S = 2), read back by the z pass
    static constexpr bool PARF = !FIVE && S == 2 && ztile_par_ok<N, ztile<T, N>()>();
    static constexpr int PC = par_chunk<T, ztile<T, N>()>();  // parity-layout chunk
    // FP64 256^3, whose half plane does not fit in LDS: the fused pass in
    // quarter planes (S = 4, 132 KiB, one workgroup per CU) with its own
    // first forward pass and the four-quarter z pass (tiles of one column x
    // four quarters, 48 KiB; parity chunks of one column); the other passes
    // keep the five-pass form.  The fused pass writes the five-pass form's
    // partial slots (N / G per plane).
    static constexpr bool QF = FIVE && sizeof(T) == 8 && N == 256;
    static constexpr int NTQ = 512, WQ = 4;
    static constexpr bool PARX = PARF || QF;  // a parity-layout fused path
    template <bool PHI, bool PAR = false> static void fwd_t(const LaunchArgs &a, hipStream_t s, int lc_sel) {
        if constexpr (PAR && QF) {
            hipLaunchKernelGGL((k_fwd_plane<T, N, 4, NTQ, false, 3, true, WQ / 4>), dim3((lc_sel < 0 ? 9 : 3) * N * 4),
                               dim3(NTQ), 0, s, (const T *)a.e, a.ph, (Cx<T> *)a.spec2, (Cx<T> *)a.nyq2,
                               (const Cx<T> *)a.tw, a.prm, (const DevState *)a.st, ch0(lc_sel));
        } else if constexpr (FIVE) {
            hipLaunchKernelGGL((k_fwd_rows<T, N, G, NTR, PHI>), dim3(9 * N * (N / G)), dim3(NTR), 0, s,
                               (const T *)a.e, a.ph, (Cx<T> *)a.spec, (Cx<T> *)a.nyq,
                               (const Cx<T> *)a.tw, a.prm, (const DevState *)a.st);
            hipLaunchKernelGGL((k_cols<T, N, WC, NTR, false, PHI>), dim3(ColTiles<N, WC>::ALL), dim3(NTR), 0,
                               s, (Cx<T> *)a.spec, (Cx<T> *)a.nyq, (const Cx<T> *)a.tw,
                               (const DevState *)a.st);
        } else if constexpr (PAR) {
            hipLaunchKernelGGL((k_fwd_plane<T, N, SP, NTP, false, 3, true, PC>), dim3(pgrid(lc_sel)), dim3(NTP), 0, s,
                               (const T *)a.e, a.ph, (Cx<T> *)a.spec2, (Cx<T> *)a.nyq2,
                               (const Cx<T> *)a.tw, a.prm, (const DevState *)a.st, ch0(lc_sel));
        } else {
            hipLaunchKernelGGL((k_fwd_plane<T, N, SP, NTP, PHI>), dim3(pgrid(lc_sel)), dim3(NTP), 0, s,
                               (const T *)a.e, a.ph, (Cx<T> *)a.spec, (Cx<T> *)a.nyq,
                               (const Cx<T> *)a.tw, a.prm, (const DevState *)a.st, ch0(lc_sel));
        }
    }
    static void fwd(const LaunchArgs &a, hipStream_t s, int lc_sel) { fwd_t<false>(a, s, lc_sel); }
    static void fwd_par(const LaunchArgs &a, hipStream_t s, int lc_sel) {
        if constexpr (PARX) fwd_t<false, true>(a, s, lc_sel);
    }
    static void fwd_phi(const LaunchArgs &a, hipStream_t s) { fwd_t<true>(a, s, -1); }
    static void zeq(const LaunchArgs &a, hipStream_t s) {
        hipLaunchKernelGGL((k_zeq<T, N, W, NTZ>), dim3(3 * ZTiles<N, W>::PER_LC), dim3(NTZ), 0, s,
                           (const Cx<T> *)a.spec, (const Cx<T> *)a.nyq, (const Cx<T> *)a.tw,
                           (const DevState *)a.st, a.peq);
    }
    // red_nper > 0: one extra workgroup reduces the previous inverse pass
    template <int WV, bool PAR = false>
    static void zgreen_w(const LaunchArgs &a, hipStream_t s, int red_nper, int lc_sel) {
        const int lcs = FIVE || lc_sel < 0 ? 3 : 1;
        hipLaunchKernelGGL((k_zgreen<T, N, WV, NTZ, PAR, (PAR && QF) ? 4 : 2>),
                           dim3(lcs * ZTiles<N, WV>::PER_LC + (red_nper > 0 ? 1 : 0)), dim3(NTZ), 0, s,
                           (Cx<T> *)a.spec, (Cx<T> *)a.nyq, (const Cx<T> *)a.tw, a.prm, a.st,
                           (const double *)a.part, red_nper, a.hist, lcs == 3 ? 0 : lc_sel,
                           (const Cx<T> *)a.spec2, (const Cx<T> *)a.nyq2);
    }
    static void zgreen(const LaunchArgs &a, hipStream_t s, int red_nper, int lc_sel) {
        zgreen_w<W>(a, s, red_nper, lc_sel);
    }
    static void zgreen_alt(const LaunchArgs &a, hipStream_t s, int red_nper, int lc_sel) {
        zgreen_w<W2>(a, s, red_nper, lc_sel);
    }
    // the parity layout's z pass (tiles of rows ky and ky + N/2 read the same
    // two parity rows)
    static void zgreen_par(const LaunchArgs &a, hipStream_t s, int red_nper, int lc_sel) {
        if constexpr (PARX) zgreen_w<QF ? WQ : W, true>(a, s, red_nper, lc_sel);
    }
    template <int AL> static void inv_t(const LaunchArgs &a, hipStream_t s, int lc_sel) {
        if constexpr (FIVE) {
            hipLaunchKernelGGL((k_cols<T, N, WC, NTR, true>), dim3(ColTiles<N, WC>::ALL), dim3(NTR), 0, s,
                               (Cx<T> *)a.spec, (Cx<T> *)a.nyq, (const Cx<T> *)a.tw, (const DevState *)a.st);
            hipLaunchKernelGGL((k_inv_rows<T, N, G, NTR, AL>), dim3(9 * N * (N / G)), dim3(NTR), 0, s, (T *)a.e,
                               a.ph, (const Cx<T> *)a.spec, (const Cx<T> *)a.nyq, (const Cx<T> *)a.tw,
                               a.prm, (const DevState *)a.st, a.part);
        } else {
            hipLaunchKernelGGL((k_inv_plane<T, N, SP, NTP, false, AL>), dim3(pgrid(lc_sel)), dim3(NTP), 0, s,
                               (T *)a.e, a.ph, (Cx<T> *)a.spec, (Cx<T> *)a.nyq, (const Cx<T> *)a.tw, a.prm,
                               (const DevState *)a.st, a.part, ch0(lc_sel), (Cx<T> *)nullptr, (Cx<T> *)nullptr);
        }
    }
    static void inv(const LaunchArgs &a, hipStream_t s, int lc_sel) { inv_t<0>(a, s, lc_sel); }
    static void inv_al(const LaunchArgs &a, hipStream_t s, int lc_sel) { inv_t<1>(a, s, lc_sel); }
    static void inv_dual(const LaunchArgs &a, hipStream_t s, int lc_sel) { inv_t<2>(a, s, lc_sel); }
    static void to_tau(const LaunchArgs &a, size_t M, hipStream_t s) {
        hipLaunchKernelGGL((k_to_tau<T>), dim3(1024), dim3(256), 0, s, (T *)a.e, a.ph, M, a.prm);
    }
    // fused inverse + next forward pass (whole planes in LDS); FP32 96^3
    // runs it at 512 threads per workgroup (at 256 it spills registers)
    static constexpr bool FUSED = !FIVE && S == 1;
    static constexpr int NTF = (sizeof(T) == 4 && N == 96) ? 512 : NTP;
    template <int AL> static void inv_fwd_t(const LaunchArgs &a, hipStream_t s, int lc_sel) {
        if constexpr (FUSED) {
            hipLaunchKernelGGL((k_inv_plane<T, N, 1, NTF, true, AL>), dim3(pgrid(lc_sel)), dim3(NTF), 0, s,
                               (T *)a.e, a.ph, (Cx<T> *)a.spec, (Cx<T> *)a.nyq, (const Cx<T> *)a.tw, a.prm,
                               (const DevState *)a.st, a.part, ch0(lc_sel), (Cx<T> *)nullptr, (Cx<T> *)nullptr);
        } else if constexpr (PARF) {
            hipLaunchKernelGGL((k_inv_plane<T, N, 2, NTP, true, AL, 3, PC>), dim3(pgrid(lc_sel)), dim3(NTP), 0, s,
                               (T *)a.e, a.ph, (Cx<T> *)a.spec, (Cx<T> *)a.nyq, (const Cx<T> *)a.tw, a.prm,
                               (const DevState *)a.st, a.part, ch0(lc_sel), (Cx<T> *)a.spec2, (Cx<T> *)a.nyq2);
        } else if constexpr (QF) {
            hipLaunchKernelGGL((k_inv_plane<T, N, 4, NTQ, true, AL, 3, WQ / 4, N / G>), dim3((lc_sel < 0 ? 9 : 3) * N * 4),
                               dim3(NTQ), 0, s, (T *)a.e, a.ph, (Cx<T> *)a.spec, (Cx<T> *)a.nyq,
                               (const Cx<T> *)a.tw, a.prm, (const DevState *)a.st, a.part, ch0(lc_sel),
                               (Cx<T> *)a.spec2, (Cx<T> *)a.nyq2);
        }
    }
    static constexpr int NTP2 = NTF != NTP ? NTF : plane_threads_alt<T, N>();
    static constexpr bool FUSED2 = FUSED && NTP2 != NTF;
    template <int AL> static void inv_fwd2_t(const LaunchArgs &a, hipStream_t s, int lc_sel) {
        if constexpr (FUSED2) {
            hipLaunchKernelGGL((k_inv_plane<T, N, 1, NTP2, true, AL>), dim3(pgrid(lc_sel)), dim3(NTP2), 0, s,
                               (T *)a.e, a.ph, (Cx<T> *)a.spec, (Cx<T> *)a.nyq, (const Cx<T> *)a.tw, a.prm,
                               (const DevState *)a.st, a.part, ch0(lc_sel), (Cx<T> *)nullptr, (Cx<T> *)nullptr);
        }
    }
    static void inv_fwd2(const LaunchArgs &a, hipStream_t s, int lc_sel) { inv_fwd2_t<0>(a, s, lc_sel); }
    static void inv_fwd2_al(const LaunchArgs &a, hipStream_t s, int lc_sel) { inv_fwd2_t<1>(a, s, lc_sel); }
    static void inv_fwd2_dual(const LaunchArgs &a, hipStream_t s, int lc_sel) { inv_fwd2_t<2>(a, s, lc_sel); }
    static void inv_fwd(const LaunchArgs &a, hipStream_t s, int lc_sel) { inv_fwd_t<0>(a, s, lc_sel); }
    static void inv_fwd_al(const LaunchArgs &a, hipStream_t s, int lc_sel) { inv_fwd_t<1>(a, s, lc_sel); }
    static void inv_fwd_dual(const LaunchArgs &a, hipStream_t s, int lc_sel) { inv_fwd_t<2>(a, s, lc_sel); }
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
        // Field bytes (all three load cases; the phase image, read by P1, P3
        // and the fused pass, is counted once per launch in phase_bytes):
        // P1: read e, write spectrum (five-pass: plus a read and write of the
        // spectrum for y).  P2: read + write spectrum.  P3: read spectrum and
        // e, write e (five-pass: plus y).
        constexpr double extra = FIVE ? 2.0 * spec_b : 0.0;
        static const SolverOps o = {
            N,
            precision,
            FIVE ? 0 : S,
            W,
            NPER,
            sizeof(T),
            (size_t)9 * N * N * H,
            (size_t)9 * N * N,
            {FIVE ? 9 * N * (N / G) : 9 * N * S, 3 * ZTiles<N, W>::PER_LC, FIVE ? 9 * N * (N / G) : 9 * N * S},
            {FIVE ? NTR : NTP, NTZ, FIVE ? NTR : NTP},
            {9.0 * M * rb + spec_b + extra, 2.0 * spec_b, spec_b + 2.0 * 9.0 * M * rb + extra},
            ZTiles<N, W>::PER_LC,
            (FUSED || PARX) ? 2.0 * spec_b + 2.0 * 9.0 * M * rb : 0.0,
            (FUSED || PARX) ? &inv_fwd : nullptr,
            &fwd,
            &fwd_phi,
            &zeq,
            &zgreen,
            W2,
            W2 != W ? &zgreen_alt : nullptr,
            &inv,
            &init,
            &from_f64,
            &to_f64,
            (FUSED || PARX) ? &inv_fwd_al : nullptr,
            &inv_al,
            &to_tau,
            3,
            &launch_reduce,
            (double)M,
            PARX ? &fwd_par : nullptr,
            PARX ? &zgreen_par : nullptr,
            (FUSED || PARX) ? &inv_fwd_dual : nullptr,
            &inv_dual,
            FUSED2 ? NTP2 : 0,
            {FUSED2 ? &inv_fwd2 : nullptr, FUSED2 ? &inv_fwd2_al : nullptr, FUSED2 ? &inv_fwd2_dual : nullptr},
        };
        return &o;
    }
};

}  // namespace rvehom
