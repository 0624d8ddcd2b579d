// elastic_kernels.hpp -- the elastic case of the accelerated scheme (linear
// elasticity with isotropic phases, which Sec. 6 names as the extension of
// the method): the z pass with the isotropic elastic Green operator, and the
// launcher table of one (T, N).  The plane passes are the conductivity
// kernels with six components per load case (NC = 6).
//
// Components are taken in an orthonormal basis of symmetric tensors,
//   B0 = I / sqrt3,              B1 = (e1e1 - e2e2) / sqrt2,
//   B2 = (e1e1 + e2e2 - 2 e3e3) / sqrt6,
//   B3 = (e2e3 + e3e2) / sqrt2,  B4 = (e1e3 + e3e1) / sqrt2,
//   B5 = (e1e2 + e2e1) / sqrt2,
// where an isotropic stiffness is diagonal, diag(3 kappa, 2 mu, ..., 2 mu):
// the update e+ = e + 2 (C + C0)^-1 C0 (c - e) and tau = (C - C0) e then act
// on each component alone (hydrostatic channel: 3 kappa, deviatoric ones:
// 2 mu), exactly as the conductivity update acts on each vector component.
// Load case j imposes E = Bj; the mean stress component k is C_hom's entry
// (k, j) in this basis.
#pragma once

#include "kernel_instances.hpp"

namespace rvehom {

// z-tile width for six components: largest even W <= 16 dividing N/2 with
// 6 N W complex values in 64 KiB of LDS (96 KiB if that leaves W < 4).
template <typename T, int N> constexpr int ztile_el_cap(size_t cap) {
    for (int w = 16; w >= 2; w -= 2)
        if ((N / 2) % w == 0 && N % w == 0 && (size_t)6 * N * w * sizeof(Cx<T>) <= cap) return w;
    return 0;
}
template <typename T, int N> constexpr int ztile_el() {
    // FP32 256^3: 8-column tiles (64-byte rows, 96 KiB for the six
    // components), transformed in two halves of 48 KiB by the parity-layout
    // z pass (one solve: 214 ms, against 264 ms with 4-column tiles)
    if constexpr (sizeof(T) == 4 && N == 256) return 8;
    return ztile_el_cap<T, N>(64 * 1024) >= 4 ? ztile_el_cap<T, N>(64 * 1024) : ztile_el_cap<T, N>(96 * 1024);
}

// The Green operator of the elastic case at one frequency (ki0, ki1, ki2)
// of the grid (indices in 0 .. N-1): the six basis components tv of the
// transformed polarization in, those of c^ out.  A0 = 1 / (mu0 M),
// B0c = beta / M.
template <typename T, int N>
__device__ __forceinline__ void green_el_point(const Cx<T> *tv, Cx<T> *o, int ki0, int ki1, int ki2, T A0, T B0c) {
    constexpr int H = N / 2, NC = 6;
    const double s2 = 0.70710678118654752440, s3 = 0.57735026918962576451, s6 = 0.40824829046386301637;
    const int ki[3] = {ki0, ki1, ki2};
    T xi[3];
    int flip = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (ki[d] == H) flip |= 1 << d;
        xi[d] = (T)(ki[d] <= H ? ki[d] : ki[d] - N);
    }
    if (ki[0] == 0 && ki[1] == 0 && ki[2] == 0) {
#pragma unroll
        for (int c = 0; c < NC; ++c) o[c] = Cx<T>{(T)0, (T)0};
    } else {
        // T^ as a symmetric tensor: t[0..2] = 11, 22, 33; t[3..5] = 23, 13, 12
        Cx<T> tt[6];
        tt[0] = scale(tv[0], (T)s3) + scale(tv[1], (T)s2) + scale(tv[2], (T)s6);
        tt[1] = scale(tv[0], (T)s3) - scale(tv[1], (T)s2) + scale(tv[2], (T)s6);
        tt[2] = scale(tv[0], (T)s3) - scale(tv[2], (T)(2.0 * s6));
        tt[3] = scale(tv[3], (T)s2);
        tt[4] = scale(tv[4], (T)s2);
        tt[5] = scale(tv[5], (T)s2);
        Cx<T> cc[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) cc[q] = Cx<T>{(T)0, (T)0};
        int count = 0;
        for (int sgn = 0; sgn < 8; ++sgn) {
            if (sgn & ~flip) continue;  // only Nyquist components change sign
            T v[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) v[d] = ((sgn >> d) & 1) ? -xi[d] : xi[d];
            const T v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
            // u = T^ v, s = v . u
            const Cx<T> u0 = scale(tt[0], v[0]) + scale(tt[5], v[1]) + scale(tt[4], v[2]);
            const Cx<T> u1 = scale(tt[5], v[0]) + scale(tt[1], v[1]) + scale(tt[3], v[2]);
            const Cx<T> u2 = scale(tt[4], v[0]) + scale(tt[3], v[1]) + scale(tt[2], v[2]);
            const Cx<T> sv = scale(u0, v[0]) + scale(u1, v[1]) + scale(u2, v[2]);
            const T a = A0 / v2, b = B0c / (v2 * v2);
            const Cx<T> bs = scale(sv, b);
            cc[0] = cc[0] + scale(u0, a * v[0]) - scale(bs, v[0] * v[0]);
            cc[1] = cc[1] + scale(u1, a * v[1]) - scale(bs, v[1] * v[1]);
            cc[2] = cc[2] + scale(u2, a * v[2]) - scale(bs, v[2] * v[2]);
            cc[3] = cc[3] + scale(scale(u1, v[2]) + scale(u2, v[1]), (T)0.5 * a) - scale(bs, v[1] * v[2]);
            cc[4] = cc[4] + scale(scale(u0, v[2]) + scale(u2, v[0]), (T)0.5 * a) - scale(bs, v[0] * v[2]);
            cc[5] = cc[5] + scale(scale(u0, v[1]) + scale(u1, v[0]), (T)0.5 * a) - scale(bs, v[0] * v[1]);
            ++count;
        }
        const T f = (T)-1 / (T)count;
        // back to the basis components: c_k = B_k : C
        o[0] = scale(cc[0] + cc[1] + cc[2], f * (T)s3);
        o[1] = scale(cc[0] - cc[1], f * (T)s2);
        o[2] = scale(cc[0] + cc[1] - scale(cc[2], (T)2), f * (T)s6);
        o[3] = scale(cc[3], f * (T)(2.0 * s2));
        o[4] = scale(cc[4], f * (T)(2.0 * s2));
        o[5] = scale(cc[5], f * (T)(2.0 * s2));
    }
}

// P2 of the elastic case: z FFT of the six components' pencils, the Green
// operator of the isotropic reference medium (lambda0, mu0),
//   c^ = -[ sym((T^ xi) (x) xi) / (mu0 |xi|^2)
//           - beta (xi . T^ xi) xi (x) xi / |xi|^4 ] / M,
//   beta = (lambda0 + mu0) / (mu0 (lambda0 + 2 mu0)),
// with T^ = sum_l tau^_l B_l, averaged over the signs of the Nyquist
// components (the conductivity reading of even grids), c^(0) = 0 (E is added
// after the inverse transform), inverse z FFT.  PAR: the forward spectrum
// arrives in the parity layout of the split-plane fused pass (specB, nyqB),
// combined as X = E +- w O while it loads, as in k_zgreen<PAR>.
template <typename T, int N, int W, int NT, bool PAR = false>
__global__ __launch_bounds__(NT) void k_zgreen_el(Cx<T> *__restrict__ spec, Cx<T> *__restrict__ nyq,
                                                  const Cx<T> *__restrict__ twg,
                                                  const DevParams *__restrict__ prm,
                                                  const DevState *__restrict__ st,
                                                  const Cx<T> *__restrict__ specB = nullptr,
                                                  const Cx<T> *__restrict__ nyqB = nullptr) {
    using TL = ZTiles<N, W>;
    constexpr int H = N / 2, NW = N * W, NC = 6;
    static_assert(H % W == 0 && N % W == 0 && W % 2 == 0, "tile width must be even and divide N/2");
    __shared__ Cx<T> buf[NC * NW];
    const int tid = threadIdx.x;
    const int lc = blockIdx.x / TL::PER_LC;
    int t;
    if constexpr (PAR) t = ztile_par<N, W>(blockIdx.x - lc * TL::PER_LC);
    else t = ztile_of<T, N, W>(blockIdx.x - lc * TL::PER_LC);
    if (st->done[lc]) return;
    Cx<T> *base;
    const Cx<T> *pbase = nullptr;  // PAR: row ky mod N/2 of the parity layout
    size_t cstride, zstride, poff = 0;  // poff: from parity 0 to parity 1
    int kx0, ky0, dkx, dky;
    if (t < TL::MAIN) {
        const int ky = t / (H / W);
        kx0 = (t - ky * (H / W)) * W;
        ky0 = ky;
        dkx = 1;
        dky = 0;
        base = spec + (size_t)(NC * lc) * N * N * H + (size_t)ky * H + kx0;
        constexpr int PC = par_chunk<T, W>();
        static_assert(!PAR || (PC % W == 0 && H % PC == 0), "z tiles inside parity chunks");
        if constexpr (PAR)
            pbase = specB + (size_t)(NC * lc) * N * N * H + (size_t)(ky % H) * N + (kx0 / PC) * (2 * PC) + kx0 % PC;
        poff = PC;
        cstride = (size_t)N * N * H;
        zstride = (size_t)N * H;
    } else {
        kx0 = H;
        ky0 = (t - TL::MAIN) * W;
        dkx = 0;
        dky = 1;
        base = nyq + (size_t)(NC * lc) * N * N + ky0;
        if constexpr (PAR) pbase = nyqB + (size_t)(NC * lc) * N * N + (ky0 % H);
        poff = H;
        cstride = (size_t)N * N;
        zstride = N;
    }
    // the six components' pencils straight to the registers of the first z
    // stage, and the last inverse stage straight back (measured faster below
    // 256^3 in FP32 and below 128^3 in FP64; the 4-column tiles of the larger
    // grids keep the staged form)
    constexpr bool DIRECT = !(N >= 256 || (sizeof(T) == 8 && N >= 128)) && !PAR;
    constexpr int NP = NC * NW / 2;
    ZFirstStage<T, N, W, NT, NC> z0;
    if constexpr (DIRECT) {
        z0.load(base, cstride, zstride, tid);
    } else if constexpr (PAR) {
        // X = E +- w O from the two parity rows (a tile's rows lie in one
        // half: W divides N/2)
        const bool upper = ky0 >= H;
        for (int idx = tid; idx < NP; idx += NT) {
            const int e0 = 2 * idx, c = e0 / NW, r = e0 - c * NW, zz = r / W, w = r - zz * W;
            const Cx<T> *src = pbase + c * cstride + zz * zstride + w;
            Cx<T> a, b, u, v;
            gload2<T>(src, a, b);
            gload2<T>(src + poff, u, v);
            buf[e0] = upper ? a - u : a + u;
            buf[e0 + 1] = upper ? b - v : b + v;
        }
    } else {
        for (int idx = tid; idx < NP; idx += NT) {
            const int e0 = 2 * idx, c = e0 / NW, r = e0 - c * NW, zz = r / W, w = r - zz * W;
            Cx<T> a, b;
            gload2<T>(base + c * cstride + zz * zstride + w, a, b);
            buf[e0] = a;
            buf[e0 + 1] = b;
        }
    }
    __shared__ Cx<T> tws[N];
    table_to_lds<T, N, NT>(tws, twg, tid);
    const Cx<T> *tw = tws;
    if constexpr (DIRECT) {
        z0.finish(buf, tid);
        fft_stages<T, N, 1, num_stages(N), false, NC * W, W, NT, N, SeqBlocked<W, NW>, kPairNone>(buf, tw, tid);
    } else {
        __syncthreads();
        fft_lds<T, N, false, NC * W, W, NT, N, SeqBlocked<W, NW>>(buf, tw, tid);
    }
    const T A0 = (T)prm->el_inv_mu0M, B0c = (T)prm->el_betaM;
    for (int idx = tid; idx < NW; idx += NT) {
        const int kz = idx / W, w = idx - kz * W;
        Cx<T> tv[NC], o[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) tv[c] = buf[c * NW + idx];
        green_el_point<T, N>(tv, o, kx0 + dkx * w, ky0 + dky * w, kz, A0, B0c);
#pragma unroll
        for (int c = 0; c < NC; ++c) buf[c * NW + idx] = o[c];
    }
    __syncthreads();
    if constexpr (DIRECT) {
        fft_stages<T, N, 0, num_stages(N) - 1, true, NC * W, W, NT, N, SeqBlocked<W, NW>, kPairNone>(buf, tw, tid);
        z_last_stage_store<T, N, W, NT, NC>(buf, tw, base, cstride, zstride, tid);
    } else {
        fft_lds<T, N, true, NC * W, W, NT, N, SeqBlocked<W, NW>>(buf, tw, tid);
        for (int idx = tid; idx < NP; idx += NT) {
            const int e0 = 2 * idx, c = e0 / NW, r = e0 - c * NW, zz = r / W, w = r - zz * W;
            gstore2<T>(base + c * cstride + zz * zstride + w, buf[e0], buf[e0 + 1]);
        }
    }
}

// The z pass of k_zgreen_el in two halves, for tiles whose six components
// would fill a CU's LDS (96 KiB at FP32 256^3 and 512^3, FP64 256^3 and
// 512^3); PAR as in k_zgreen_el (the parity layout, FP32 256^3).  The
// tile is transformed three components at a time in 48 KiB: components
// 0-2 forward, then held in registers at the Green points each thread
// evaluates, while components 3-5 go forward in the same LDS; the Green
// operator then takes its six inputs from registers and LDS, components
// 3-5 go back and are stored, and components 0-2 return from registers,
// go back and are stored.  Two or three tiles then share a CU, so one
// tile's loads and stores run beside another's transforms.
template <typename T, int N, int W, int NT, bool PAR = true>
__global__ __launch_bounds__(NT) void k_zgreen_el_half(Cx<T> *__restrict__ spec, Cx<T> *__restrict__ nyq,
                                                       const Cx<T> *__restrict__ twg,
                                                       const DevParams *__restrict__ prm,
                                                       const DevState *__restrict__ st,
                                                       const Cx<T> *__restrict__ specB,
                                                       const Cx<T> *__restrict__ nyqB) {
    using TL = ZTiles<N, W>;
    constexpr int H = N / 2, NW = N * W, NC = 6, NH = 3, NPH = NH * NW / 2, GP = NW / NT;
    constexpr int PC = par_chunk<T, W>();
    static_assert(NW % NT == 0, "whole Green points per thread");
    static_assert(!PAR || (PC % W == 0 && H % PC == 0), "z tiles inside parity chunks");
    static_assert(H % W == 0 && N % W == 0 && W % 2 == 0, "tile width must be even and divide N/2");
    __shared__ Cx<T> buf[NH * NW];
    __shared__ Cx<T> tws[N];
    const int tid = threadIdx.x;
    const int lc = blockIdx.x / TL::PER_LC;
    int t;
    if constexpr (PAR) t = ztile_par<N, W>(blockIdx.x - lc * TL::PER_LC);
    else t = ztile_of<T, N, W>(blockIdx.x - lc * TL::PER_LC);
    if (st->done[lc]) return;
    Cx<T> *base;
    const Cx<T> *pbase = nullptr;
    size_t cstride, zstride, poff;
    int kx0, ky0, dkx, dky;
    if (t < TL::MAIN) {
        const int ky = t / (H / W);
        kx0 = (t - ky * (H / W)) * W;
        ky0 = ky;
        dkx = 1;
        dky = 0;
        base = spec + (size_t)(NC * lc) * N * N * H + (size_t)ky * H + kx0;
        if constexpr (PAR)
            pbase = specB + (size_t)(NC * lc) * N * N * H + (size_t)(ky % H) * N + (kx0 / PC) * (2 * PC) + kx0 % PC;
        poff = PC;
        cstride = (size_t)N * N * H;
        zstride = (size_t)N * H;
    } else {
        kx0 = H;
        ky0 = (t - TL::MAIN) * W;
        dkx = 0;
        dky = 1;
        base = nyq + (size_t)(NC * lc) * N * N + ky0;
        if constexpr (PAR) pbase = nyqB + (size_t)(NC * lc) * N * N + (ky0 % H);
        poff = H;
        cstride = (size_t)N * N;
        zstride = N;
    }
    const bool upper = ky0 >= H;  // a tile's rows lie in one half
    // components c0 .. c0 + 2 into LDS as X = E +- w O
    auto load_half = [&](int c0) {
        for (int idx = tid; idx < NPH; idx += NT) {
            const int e0 = 2 * idx, c = e0 / NW, r = e0 - c * NW, zz = r / W, w = r - zz * W;
            if constexpr (PAR) {
                const Cx<T> *src = pbase + (c0 + c) * cstride + zz * zstride + w;
                Cx<T> a, b, u, v;
                gload2<T>(src, a, b);
                gload2<T>(src + poff, u, v);
                buf[e0] = upper ? a - u : a + u;
                buf[e0 + 1] = upper ? b - v : b + v;
            } else {
                Cx<T> a, b;
                gload2<T>(base + (c0 + c) * cstride + zz * zstride + w, a, b);
                buf[e0] = a;
                buf[e0 + 1] = b;
            }
        }
    };
    auto store_half = [&](int c0) {
        for (int idx = tid; idx < NPH; idx += NT) {
            const int e0 = 2 * idx, c = e0 / NW, r = e0 - c * NW, zz = r / W, w = r - zz * W;
            gstore2<T>(base + (c0 + c) * cstride + zz * zstride + w, buf[e0], buf[e0 + 1]);
        }
    };
    load_half(0);
    table_to_lds<T, N, NT>(tws, twg, tid);
    __syncthreads();
    fft_lds<T, N, false, NH * W, W, NT, N, SeqBlocked<W, NW>>(buf, tws, tid);
    Cx<T> keep[GP][NH];  // components 0-2 at this thread's Green points tid + g NT
#pragma unroll
    for (int g = 0; g < GP; ++g)
#pragma unroll
        for (int c = 0; c < NH; ++c) keep[g][c] = buf[c * NW + tid + g * NT];
    __syncthreads();
    load_half(NH);
    __syncthreads();
    fft_lds<T, N, false, NH * W, W, NT, N, SeqBlocked<W, NW>>(buf, tws, tid);
    const T A0 = (T)prm->el_inv_mu0M, B0c = (T)prm->el_betaM;
#pragma unroll
    for (int g = 0; g < GP; ++g) {
        const int idx = tid + g * NT, kz = idx / W, w = idx - kz * W;
        Cx<T> tv[NC], o[NC];
#pragma unroll
        for (int c = 0; c < NH; ++c) {
            tv[c] = keep[g][c];
            tv[NH + c] = buf[c * NW + idx];
        }
        green_el_point<T, N>(tv, o, kx0 + dkx * w, ky0 + dky * w, kz, A0, B0c);
#pragma unroll
        for (int c = 0; c < NH; ++c) {
            keep[g][c] = o[c];
            buf[c * NW + idx] = o[NH + c];
        }
    }
    __syncthreads();
    fft_lds<T, N, true, NH * W, W, NT, N, SeqBlocked<W, NW>>(buf, tws, tid);
    store_half(NH);
    __syncthreads();  // every wave has read components 3-5 out of buf
#pragma unroll
    for (int g = 0; g < GP; ++g)
#pragma unroll
        for (int c = 0; c < NH; ++c) buf[c * NW + tid + g * NT] = keep[g][c];
    __syncthreads();
    fft_lds<T, N, true, NH * W, W, NT, N, SeqBlocked<W, NW>>(buf, tws, tid);
    store_half(0);
}

// Reduction of the elastic partials as a kernel of its own (576 threads).
__global__ void k_reduce_el(const double *part, int nper, const DevParams *prm, DevState *st, double *hist);

template <typename T, int N> struct ElasticInstance {
    static constexpr int NC = 6, CH = NC * NC;
    static constexpr int S = plane_split<T, N>();
    // planes that do not fit in LDS (FP64 256^3, 512^3): the five-pass form
    // of the conductivity case with six components per load case
    static constexpr bool FIVE = (S == 0);
    static constexpr int G = row_group<T, N>();
    static constexpr int WC = col_tile<T, N>();
    static constexpr int NTR = 256;
    static constexpr int W = ztile_el<T, N>();
    static_assert(W >= 2, "no z tile fits in LDS");
    static constexpr int NTP = plane_threads<T, N>();
    // FP32: 512-thread z tiles (the six-component tile needs ~128 VGPRs, so
    // the waves per CU are set by registers, not by LDS; measured 7 % faster
    // than 256 threads at 128^3), 1024 for the one 96 KiB tile per CU of
    // the plain-layout z pass at 256^3; FP64: 256 (measured faster)
    static constexpr int NTZ = sizeof(T) == 4 ? (N == 256 ? 1024 : 512) : 256;
    static constexpr int NPER = FIVE ? N * (N / G) : N * S;
    // the fused inverse + next forward pass: whole planes (not FP32 96^3,
    // whose fused pass spills at 256 threads and at 512 measured no faster
    // than the separate passes), and split planes writing the parity layout
    // that the z pass combines (FP32 256^3)
    static constexpr bool FUSED = S == 1 && !(sizeof(T) == 4 && N == 96);
    static constexpr bool PARF = S == 2 && ztile_par_ok<N, W>();
    static constexpr int PC = par_chunk<T, W>();
    // the parity-layout z pass in two halves of three components where the
    // six-component tile would fill a CU's LDS (FP32 256^3): 512 threads,
    // 120 VGPRs, two workgroups per CU (2118 -> 1769 us per launch; 256
    // threads at 198 VGPRs 2248 us)
    static constexpr bool HALF = PARF && sizeof(T) == 4 && N == 256;
    static constexpr int NTH = 512;
    // the plain-layout z pass in two halves wherever the six-component tile
    // needs more than 64 KiB (FP32 256^3 outside the parity layout, 512^3;
    // FP64 256^3, 512^3): two workgroups per CU, 512 threads in FP32 (107-121
    // VGPRs), 256 in FP64 (208-220); per launch FP64 256^3 5195 -> 3224 us,
    // FP32 512^3 30.8 -> 21.9 ms, FP64 512^3 77.5 -> 54.4 ms
    static constexpr bool HALFZ = (size_t)6 * N * W * sizeof(Cx<T>) > 64 * 1024;
    static constexpr int NTZH = sizeof(T) == 4 ? 512 : 256;
    static constexpr int PGRID = FIVE ? CH * N * (N / G) : CH * N * S;
    static constexpr int SP = FIVE ? 1 : S;

    static void fwd(const LaunchArgs &a, hipStream_t s, int) {
        if constexpr (FIVE) {
            hipLaunchKernelGGL((k_fwd_rows<T, N, G, NTR, false, NC>), dim3(PGRID), dim3(NTR), 0, s, (const T *)a.e,
                               a.ph, (Cx<T> *)a.spec, (Cx<T> *)a.nyq, (const Cx<T> *)a.tw, a.prm,
                               (const DevState *)a.st);
            hipLaunchKernelGGL((k_cols<T, N, WC, NTR, false, false, NC>), dim3(ColTiles<N, WC, CH>::ALL), dim3(NTR),
                               0, s, (Cx<T> *)a.spec, (Cx<T> *)a.nyq, (const Cx<T> *)a.tw, (const DevState *)a.st);
        } else {
            hipLaunchKernelGGL((k_fwd_plane<T, N, SP, NTP, false, NC>), dim3(PGRID), dim3(NTP), 0, s, (const T *)a.e,
                               a.ph, (Cx<T> *)a.spec, (Cx<T> *)a.nyq, (const Cx<T> *)a.tw, a.prm,
                               (const DevState *)a.st, 0);
        }
    }
    static void zgreen(const LaunchArgs &a, hipStream_t s, int, int) {
        if constexpr (HALFZ)
            hipLaunchKernelGGL((k_zgreen_el_half<T, N, W, NTZH, false>), dim3(NC * ZTiles<N, W>::PER_LC), dim3(NTZH),
                               0, s, (Cx<T> *)a.spec, (Cx<T> *)a.nyq, (const Cx<T> *)a.tw, a.prm,
                               (const DevState *)a.st, (const Cx<T> *)nullptr, (const Cx<T> *)nullptr);
        else
            hipLaunchKernelGGL((k_zgreen_el<T, N, W, NTZ>), dim3(NC * ZTiles<N, W>::PER_LC), dim3(NTZ), 0, s,
                               (Cx<T> *)a.spec, (Cx<T> *)a.nyq, (const Cx<T> *)a.tw, a.prm, (const DevState *)a.st,
                               (const Cx<T> *)nullptr, (const Cx<T> *)nullptr);
    }
    // split planes: the first forward pass and the z pass of the parity layout
    static void fwd_par(const LaunchArgs &a, hipStream_t s, int) {
        if constexpr (PARF)
            hipLaunchKernelGGL((k_fwd_plane<T, N, 2, NTP, false, NC, true, PC>), dim3(PGRID), dim3(NTP), 0, s,
                               (const T *)a.e, a.ph, (Cx<T> *)a.spec2, (Cx<T> *)a.nyq2, (const Cx<T> *)a.tw, a.prm,
                               (const DevState *)a.st, 0);
    }
    static void zgreen_par(const LaunchArgs &a, hipStream_t s, int, int) {
        if constexpr (HALF)
            hipLaunchKernelGGL((k_zgreen_el_half<T, N, W, NTH, true>), dim3(NC * ZTiles<N, W>::PER_LC), dim3(NTH), 0, s,
                               (Cx<T> *)a.spec, (Cx<T> *)a.nyq, (const Cx<T> *)a.tw, a.prm, (const DevState *)a.st,
                               (const Cx<T> *)a.spec2, (const Cx<T> *)a.nyq2);
        else if constexpr (PARF)
            hipLaunchKernelGGL((k_zgreen_el<T, N, W, NTZ, true>), dim3(NC * ZTiles<N, W>::PER_LC), dim3(NTZ), 0, s,
                               (Cx<T> *)a.spec, (Cx<T> *)a.nyq, (const Cx<T> *)a.tw, a.prm, (const DevState *)a.st,
                               (const Cx<T> *)a.spec2, (const Cx<T> *)a.nyq2);
    }
    static void inv(const LaunchArgs &a, hipStream_t s, int) {
        if constexpr (FIVE) {
            hipLaunchKernelGGL((k_cols<T, N, WC, NTR, true, false, NC>), dim3(ColTiles<N, WC, CH>::ALL), dim3(NTR), 0,
                               s, (Cx<T> *)a.spec, (Cx<T> *)a.nyq, (const Cx<T> *)a.tw, (const DevState *)a.st);
            hipLaunchKernelGGL((k_inv_rows<T, N, G, NTR, 0, NC>), dim3(PGRID), dim3(NTR), 0, s, (T *)a.e, a.ph,
                               (const Cx<T> *)a.spec, (const Cx<T> *)a.nyq, (const Cx<T> *)a.tw, a.prm,
                               (const DevState *)a.st, a.part);
        } else {
            hipLaunchKernelGGL((k_inv_plane<T, N, SP, NTP, false, 0, NC>), dim3(PGRID), dim3(NTP), 0, s, (T *)a.e,
                               a.ph, (Cx<T> *)a.spec, (Cx<T> *)a.nyq, (const Cx<T> *)a.tw, a.prm,
                               (const DevState *)a.st, a.part, 0, (Cx<T> *)nullptr, (Cx<T> *)nullptr);
        }
    }
    static void inv_fwd(const LaunchArgs &a, hipStream_t s, int) {
        if constexpr (FUSED) {
            hipLaunchKernelGGL((k_inv_plane<T, N, 1, NTP, true, 0, NC>), dim3(PGRID), dim3(NTP), 0, s, (T *)a.e,
                               a.ph, (Cx<T> *)a.spec, (Cx<T> *)a.nyq, (const Cx<T> *)a.tw, a.prm,
                               (const DevState *)a.st, a.part, 0, (Cx<T> *)nullptr, (Cx<T> *)nullptr);
        } else if constexpr (PARF) {
            hipLaunchKernelGGL((k_inv_plane<T, N, 2, NTP, true, 0, NC, PC>), dim3(PGRID), dim3(NTP), 0, s, (T *)a.e,
                               a.ph, (Cx<T> *)a.spec, (Cx<T> *)a.nyq, (const Cx<T> *)a.tw, a.prm,
                               (const DevState *)a.st, a.part, 0, (Cx<T> *)a.spec2, (Cx<T> *)a.nyq2);
        }
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
    static void reduce(const LaunchArgs &a, int nper, hipStream_t s) {
        hipLaunchKernelGGL(k_reduce_el, dim3(1), dim3(576), 0, s, (const double *)a.part, nper, a.prm, a.st, a.hist);
    }

    static const SolverOps *ops(int precision) {
        constexpr size_t M = (size_t)N * N * N;
        constexpr size_t H = N / 2;
        constexpr double cb = (double)sizeof(Cx<T>);
        constexpr double rb = (double)sizeof(T);
        constexpr double spec_b = (double)CH * N * N * (H + 1) * cb;
        // the five-pass form's column passes read and write the spectrum once more each way
        constexpr double extra = FIVE ? 2.0 * spec_b : 0.0;
        static const SolverOps o = {
            N,
            precision,
            FIVE ? 0 : S,
            W,
            NPER,
            sizeof(T),
            (size_t)CH * N * N * H,
            (size_t)CH * N * N,
            {PGRID, NC * ZTiles<N, W>::PER_LC, PGRID},
            {FIVE ? NTR : NTP, NTZ, FIVE ? NTR : NTP},
            {CH * (double)M * rb + spec_b + extra, 2.0 * spec_b, spec_b + 2.0 * CH * (double)M * rb + extra},
            0,
            (FUSED || PARF) ? 2.0 * spec_b + 2.0 * CH * (double)M * rb : 0.0,
            (FUSED || PARF) ? &inv_fwd : nullptr,
            &fwd,
            nullptr,
            nullptr,
            &zgreen,
            W,
            nullptr,
            &inv,
            &init,
            &from_f64,
            &to_f64,
            nullptr,
            nullptr,
            nullptr,
            NC,
            &reduce,
            (double)M,
            PARF ? &fwd_par : nullptr,
            PARF ? &zgreen_par : nullptr,
            nullptr,
            nullptr,
        };
        return &o;
    }
};

}  // namespace rvehom
