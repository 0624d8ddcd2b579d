// solver_kernels.hpp -- gfx950 kernels of one iteration of the accelerated
// (Eyre-Milton) FFT scheme for the thermal conductivity of a periodic voxel
// RVE (arXiv:1504.07499, Sec. 3, Algorithm steps 2-7; Sec. 5 for L0).
//
// Data in HBM (T = float or double, M = N^3, 9 channels ch = 3*lc + comp):
//   e     [ch][z][y][x]            real gradient iterate, x fastest
//   ph    [z][y][x]                uint8 phase id (0 matrix, 1 inclusion, 2 coating)
//   spec  [ch][z][ky][kx], kx<N/2  half spectrum without the kx = N/2 column
//   nyq   [ch][z][ky]              the kx = N/2 column
//   part  [ch][block][3]           FP64 partials {sum |e - c|^2, sum k e+, sum e+}
//
// One iteration = three passes over HBM plus a tiny reduction:
//   P1 (k_fwd_plane):   tau = (k - k0) e (step 2) fused into the load, then the
//                       2D real-to-complex FFT of each (ch, z) xy-plane in LDS;
//   P2 (k_zgreen):      z-FFT of the three components of one load case, the
//                       Green operator with the xi = 0 pin (step 4), inverse
//                       z-FFT, in place;
//   P3 (k_inv_plane):   2D complex-to-real inverse of each xy-plane in LDS,
//                       then the residual (step 6), the update (step 7) and the
//                       flux <k e+>, with FP64 block partials;
//   k_reduce:           fixed-order FP64 reduction, convergence test and
//                       per-load-case freeze, all on the device.
// With L0 = -k0 I (Sec. 5) the steps read tau = (k - k0) e,
// c^ = -xi (xi . tau^) / (k0 |xi|^2) for xi != 0, c^(0) = E, and
// e+ = e + 2 k0 / (k + k0) (c - e).
//
// Nyquist modes (even N): the index N/2 stands for both +N/2 and -N/2, so the
// operator used is xi xi^T / |xi|^2 averaged over both signs of every Nyquist
// component.  With A the non-Nyquist and B the Nyquist components of a mode,
// that average is (xi_A xi_A^T + diag(xi_B^2)) / |xi|^2: components in A see
// xi_i (xi_A . tau^), each component in B sees xi_i^2 tau^_i.  The result is
// even in xi (so the half-spectrum inverse is exact) and keeps the discrete
// problem covariant under mirroring any axis.
//
// Planes too large for LDS are split in S row-parities (S = 2): the first
// radix-2 step of the y transform is done while loading, so each workgroup
// holds N/2 rows.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_lds.hpp"
#include "reduce_block.hpp"
#include "solver_state.hpp"

namespace rvehom {

template <typename T> struct VecOf;
template <> struct VecOf<float> {
    static constexpr int V = 4;
    using type = float4;
    using ptype = uchar4;
};
template <> struct VecOf<double> {
    static constexpr int V = 2;
    using type = double2;
    using ptype = uchar2;
};

template <typename T> __device__ __forceinline__ void vload(const T *p, T *out);
template <> __device__ __forceinline__ void vload<float>(const float *p, float *o) {
    float4 v = *reinterpret_cast<const float4 *>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
template <> __device__ __forceinline__ void vload<double>(const double *p, double *o) {
    double2 v = *reinterpret_cast<const double2 *>(p);
    o[0] = v.x; o[1] = v.y;
}
template <typename T> __device__ __forceinline__ void vstore(T *p, const T *in);
template <> __device__ __forceinline__ void vstore<float>(float *p, const float *i) {
    *reinterpret_cast<float4 *>(p) = make_float4(i[0], i[1], i[2], i[3]);
}
template <> __device__ __forceinline__ void vstore<double>(double *p, const double *i) {
    *reinterpret_cast<double2 *>(p) = make_double2(i[0], i[1]);
}
// V phase ids (one byte each) kept packed in one register; ph_at extracts id j.
template <int V> __device__ __forceinline__ unsigned pload(const uint8_t *p);
template <> __device__ __forceinline__ unsigned pload<4>(const uint8_t *p) {
    return *reinterpret_cast<const unsigned *>(p);
}
template <> __device__ __forceinline__ unsigned pload<2>(const uint8_t *p) {
    return *reinterpret_cast<const unsigned short *>(p);
}
__device__ __forceinline__ int ph_at(unsigned pk, int j) { return (int)((pk >> (8 * j)) & 0xffu); }

// Two consecutive complex values as one 16-byte global access (FP32) or two
// (FP64); dst/src must be aligned to 2 complex values.
template <typename T> __device__ __forceinline__ void gload2(const Cx<T> *src, Cx<T> &a, Cx<T> &b);
template <> __device__ __forceinline__ void gload2<float>(const Cx<float> *src, Cx<float> &a, Cx<float> &b) {
    const float4 v = *reinterpret_cast<const float4 *>(src);
    a = Cx<float>{v.x, v.y};
    b = Cx<float>{v.z, v.w};
}
template <> __device__ __forceinline__ void gload2<double>(const Cx<double> *src, Cx<double> &a, Cx<double> &b) {
    a = src[0];
    b = src[1];
}
template <typename T> __device__ __forceinline__ void gstore2(Cx<T> *dst, Cx<T> a, Cx<T> b);
template <> __device__ __forceinline__ void gstore2<float>(Cx<float> *dst, Cx<float> a, Cx<float> b) {
    *reinterpret_cast<float4 *>(dst) = make_float4(a.x, a.y, b.x, b.y);
}
template <> __device__ __forceinline__ void gstore2<double>(Cx<double> *dst, Cx<double> a, Cx<double> b) {
    dst[0] = a;
    dst[1] = b;
}

// phase-indexed lookup without a memory table: p in {0,1,2}
template <typename T> __device__ __forceinline__ T pick(int p, T a0, T a1, T a2) {
    return p == 0 ? a0 : (p == 1 ? a1 : a2);
}

// Two neighbouring complex values of a plane row: one 16-byte LDS access
// when the pair is 16-byte aligned (even row pitch), else two.
template <typename T, bool ALIGNED>
__device__ __forceinline__ void ld_pair(const Cx<T> *p, Cx<T> &a, Cx<T> &b) {
    if constexpr (ALIGNED) {
        lds_ld2<T>(p, a, b);
    } else {
        a = p[0];
        b = p[1];
    }
}
template <typename T, bool ALIGNED> __device__ __forceinline__ void st_pair(Cx<T> *p, Cx<T> a, Cx<T> b) {
    if constexpr (ALIGNED) {
        lds_st2<T>(p, a, b);
    } else {
        p[0] = a;
        p[1] = b;
    }
}

// R2C unpack, item k in [0, N/4] of one row: the length-N/2 FFT Z of the
// packed even/odd samples becomes X[k] and X[N/2 - k] of the real-input
// spectrum (X[0] and X[N/2] for k = 0), optionally times a row factor.
// P0: the two real values X[0] and X[N/2] go to row[0] as X[0] + i X[N/2]
// (the y transform then handles both columns as one complex column).
template <typename T, int N, bool ROT, bool P0 = false>
__device__ __forceinline__ void r2c_unpack(Cx<T> *row, int k, const Cx<T> *__restrict__ tw, Cx<T> rot) {
    constexpr int H = N / 2;
    if (k == 0) {
        const Cx<T> z0 = row[0];
        if constexpr (P0) {
            row[0] = Cx<T>{z0.x + z0.y, z0.x - z0.y};
        } else {
            Cx<T> x0 = {z0.x + z0.y, (T)0}, xh = {z0.x - z0.y, (T)0};
            if (ROT) {
                x0 = x0 * rot;
                xh = xh * rot;
            }
            row[0] = x0;
            row[H] = xh;
        }
    } else {
        const Cx<T> a = row[k], b = conj(row[H - k]);
        const Cx<T> A = scale(a + b, (T)0.5);
        const Cx<T> D = scale(a - b, (T)0.5);
        const Cx<T> B = {D.y, -D.x};  // (a - b) / (2 i)
        const Cx<T> wB = B * tw[k];
        Cx<T> xk = A + wB, xm = conj(A - wB);
        if (ROT) {
            xk = xk * rot;
            xm = xm * rot;
        }
        row[k] = xk;
        if (k != H - k) row[H - k] = xm;
    }
}

// C2R pack, item k in [0, N/4]: Hermitian half row X[0..N/2] -> the
// length-N/2 sequence whose inverse FFT holds the even/odd output samples.
// P0: X[0] and X[N/2] arrive packed in row[0] as X[0] + i X[N/2].
template <typename T, int N, bool P0 = false>
__device__ __forceinline__ void c2r_pack(Cx<T> *row, int k, const Cx<T> *__restrict__ tw) {
    constexpr int H = N / 2;
    if (k == 0) {
        const T x0 = row[0].x, xh = P0 ? row[0].y : row[H].x;
        row[0] = Cx<T>{x0 + xh, x0 - xh};
    } else {
        const Cx<T> a = row[k], b = conj(row[H - k]);
        const Cx<T> A = a + b;
        const Cx<T> B = (a - b) * conj(tw[k]);
        row[k] = A + Cx<T>{-B.y, B.x};                               // A + i B
        if (k != H - k) row[H - k] = conj(A) + Cx<T>{B.y, B.x};      // conj(A) + i conj(B)
    }
}

// Unpack / pack loops over the rows of a plane: per row the items k and
// N/4 share one thread (N/4 is its own partner), N/4 items per row.
template <typename T, int N, int ROWS, int NT, bool P0, int RS>
__device__ __forceinline__ void r2c_unpack_rows(Cx<T> *plane, const Cx<T> *__restrict__ tw, int tid) {
    constexpr int H = N / 2, Q = H / 2;
    for (int idx = tid; idx < ROWS * Q; idx += NT) {
        const int y = idx / Q, k = idx - y * Q;
        r2c_unpack<T, N, false, P0>(plane + y * RS, k, tw, Cx<T>{(T)1, (T)0});
        if (k == 0) r2c_unpack<T, N, false, P0>(plane + y * RS, Q, tw, Cx<T>{(T)1, (T)0});
    }
}
template <typename T, int N, int ROWS, int NT, bool P0, int RS>
__device__ __forceinline__ void c2r_pack_rows(Cx<T> *plane, const Cx<T> *__restrict__ tw, int tid) {
    constexpr int H = N / 2, Q = H / 2;
    for (int idx = tid; idx < ROWS * Q; idx += NT) {
        const int y = idx / Q, k = idx - y * Q;
        c2r_pack<T, N, P0>(plane + y * RS, k, tw);
        if (k == 0) c2r_pack<T, N, P0>(plane + y * RS, Q, tw);
    }
}

// Last stage of the forward y transform of a whole plane (S = 1), its outputs
// stored straight to the spectrum rows ky in global memory instead of going
// back through LDS: butterfly b = j H + q reads column q as the self-sorting
// stage does, and row ky = d + r NS of column q leaves as one 8- or 16-byte
// store (neighbouring threads: neighbouring columns).  Column 0 holds
// Z = Y0 + i YH, the y transforms of the two real columns kx = 0 and N/2; it
// also goes to LDS, and after a barrier (which orders the workgroup's two
// stores to each of its addresses) Y0 = (Z[ky] + conj Z[-ky]) / 2 replaces it
// and YH = (Z[ky] - conj Z[-ky]) / (2 i) is stored (Hermitian symmetry).
template <typename T, int N, int NT, int RS>
__device__ __forceinline__ void y_last_stage_store(Cx<T> *plane, const Cx<T> *__restrict__ tw, Cx<T> *sb, Cx<T> *nb,
                                                   int tid) {
    constexpr int H = N / 2, SL = num_stages(N) - 1, R = radix_of(N, SL), NS = ns_before(N, SL), NB = N / R;
    // FP32: the same butterfly of columns 2p and 2p + 1 per thread (16-byte
    // accesses) where the pairs still give every thread work
    constexpr int P = (sizeof(T) == 4 && (H / 2) * NB >= NT) ? 2 : 1, NQ = H / P;
    constexpr int TOT = NQ * NB, PER = (TOT + NT - 1) / NT, TWS = N / (NS * R);
    Cx<T> v[PER][P][R];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int b = tid + i * NT;
        if (TOT % NT == 0 || b < TOT) {
            const int j = b / NQ, q = (b - j * NQ) * P;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if constexpr (P == 2) lds_ld2<T>(plane + q + (j + r * NB) * RS, v[i][0][r], v[i][1][r]);
                else v[i][0][r] = plane[q + (j + r * NB) * RS];
            }
            if constexpr (NS > 1) {
                const int k = j % NS;
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    const Cx<T> w = tw[r * k * TWS];
#pragma unroll
                    for (int u = 0; u < P; ++u) v[i][u][r] = twmul<T, false>(v[i][u][r], w);
                }
            }
#pragma unroll
            for (int u = 0; u < P; ++u) dft<T, R, false>(v[i][u]);
        }
    }
    __syncthreads();  // every read of the plane is done before column 0 is rewritten
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int b = tid + i * NT;
        if (TOT % NT == 0 || b < TOT) {
            const int j = b / NQ, q = (b - j * NQ) * P;
            const int k = j % NS, d = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) {  // column 0: rewritten below
                if constexpr (P == 2) gstore2<T>(sb + (size_t)(d + r * NS) * H + q, v[i][0][r], v[i][1][r]);
                else sb[(size_t)(d + r * NS) * H + q] = v[i][0][r];
            }
        }
    }
    // compiler-only fence: keeps the column-0 LDS stores from being merged
    // with the global ones into flat stores through a selected pointer
    asm volatile("" ::: "memory");
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int b = tid + i * NT;
        if ((TOT % NT == 0 || b < TOT) && b % NQ == 0) {
            const int j = b / NQ, k = j % NS, d = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) plane[(d + r * NS) * RS] = v[i][0][r];
        }
    }
    __syncthreads();
    for (int m = tid; m < N; m += NT) {
        const Cx<T> a = plane[m * RS], b = conj(plane[(m == 0 ? 0 : N - m) * RS]);
        const Cx<T> dd = scale(a - b, (T)0.5);
        nb[m] = Cx<T>{dd.y, -dd.x};
        sb[(size_t)m * H] = scale(a + b, (T)0.5);
    }
}

// Steps 6-7 and the flux on V voxels of one row: e+ = e + w (c - e),
// r2 += |e - c|^2, fl += k e+ (FP64 accumulation).
// c arrives without its mean E (added here).  Also sums e+ (its mean gives
// the mean of tau for the next forward pass).
template <typename T, int V>
__device__ __forceinline__ void em_update(T *a, const T *c, unsigned p, T w0, T w1, T w2, double k0d,
                                          double k1d, double k2d, T ec, double &r2, double &fl,
                                          double &se) {
#pragma unroll
    for (int i = 0; i < V; ++i) {
        const T ci = c[i] + ec;
        const T d = a[i] - ci;
        r2 += (double)d * (double)d;
        const int pi = ph_at(p, i);
        const T wi = pick<T>(pi, w0, w1, w2);
        a[i] = a[i] + wi * (ci - a[i]);
        fl += pick<double>(pi, k0d, k1d, k2d) * (double)a[i];
        se += (double)a[i];
    }
}

// Copy a table of L complex values from global memory into LDS (the caller
// synchronises before the first read).
template <typename T, int L, int NT>
__device__ __forceinline__ void table_to_lds(Cx<T> *dst, const Cx<T> *__restrict__ src, int tid) {
    for (int i = tid; i < L; i += NT) dst[i] = src[i];
}

// The same pointer, opaque to the optimiser: loads through it are not merged
// with earlier loads of the same addresses (keeps the inverse pass's twiddles
// from being held in registers through the update of the fused pass).
template <typename E> __device__ __forceinline__ const E *opaque_ptr(const E *p) {
    int zero = 0;  // an offset the optimiser cannot see through (p stays a global pointer)
    asm volatile("" : "+s"(zero));
    return p + zero;
}

// Steps 6-7 as em_update, and the next iteration's tau = (k - k0) e+ - tm
// (tm: a constant the mean mode absorbs).  Instead of the flux, fl collects
// sum tau in FP64: k e+ = (tau + tm) + k0 e+, so the caller adds
// count * tm + k0 * (sum e+) -- no per-voxel FP64 conductivity lookup.
// lut[phase] = {w, k - k0} (LDS).
// The V neighbouring voxels' terms are summed in the working precision, then
// accumulated in FP64 (a V-term FP32 sum adds ~1e-7 relative error).
template <typename T, int V>
__device__ __forceinline__ void em_update_tau(T *a, const T *c, unsigned p, const Cx<T> *lut, T tm, T ec,
                                              double &r2, double &st, double &se, T *tau) {
    T r2v = (T)0, stv = (T)0, sev = (T)0;
#pragma unroll
    for (int i = 0; i < V; ++i) {
        const T ci = c[i] + ec;
        const T d = a[i] - ci;
        r2v += d * d;
        const Cx<T> wd = lut[ph_at(p, i)];
        a[i] = a[i] + wd.x * (ci - a[i]);
        tau[i] = wd.y * a[i] - tm;
        stv += tau[i];
        sev += a[i];
    }
    r2 += (double)r2v;
    st += (double)stv;
    se += (double)sev;
}

// The augmented-Lagrangian scheme (named in Sec. 3 beside the accelerated
// one; k0 of Sec. 5) in the variable tau = lam - k0 d that its compatible step
// transforms (d: local field, lam: multiplier).  With c = e+ the compatible
// field, the multiplier step gives lam+ = tau + k0 c and the local step
// d+ = (lam+ + k0 c) / (k + k0), so that
//     g    = c - d+ = ((k - k0) c - tau) / (k + k0)   (residual),
//     tau+ = lam+ - k0 d+ = tau + k0 g,
//     k d+ = tau+ + k0 c                               (flux).
// tau is the one field carried between iterations: the buffer that holds e
// for the accelerated scheme holds tau here (k_to_tau writes
// tau^0 = (k - k0) e^0 from the start field before the first pass).
// lut[phase] = {k - k0, 1 / (k + k0)} (LDS).  As em_update_tau, st collects
// sum (tau+ - tm) and se sum c, so that the caller's
// count * tm + k0 * (sum c) completes the flux.
template <typename T, int V>
__device__ __forceinline__ void al_update_tau(T *a, const T *c, unsigned p, const Cx<T> *lut, T k0, T tm, T ec,
                                              double &r2, double &st, double &se, T *tau) {
    T r2v = (T)0, stv = (T)0, sev = (T)0;
#pragma unroll
    for (int i = 0; i < V; ++i) {
        const T ci = c[i] + ec;
        const Cx<T> dg = lut[ph_at(p, i)];
        const T g = (dg.x * ci - a[i]) * dg.y;
        r2v += g * g;
        a[i] = a[i] + k0 * g;
        tau[i] = a[i] - tm;
        stv += tau[i];
        sev += ci;
    }
    r2 += (double)r2v;
    st += (double)stv;
    se += (double)sev;
}

// The augmented-Lagrangian update of the separate inverse passes: as
// al_update_tau, with the flux k d+ = tau+ + k0 c summed per voxel in FP64
// (fl) and se = sum c.  step is the multiple of g added to tau: k0 for the
// augmented Lagrangian, alpha k0 for the polarization scheme.
template <typename T, int V>
__device__ __forceinline__ void al_update(T *a, const T *c, unsigned p, T dk0, T dk1, T dk2, T gm0, T gm1, T gm2,
                                          T k0, T step, T ec, double &r2, double &fl, double &se) {
#pragma unroll
    for (int i = 0; i < V; ++i) {
        const T ci = c[i] + ec;
        const int pi = ph_at(p, i);
        const T g = (pick<T>(pi, dk0, dk1, dk2) * ci - a[i]) * pick<T>(pi, gm0, gm1, gm2);
        r2 += (double)g * (double)g;
        a[i] = a[i] + step * g;
        fl += (double)a[i] + (double)k0 * (double)ci;
        se += (double)ci;
    }
}

// The dual scheme (named in Sec. 3 beside the accelerated one): the buffer
// holds the flux phi, the forward pass transforms tau = -k0^2 phi / k, so
// that the z pass, with the divergence-free projection of the dual scheme
// in place of the Green symbol, returns c = k0 G*(phi / k) (G* = I - P) and
//     phi+ = phi - Delta0 (phi / k - E) = (1 - k0 / k) phi + c + k0 E.
// Residual: the increment |phi+ - phi| / k0; flux: phi+ itself.  wd[p] =
// 1 - k0 / k, dd[p] = -k0^2 / k; e0 is k0 for the diagonal channel of the
// load case, else 0.  For the fused pass: tau of the next iteration is
// dd phi+ - tm, st collects sum (tau - tm) and se sum (phi+ - tau) / k0,
// so that the caller's count tm + k0 se completes sum phi+ as for the other
// updates (and the mean of tau follows in the reduction).
template <typename T, int V>
__device__ __forceinline__ void dual_update_tau(T *a, const T *c, unsigned p, const Cx<T> *lut, T tm, T e0, T ik0,
                                                double &r2, double &st, double &se, T *tau) {
    T r2v = (T)0, stv = (T)0, sev = (T)0;
#pragma unroll
    for (int i = 0; i < V; ++i) {
        const Cx<T> wd = lut[ph_at(p, i)];
        const T f = wd.x * a[i] + c[i] + e0;
        const T d = (f - a[i]) * ik0;
        r2v += d * d;
        a[i] = f;
        const T t = wd.y * f;
        tau[i] = t - tm;
        stv += tau[i];
        sev += (f - t) * ik0;
    }
    r2 += (double)r2v;
    st += (double)stv;
    se += (double)sev;
}

// The dual update of the separate inverse passes: fl = sum phi+, and se as
// in dual_update_tau so that the reduction's mean of tau is that of
// dd phi+ (the next forward pass subtracts it).
template <typename T, int V>
__device__ __forceinline__ void dual_update(T *a, const T *c, unsigned p, T wd0, T wd1, T wd2, T dd0, T dd1, T dd2,
                                            T e0, T ik0, double &r2, double &fl, double &se) {
#pragma unroll
    for (int i = 0; i < V; ++i) {
        const int pi = ph_at(p, i);
        const T f = pick<T>(pi, wd0, wd1, wd2) * a[i] + c[i] + e0;
        const T d = (f - a[i]) * ik0;
        r2 += (double)d * (double)d;
        a[i] = f;
        fl += (double)f;
        se += (double)((f - pick<T>(pi, dd0, dd1, dd2) * f) * ik0);
    }
}

// The parity layout of split planes interleaves the S parities' rows in
// chunks of PC columns: element (parity h, row m < N/S, column kx) of a
// (channel, z) plane sits at m S N/2 + (kx / PC) S PC + h PC + kx % PC.  PC
// is the smallest multiple of the z-tile width W that fills a 128-byte line,
// so each workgroup of the plane pass writes whole lines, and a z tile finds
// the S parities of its row next to each other (one DRAM page) instead of
// N/S rows apart.
template <typename T, int W> constexpr int par_chunk() {
    constexpr int wb = W * (int)sizeof(Cx<T>);
    return W * ((128 + wb - 1) / wb);
}

// Forward transform of a split plane after its x transform (S parities,
// rows of pitch N/2 + 1 in LDS, the N/S rows of parity h).  Without PAR
// (S = 2 only) the rows are the parity-h combinations of a decimation in
// frequency (rows y and y + N/2 summed, or subtracted and turned by w_N^y),
// and the length-N/2 y transform gives the output rows ky = 2 m + h of the
// spectrum.  With PAR the rows are the samples y = S m + h themselves
// (decimation in time): the length-N/S y transform gives Z_h, with
//     X[k + q N/S] = sum_h exp(-2 pi i q h / S) w_N^(k h) Z_h[k],  k < N/S,
// and this pass stores T_h = w_N^(k h) Z_h as parity h of row k of the
// parity layout (chunks of PC columns, par_chunk; S = 4: PC = 2), which the
// z pass combines; the kx = N/2 column goes to row h N/S + k of its own
// array (S = 4: to (k / PC) 4 PC + h PC + k % PC, rows grouped as the
// columns).
template <typename T, int N, int NT, bool PAR, int PC = 2, int S = 2>
__device__ __forceinline__ void split_fwd_tail(Cx<T> *plane, const Cx<T> *__restrict__ tw, Cx<T> *sb, Cx<T> *nb,
                                               int h, int tid) {
    constexpr int H = N / 2, RS = H + 1, ROWS = N / S;
    static_assert(!PAR || ((PC == 1 || PC % 2 == 0) && H % PC == 0), "parity chunks that tile a row");
    static_assert(PAR || S == 2, "the frequency-decimated split is a two-parity one");
    for (int idx = tid; idx < ROWS * (H / 2 + 1); idx += NT) {
        const int y = idx / (H / 2 + 1), k = idx - y * (H / 2 + 1);
        if (!PAR && h) r2c_unpack<T, N, true>(plane + y * RS, k, tw, tw[y]);  // w_N^y of the parity split
        else r2c_unpack<T, N, false>(plane + y * RS, k, tw, Cx<T>{(T)1, (T)0});
    }
    __syncthreads();
    // y: complex FFT of length N/S down the N/2 + 1 columns
    fft_lds<T, ROWS, false, RS, RS, NT, N, SeqStride<1>>(plane, tw, tid);
    if constexpr (PAR) {
        for (int idx = tid; idx < ROWS * H / 2; idx += NT) {
            const int m = idx / (H / 2), kx = (idx - m * (H / 2)) * 2;
            Cx<T> v0 = plane[m * RS + kx], v1 = plane[m * RS + kx + 1];
            if (h) {
                const Cx<T> w = tw[m * h];
                v0 = v0 * w;
                v1 = v1 * w;
            }
            Cx<T> *o = sb + (size_t)m * (S * H) + (kx / PC) * (S * PC) + h * PC + kx % PC;
            if constexpr (PC == 1) {
                o[0] = v0;
                o[S] = v1;  // column kx + 1: the next chunk
            } else {
                gstore2<T>(o, v0, v1);
            }
        }
        for (int m = tid; m < ROWS; m += NT) {
            const int o = S == 4 ? (m / PC) * (4 * PC) + h * PC + m % PC : h * ROWS + m;
            nb[o] = h ? plane[m * RS + H] * tw[m * h] : plane[m * RS + H];
        }
    } else {
        for (int idx = tid; idx < ROWS * H / 2; idx += NT) {
            const int m = idx / (H / 2), kx = (idx - m * (H / 2)) * 2;
            gstore2<T>(sb + (size_t)(2 * m + h) * H + kx, plane[m * RS + kx], plane[m * RS + kx + 1]);
        }
        for (int m = tid; m < ROWS; m += NT) nb[2 * m + h] = plane[m * RS + H];
    }
}

// Waves per SIMD asked of the plane kernels: as many workgroups per CU as
// their LDS plane allows, capped at 4 waves per SIMD (at most 128 VGPRs).
template <typename T, int N, int S, int NT> constexpr int plane_min_waves() {
    constexpr size_t lds = (size_t)(N / S) * (N / 2 + (S == 1 ? 2 : 1)) * sizeof(Cx<T>) + (size_t)N * sizeof(Cx<T>) + 512;
    constexpr int per_cu = (int)((160 * 1024) / lds);
    constexpr int waves = per_cu * (NT / 256);
    return waves < 1 ? 1 : (waves > 4 ? 4 : waves);
}

// Block index -> (channel, z, parity).  Workgroups are dealt round-robin to
// the 8 XCDs (block b to XCD b mod 8, as the (b / 8)-th there), each with its
// own L2: the nch x S blocks of one z-plane (nch channels in the grid, S
// parities) take consecutive places on XCD z mod 8, so that the plane's
// phase image comes from HBM once for all channels and, for S = 2, the second
// parity's read of the plane's spectrum hits L2.  Grids whose N is not a
// multiple of 8 keep the channel-major order.
template <int N, int S> __device__ __forceinline__ void plane_of_block(int b, int &ch, int &z, int &h) {
    if constexpr (N % 8 == 0) {
        const int nch = (int)gridDim.x / (N * S), g = nch * S;
        const int x = b & 7, slot = b >> 3, zq = slot / g, r = slot - zq * g;
        z = zq * 8 + x;
        ch = r / S;
        h = r - ch * S;
    } else {
        static_assert(S == 1 || N % 8 == 0, "split planes need N % 8 == 0");
        ch = b / N;
        z = b - ch * N;
        h = 0;
    }
}

// ---------------------------------------------------------------------------
// P1: tau = (k - k0) e fused into the load; 2D R2C of the (ch, z) plane.
// With PHI the same pass transforms the flux k e for the equilibrium check.
// ---------------------------------------------------------------------------
template <typename T, int N, int S, int NT, bool PHI = false, int NC = 3, bool PAR = false, int PC = 2>
__global__ __launch_bounds__(NT, (plane_min_waves<T, N, S, NT>())) void k_fwd_plane(const T *__restrict__ e, const uint8_t *__restrict__ ph,
                                                  Cx<T> *__restrict__ spec, Cx<T> *__restrict__ nyq,
                                                  const Cx<T> *__restrict__ twg,
                                                  const DevParams *__restrict__ prm,
                                                  const DevState *__restrict__ st, int ch0) {
    // row pitch: even for whole planes (16-byte pair accesses, paired FFT
    // stages), N/2 + 1 for split planes
    constexpr int H = N / 2, RS = (S == 1) ? H + 2 : H + 1, ROWS = N / S, V = VecOf<T>::V, NN = N * N;
    // paired FFT stages: FP32 whole planes (an FP64 complex already fills a
    // 16-byte access, and pairs would double the registers of a butterfly)
    constexpr int PMX = (S == 1 && sizeof(T) == 4) ? kPairElem : kPairNone;
    constexpr int PMY = (S == 1 && sizeof(T) == 4) ? kPairSeq : kPairNone;
    static_assert(N % 4 == 0 && (S == 1 || S == 2 || (S == 4 && PAR)), "plane kernel needs N % 4 == 0");
    static_assert(!PAR || (S >= 2 && !PHI), "the parity layout is a split-plane forward pass");
    __shared__ Cx<T> plane[ROWS * RS];
    const int tid = threadIdx.x;
    int ch, z, h;
    plane_of_block<N, S>(blockIdx.x, ch, z, h);
    ch += ch0;  // the grid covers channels ch0 .. (all nine, or one load case's three)
    const int lc = ch / NC;
    // PHI: the flux k e of the equilibrium check (step 1); else tau = (k - k0) e
    // (augmented Lagrangian: the buffer already holds tau; elasticity: the
    // deviatoric channels take their own table)
    if (PHI ? !st->eq_pending[lc] : st->done[lc]) return;
    const bool dev = NC == 6 && ch % NC != 0;
    const double *lut = PHI ? prm->k : (dev ? prm->dk_dev : prm->dk);
    const bool tau_in = !PHI && (prm->scheme == 2 || prm->scheme == 4);
    const T d0 = tau_in ? (T)1 : (T)lut[0], d1 = tau_in ? (T)1 : (T)lut[1], d2 = tau_in ? (T)1 : (T)lut[2];
    const T tm = PHI ? (T)0 : (T)st->tau_mean[ch];  // only the discarded mean mode changes
    const T *eb = e + (size_t)ch * N * NN + (size_t)z * NN;
    const uint8_t *pb = ph + (size_t)z * NN;

    // load rows (S = 2: combine rows y and y + N/2 with sign (-1)^h; PAR:
    // the rows S y + h of parity h alone); each batch issues all of its
    // global loads before the first use
    constexpr int TOTL = ROWS * N / V, PERL = (TOTL + NT - 1) / NT;
    constexpr int BL = (S == 2 && !PAR) ? 4 : 8;
#pragma unroll
    for (int i0 = 0; i0 < PERL; i0 += BL) {
        T a[BL][V], b[BL][V];
        unsigned p[BL], q[BL];
#pragma unroll
        for (int i = 0; i < BL; ++i) {
            const int idx = tid + (i0 + i) * NT;
            if (i0 + i < PERL && (TOTL % NT == 0 || idx < TOTL)) {
                const int y = idx / (N / V), x = (idx - y * (N / V)) * V;
                const int ys = PAR ? S * y + h : y;
                vload<T>(eb + ys * N + x, a[i]);
                p[i] = pload<V>(pb + ys * N + x);
                if constexpr (S == 2 && !PAR) {
                    vload<T>(eb + (y + ROWS) * N + x, b[i]);
                    q[i] = pload<V>(pb + (y + ROWS) * N + x);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < BL; ++i) {
            const int idx = tid + (i0 + i) * NT;
            if (i0 + i < PERL && (TOTL % NT == 0 || idx < TOTL)) {
                const int y = idx / (N / V), x = (idx - y * (N / V)) * V;
                T u[V];
#pragma unroll
                for (int j = 0; j < V; ++j) {
                    u[j] = pick<T>(ph_at(p[i], j), d0, d1, d2) * a[i][j] - tm;
                    if constexpr (S == 2 && !PAR) {
                        const T t2 = pick<T>(ph_at(q[i], j), d0, d1, d2) * b[i][j] - tm;
                        u[j] = h ? u[j] - t2 : u[j] + t2;
                    }
                }
                if constexpr (V == 4) {
                    st_pair<T, RS % 2 == 0>(plane + y * RS + x / 2, Cx<T>{u[0], u[1]}, Cx<T>{u[2], u[3]});
                } else {
#pragma unroll
                    for (int j = 0; j < V; j += 2) plane[y * RS + (x + j) / 2] = Cx<T>{u[j], u[j + 1]};
                }
            }
        }
    }
    // twiddle table (length N) in LDS: short-latency loads inside the stages
    __shared__ Cx<T> tws[N];
    table_to_lds<T, N, NT>(tws, twg, tid);
    const Cx<T> *tw = tws;
    __syncthreads();
    // x: complex FFT of length N/2 of the packed even/odd samples
    fft_lds<T, H, false, ROWS, 1, NT, N, SeqStride<RS>, PMX>(plane, tw, tid);
    // unpack to the real-input spectrum X[0..N/2]
    Cx<T> *sb = spec + ((size_t)ch * N + z) * N * H;
    Cx<T> *nb = nyq + ((size_t)ch * N + z) * N;
    if constexpr (S == 1) {
        // whole plane: columns kx = 0 and N/2 are real, one complex column
        r2c_unpack_rows<T, N, ROWS, NT, true, RS>(plane, tw, tid);
        __syncthreads();
        fft_stages<T, ROWS, 0, num_stages(ROWS) - 1, false, H, RS, NT, N, SeqStride<1>, PMY>(plane, tw, tid);
        y_last_stage_store<T, N, NT, RS>(plane, tw, sb, nb, tid);
    } else {
        split_fwd_tail<T, N, NT, PAR, PC, S>(plane, tw, sb, nb, h, tid);
    }
}

// ---------------------------------------------------------------------------
// P2: z-FFT, Green operator (step 4), inverse z-FFT for one load case.
// Tiles: W consecutive kx of one ky (main), or W consecutive ky of the
// kx = N/2 column (nyq).  All three components sit in LDS together.
// ---------------------------------------------------------------------------
template <int N, int W> struct ZTiles {
    static constexpr int H = N / 2;
    static constexpr int MAIN = N * (H / W);
    static constexpr int NYQ = N / W;
    static constexpr int PER_LC = MAIN + NYQ;
};

// Tile of the t-th workgroup of a load case.  When a tile row is shorter than
// a 128-byte line, the tiles that share each line (neighbouring kx chunks of
// one ky, or neighbouring ky groups of the kx = N/2 column: two of 64-byte
// rows, four of 32-byte rows) go to workgroups 8 apart: workgroups are dealt
// round-robin to the 8 XCDs, so they run on one XCD and the repeated reads
// of the line hit its L2.  Within each block of 16 (pairs) or 32 (quads)
// workgroups this is a permutation, so every tile is taken once.
template <typename T, int N, int W> __device__ __forceinline__ int ztile_of(int t) {
    using TL = ZTiles<N, W>;
    constexpr int RB = W * (int)sizeof(Cx<T>);
    constexpr bool QUAD = RB <= 32 && TL::MAIN % 32 == 0 && TL::NYQ % 32 == 0 && (TL::H / W) % 4 == 0;
    constexpr bool PAIR = !QUAD && RB < 128 && TL::MAIN % 16 == 0 && TL::NYQ % 16 == 0 && (TL::H / W) % 2 == 0;
    if constexpr (QUAD) return (t & ~31) | ((t & 7) << 2) | ((t >> 3) & 3);
    if constexpr (PAIR) return (t & ~15) | ((t & 7) << 1) | ((t >> 3) & 1);
    return t;
}

// Tile of the t-th workgroup of a load case when the z pass reads a
// parity-layout spectrum: the tiles of rows ky and ky + N/2 read the same
// parity data of row ky mod N/2, and neighbouring kx tiles share 128-byte
// lines, so the four tiles {ky, ky + N/2} x {tiles 2j, 2j + 1} get
// workgroups 8 apart (one XCD, whose L2 then serves the repeated reads).
// The same for the Nyquist column's tiles of W rows.
template <int N, int W> constexpr bool ztile_par_ok() {
    return (N / 2 / W) % 2 == 0 && ZTiles<N, W>::MAIN % 32 == 0 && ZTiles<N, W>::NYQ % 32 == 0;
}
template <int N, int W> __device__ __forceinline__ int ztile_par(int b) {
    using TL = ZTiles<N, W>;
    constexpr int H = N / 2, C = H / W;
    static_assert(ztile_par_ok<N, W>(), "parity tiles come in groups of 32");
    const bool main = b < TL::MAIN;
    const int bb = main ? b : b - TL::MAIN;
    const int lane = bb & 7, q = (bb >> 3) & 3, quad = (bb >> 5) * 8 + lane;
    if (main) {
        const int kyp = quad / (C / 2), j = quad - kyp * (C / 2);
        return (kyp + (q >> 1) * H) * C + 2 * j + (q & 1);
    }
    return TL::MAIN + 2 * quad + (q & 1) + (q >> 1) * C;
}

// z * exp(2 pi i s / 4), a quarter turn s mod 4 (exact: a swap and signs)
template <int QS, typename T> __device__ __forceinline__ Cx<T> quarter_turn(Cx<T> v) {
    constexpr int s = QS & 3;
    if constexpr (s == 0) return v;
    else if constexpr (s == 1) return Cx<T>{-v.y, v.x};
    else if constexpr (s == 2) return Cx<T>{-v.x, -v.y};
    else return Cx<T>{v.y, -v.x};
}

// sum_h exp(SGN 2 pi i K h / SP) v[h] with K fixed (a DFT of length SP = 2 or
// 4 at one output index: sums of swapped and negated inputs)
template <int SP, int K, int SGN, typename T> __device__ __forceinline__ Cx<T> parity_sum(const Cx<T> *v) {
    Cx<T> x = v[0];
    if constexpr (SP > 1) x = x + quarter_turn<SGN * (4 / SP) * K * 1>(v[1]);
    if constexpr (SP > 2) x = x + quarter_turn<SGN * (4 / SP) * K * 2>(v[2]);
    if constexpr (SP > 3) x = x + quarter_turn<SGN * (4 / SP) * K * 3>(v[3]);
    return x;
}

// First stage of a length-N transform (forward, or inverse with INV) of a
// tile of NCOMP x W pencils, its inputs read straight from global memory:
// butterfly b = j NCOMP W + q takes elements j + r N/R of pencil q
// (component q / W at cstride, column q % W at wstride, elements at
// estride), neighbouring threads neighbouring pencils.  finish() runs the
// radix-R DFTs (stage 0 has no twiddles) and writes the outputs to LDS
// (pencil q at (q / W) N W + q % W, element stride W) in the self-sorting
// order of stage 0.
template <typename T, int N, int W, int NT, int NCOMP = 3, bool INV = false> struct ZFirstStage {
    static constexpr int NSEQ = NCOMP * W, NW = N * W, R = radix_of(N, 0), NB = N / R, TOT = NSEQ * NB,
                         PER = (TOT + NT - 1) / NT;
    Cx<T> v[PER][R];
    __device__ __forceinline__ void load(const Cx<T> *base, size_t cstride, size_t estride, int tid,
                                         size_t wstride = 1) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int b = tid + i * NT;
            if (TOT % NT == 0 || b < TOT) {
                const int j = b / NSEQ, q = b - j * NSEQ, c = q / W, w = q - c * W;
#pragma unroll
                for (int r = 0; r < R; ++r) v[i][r] = base[c * cstride + (j + r * NB) * estride + w * wstride];
            }
        }
    }
    __device__ __forceinline__ void finish(Cx<T> *buf, int tid) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int b = tid + i * NT;
            if (TOT % NT == 0 || b < TOT) {
                const int j = b / NSEQ, q = b - j * NSEQ, c = q / W, w = q - c * W;
                dft<T, R, INV>(v[i]);
#pragma unroll
                for (int r = 0; r < R; ++r) buf[c * NW + w + (j * R + r) * W] = v[i][r];
            }
        }
        __syncthreads();
    }
};

// Last stage of a length-N transform (inverse, or forward without INV) of a
// tile of pencils, its outputs stored straight to global memory (the layouts
// of ZFirstStage).
template <typename T, int N, int W, int NT, int NCOMP = 3, bool INV = true>
__device__ __forceinline__ void z_last_stage_store(const Cx<T> *buf, const Cx<T> *__restrict__ tw, Cx<T> *base,
                                                   size_t cstride, size_t estride, int tid, size_t wstride = 1) {
    constexpr int NSEQ = NCOMP * W, NW = N * W, SL = num_stages(N) - 1, R = radix_of(N, SL), NS = ns_before(N, SL),
                  NB = N / R, TOT = NSEQ * NB, PER = (TOT + NT - 1) / NT, TWS = N / (NS * R);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int b = tid + i * NT;
        if (TOT % NT == 0 || b < TOT) {
            const int j = b / NSEQ, q = b - j * NSEQ, c = q / W, w = q - c * W;
            Cx<T> v[R];
#pragma unroll
            for (int r = 0; r < R; ++r) v[r] = buf[c * NW + w + (j + r * NB) * W];
            const int k = j % NS, d = (j - k) * R + k;
            if constexpr (NS > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) v[r] = twmul<T, INV>(v[r], tw[r * k * TWS]);
            }
            dft<T, R, INV>(v);
#pragma unroll
            for (int r = 0; r < R; ++r) base[c * cstride + (d + r * NS) * estride + w * wstride] = v[r];
        }
    }
}

// With red_nper > 0 the first workgroup instead runs the reduction of the
// previous inverse pass's partials (nper per channel) while the others do
// the tiles.  The tiles then read the convergence flags as of the iteration
// before: a load case that has just converged may be transformed once more,
// which is harmless (its spectrum is not used again).
// Waves per SIMD asked of the z pass: six for FP32 128^3 (8-column tiles,
// six workgroups per CU fit in LDS; measured faster despite a few spills),
// otherwise no bound.
// z pass with its first and last stages on the pencils in global memory:
// measured faster at every grid but FP32 256^3 and 512^3 (1-2 %).
template <typename T, int N> constexpr bool zpass_direct() { return !(sizeof(T) == 4 && N >= 256); }

template <typename T, int N, int W> constexpr int zpass_min_waves() {
    return (sizeof(T) == 4 && N == 128 && W == 8) ? 6 : 1;
}

// PAR: the forward spectrum arrives in the parity layout of split_fwd_tail
// (specB, nyqB).  SP = 2: the tile of row ky reads both parities E, w O of
// row ky mod N/2 (neighbouring chunks of one row in specB; rows ky mod N/2
// and N/2 + ky mod N/2 in nyqB) and forms X[ky] = E +- w O (+ for ky < N/2)
// as it loads; the result goes to spec / nyq in the plain layout.  SP = 4
// (W = 4 CW, CW = 2 in FP32, 1 in FP64): a tile holds CW columns
// kx0 .. kx0 + CW - 1 (or CW rows of the kx = N/2 column) of row k < N/4 in
// all four quarters ky = k + q N/4, W pencils per component ordered
// p = 4 w + q.  It reads the four parities of its columns (one 64-byte run
// per z and component: the parity layout's chunks are CW columns), forms
// X_q = sum_h exp(-2 pi i q h / 4) T_h (a length-4 DFT per column) in LDS,
// and writes the result in the quarter layout that the quarter-plane pass
// reads: element (q, k, kx) at k 2N + 4 kx + q (kx = N/2 column: 4 k + q),
// again one 64-byte run per z and component.
template <typename T, int N, int W, int NT, bool PAR = false, int SP = 2>
__global__ __launch_bounds__(NT, (zpass_min_waves<T, N, W>())) void k_zgreen(Cx<T> *__restrict__ spec, Cx<T> *__restrict__ nyq,
                                               const Cx<T> *__restrict__ twg,
                                               const DevParams *__restrict__ prm,
                                               DevState *__restrict__ st, const double *__restrict__ part,
                                               int red_nper, double *__restrict__ hist, int lc0,
                                               const Cx<T> *__restrict__ specB, const Cx<T> *__restrict__ nyqB) {
    using TL = ZTiles<N, W>;
    constexpr int H = N / 2, NW = N * W;
    constexpr bool Q4 = PAR && SP == 4;
    static_assert(H % W == 0 && N % W == 0 && W % 2 == 0, "tile width must be even and divide N/2");
    static_assert(SP == 2 || (Q4 && (W == 8 || W == 4) && N % 8 == 0),
                  "four parities: tiles of W / 4 columns x 4 quarters");
    constexpr int CW = Q4 ? W / 4 : 1;  // Q4: columns (or kx = N/2 rows) per tile
    static_assert(NT == 256, "the merged reduction runs on a 256-thread workgroup");
    __shared__ Cx<T> buf[3 * NW];
    const int tid = threadIdx.x;
    if (red_nper > 0 && blockIdx.x == 0) {
        reduce_block(part, red_nper, prm, st, hist, tid);
        return;
    }
    const int bt = blockIdx.x - (red_nper > 0 ? 1 : 0);
    const int lt = bt / TL::PER_LC;
    int t;
    if constexpr (PAR && !Q4) t = ztile_par<N, W>(bt - lt * TL::PER_LC);
    else t = ztile_of<T, N, W>(bt - lt * TL::PER_LC);
    const int lc = lc0 + lt;  // the grid covers load cases lc0 .. (all three, or one)
    // the freeze flag, read once for the workgroup (the merged reduction of
    // workgroup 0 may write it meanwhile) so that every wave takes the same
    // exit; a load case frozen during this pass may leave its spectrum
    // unprocessed, which is harmless (it is not read again)
    __shared__ int s_done;
    if (tid == 0) s_done = __hip_atomic_load(&st->done[lc], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (s_done) return;
    Cx<T> *base;
    const Cx<T> *pbase = nullptr;  // PAR: row ky mod N/2 of the parity layout
    size_t cstride, zstride, poff = 0;  // poff: from parity 0 to parity 1
    int kx0, ky0, dkx, dky;  // kx(w) = kx0 + dkx*w, ky(w) = ky0 + dky*w
    if constexpr (Q4) {
        // the same offset in both layouts: parity layout k 2N + 4 CW j +
        // CW h + w, quarter layout k 2N + 4 CW j + 4 w + q (j: the tile's
        // group of CW columns)
        if (t < TL::MAIN) {
            const int k = t / (H / CW), j = t - k * (H / CW);
            kx0 = CW * j;
            ky0 = k;
            dkx = 1;
            dky = 0;
            const size_t off = (size_t)(3 * lc) * N * N * H + (size_t)k * (4 * H) + 4 * CW * j;
            base = spec + off;
            pbase = specB + off;
            cstride = (size_t)N * N * H;
            zstride = (size_t)N * H;
        } else {
            const int j = t - TL::MAIN;
            kx0 = H;
            ky0 = CW * j;
            dkx = 0;
            dky = 1;
            const size_t off = (size_t)(3 * lc) * N * N + 4 * CW * j;
            base = nyq + off;
            pbase = nyqB + off;
            cstride = (size_t)N * N;
            zstride = N;
        }
    } else if (t < TL::MAIN) {
        const int ky = t / (H / W);
        kx0 = (t - ky * (H / W)) * W;
        ky0 = ky;
        dkx = 1;
        dky = 0;
        base = spec + (size_t)(3 * lc) * N * N * H + (size_t)ky * H + kx0;
        // the parity layout: row ky mod N/2, the tile's chunk, parity 0 and
        // (poff further) parity 1
        constexpr int PC = par_chunk<T, W>();
        static_assert(!PAR || (PC % W == 0 && H % PC == 0), "z tiles inside parity chunks");
        if constexpr (PAR)
            pbase = specB + (size_t)(3 * lc) * N * N * H + (size_t)(ky % H) * N + (kx0 / PC) * (2 * PC) + kx0 % PC;
        poff = PC;
        cstride = (size_t)N * N * H;
        zstride = (size_t)N * H;
    } else {
        kx0 = H;
        ky0 = (t - TL::MAIN) * W;
        dkx = 0;
        dky = 1;
        base = nyq + (size_t)(3 * lc) * N * N + ky0;
        if constexpr (PAR) pbase = nyqB + (size_t)(3 * lc) * N * N + (ky0 % H);
        poff = H;
        cstride = (size_t)N * N;
        zstride = N;
    }
    // the three components' pencils straight to the registers of the first
    // z stage, and the last inverse stage straight back (except FP32 from
    // 256^3 on, measured faster with the pencils staged through LDS)
    // the parity layout is read through the staged load
    constexpr bool DIRECT = zpass_direct<T, N>() && !PAR;
    constexpr int NP = 3 * NW / 2, PERP = (NP + NT - 1) / NT;
    ZFirstStage<T, N, W, NT> z0;
    if constexpr (DIRECT) {
        z0.load(base, cstride, zstride, tid);
    } else if constexpr (PAR && !Q4) {
        // X = E +- w O from the two parity rows, in batches of loads
        const bool upper = ky0 >= H;  // a tile's rows lie in one half (W divides N/2)
        constexpr int BP = 6;
#pragma unroll
        for (int i0 = 0; i0 < PERP; i0 += BP) {
            Cx<T> va[BP], vb[BP], ua[BP], ub[BP];
#pragma unroll
            for (int i = 0; i < BP; ++i) {
                const int idx = tid + (i0 + i) * NT;
                if (i0 + i < PERP && (NP % NT == 0 || idx < NP)) {
                    const int e0 = 2 * idx, c = e0 / NW, r = e0 - c * NW, zz = r / W, w = r - zz * W;
                    const Cx<T> *src = pbase + c * cstride + zz * zstride + w;
                    gload2<T>(src, va[i], vb[i]);
                    gload2<T>(src + poff, ua[i], ub[i]);
                }
            }
#pragma unroll
            for (int i = 0; i < BP; ++i) {
                const int idx = tid + (i0 + i) * NT;
                if (i0 + i < PERP && (NP % NT == 0 || idx < NP)) {
                    buf[2 * idx] = upper ? va[i] - ua[i] : va[i] + ua[i];
                    buf[2 * idx + 1] = upper ? vb[i] - ub[i] : vb[i] + ub[i];
                }
            }
        }
    } else {
        // two complex values per access, every load of a thread in flight
        // before the first LDS store (Q4: the raw parities, combined below)
        const Cx<T> *src = Q4 ? pbase : base;
        Cx<T> va[PERP], vb[PERP];
#pragma unroll
        for (int i = 0; i < PERP; ++i) {
            const int idx = tid + i * NT;
            if (NP % NT == 0 || idx < NP) {
                const int e0 = 2 * idx, c = e0 / NW, r = e0 - c * NW, zz = r / W, w = r - zz * W;
                gload2<T>(src + c * cstride + zz * zstride + w, va[i], vb[i]);
            }
        }
#pragma unroll
        for (int i = 0; i < PERP; ++i) {
            const int idx = tid + i * NT;
            if (NP % NT == 0 || idx < NP) {
                buf[2 * idx] = va[i];
                buf[2 * idx + 1] = vb[i];
            }
        }
    }
    // twiddle table (length N) in LDS: short-latency loads inside the stages
    __shared__ Cx<T> tws[N];
    table_to_lds<T, N, NT>(tws, twg, tid);
    const Cx<T> *tw = tws;
    if constexpr (DIRECT) {
        z0.finish(buf, tid);
        fft_stages<T, N, 1, num_stages(N), false, 3 * W, W, NT, N, SeqBlocked<W, NW>, kPairNone>(buf, tw, tid);
    } else {
        __syncthreads();
        if constexpr (Q4) {
            // per (component, z) row: slots CW h + w -> 4 w + q, X_q the
            // length-4 DFT over h of column w
            for (int row = tid; row < 3 * N; row += NT) {
                Cx<T> v[W];
#pragma unroll
                for (int i = 0; i < W; ++i) v[i] = buf[row * W + i];
#pragma unroll
                for (int w = 0; w < CW; ++w) {
                    Cx<T> a[4];
#pragma unroll
                    for (int hh = 0; hh < 4; ++hh) a[hh] = v[CW * hh + w];
                    dft4<T, false>(a);
#pragma unroll
                    for (int q = 0; q < 4; ++q) buf[row * W + 4 * w + q] = a[q];
                }
            }
            __syncthreads();
        }
        fft_lds<T, N, false, 3 * W, W, NT, N, SeqBlocked<W, NW>>(buf, tw, tid);
    }
    const T sc = (T)prm->inv_k0M;
    // the dual scheme takes G* = I - P, P the projection on the fields whose
    // divergence vanishes for every sign of the Nyquist components (Nyquist
    // components pass unchanged, the others see xi_A xi_A^T / |xi_A|^2 with
    // xi_A the non-Nyquist part of xi)
    const bool dual = prm->scheme == 3;
    for (int idx = tid; idx < NW; idx += NT) {
        const int kz = idx / W, p = idx - kz * W;
        // Q4: pencil p = 4 w + q in quarter q of the rows
        const int w = Q4 ? p >> 2 : p, qq = Q4 ? p & 3 : 0;
        const int ki[3] = {kx0 + dkx * w, ky0 + dky * w + qq * (N / 4), kz};
        T xi[3];
        bool nq[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            nq[d] = (ki[d] == H);
            xi[d] = (T)(ki[d] <= H ? ki[d] : ki[d] - N);
        }
        Cx<T> tv[3] = {buf[idx], buf[NW + idx], buf[2 * NW + idx]};
        Cx<T> out[3];
        if (ki[0] == 0 && ki[1] == 0 && ki[2] == 0) {
            // step 4 pins the mean to E; E is added after the inverse
            // transform instead (exact), so the mean mode carries 0 here
#pragma unroll
            for (int c = 0; c < 3; ++c) out[c] = Cx<T>{(T)0, (T)0};
        } else {
            Cx<T> sA = {(T)0, (T)0};
            T a2 = (T)0;
#pragma unroll
            for (int d = 0; d < 3; ++d)
                if (!nq[d]) {
                    sA = sA + scale(tv[d], xi[d]);
                    a2 += xi[d] * xi[d];
                }
            if (dual) {
                const T fa = a2 > (T)0 ? -sc / a2 : (T)0;
#pragma unroll
                for (int c = 0; c < 3; ++c) out[c] = nq[c] ? scale(tv[c], -sc) : scale(sA, fa * xi[c]);
            } else {
                const T x2 = xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2];
                const T f = -sc / x2;
#pragma unroll
                for (int c = 0; c < 3; ++c) out[c] = scale(nq[c] ? scale(tv[c], xi[c]) : sA, f * xi[c]);
            }
        }
        buf[idx] = out[0];
        buf[NW + idx] = out[1];
        buf[2 * NW + idx] = out[2];
    }
    __syncthreads();
    if constexpr (DIRECT) {
        fft_stages<T, N, 0, num_stages(N) - 1, true, 3 * W, W, NT, N, SeqBlocked<W, NW>, kPairNone>(buf, tw, tid);
        z_last_stage_store<T, N, W, NT>(buf, tw, base, cstride, zstride, tid);
    } else {
        fft_lds<T, N, true, 3 * W, W, NT, N, SeqBlocked<W, NW>>(buf, tw, tid);
        for (int idx = tid; idx < NP; idx += NT) {
            const int e0 = 2 * idx, c = e0 / NW, r = e0 - c * NW, zz = r / W, w = r - zz * W;
            gstore2<T>(base + c * cstride + zz * zstride + w, buf[e0], buf[e0 + 1]);
        }
    }
}

// One DPP step on an FP64 value (both 32-bit halves): lanes the pattern
// does not feed, or whose row is masked off, receive 0.
template <int CTRL, int ROWS> __device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Fixed-order sum over a wave of 64 lanes in registers (no LDS traffic):
// row shifts by 1, 2, 4 and 8 leave each 16-lane row's prefix sums, the
// broadcasts of lanes 15 and 31 carry them across rows.  The total is in
// lane 63.
__device__ __forceinline__ double wave_sum_f64(double v) {
    v += dpp_f64<0x111, 0xf>(v);  // row_shr:1
    v += dpp_f64<0x112, 0xf>(v);  // row_shr:2
    v += dpp_f64<0x114, 0xf>(v);  // row_shr:4
    v += dpp_f64<0x118, 0xf>(v);  // row_shr:8
    v += dpp_f64<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_f64<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

// FP64 block sums of NV values; results valid in thread 0.  red holds
// NV * (NT / 64) doubles.
template <int NT, int NV> __device__ __forceinline__ void block_sum(double *v, double *red) {
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = wave_sum_f64(v[q]);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 63)
        for (int q = 0; q < NV; ++q) red[NV * wv + q] = v[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 0; q < NV; ++q) {
            double t = 0.0;
            for (int i = 0; i < NT / 64; ++i) t += red[NV * i + q];
            v[q] = t;
        }
    }
}

template <int NT> __device__ __forceinline__ void block_sum2(double &a, double &b, double *red) {
    double v[2] = {a, b};
    block_sum<NT, 2>(v, red);
    a = v[0];
    b = v[1];
}

// Equilibrium error of step 1 (option): after P1<PHI> the z-FFT of the flux
// spectrum, then per block sum' |xi . phi^|^2 / |xi|^2 over the modes where
// the sign-averaged operator is the projection on xi (no Nyquist component,
// or a single Nyquist component and nothing else), each half-spectrum mode
// counted with its Hermitian partner, and |phi^(0)|^2 from the tile holding
// mode 0.  Partials: peq[lc][tile] = {num, den}.
template <typename T, int N, int W, int NT>
__global__ __launch_bounds__(NT) void k_zeq(const Cx<T> *__restrict__ spec, const Cx<T> *__restrict__ nyq,
                                            const Cx<T> *__restrict__ twg, const DevState *__restrict__ st,
                                            double *__restrict__ peq) {
    using TL = ZTiles<N, W>;
    constexpr int H = N / 2, NW = N * W;
    __shared__ Cx<T> buf[3 * NW];
    __shared__ double red[2 * (NT / 64)];
    const int tid = threadIdx.x;
    const int lc = blockIdx.x / TL::PER_LC, t = ztile_of<T, N, W>(blockIdx.x - lc * TL::PER_LC);
    if (!st->eq_pending[lc]) return;
    const Cx<T> *base;
    size_t cstride, zstride;
    int kx0, ky0, dkx, dky;
    if (t < TL::MAIN) {
        const int ky = t / (H / W);
        kx0 = (t - ky * (H / W)) * W;
        ky0 = ky;
        dkx = 1;
        dky = 0;
        base = spec + (size_t)(3 * lc) * N * N * H + (size_t)ky * H + kx0;
        cstride = (size_t)N * N * H;
        zstride = (size_t)N * H;
    } else {
        kx0 = H;
        ky0 = (t - TL::MAIN) * W;
        dkx = 0;
        dky = 1;
        base = nyq + (size_t)(3 * lc) * N * N + ky0;
        cstride = (size_t)N * N;
        zstride = N;
    }
    for (int idx = tid; idx < 3 * NW; idx += NT) {
        const int c = idx / NW, r = idx - c * NW, zz = r / W, w = r - zz * W;
        buf[idx] = base[c * cstride + zz * zstride + w];
    }
    // twiddle table (length N) in LDS: short-latency loads inside the stages
    __shared__ Cx<T> tws[N];
    table_to_lds<T, N, NT>(tws, twg, tid);
    const Cx<T> *tw = tws;
    __syncthreads();
    fft_lds<T, N, false, 3 * W, W, NT, N, SeqBlocked<W, NW>>(buf, tw, tid);
    double num = 0.0, den = 0.0;
    for (int idx = tid; idx < NW; idx += NT) {
        const int kz = idx / W, w = idx - kz * W;
        const int ki[3] = {kx0 + dkx * w, ky0 + dky * w, kz};
        Cx<double> v[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const Cx<T> q = buf[c * NW + idx];
            v[c] = Cx<double>{(double)q.x, (double)q.y};
        }
        if (ki[0] == 0 && ki[1] == 0 && ki[2] == 0) {
            den = v[0].x * v[0].x + v[0].y * v[0].y + v[1].x * v[1].x + v[1].y * v[1].y +
                  v[2].x * v[2].x + v[2].y * v[2].y;
            continue;
        }
        int nnyq = 0, nreg = 0;
        double xi[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (ki[d] == H) ++nnyq;
            else if (ki[d] != 0) ++nreg;
            xi[d] = (double)(ki[d] <= H ? ki[d] : ki[d] - N);
        }
        if (!(nnyq == 0 || (nnyq == 1 && nreg == 0))) continue;
        const double dr = xi[0] * v[0].x + xi[1] * v[1].x + xi[2] * v[2].x;
        const double di = xi[0] * v[0].y + xi[1] * v[1].y + xi[2] * v[2].y;
        const double wgt = (ki[0] == 0 || ki[0] == H) ? 1.0 : 2.0;  // Hermitian partner
        num += wgt * (dr * dr + di * di) / (xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]);
    }
    block_sum2<NT>(num, den, red);
    if (tid == 0) {
        peq[((size_t)lc * TL::PER_LC + t) * 2] = num;
        peq[((size_t)lc * TL::PER_LC + t) * 2 + 1] = den;
    }
}

// First stage of the inverse y transform of a whole plane (S = 1), its inputs
// read straight from the spectrum rows in global memory rather than staged
// through LDS: butterfly b = j H + q takes rows j + r N/R of column q, so
// neighbouring threads read neighbouring columns (coalesced).  load() issues
// the reads; finish() (after a barrier that published LDS column H) forms
// column 0 as Y0 + i YH from the kx = N/2 column held in LDS column H, which
// no stage writes, runs the radix-R DFTs (stage 0 has no twiddles) and writes
// the outputs to LDS in the self-sorting order of stage 0.  The caller runs
// the later stages.
template <typename T, int N, int NT, int RS> struct YFirstStage {
    static constexpr int H = N / 2, R = radix_of(N, 0), NB = N / R, TOT = H * NB, PER = (TOT + NT - 1) / NT;
    Cx<T> v[PER][R];
    __device__ __forceinline__ void load(const Cx<T> *__restrict__ sb, int tid) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int b = tid + i * NT;
            if (TOT % NT == 0 || b < TOT) {
                const int j = b / H, q = b - j * H;
#pragma unroll
                for (int r = 0; r < R; ++r) v[i][r] = sb[(size_t)(j + r * NB) * H + q];
            }
        }
    }
    __device__ __forceinline__ void finish(Cx<T> *plane, int tid) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int b = tid + i * NT;
            if (TOT % NT == 0 || b < TOT) {
                const int j = b / H, q = b - j * H;
                if (q == 0) {
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const Cx<T> yh = plane[(j + r * NB) * RS + H];
                        v[i][r] = Cx<T>{v[i][r].x - yh.y, v[i][r].y + yh.x};
                    }
                }
                dft<T, R, true>(v[i]);
#pragma unroll
                for (int r = 0; r < R; ++r) plane[(j * R + r) * RS + q] = v[i][r];
            }
        }
        __syncthreads();
    }
};

// ---------------------------------------------------------------------------
// P3: 2D C2R of the (ch, z) plane, then steps 6-7 and the flux, fused.
// ---------------------------------------------------------------------------
// FWD: the same workgroup then forms tau = (k - k0) e+ of the next
// iteration from the updated values it holds, runs the forward 2D R2C of
// pass 1 and writes the plane's next spectrum -- one read and one write of
// the plane per iteration instead of two of each.  Whole planes (S = 1)
// overwrite their spectrum in place; split planes (S = 2), each of whose
// two workgroups reads the whole plane's spectrum, write the parity layout
// of split_fwd_tail to specB / nyqB instead.  The mean subtracted from tau
// is the previous iteration's (any constant is exact: the mean mode of tau
// is replaced by E).
// UPD: the update of steps 6-7: 0 accelerated (and basic), 1 augmented
// Lagrangian / polarization, 2 dual.
// The value of the neighbouring lane within each pair (lanes 2j <-> 2j + 1,
// a DPP quad permutation [1, 0, 3, 2]).
__device__ __forceinline__ float dpp_quad_swap1(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xf, 0xf, false));
}
__device__ __forceinline__ double dpp_quad_swap1(double v) {
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(x >> 32), 0xB1, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Load of a split plane's parity HP of S from the half spectrum (main
// columns, two complex values per access, all loads of a batch in flight
// before the LDS stores; the kx = N/2 column into LDS column N/2): row
// m < N/S gets Y[m] = w_N^(-m HP) sum_q exp(2 pi i q HP / S) X[m + q N/S] (a
// decimation in frequency), whose length-N/S inverse transform gives the
// rows y = S m' + HP of the plane.  S = 2 reads the plain layout (rows
// m + q N/2), S = 4 the quarter layout of the z pass (X[m + q N/4][kx] at
// m 2N + 4 kx + q, the kx = N/2 column at 4 m + q): the eight values of a
// column pair in one 64-byte run.
template <typename T, int N, int S, int NT, int RS, int HP>
__device__ __forceinline__ void split_inv_load(Cx<T> *plane, const Cx<T> *__restrict__ sb,
                                               const Cx<T> *__restrict__ nb, const Cx<T> *__restrict__ twg,
                                               int tid) {
    constexpr int H = N / 2, ROWS = N / S;
    if constexpr (S == 4) {
        // 16-byte units u of row m in lane order (each load instruction one
        // contiguous run): unit u holds quarters 2b, 2b + 1 (b = u & 1) of
        // column u / 2, so the four lanes of a quad hold one column pair.
        // Each lane forms its two quarters' share of the sum,
        // (-1)^(b HP) (X_2b + i^HP X_2b+1), and adds its neighbour's (lane
        // b ^ 1) by a DPP swap; lanes b = 0 store the column.
        constexpr int NU = ROWS * 2 * H, PERU = NU / NT, BU = 8;
        static_assert(NU % NT == 0 && PERU % BU == 0 && NT % 64 == 0 && (2 * H) % 4 == 0,
                      "units of a row in whole quads");
        const int b = tid & 1;  // u = tid (mod 4): NT and the row's 2 H units are multiples of 4
#pragma unroll
        for (int i0 = 0; i0 < PERU; i0 += BU) {
            Cx<T> lo[BU], hi[BU];
#pragma unroll
            for (int i = 0; i < BU; ++i) {
                const int idx = tid + (i0 + i) * NT, m = idx / (2 * H), u = idx - m * (2 * H);
                gload2<T>(sb + (size_t)m * (4 * H) + 2 * u, lo[i], hi[i]);
            }
#pragma unroll
            for (int i = 0; i < BU; ++i) {
                const int idx = tid + (i0 + i) * NT, m = idx / (2 * H), u = idx - m * (2 * H);
                Cx<T> pp = lo[i] + quarter_turn<HP>(hi[i]);
                if ((HP & 1) && b) pp = Cx<T>{-pp.x, -pp.y};
                Cx<T> y = pp + Cx<T>{dpp_quad_swap1(pp.x), dpp_quad_swap1(pp.y)};
                if constexpr (HP > 0) y = y * conj(twg[m * HP]);
                if (!b) plane[m * RS + (u >> 1)] = y;
            }
        }
    } else {
        constexpr int NP = ROWS * H / 2, PERP = (NP + NT - 1) / NT, BP = 4;
#pragma unroll
        for (int i0 = 0; i0 < PERP; i0 += BP) {
            Cx<T> va[BP][S], vb[BP][S];
#pragma unroll
            for (int i = 0; i < BP; ++i) {
                const int idx = tid + (i0 + i) * NT;
                if (i0 + i < PERP && (NP % NT == 0 || idx < NP)) {
                    const int m = idx / (H / 2), kx = (idx - m * (H / 2)) * 2;
#pragma unroll
                    for (int q = 0; q < S; ++q) gload2<T>(sb + (size_t)(m + q * ROWS) * H + kx, va[i][q], vb[i][q]);
                }
            }
#pragma unroll
            for (int i = 0; i < BP; ++i) {
                const int idx = tid + (i0 + i) * NT;
                if (i0 + i < PERP && (NP % NT == 0 || idx < NP)) {
                    const int m = idx / (H / 2), kx = (idx - m * (H / 2)) * 2;
                    Cx<T> a0 = parity_sum<S, HP, 1>(va[i]), a1 = parity_sum<S, HP, 1>(vb[i]);
                    if constexpr (HP > 0) {
                        const Cx<T> r = conj(twg[m * HP]);
                        a0 = a0 * r;
                        a1 = a1 * r;
                    }
                    st_pair<T, RS % 2 == 0>(plane + m * RS + kx, a0, a1);
                }
            }
        }
    }
    for (int m = tid; m < ROWS; m += NT) {
        Cx<T> v[S];
#pragma unroll
        for (int q = 0; q < S; ++q) v[q] = S == 4 ? nb[4 * m + q] : nb[m + q * ROWS];
        const Cx<T> x = parity_sum<S, HP, 1>(v);
        plane[m * RS + H] = HP > 0 ? x * conj(twg[m * HP]) : x;
    }
}

template <typename T, int N, int S, int NT, bool FWD = false, int UPD = 0, int NC = 3, int PC = 2, int PS = S>
__global__ __launch_bounds__(NT, (plane_min_waves<T, N, S, NT>())) void k_inv_plane(T *__restrict__ e, const uint8_t *__restrict__ ph,
                                                  Cx<T> *__restrict__ spec,
                                                  Cx<T> *__restrict__ nyq,
                                                  const Cx<T> *__restrict__ twg,
                                                  const DevParams *__restrict__ prm,
                                                  const DevState *__restrict__ st,
                                                  double *__restrict__ part, int ch0,
                                                  Cx<T> *__restrict__ specB, Cx<T> *__restrict__ nyqB) {
    // row pitch: even for whole planes (16-byte pair accesses, paired FFT
    // stages), N/2 + 1 for split planes
    constexpr int H = N / 2, RS = (S == 1) ? H + 2 : H + 1, ROWS = N / S, V = VecOf<T>::V, NN = N * N;
    // paired FFT stages: FP32 whole planes (an FP64 complex already fills a
    // 16-byte access, and pairs would double the registers of a butterfly)
    constexpr int PMX = (S == 1 && sizeof(T) == 4) ? kPairElem : kPairNone;
    constexpr int PMY = (S == 1 && sizeof(T) == 4) ? kPairSeq : kPairNone;
    // S = 1: column kx = 0 becomes Y0 + i YH with YH the kx = N/2 column, one
    // complex column for the y transform (both are transforms of real
    // columns, so the inverse separates them exactly)
    __shared__ Cx<T> plane[ROWS * RS];
    __shared__ double red[3 * (NT / 64)];
    const int tid = threadIdx.x;
    int ch, z, h;
    plane_of_block<N, S>(blockIdx.x, ch, z, h);
    ch += ch0;  // the grid covers channels ch0 .. (all nine, or one load case's three)
    const int lc = ch / NC;
    if (st->done[lc]) return;
    // E_comp of this channel (ch = NC lc + comp; E of load case lc is the unit
    // vector or basis tensor lc)
    const T ec = (ch % (NC + 1) == 0) ? (T)1 : (T)0;
    // per-phase tables: the conductivities, or (elasticity) those of the
    // hydrostatic channel or of the deviatoric ones
    const bool dev = NC == 6 && ch % NC != 0;
    const double *pk = dev ? prm->k_dev : prm->k;
    const double *pdk = dev ? prm->dk_dev : prm->dk;
    const double *pw = dev ? prm->w_dev : prm->w;
    const double k0c = dev ? prm->k0_dev : prm->k0;

    const Cx<T> *sb = spec + ((size_t)ch * N + z) * N * H;
    const Cx<T> *nb = nyq + ((size_t)ch * N + z) * N;
    YFirstStage<T, N, NT, RS> y0;
    if constexpr (S == 1) {
        // the main columns straight to the registers of the first y stage,
        // the kx = N/2 column into LDS column H
        y0.load(sb, tid);
        for (int m = tid; m < ROWS; m += NT) plane[m * RS + H] = nb[m];
    } else {
        // parity h, a compile-time constant in the loads' combination
        if constexpr (S == 2) {
            if (h) split_inv_load<T, N, S, NT, RS, 1>(plane, sb, nb, twg, tid);
            else split_inv_load<T, N, S, NT, RS, 0>(plane, sb, nb, twg, tid);
        } else {
            switch (h) {
            case 0: split_inv_load<T, N, S, NT, RS, 0>(plane, sb, nb, twg, tid); break;
            case 1: split_inv_load<T, N, S, NT, RS, 1>(plane, sb, nb, twg, tid); break;
            case 2: split_inv_load<T, N, S, NT, RS, 2>(plane, sb, nb, twg, tid); break;
            default: split_inv_load<T, N, S, NT, RS, 3>(plane, sb, nb, twg, tid); break;
            }
        }
    }
    // twiddle table (length N) in LDS: short-latency loads inside the stages
    __shared__ Cx<T> tws[N];
    table_to_lds<T, N, NT>(tws, twg, tid);
    const Cx<T> *tw = tws;
    // per-phase {w, k - k0} of the update (fused form; augmented Lagrangian:
    // {k - k0, 1 / (k + k0)}; dual: {1 - k0 / k, -k0^2 / k})
    constexpr bool AL = UPD == 1;
    __shared__ Cx<T> lut[3];
    if (FWD && tid < 3) lut[tid] = AL ? Cx<T>{(T)pdk[tid], (T)prm->gam[tid]} : Cx<T>{(T)pw[tid], (T)pdk[tid]};
    __syncthreads();
    if constexpr (S == 1) {
        y0.finish(plane, tid);
        fft_stages<T, ROWS, 1, num_stages(ROWS), true, H, RS, NT, N, SeqStride<1>, PMY>(plane, tw, tid);
        c2r_pack_rows<T, N, ROWS, NT, true, RS>(plane, tw, tid);
    } else {
        fft_lds<T, ROWS, true, RS, RS, NT, N, SeqStride<1>>(plane, tw, tid);
        // pack the Hermitian half row into a length-N/2 complex sequence
        for (int idx = tid; idx < ROWS * (H / 2 + 1); idx += NT) {
            const int y = idx / (H / 2 + 1), k = idx - y * (H / 2 + 1);
            c2r_pack<T, N>(plane + y * RS, k, tw);
        }
    }
    T *eb = e + (size_t)ch * N * NN + (size_t)z * NN;
    const uint8_t *pb = ph + (size_t)z * NN;
    constexpr int TOTL = ROWS * N / V, PERL = (TOTL + NT - 1) / NT, BL = 8;
    // split planes, fused: the first NPF items of the update are loaded
    // before the x transform, which hides their latency
    constexpr int NPF = (S >= 2 && FWD) ? 4 : 0;
    T apre[NPF > 0 ? NPF : 1][V];
    unsigned ppre[NPF > 0 ? NPF : 1];
#pragma unroll
    for (int i = 0; i < NPF; ++i) {
        const int idx = tid + i * NT;
        if (i < PERL && (TOTL % NT == 0 || idx < TOTL)) {
            const int m = idx / (N / V), x = (idx - m * (N / V)) * V, y = S * m + h;
            vload<T>(eb + y * N + x, apre[i]);
            ppre[i] = pload<V>(pb + y * N + x);
        }
    }
    __syncthreads();
    fft_lds<T, H, true, ROWS, 1, NT, N, SeqStride<RS>, PMX>(plane, tw, tid);

    const T w0 = (T)pw[0], w1 = (T)pw[1], w2 = (T)pw[2];
    const double k0d = pk[0], k1d = pk[1], k2d = pk[2];
    const T d0 = (T)pdk[0], d1 = (T)pdk[1], d2 = (T)pdk[2];
    const T tm = (T)st->tau_mean[ch];
    const T k0t = (T)k0c;
    const T stp = (T)(prm->relax * k0c);  // the step of the augmented-Lagrangian family
    const T g0 = (T)prm->gam[0], g1 = (T)prm->gam[1], g2 = (T)prm->gam[2];
    const T e0 = (T)(ec * k0c), ik0 = (T)(1.0 / k0c);  // dual: k0 E, 1 / k0
    (void)d0, (void)d1, (void)d2, (void)tm, (void)k0t, (void)stp, (void)g0, (void)g1, (void)g2, (void)e0, (void)ik0;
    double r2 = 0.0, fl = 0.0, se = 0.0;
#pragma unroll
    for (int i0 = 0; i0 < PERL; i0 += BL) {
        T a[BL][V];
        unsigned p[BL];
#pragma unroll
        for (int i = 0; i < BL; ++i) {
            const int idx = tid + (i0 + i) * NT;
            if (i0 + i < PERL && (TOTL % NT == 0 || idx < TOTL)) {
                const int m = idx / (N / V), x = (idx - m * (N / V)) * V, y = S * m + h;
                if (i0 + i < NPF) {
#pragma unroll
                    for (int j = 0; j < V; ++j) a[i][j] = apre[(i0 + i) % (NPF > 0 ? NPF : 1)][j];
                    p[i] = ppre[(i0 + i) % (NPF > 0 ? NPF : 1)];
                } else {
                    vload<T>(eb + y * N + x, a[i]);
                    p[i] = pload<V>(pb + y * N + x);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < BL; ++i) {
            const int idx = tid + (i0 + i) * NT;
            if (i0 + i < PERL && (TOTL % NT == 0 || idx < TOTL)) {
                const int m = idx / (N / V), x = (idx - m * (N / V)) * V, y = S * m + h;
                T c[V];
                if constexpr (V == 4) {
                    Cx<T> z0, z1;
                    ld_pair<T, RS % 2 == 0>(plane + m * RS + x / 2, z0, z1);
                    c[0] = z0.x, c[1] = z0.y, c[2] = z1.x, c[3] = z1.y;
                } else {
#pragma unroll
                    for (int j = 0; j < V; j += 2) {
                        const Cx<T> zz = plane[m * RS + (x + j) / 2];
                        c[j] = zz.x;
                        c[j + 1] = zz.y;
                    }
                }
                if constexpr (FWD) {
                    // next iteration's tau, packed in place of the c values just
                    // read; fl collects sum tau here (the flux follows below)
                    T tau[V];
                    if constexpr (UPD == 1)
                        al_update_tau<T, V>(a[i], c, p[i], lut, stp, tm, ec, r2, fl, se, tau);
                    else if constexpr (UPD == 2)
                        dual_update_tau<T, V>(a[i], c, p[i], lut, tm, e0, ik0, r2, fl, se, tau);
                    else
                        em_update_tau<T, V>(a[i], c, p[i], lut, tm, ec, r2, fl, se, tau);
                    vstore<T>(eb + y * N + x, a[i]);
                    if constexpr (V == 4) {
                        st_pair<T, RS % 2 == 0>(plane + m * RS + x / 2, Cx<T>{tau[0], tau[1]}, Cx<T>{tau[2], tau[3]});
                    } else {
#pragma unroll
                        for (int j = 0; j < V; j += 2) plane[m * RS + (x + j) / 2] = Cx<T>{tau[j], tau[j + 1]};
                    }
                } else {
                    if constexpr (UPD == 1)
                        al_update<T, V>(a[i], c, p[i], d0, d1, d2, g0, g1, g2, k0t, stp, ec, r2, fl, se);
                    else if constexpr (UPD == 2)
                        dual_update<T, V>(a[i], c, p[i], w0, w1, w2, d0, d1, d2, e0, ik0, r2, fl, se);
                    else
                        em_update<T, V>(a[i], c, p[i], w0, w1, w2, k0d, k1d, k2d, ec, r2, fl, se);
                    vstore<T>(eb + y * N + x, a[i]);
                }
            }
        }
    }
    if constexpr (FWD) {
        // flux k e+ = (k - k0) e+ + k0 e+ = (tau + tm) + k0 e+ per voxel, summed
        // over the voxels of this thread (V per item idx = tid + i NT < TOTL)
        const int items = tid < TOTL ? (TOTL - 1 - tid) / NT + 1 : 0;
        fl += (double)(items * V) * (double)tm + k0c * se;
    }
    double v3[3] = {r2, fl, se};
    block_sum<NT, 3>(v3, red);
    // PS partial slots per plane (PS >= S: a grid whose other plane passes
    // split planes further; the first workgroup of a plane clears the spare
    // slots, whose zeros leave the fixed-order sums unchanged)
    if (tid == 0) {
        double *pp = part + ((size_t)ch * (N * PS) + (size_t)z * PS + h) * 3;
        pp[0] = v3[0];
        pp[1] = v3[1];
        pp[2] = v3[2];
        if (PS > S && h == 0)
            for (int j = 3 * S; j < 3 * PS; ++j) pp[j] = 0.0;
    }
    if constexpr (FWD) {
        __syncthreads();
        const Cx<T> *twf = opaque_ptr(tw);
        fft_lds<T, H, false, ROWS, 1, NT, N, SeqStride<RS>, PMX>(plane, twf, tid);
        if constexpr (S == 1) {
            r2c_unpack_rows<T, N, ROWS, NT, true, RS>(plane, twf, tid);
            __syncthreads();
            fft_stages<T, ROWS, 0, num_stages(ROWS) - 1, false, H, RS, NT, N, SeqStride<1>, PMY>(plane, twf, tid);
            y_last_stage_store<T, N, NT, RS>(plane, twf, spec + ((size_t)ch * N + z) * N * H,
                                             nyq + ((size_t)ch * N + z) * N, tid);
        } else {
            split_fwd_tail<T, N, NT, true, PC, S>(plane, twf, specB + ((size_t)ch * N + z) * N * H,
                                           nyqB + ((size_t)ch * N + z) * N, h, tid);
        }
    }
}

// ---------------------------------------------------------------------------
// Five-pass form for grids whose xy-plane does not fit in LDS (FP64 256^3,
// 512^3): the x and y transforms get passes of their own.
//   k_fwd_rows:  tau (or flux) fused into the load, R2C of G rows;
//   k_cols:      complex FFT down W columns of one (ch, z) plane (forward or
//                inverse); the kx = N/2 column is a tile of W planes;
//   k_zgreen:    as in the three-pass form;
//   k_inv_rows:  C2R of G rows fused with steps 6-7 and the flux.
// ---------------------------------------------------------------------------
// NC: components per load case (3 conductivity, 6 elasticity: the grid then
// covers 36 channels, the deviatoric ones with their own table).
template <typename T, int N, int G, int NT, bool PHI = false, int NC = 3>
__global__ __launch_bounds__(NT) void k_fwd_rows(const T *__restrict__ e, const uint8_t *__restrict__ ph,
                                                 Cx<T> *__restrict__ spec, Cx<T> *__restrict__ nyq,
                                                 const Cx<T> *__restrict__ twg,
                                                 const DevParams *__restrict__ prm,
                                                 const DevState *__restrict__ st) {
    constexpr int H = N / 2, RS = H + 1, V = VecOf<T>::V, NN = N * N, GP = N / G;
    __shared__ Cx<T> rows[G * RS];
    const int tid = threadIdx.x;
    const int ch = blockIdx.x / (N * GP), rem = blockIdx.x - ch * (N * GP);
    const int z = rem / GP, y0 = (rem - z * GP) * G;
    const int lc = ch / NC;
    if (PHI ? !st->eq_pending[lc] : st->done[lc]) return;
    const bool dev = NC == 6 && ch % NC != 0;
    const double *lut = PHI ? prm->k : (dev ? prm->dk_dev : prm->dk);
    // augmented Lagrangian, polarization: the buffer holds tau
    const bool tau_in = NC == 3 && !PHI && (prm->scheme == 2 || prm->scheme == 4);
    const T d0 = tau_in ? (T)1 : (T)lut[0], d1 = tau_in ? (T)1 : (T)lut[1], d2 = tau_in ? (T)1 : (T)lut[2];
    const T tm = PHI ? (T)0 : (T)st->tau_mean[ch];
    const T *eb = e + (size_t)ch * N * NN + (size_t)z * NN + (size_t)y0 * N;
    const uint8_t *pb = ph + (size_t)z * NN + (size_t)y0 * N;
    for (int idx = tid; idx < G * N / V; idx += NT) {
        const int y = idx / (N / V), x = (idx - y * (N / V)) * V;
        T a[V];
        vload<T>(eb + y * N + x, a);
        const unsigned p = pload<V>(pb + y * N + x);
#pragma unroll
        for (int i = 0; i < V; i += 2)
            rows[y * RS + (x + i) / 2] = Cx<T>{pick<T>(ph_at(p, i), d0, d1, d2) * a[i] - tm,
                                               pick<T>(ph_at(p, i + 1), d0, d1, d2) * a[i + 1] - tm};
    }
    // twiddle table (length N) in LDS: short-latency loads inside the stages
    __shared__ Cx<T> tws[N];
    table_to_lds<T, N, NT>(tws, twg, tid);
    const Cx<T> *tw = tws;
    __syncthreads();
    fft_lds<T, H, false, G, 1, NT, N, SeqStride<RS>>(rows, tw, tid);
    for (int idx = tid; idx < G * (H / 2 + 1); idx += NT) {
        const int y = idx / (H / 2 + 1), k = idx - y * (H / 2 + 1);
        r2c_unpack<T, N, false>(rows + y * RS, k, tw, Cx<T>{(T)1, (T)0});
    }
    __syncthreads();
    Cx<T> *sb = spec + (((size_t)ch * N + z) * N + y0) * H;
    for (int idx = tid; idx < G * H; idx += NT) {
        const int y = idx / H, kx = idx - y * H;
        sb[(size_t)y * H + kx] = rows[y * RS + kx];
    }
    Cx<T> *nb = nyq + ((size_t)ch * N + z) * N + y0;
    for (int y = tid; y < G; y += NT) nb[y] = rows[y * RS + H];
}

template <int N, int W, int NCH = 9> struct ColTiles {
    static constexpr int H = N / 2;
    static constexpr int MAIN = NCH * N * (H / W);  // (ch, z, kx chunk)
    static constexpr int NYQ = NCH * (N / W);       // (ch, chunk of W planes) of the kx = N/2 column
    static constexpr int ALL = MAIN + NYQ;
};

// GATE_EQ: run for load cases awaiting the equilibrium check instead of the
// ones still iterating.
template <typename T, int N, int W, int NT, bool INV, bool GATE_EQ = false, int NC = 3>
__global__ __launch_bounds__(NT) void k_cols(Cx<T> *__restrict__ spec, Cx<T> *__restrict__ nyq,
                                             const Cx<T> *__restrict__ twg, const DevState *__restrict__ st) {
    using TL = ColTiles<N, W, NC * NC>;
    constexpr int H = N / 2, NW = N * W;
    __shared__ Cx<T> buf[NW];  // [ky][w]
    const int tid = threadIdx.x;
    const int b = blockIdx.x;
    Cx<T> *base;
    int ch;
    size_t es, ss;  // global stride between ky and between w
    if (b < TL::MAIN) {
        ch = b / (N * (H / W));
        const int rem = b - ch * (N * (H / W));
        const int z = rem / (H / W), c0 = (rem - z * (H / W)) * W;
        base = spec + ((size_t)ch * N + z) * N * H + c0;
        es = H;
        ss = 1;
    } else {
        const int t = b - TL::MAIN;
        ch = t / (N / W);
        const int z0 = (t - ch * (N / W)) * W;
        base = nyq + ((size_t)ch * N + z0) * N;
        es = 1;
        ss = N;
    }
    const int lc = ch / NC;
    if (GATE_EQ ? !st->eq_pending[lc] : st->done[lc]) return;
    // the columns straight to the registers of the first stage, and the last
    // stage straight back
    constexpr int PM = (W % 2 == 0 && sizeof(T) == 4) ? kPairSeq : kPairNone;
    ZFirstStage<T, N, W, NT, 1, INV> c0;
    c0.load(base, 0, es, tid, ss);
    // twiddle table (length N) in LDS: short-latency loads inside the stages
    __shared__ Cx<T> tws[N];
    table_to_lds<T, N, NT>(tws, twg, tid);
    const Cx<T> *tw = tws;
    c0.finish(buf, tid);
    fft_stages<T, N, 1, num_stages(N) - 1, INV, W, W, NT, N, SeqStride<1>, PM>(buf, tw, tid);
    z_last_stage_store<T, N, W, NT, 1, INV>(buf, tw, base, 0, es, tid, ss);
}

template <typename T, int N, int G, int NT, int UPD = 0, int NC = 3>
__global__ __launch_bounds__(NT) void k_inv_rows(T *__restrict__ e, const uint8_t *__restrict__ ph,
                                                 const Cx<T> *__restrict__ spec, const Cx<T> *__restrict__ nyq,
                                                 const Cx<T> *__restrict__ twg,
                                                 const DevParams *__restrict__ prm,
                                                 const DevState *__restrict__ st, double *__restrict__ part) {
    constexpr int H = N / 2, RS = H + 1, V = VecOf<T>::V, NN = N * N, GP = N / G;
    static_assert(NC == 3 || UPD == 0, "the elastic case runs the accelerated update");
    __shared__ Cx<T> rows[G * RS];
    __shared__ double red[3 * (NT / 64)];
    const int tid = threadIdx.x;
    const int ch = blockIdx.x / (N * GP), rem = blockIdx.x - ch * (N * GP);
    const int z = rem / GP, yg = rem - z * GP, y0 = yg * G;
    const int lc = ch / NC;
    if (st->done[lc]) return;
    // E_comp of this channel (ch = NC lc + comp: the unit vector or basis
    // tensor lc), and (elasticity) the deviatoric channels' own tables
    const T ec = (ch % (NC + 1) == 0) ? (T)1 : (T)0;
    const bool dev = NC == 6 && ch % NC != 0;
    const double *pk = dev ? prm->k_dev : prm->k;
    const double *pw = dev ? prm->w_dev : prm->w;
    const Cx<T> *sb = spec + (((size_t)ch * N + z) * N + y0) * H;
    const Cx<T> *nb = nyq + ((size_t)ch * N + z) * N + y0;
    for (int idx = tid; idx < G * RS; idx += NT) {
        const int y = idx / RS, kx = idx - y * RS;
        rows[idx] = (kx < H) ? sb[(size_t)y * H + kx] : nb[y];
    }
    // twiddle table (length N) in LDS: short-latency loads inside the stages
    __shared__ Cx<T> tws[N];
    table_to_lds<T, N, NT>(tws, twg, tid);
    const Cx<T> *tw = tws;
    __syncthreads();
    for (int idx = tid; idx < G * (H / 2 + 1); idx += NT) {
        const int y = idx / (H / 2 + 1), k = idx - y * (H / 2 + 1);
        c2r_pack<T, N>(rows + y * RS, k, tw);
    }
    __syncthreads();
    fft_lds<T, H, true, G, 1, NT, N, SeqStride<RS>>(rows, tw, tid);
    const T w0 = (T)pw[0], w1 = (T)pw[1], w2 = (T)pw[2];
    const double k0d = pk[0], k1d = pk[1], k2d = pk[2];
    T *eb = e + (size_t)ch * N * NN + (size_t)z * NN + (size_t)y0 * N;
    const uint8_t *pb = ph + (size_t)z * NN + (size_t)y0 * N;
    double r2 = 0.0, fl = 0.0, se = 0.0;
    for (int idx = tid; idx < G * N / V; idx += NT) {
        const int y = idx / (N / V), x = (idx - y * (N / V)) * V;
        T a[V], c[V];
        vload<T>(eb + y * N + x, a);
        const unsigned p = pload<V>(pb + y * N + x);
#pragma unroll
        for (int i = 0; i < V; i += 2) {
            const Cx<T> zz = rows[y * RS + (x + i) / 2];
            c[i] = zz.x;
            c[i + 1] = zz.y;
        }
        if constexpr (UPD == 1)
            al_update<T, V>(a, c, p, (T)prm->dk[0], (T)prm->dk[1], (T)prm->dk[2], (T)prm->gam[0],
                            (T)prm->gam[1], (T)prm->gam[2], (T)prm->k0, (T)(prm->relax * prm->k0), ec, r2, fl, se);
        else if constexpr (UPD == 2)
            dual_update<T, V>(a, c, p, w0, w1, w2, (T)prm->dk[0], (T)prm->dk[1], (T)prm->dk[2],
                              (T)(ec * prm->k0), (T)(1.0 / prm->k0), r2, fl, se);
        else
            em_update<T, V>(a, c, p, w0, w1, w2, k0d, k1d, k2d, ec, r2, fl, se);
        vstore<T>(eb + y * N + x, a);
    }
    double v3[3] = {r2, fl, se};
    block_sum<NT, 3>(v3, red);
    if (tid == 0) {
        double *pp = part + ((size_t)ch * (N * GP) + (size_t)z * GP + yg) * 3;
        pp[0] = v3[0];
        pp[1] = v3[1];
        pp[2] = v3[2];
    }
}

// e = E_lc for every voxel; solver state reset.  Load cases outside the mask
// start frozen.
// Augmented Lagrangian: the start field e^0 becomes tau^0 = (k - k0) e^0 in
// place, for the load cases being solved (lam^0 = k e^0, d^0 = e^0).
template <typename T>
__global__ void k_to_tau(T *__restrict__ e, const uint8_t *__restrict__ ph, size_t M,
                         const DevParams *__restrict__ prm) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < 9 * M; i += stride) {
        const int lc = (int)(i / (3 * M));
        if (!((prm->lc_mask >> lc) & 1)) continue;
        e[i] = (T)(prm->dk[ph[i % M]] * (double)e[i]);
    }
}

template <typename T>
__global__ void k_init(T *__restrict__ e, size_t M, const DevParams *__restrict__ prm, DevState *__restrict__ st) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const int nc = prm->nc;
    // the dual scheme's iterate is the flux, which starts at k0 E
    const T one = prm->scheme == 3 ? (T)prm->k0 : (T)1;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (size_t)(nc * nc) * M; i += stride) {
        const int ch = (int)(i / M);
        e[i] = (ch % (nc + 1) == 0) ? one : (T)0;  // ch = nc lc + comp, comp == lc
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->iter = 0;
        int all = 1;
        for (int lc = 0; lc < 6; ++lc) {
            const int on = lc < nc && ((prm->lc_mask >> lc) & 1);
            st->done[lc] = on ? 0 : 1;
            all &= !on;
            st->status[lc] = on ? ST_NOT_CONVERGED : ST_OK;
            st->iters[lc] = 0;
            st->best_it[lc] = 0;
            st->eq_pending[lc] = 0;
            st->res[lc] = 0.0;
            st->best[lc] = 1e308;
            st->eps_eq[lc] = -1.0;
        }
        for (int i = 0; i < 36; ++i) {
            st->K[i] = 0.0;
            st->tau_mean[i] = 0.0;
        }
        st->all_done = all;
    }
}

// Warm start / field export between FP64 host staging and the working field.
template <typename T> __global__ void k_from_f64(T *__restrict__ e, const double *__restrict__ src, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) e[i] = (T)src[i];
}
template <typename T> __global__ void k_to_f64(double *__restrict__ dst, const T *__restrict__ e, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = (double)e[i];
}

}  // namespace rvehom
