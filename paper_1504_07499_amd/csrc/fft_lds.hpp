// fft_lds.hpp -- device building blocks for batched FFTs held in LDS (gfx950).
//
// Complex arithmetic, small in-register DFTs (radix 2, 3, 4, 8, 16) and a
// self-sorting (Stockham) radix stage over many sequences that live in LDS.
// Every stage reads all of its butterflies into registers, waits at a
// workgroup barrier, then writes, so the transform is in place in LDS.
//
// Forward transforms use exp(-2 pi i k n / L); inverse transforms use the
// conjugate kernel and are unnormalised.  Twiddles come from a table
// tw[m] = exp(-2 pi i m / NT) of the top-level length, computed in FP64 on the
// host and rounded once to the working precision.
#pragma once

#include <hip/hip_runtime.h>

namespace rvehom {

template <typename T> struct Cx {
    T x, y;
};

template <typename T> __device__ __forceinline__ Cx<T> cx(T a, T b) { return Cx<T>{a, b}; }
template <typename T> __device__ __forceinline__ Cx<T> operator+(Cx<T> a, Cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __device__ __forceinline__ Cx<T> operator-(Cx<T> a, Cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> __device__ __forceinline__ Cx<T> operator*(Cx<T> a, Cx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T> __device__ __forceinline__ Cx<T> scale(Cx<T> a, T s) { return {a.x * s, a.y * s}; }
template <typename T> __device__ __forceinline__ Cx<T> conj(Cx<T> a) { return {a.x, -a.y}; }
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV> __device__ __forceinline__ Cx<T> mul_mi(Cx<T> a) {
    return INV ? Cx<T>{-a.y, a.x} : Cx<T>{a.y, -a.x};
}
// twiddle w (forward table value) applied in the transform's direction
template <typename T, bool INV> __device__ __forceinline__ Cx<T> twmul(Cx<T> a, Cx<T> w) {
    return INV ? a * conj(w) : a * w;
}

// ---------------------------------------------------------------------------
// In-register DFTs, out[s] = sum_r v[r] w_R^(r s) (w_R = exp(-+2 pi i / R)).
// ---------------------------------------------------------------------------
template <typename T, bool INV> __device__ __forceinline__ void dft2(Cx<T> *v) {
    Cx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
}

template <typename T, bool INV> __device__ __forceinline__ void dft3(Cx<T> *v) {
    const T s = (T)0.86602540378443864676;  // sin(2 pi / 3)
    Cx<T> t1 = v[1] + v[2];
    Cx<T> t2 = v[0] - scale(t1, (T)0.5);
    Cx<T> d = scale(v[1] - v[2], s);
    Cx<T> rd = mul_mi<T, INV>(d);  // -i s (v1 - v2) forward
    v[0] = v[0] + t1;
    v[1] = t2 + rd;
    v[2] = t2 - rd;
}

template <typename T, bool INV> __device__ __forceinline__ void dft4(Cx<T> *v) {
    Cx<T> a0 = v[0] + v[2], a1 = v[0] - v[2];
    Cx<T> a2 = v[1] + v[3], a3 = mul_mi<T, INV>(v[1] - v[3]);
    v[0] = a0 + a2;
    v[2] = a0 - a2;
    v[1] = a1 + a3;
    v[3] = a1 - a3;
}

template <typename T, bool INV> __device__ __forceinline__ void dft8(Cx<T> *v) {
    const T h = (T)0.70710678118654752440;  // 1/sqrt(2)
    Cx<T> e[4] = {v[0], v[2], v[4], v[6]};
    Cx<T> o[4] = {v[1], v[3], v[5], v[7]};
    dft4<T, INV>(e);
    dft4<T, INV>(o);
    // w8^1 = (1 - i)/sqrt2, w8^2 = -i, w8^3 = (-1 - i)/sqrt2 (forward)
    Cx<T> o1 = INV ? Cx<T>{h * (o[1].x - o[1].y), h * (o[1].x + o[1].y)}
                   : Cx<T>{h * (o[1].x + o[1].y), h * (o[1].y - o[1].x)};
    Cx<T> o2 = mul_mi<T, INV>(o[2]);
    Cx<T> o3 = INV ? Cx<T>{-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y)}
                   : Cx<T>{h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y)};
    v[0] = e[0] + o[0];
    v[4] = e[0] - o[0];
    v[1] = e[1] + o1;
    v[5] = e[1] - o1;
    v[2] = e[2] + o2;
    v[6] = e[2] - o2;
    v[3] = e[3] + o3;
    v[7] = e[3] - o3;
}

template <typename T, bool INV> __device__ __forceinline__ void dft16(Cx<T> *v) {
    // 16 = 4 x 4: inner DFT4 over n1 for each n2, twiddle w16^(n2 k1), outer DFT4.
    const T c1 = (T)0.92387953251128675613;  // cos(pi/8)
    const T s1 = (T)0.38268343236508977173;  // sin(pi/8)
    const T h = (T)0.70710678118654752440;
    Cx<T> y[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        Cx<T> t[4] = {v[n2], v[4 + n2], v[8 + n2], v[12 + n2]};
        dft4<T, INV>(t);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) y[n2][k1] = t[k1];
    }
    // twiddles w16^m, m = n2 k1 in {1,2,3,2,4,6,3,6,9}; forward w = cos - i sin
    const T sg = INV ? (T)1 : (T)-1;
    const Cx<T> w1 = {c1, sg * s1}, w2 = {h, sg * h}, w3 = {s1, sg * c1};
    const Cx<T> w6 = {-h, sg * h}, w9 = {-c1, -sg * s1};
    y[1][1] = y[1][1] * w1;
    y[1][2] = y[1][2] * w2;
    y[1][3] = y[1][3] * w3;
    y[2][1] = y[2][1] * w2;
    y[2][2] = mul_mi<T, INV>(y[2][2]);
    y[2][3] = y[2][3] * w6;
    y[3][1] = y[3][1] * w3;
    y[3][2] = y[3][2] * w6;
    y[3][3] = y[3][3] * w9;
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        Cx<T> t[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
        dft4<T, INV>(t);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
    }
}

template <typename T, int R, bool INV> __device__ __forceinline__ void dft(Cx<T> *v) {
    if constexpr (R == 2) dft2<T, INV>(v);
    else if constexpr (R == 3) dft3<T, INV>(v);
    else if constexpr (R == 4) dft4<T, INV>(v);
    else if constexpr (R == 8) dft8<T, INV>(v);
    else if constexpr (R == 16) dft16<T, INV>(v);
    else static_assert(R == 2, "unsupported radix");
}

// ---------------------------------------------------------------------------
// Radix plans.  Stage s of a length-L transform uses radix radix_of(L, s).
// Powers of two use 16/8/4 stages; factors of 3 get a radix-3 stage each.
// ---------------------------------------------------------------------------
constexpr int pow2_part(int L) { return (L % 2 == 0) ? 2 * pow2_part(L / 2) : 1; }

constexpr int pow2_stages(int p) {
    return p == 1 ? 0 : p <= 16 ? 1 : p <= 256 ? 2 : p <= 4096 ? 3 : 4;
}

// radix of stage s (0-based) for the power-of-two part p
constexpr int pow2_radix(int p, int s) {
    return p <= 16    ? p
           : p == 32  ? (s == 0 ? 8 : 4)
           : p == 64  ? 8
           : p == 128 ? (s == 0 ? 16 : 8)
           : p == 256 ? 16
           : p == 512 ? 8
           : p == 1024 ? (s == 0 ? 16 : 8)
                       : 16;
}

constexpr int three_count(int L) { return (L % 3 == 0) ? 1 + three_count(L / 3) : 0; }

constexpr int num_stages(int L) { return pow2_stages(pow2_part(L)) + three_count(L); }

constexpr int radix_of(int L, int s) {
    return s < pow2_stages(pow2_part(L)) ? pow2_radix(pow2_part(L), s) : 3;
}

constexpr int ns_before(int L, int s) { return s == 0 ? 1 : ns_before(L, s - 1) * radix_of(L, s - 1); }

constexpr bool plan_ok(int L) {
    int p = 1;
    for (int s = 0; s < num_stages(L); ++s) p *= radix_of(L, s);
    return p == L;
}

// ---------------------------------------------------------------------------
// One Stockham stage over NSEQ sequences of length L in LDS.  Element e of
// sequence q sits at buf[Seq::base(q) + e * ES].  TW = top-level table
// length (L divides TW).  NT threads take part; each owns up to PER
// butterflies of radix R.
// ---------------------------------------------------------------------------
template <typename T, int L, int S, bool INV, int NSEQ, int ES, int NT, int TW, class Seq>
__device__ __forceinline__ void fft_stage(Cx<T> *buf, const Cx<T> *__restrict__ tw, int tid) {
    constexpr int R = radix_of(L, S);
    constexpr int NS = ns_before(L, S);
    constexpr int NB = L / R;
    constexpr int TOT = NSEQ * NB;
    constexpr int PER = (TOT + NT - 1) / NT;
    constexpr int TWS = TW / (NS * R);  // table stride of one twiddle step
    Cx<T> v[PER][R];
    // Butterfly b = j * NSEQ + q: neighbouring threads take the same butterfly
    // of neighbouring sequences, so they share one twiddle (a broadcast load)
    // and, for sequences side by side in LDS, touch consecutive addresses.
    // Reads, twiddles and the radix-R DFT all happen before the barrier (the
    // twiddle loads' latency overlaps the wait); only the writes follow it.
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int b = tid + i * NT;
        if (TOT % NT == 0 || b < TOT) {
            const int j = b / NSEQ, q = b - j * NSEQ;
            const int off = Seq::base(q);
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = buf[off + (j + r * NB) * ES];
        }
    }
    if (NS > 1) {
        Cx<T> w[PER][R];
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int b = tid + i * NT;
            if (TOT % NT == 0 || b < TOT) {
                const int k = (b / NSEQ) % NS;
#pragma unroll
                for (int r = 1; r < R; ++r) w[i][r] = tw[r * k * TWS];
            }
        }
#pragma unroll
        for (int i = 0; i < PER; ++i)
#pragma unroll
            for (int r = 1; r < R; ++r) v[i][r] = twmul<T, INV>(v[i][r], w[i][r]);
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) dft<T, R, INV>(v[i]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int b = tid + i * NT;
        if (TOT % NT == 0 || b < TOT) {
            const int j = b / NSEQ, q = b - j * NSEQ;
            const int k = j % NS;
            const int off = Seq::base(q);
            const int d = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[off + (d + r * NS) * ES] = v[i][r];
        }
    }
    __syncthreads();
}

// Two neighbouring complex values in LDS as one 16-byte access (FP32; the
// address must be 16-byte aligned) or two (FP64).
template <typename T> __device__ __forceinline__ void lds_ld2(const Cx<T> *p, Cx<T> &a, Cx<T> &b) {
    if constexpr (sizeof(T) == 4) {
        const float4 t = *reinterpret_cast<const float4 *>(p);
        a = Cx<T>{t.x, t.y};
        b = Cx<T>{t.z, t.w};
    } else {
        a = p[0];
        b = p[1];
    }
}
template <typename T> __device__ __forceinline__ void lds_st2(Cx<T> *p, Cx<T> a, Cx<T> b) {
    if constexpr (sizeof(T) == 4) {
        *reinterpret_cast<float4 *>(p) = make_float4(a.x, a.y, b.x, b.y);
    } else {
        p[0] = a;
        p[1] = b;
    }
}

// Paired stages: each thread owns two butterflies whose data sit side by
// side in LDS, so every LDS access moves two complex values.
//  * PairSeq: the same butterfly of sequences 2p and 2p + 1, which must be
//    adjacent (Seq::base(2p + 1) = Seq::base(2p) + 1, base even, ES even).
//  * PairElem: butterflies 2p and 2p + 1 of one sequence whose elements are
//    contiguous (ES = 1, Seq::base even); needs R and NB even.  A first stage
//    (NS = 1) writes each butterfly's R outputs contiguously (pairs along r);
//    later stages write the two butterflies' outputs side by side.
enum PairMode { kPairNone = 0, kPairSeq = 1, kPairElem = 2 };

template <typename T, int L, int S, bool INV, int NSEQ, int ES, int NT, int TW, class Seq>
__device__ __forceinline__ void fft_stage_pseq(Cx<T> *buf, const Cx<T> *__restrict__ tw, int tid) {
    constexpr int R = radix_of(L, S);
    constexpr int NS = ns_before(L, S);
    constexpr int NB = L / R;
    constexpr int NP = NSEQ / 2;
    constexpr int TOT = NP * NB;
    constexpr int PER = (TOT + NT - 1) / NT;
    constexpr int TWS = TW / (NS * R);
    static_assert(NSEQ % 2 == 0 && ES % 2 == 0, "sequence pairs need an even count and an even stride");
    Cx<T> v[PER][2][R];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int u = tid + i * NT;
        if (TOT % NT == 0 || u < TOT) {
            const int j = u / NP, qp = u - j * NP;
            const int off = Seq::base(2 * qp);
#pragma unroll
            for (int r = 0; r < R; ++r) lds_ld2<T>(buf + off + (j + r * NB) * ES, v[i][0][r], v[i][1][r]);
        }
    }
    if (NS > 1) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int u = tid + i * NT;
            if (TOT % NT == 0 || u < TOT) {
                const int k = (u / NP) % NS;
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    const Cx<T> w = tw[r * k * TWS];
                    v[i][0][r] = twmul<T, INV>(v[i][0][r], w);
                    v[i][1][r] = twmul<T, INV>(v[i][1][r], w);
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        dft<T, R, INV>(v[i][0]);
        dft<T, R, INV>(v[i][1]);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int u = tid + i * NT;
        if (TOT % NT == 0 || u < TOT) {
            const int j = u / NP, qp = u - j * NP;
            const int k = j % NS;
            const int off = Seq::base(2 * qp);
            const int d = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) lds_st2<T>(buf + off + (d + r * NS) * ES, v[i][0][r], v[i][1][r]);
        }
    }
    __syncthreads();
}

template <typename T, int L, int S, bool INV, int NSEQ, int NT, int TW, class Seq>
__device__ __forceinline__ void fft_stage_pelem(Cx<T> *buf, const Cx<T> *__restrict__ tw, int tid) {
    constexpr int R = radix_of(L, S);
    constexpr int NS = ns_before(L, S);
    constexpr int NB = L / R;
    constexpr int NBP = NB / 2;
    constexpr int TOT = NSEQ * NBP;
    constexpr int PER = (TOT + NT - 1) / NT;
    constexpr int TWS = TW / (NS * R);
    static_assert(R % 2 == 0 && NB % 2 == 0 && (NS == 1 || NS % 2 == 0), "element pairs need even R, NB, NS");
    Cx<T> v[PER][2][R];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int u = tid + i * NT;
        if (TOT % NT == 0 || u < TOT) {
            const int jp = u / NSEQ, q = u - jp * NSEQ;
            const int off = Seq::base(q) + 2 * jp;
#pragma unroll
            for (int r = 0; r < R; ++r) lds_ld2<T>(buf + off + r * NB, v[i][0][r], v[i][1][r]);
        }
    }
    if (NS > 1) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int u = tid + i * NT;
            if (TOT % NT == 0 || u < TOT) {
                const int k0 = (2 * (u / NSEQ)) % NS;
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    v[i][0][r] = twmul<T, INV>(v[i][0][r], tw[r * k0 * TWS]);
                    v[i][1][r] = twmul<T, INV>(v[i][1][r], tw[r * (k0 + 1) * TWS]);
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        dft<T, R, INV>(v[i][0]);
        dft<T, R, INV>(v[i][1]);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int u = tid + i * NT;
        if (TOT % NT == 0 || u < TOT) {
            const int jp = u / NSEQ, q = u - jp * NSEQ;
            const int j0 = 2 * jp;
            const int base = Seq::base(q);
            if constexpr (NS == 1) {
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int r = 0; r < R; r += 2) lds_st2<T>(buf + base + (j0 + h) * R + r, v[i][h][r], v[i][h][r + 1]);
            } else {
                const int k0 = j0 % NS;
                const int d = (j0 - k0) * R + k0;
#pragma unroll
                for (int r = 0; r < R; ++r) lds_st2<T>(buf + base + d + r * NS, v[i][0][r], v[i][1][r]);
            }
        }
    }
    __syncthreads();
}

// stage S with pairing where its radix allows it
template <typename T, int L, int S, bool INV, int NSEQ, int ES, int NT, int TW, class Seq, int PM>
__device__ __forceinline__ void fft_stage_any(Cx<T> *buf, const Cx<T> *__restrict__ tw, int tid) {
    constexpr int R = radix_of(L, S);
    constexpr int NB = L / R;
    constexpr int NS = ns_before(L, S);
    // sequence pairs only where they give every thread a butterfly pair (a
    // radix-16 stage over few sequences would leave half the block idle)
    if constexpr (PM == kPairSeq && (NSEQ / 2) * NB >= NT) {
        fft_stage_pseq<T, L, S, INV, NSEQ, ES, NT, TW, Seq>(buf, tw, tid);
    } else if constexpr (PM == kPairElem && ES == 1 && R % 2 == 0 && NB % 2 == 0 && (NS == 1 || NS % 2 == 0)) {
        fft_stage_pelem<T, L, S, INV, NSEQ, NT, TW, Seq>(buf, tw, tid);
    } else {
        fft_stage<T, L, S, INV, NSEQ, ES, NT, TW, Seq>(buf, tw, tid);
    }
}

template <typename T, int L, int S, int NST, bool INV, int NSEQ, int ES, int NT, int TW, class Seq, int PM>
__device__ __forceinline__ void fft_stages(Cx<T> *buf, const Cx<T> *__restrict__ tw, int tid) {
    if constexpr (S < NST) {
        fft_stage_any<T, L, S, INV, NSEQ, ES, NT, TW, Seq, PM>(buf, tw, tid);
        fft_stages<T, L, S + 1, NST, INV, NSEQ, ES, NT, TW, Seq, PM>(buf, tw, tid);
    }
}

// Full length-L transform of NSEQ sequences in LDS (caller syncs before).
// PM selects paired stages (the layout must meet that mode's conditions).
template <typename T, int L, bool INV, int NSEQ, int ES, int NT, int TW, class Seq, int PM = kPairNone>
__device__ __forceinline__ void fft_lds(Cx<T> *buf, const Cx<T> *__restrict__ tw, int tid) {
    static_assert(plan_ok(L), "no radix plan for this length");
    static_assert(TW % L == 0, "twiddle table length must be a multiple of L");
    fft_stages<T, L, 0, num_stages(L), INV, NSEQ, ES, NT, TW, Seq, PM>(buf, tw, tid);
}

// Sequence placements
template <int SS> struct SeqStride {  // sequence q at q * SS
    __device__ static __forceinline__ int base(int q) { return q * SS; }
};
template <int W, int BLK> struct SeqBlocked {  // q = c * W + w -> c * BLK + w
    __device__ static __forceinline__ int base(int q) { return (q / W) * BLK + (q % W); }
};

}  // namespace rvehom
