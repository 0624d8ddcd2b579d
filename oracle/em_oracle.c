/*
 * em_oracle.c -- plain, slow FP64 CPU oracle for the accelerated FFT scheme
 * that computes the effective thermal conductivity tensor of a periodic
 * voxelized three-phase RVE.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU path; both only consume the same
 * phase image produced by the seeded input generator.
 *
 * Paper: S. Lemaitre, V. Salnikov, D. Choi, P. Karamian, "Computation of
 * thermal properties via 3D homogenization of multiphase materials using
 * FFT-based accelerated scheme", arXiv:1504.07499.
 *   Sec. 3  problem statement (periodic RVE, Fourier's law, div phi = 0,
 *           imposed mean gradient), eq. (1) polarization, eq. (3) Fourier
 *           Lippmann-Schwinger equation, the Green operator Gamma^0 and the
 *           Algorithm "FFT-based homogenization scheme for thermal
 *           conductivity case" (steps 1-7), and L_hom from <phi>; the basic
 *           and augmented-Lagrangian schemes named there as alternatives
 *           (orc_homogenize, scheme 1 and 2).
 *   Sec. 5  reference medium L0 = -sqrt(min k * max k) I.
 *   Sec. 6  the elastic case named as the extension (orc_homogenize_elastic,
 *           at the end of this file).
 *
 * Readings of the paper taken here (each is listed with its reason in the
 * design notes of the repository):
 *  R1  L0 = -k0 I with k0 = sqrt(min k * max k) > 0 (Sec. 5).  Putting this
 *      negative L0 into steps 2, 4 and 7 gives
 *          tau   = (k - k0) e                      (step 2, overall sign
 *                                                   cancels with step 4)
 *          c^(xi)= -xi (xi . tau^) / (k0 |xi|^2),  xi != 0   (step 4)
 *          e+    = e + 2 k0/(k + k0) (c - e)        (step 7)
 *      where e is the gradient iterate and c the compatible field.
 *  R2  c^(0) = E (step 4): with the unnormalised DFT used here this is
 *      c^(0) = M E, M = N^3.
 *  R3  xi are the signed integer wavenumbers (the 2 pi / L factor cancels in
 *      Gamma^0).  On an even grid the index N/2 is both +N/2 and -N/2: the
 *      sign of such a Nyquist component is undetermined.  The operator used
 *      at a mode is the average of xi xi^T / |xi|^2 over both signs of every
 *      Nyquist component (each axis independently).  This keeps the discrete
 *      problem covariant under the reflection of any single axis (a choice of
 *      one sign, or the average over +-xi only, does not at modes with two or
 *      more Nyquist components) and leaves every other mode unchanged.  The
 *      averaged operator is even in xi, so the inverse DFT of the compatible
 *      field is real; its real part is taken to drop rounding residue.
 *  R4  Stop when eps_comp (step 6) < tol.  With the option eq_check the
 *      paper's two-stage test of step 1 is used instead: stop only when
 *      eps_comp < tol and eps_eq < tol, with the scale-free
 *      eps_eq = sqrt(sum' |xi . phi^|^2 / |xi|^2) / |phi^(0)|, where sum'
 *      runs over the modes xi != 0 on which the averaged operator of R3 is
 *      the projection on xi: modes without a Nyquist component, and modes
 *      whose only nonzero component is one Nyquist component.  On the other
 *      Nyquist modes the sign average makes the operator a non-projection
 *      and the discrete fixed point does not zero xi . phi^ there.
 *  R5  <phi> (after the algorithm) is taken on the field updated in the
 *      stopping iteration; column j of L_hom is <k e> for E = e_j.
 *  R6  The three load cases E = e_1, e_2, e_3 are solved independently.
 *  R7  Dual scheme on an even grid: a field is divergence free at a mode when
 *      xi . v = 0 for every sign of its Nyquist components (so the averaged
 *      operator is a projection; the average of I - xi xi^T / |xi|^2 over the
 *      signs, the complement of R3's symbol, is not, and leaves eigenvalues
 *      near 0 that the dual iteration barely contracts).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define ORC_OK 0
#define ORC_NOT_CONVERGED 1
#define ORC_ERR_ARG -1
#define ORC_ERR_NONFINITE -5

/* ------------------------------------------------------------------------
 * Own FFT: recursive mixed-radix decimation in time.  Factors 2 and 3 are
 * split off recursively; any other prime length falls back to the direct
 * O(n^2) sum.  sign = -1 is the forward transform
 *     X[k] = sum_n x[n] exp(-2 pi i k n / N),
 * sign = +1 the unnormalised inverse.
 * ---------------------------------------------------------------------- */

/* w[j] = exp(sign 2 pi i j / N), j < N, computed directly in FP64. */
static void twiddle_table(int n, int sign, cplx *w)
{
    for (int j = 0; j < n; ++j) {
        double a = 2.0 * M_PI * (double)j / (double)n;
        w[j] = cos(a) + (double)sign * sin(a) * I;
    }
}

static int smallest_factor(int n)
{
    if (n % 2 == 0) return 2;
    if (n % 3 == 0) return 3;
    for (int p = 5; p * p <= n; p += 2)
        if (n % p == 0) return p;
    return n;
}

/* Transform n = ntop / stride_factor points read from in[0], in[is], ...,
 * into out[0..n-1].  w is the table for the top-level length ntop. */
static void fft_rec(const cplx *in, int is, cplx *out, int n, int ntop,
                    const cplx *w)
{
    if (n == 1) {
        out[0] = in[0];
        return;
    }
    int p = smallest_factor(n);
    int m = n / p;
    int step = ntop / n; /* w_n^j = w_ntop^(j * step) */
    if (p == n) {
        /* direct sum for a prime length that is not 2 or 3 */
        for (int k = 0; k < n; ++k) {
            cplx s = 0;
            for (int j = 0; j < n; ++j)
                s += in[j * is] * w[((long)j * k % n) * step];
            out[k] = s;
        }
        return;
    }
    /* sub-transforms of the p decimated sequences */
    for (int q = 0; q < p; ++q)
        fft_rec(in + q * is, is * p, out + q * m, m, ntop, w);
    /* combine: X[k + s m] = sum_q w_n^(q (k + s m)) Y_q[k] */
    cplx t[3];
    for (int k = 0; k < m; ++k) {
        for (int q = 0; q < p; ++q)
            t[q] = out[q * m + k] * w[(q * k) * step];
        for (int s = 0; s < p; ++s) {
            cplx acc = 0;
            for (int q = 0; q < p; ++q)
                acc += t[q] * w[((q * s * m) % n) * step];
            out[k + s * m] = acc;
        }
    }
}

/* 1D transform of a contiguous line in place; buf holds n points. */
static void fft_line(cplx *line, int n, const cplx *w, cplx *buf)
{
    memcpy(buf, line, sizeof(cplx) * (size_t)n);
    fft_rec(buf, 1, line, n, n, w);
}

/* Full complex 3D DFT of a [z][y][x] array (x fastest), in place,
 * unnormalised, applied one axis at a time. */
void orc_fft3(int n, double *data_ri, int sign)
{
    cplx *a = (cplx *)data_ri;
    size_t nn = (size_t)n * n;
    cplx *w = malloc(sizeof(cplx) * (size_t)n);
    twiddle_table(n, sign, w);
    #pragma omp parallel
    {
        cplx *line = malloc(sizeof(cplx) * (size_t)n);
        cplx *buf = malloc(sizeof(cplx) * (size_t)n);
        /* axis x */
        #pragma omp for schedule(static)
        for (long zy = 0; zy < (long)nn; ++zy)
            fft_line(a + (size_t)zy * n, n, w, buf);
        /* axis y */
        #pragma omp for schedule(static)
        for (long zx = 0; zx < (long)nn; ++zx) {
            size_t z = (size_t)zx / n, x = (size_t)zx % n;
            for (int y = 0; y < n; ++y) line[y] = a[z * nn + (size_t)y * n + x];
            fft_line(line, n, w, buf);
            for (int y = 0; y < n; ++y) a[z * nn + (size_t)y * n + x] = line[y];
        }
        /* axis z */
        #pragma omp for schedule(static)
        for (long yx = 0; yx < (long)nn; ++yx) {
            for (int z = 0; z < n; ++z) line[z] = a[(size_t)z * nn + (size_t)yx];
            fft_line(line, n, w, buf);
            for (int z = 0; z < n; ++z) a[(size_t)z * nn + (size_t)yx] = line[z];
        }
        free(line);
        free(buf);
    }
    free(w);
}

/* Signed wavenumber of index k on an n-point grid (R3). */
static double wavenumber(int k, int n)
{
    return (k < (n + 1) / 2) ? (double)k : (double)(k - n);
}

static int is_nyquist(int k, int n)
{
    return n % 2 == 0 && k == n / 2;
}

/* Green symbol xi xi^T / |xi|^2 of mode (kx, ky, kz), averaged over the two
 * signs of every Nyquist component (R3).  Mode 0 is not passed here. */
static void green_symbol(int n, const int kk[3], double G[3][3])
{
    double xi[3];
    int flip = 0;
    for (int d = 0; d < 3; ++d) {
        xi[d] = wavenumber(kk[d], n);
        if (is_nyquist(kk[d], n)) flip |= 1 << d;
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) G[i][j] = 0.0;
    int count = 0;
    for (int s = 0; s < 8; ++s) {
        if (s & ~flip) continue; /* only Nyquist components change sign */
        double v[3];
        for (int d = 0; d < 3; ++d) v[d] = ((s >> d) & 1) ? -xi[d] : xi[d];
        double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) G[i][j] += v[i] * v[j] / v2;
        ++count;
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) G[i][j] /= (double)count;
}

/* Step 4 (Sec. 3, Algorithm) with the Green operator of Sec. 3 for
 * L0 = -k0 I:  c^(xi) = -G(xi) tau^(xi) / k0 for xi != 0, where
 * G = xi xi^T / |xi|^2 (R3), and c^(0) = M E (R2).  tau_hat and c_hat are
 * three full complex spectra (interleaved re/im), [comp][z][y][x]; they may
 * alias. */
void orc_green_apply(int n, double k0, const double E[3],
                     const double *tau_hat_ri, double *c_hat_ri)
{
    size_t M = (size_t)n * n * n;
    const cplx *t = (const cplx *)tau_hat_ri;
    cplx *c = (cplx *)c_hat_ri;
    #pragma omp parallel for schedule(static)
    for (long idx = 0; idx < (long)M; ++idx) {
        int kk[3] = {(int)(idx % n), (int)((idx / n) % n), (int)(idx / ((long)n * n))};
        if (kk[0] == 0 && kk[1] == 0 && kk[2] == 0) {
            for (int i = 0; i < 3; ++i) c[i * M + idx] = (double)M * E[i];
            continue;
        }
        double G[3][3];
        green_symbol(n, kk, G);
        cplx tv[3] = {t[idx], t[M + idx], t[2 * M + idx]};
        for (int i = 0; i < 3; ++i) {
            cplx acc = 0;
            for (int j = 0; j < 3; ++j) acc += G[i][j] * tv[j];
            c[i * M + idx] = -acc / k0;
        }
    }
}

/* R7 (dual scheme): the divergence-free fields at a mode are those whose
 * divergence xi . v vanishes for every sign of the Nyquist components of xi:
 * their Nyquist components are 0 and the others are orthogonal to the
 * non-Nyquist part xi_A of xi.  P is the orthogonal projection on them:
 * 0 on the Nyquist components, I - xi_A xi_A^T / |xi_A|^2 on the others (I if
 * xi_A = 0).  Without Nyquist components this is I - xi xi^T / |xi|^2. */
static void dual_projection(int n, const int kk[3], double P[3][3])
{
    double xa[3];
    int nyq[3];
    double a2 = 0.0;
    for (int d = 0; d < 3; ++d) {
        nyq[d] = is_nyquist(kk[d], n);
        xa[d] = nyq[d] ? 0.0 : wavenumber(kk[d], n);
        a2 += xa[d] * xa[d];
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            if (nyq[i] || nyq[j]) {
                P[i][j] = 0.0;
                continue;
            }
            P[i][j] = (i == j ? 1.0 : 0.0) - (a2 > 0.0 ? xa[i] * xa[j] / a2 : 0.0);
        }
}

/* The dual Green operator of the reference medium k0 on three full spectra
 * in place: k0 P(xi) z^(xi) for xi != 0 (P of R7), k0 z^(0) at xi = 0. */
static void dual_green_apply(int n, double k0, cplx *z)
{
    size_t M = (size_t)n * n * n;
    #pragma omp parallel for schedule(static)
    for (long idx = 0; idx < (long)M; ++idx) {
        cplx zv[3] = {z[idx], z[M + idx], z[2 * M + idx]};
        if (idx == 0) {
            for (int i = 0; i < 3; ++i) z[i * M + idx] = k0 * zv[i];
            continue;
        }
        int kk[3] = {(int)(idx % n), (int)((idx / n) % n), (int)(idx / ((long)n * n))};
        double P[3][3];
        dual_projection(n, kk, P);
        for (int i = 0; i < 3; ++i) {
            cplx acc = 0;
            for (int j = 0; j < 3; ++j) acc += P[i][j] * zv[j];
            z[i * M + idx] = k0 * acc;
        }
    }
}

/* eps_eq of R4: phi^ = FFT(k e) for one load case; returns
 * sqrt(sum_{xi != 0} |xi . phi^|^2 / |xi|^2) / |phi^(0)|. */
static double equilibrium_error(int n, const double *kvox, const double *e3,
                                cplx *work3)
{
    size_t M = (size_t)n * n * n;
    for (int i = 0; i < 3; ++i) {
        for (size_t v = 0; v < M; ++v) work3[i * M + v] = kvox[v] * e3[i * M + v];
        orc_fft3(n, (double *)(work3 + i * M), -1);
    }
    double num = 0.0;
    for (size_t idx = 1; idx < M; ++idx) {
        int kk[3] = {(int)(idx % n), (int)((idx / n) % n), (int)(idx / ((size_t)n * n))};
        int nnyq = 0, nreg = 0;
        for (int d = 0; d < 3; ++d) {
            if (is_nyquist(kk[d], n)) ++nnyq;
            else if (kk[d] != 0) ++nreg;
        }
        /* R4: only modes where the averaged symbol is the projection on xi */
        if (!(nnyq == 0 || (nnyq == 1 && nreg == 0))) continue;
        double xi[3] = {wavenumber(kk[0], n), wavenumber(kk[1], n), wavenumber(kk[2], n)};
        double xi2 = xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2];
        cplx div = 0;
        for (int j = 0; j < 3; ++j) div += xi[j] * work3[j * M + idx];
        num += creal(div * conj(div)) / xi2;
    }
    double den = 0.0;
    for (int i = 0; i < 3; ++i) den += creal(work3[i * M] * conj(work3[i * M]));
    return sqrt(num) / sqrt(den);
}

/* eps_eq of R4 for one load case: kvox the M voxel conductivities, e3 the
 * field [comp][z][y][x] (3 M).  Exported so that the tests can pin it on
 * fields whose flux spectrum is known in closed form. */
double orc_equilibrium_error(int n, const double *kvox, const double *e3)
{
    size_t M = (size_t)n * n * n;
    cplx *work3 = malloc(sizeof(cplx) * 3 * M);
    if (!work3) return -1.0;
    double r = equilibrium_error(n, kvox, e3, work3);
    free(work3);
    return r;
}

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/*
 * The Algorithm of Sec. 3, run for the three load cases E = e_1, e_2, e_3.
 *
 *  n          grid points per side (M = n^3 voxels), n >= 1
 *  phase      M phase ids, [z][y][x], 0 = matrix, 1 = inclusion, 2 = coating
 *  kph        conductivities of the three phases (> 0)
 *  tol        convergence criterion acc (>= 0; 0 runs exactly max_iter)
 *  max_iter   iteration cap (>= 1)
 *  eq_check   0: stop on eps_comp < tol;  1: two-stage test of step 1
 *  init_field optional start field [lc][comp][z][y][x] (9 M), NULL = E
 *  K          out, 9 doubles, K[i*3+j] = <k e_i> for load case j
 *  iters      out, iterations (FFT round trips) per load case
 *  status     out, per load case: 0 converged, 1 not converged, -5 non-finite
 *  final_res  out, last eps_comp per load case
 *  eps_eq     out (may be NULL), eps_eq of the final field per load case
 *  hist       out (may be NULL), [lc][hist_cap] eps_comp history
 *  out_field  out (may be NULL), final field, same layout as init_field
 *  lc_mask    load cases to run (bit j = e_(j+1)); others are left at E with
 *             K column, iters and residual zero
 *  scheme     0 = the accelerated scheme of the Algorithm (k0 of Sec. 5);
 *             1 = the basic scheme named in Sec. 3 as an alternative:
 *             e+ = grad theta_comp, with k0 = (min k + max k) / 2;
 *             2 = the augmented-Lagrangian scheme named in Sec. 3 (k0 of
 *             Sec. 5), for this linear problem the alternating minimisation
 *             of  1/2 <d.k d> + <lam.(e - d)> + k0/2 <|e - d|^2>  over the
 *             local field d, the compatible field e (mean E) and the
 *             multiplier lam:
 *                 d    = (lam + k0 e) / (k + k0)
 *                 e+   = E + P(d - lam / k0)     (P: projection on gradients,
 *                                                 the Green operator times k0)
 *                 lam+ = lam + k0 (e+ - d)
 *             from d = e = E, lam = k E (the first transform is then that of
 *             the accelerated scheme; a start field replaces E in d and e);
 *             per iteration the compatible step, the multiplier step and
 *             the local step.  The residual is the gap sqrt(<|e+ - d+|^2>)
 *             between the compatible and the local field of the same
 *             iteration, the tensor column their common limit's flux
 *             <k d+>.  out_field returns lam - k0 d, the input of the next
 *             compatible step ((k - k0) e at the fixed point, where d = e
 *             and lam = k e).  eq_check is not used.
 *             Parity unpinned against the cited work (its equations are not
 *             in the paper); pinned by the same closed forms as the others.
 *             3 = the dual scheme named in Sec. 3: the flux phi is the
 *             iterate, kept divergence free, with the dual Green operator of
 *             the reference medium k0 (in Fourier space k0 P for xi != 0, P
 *             the projection on divergence-free fields of R7, and k0 at
 *             xi = 0):
 *                 e    = phi / k
 *                 phi+ = phi - Delta0 * (e - E)
 *             from phi = k0 E, with k0 = 2 min k max k / (min k + max k)
 *             (the mean of the extreme resistivities, the dual of the basic
 *             scheme's choice).  At the fixed point e - E is a gradient of
 *             zero mean, so e is compatible with <e> = E and phi = k e is
 *             divergence free.  The residual is sqrt(<|phi+ - phi|^2>) / k0,
 *             the distance of e from the compatible fields of mean E; the
 *             tensor column is <phi+>; out_field returns phi.  init_field
 *             and eq_check are refused.
 *             4 = the polarization scheme named in Sec. 3, read as the
 *             relaxed iteration on the polarization tau = (k - k0) e with
 *             the compatible field of step 4 (k0 of Sec. 5):
 *                 c    = E - Gamma0 tau
 *                 g    = ((k - k0) c - tau) / (k + k0)
 *                 tau+ = tau + alpha k0 g,   0 < alpha <= 2
 *             from tau = (k - k0) E (or the start field); residual
 *             sqrt(<g^2>), tensor column <tau+ + k0 c>.  alpha = 1 gives the
 *             augmented-Lagrangian scheme (2), alpha = 2 the iterates of the
 *             accelerated scheme (tau = (k - k0) e of scheme 0).  out_field
 *             returns tau; eq_check is refused.
 *             Both: parity unpinned against the cited works (their equations
 *             are not in the paper); pinned by closed forms, the dense
 *             solves of the discrete problem and their rate bounds.
 *  alpha      relaxation of scheme 4 (ignored by the others)
 */
int orc_homogenize(int n, const uint8_t *phase, const double kph[3], double tol,
                   int max_iter, int eq_check, const double *init_field,
                   double *K, int *iters, int *status, double *final_res,
                   double *eps_eq, double *hist, int hist_cap, double *out_field,
                   int lc_mask, int scheme, double alpha)
{
    if (n < 1 || max_iter < 1 || !(tol >= 0.0) || !phase || !kph || !K) return ORC_ERR_ARG;
    for (int p = 0; p < 3; ++p)
        if (!(kph[p] > 0.0) || !isfinite(kph[p])) return ORC_ERR_ARG;
    size_t M = (size_t)n * n * n;
    for (size_t v = 0; v < M; ++v)
        if (phase[v] > 2) return ORC_ERR_ARG;

    if (scheme < 0 || scheme > 4) return ORC_ERR_ARG;
    if (scheme >= 3 && eq_check) return ORC_ERR_ARG;
    if (scheme == 3 && init_field) return ORC_ERR_ARG;
    if (scheme == 4 && !(alpha > 0.0 && alpha <= 2.0)) return ORC_ERR_ARG;
    /* Sec. 5: L0 = -sqrt(min k * max k) I over the three given k (R1);
     * the basic scheme takes the arithmetic mean of the extremes, the dual
     * scheme their harmonic mean. */
    double kmin = fmin(kph[0], fmin(kph[1], kph[2]));
    double kmax = fmax(kph[0], fmax(kph[1], kph[2]));
    double k0 = scheme == 1 ? 0.5 * (kmin + kmax)
              : scheme == 3 ? 2.0 * kmin * kmax / (kmin + kmax)
                            : sqrt(kmin * kmax);

    double *kvox = malloc(sizeof(double) * M);
    double *e = malloc(sizeof(double) * 3 * M);
    cplx *t = malloc(sizeof(cplx) * 3 * M);
    /* augmented Lagrangian: the local field d and the multiplier lam */
    double *d = scheme == 2 ? malloc(sizeof(double) * 3 * M) : NULL;
    double *lam = scheme == 2 ? malloc(sizeof(double) * 3 * M) : NULL;
    if (!kvox || !e || !t || (scheme == 2 && (!d || !lam))) {
        free(kvox); free(e); free(t); free(d); free(lam);
        return ORC_ERR_ARG;
    }
    for (size_t v = 0; v < M; ++v) kvox[v] = kph[phase[v]];

    for (int lc = 0; lc < 3; ++lc) {
        double E[3] = {0.0, 0.0, 0.0};
        E[lc] = 1.0;
        if (!((lc_mask >> lc) & 1)) {
            for (int i = 0; i < 3; ++i) K[i * 3 + lc] = 0.0;
            if (iters) iters[lc] = 0;
            if (status) status[lc] = ORC_OK;
            if (final_res) final_res[lc] = 0.0;
            if (eps_eq) eps_eq[lc] = -1.0;
            if (out_field)
                for (int i = 0; i < 3; ++i)
                    for (size_t v = 0; v < M; ++v)
                        out_field[(size_t)(lc * 3 + i) * M + v] = E[i];
            continue;
        }
        /* Initialize: grad theta^0 = grad Theta */
        for (int i = 0; i < 3; ++i)
            for (size_t v = 0; v < M; ++v)
                e[i * M + v] = init_field ? init_field[(lc * 3 + i) * M + v] : E[i];

        double F[3] = {0.0, 0.0, 0.0}, r = 0.0, eq = -1.0;
        int st = ORC_NOT_CONVERGED, it = 0;
        if (scheme == 2)
            for (int i = 0; i < 3; ++i)
                for (size_t v = 0; v < M; ++v) {
                    d[i * M + v] = e[i * M + v];                 /* d^0 = e^0 */
                    lam[i * M + v] = kvox[v] * e[i * M + v];     /* lam^0 = k e^0 */
                }
        while (scheme == 2 && it < max_iter) {
            /* compatible step: e+ = E + P(d - lam/k0) = E - Gamma0 * (lam - k0 d),
             * through the transform, the Green operator and the inverse */
            for (int i = 0; i < 3; ++i)
                for (size_t v = 0; v < M; ++v) t[i * M + v] = lam[i * M + v] - k0 * d[i * M + v];
            for (int i = 0; i < 3; ++i) orc_fft3(n, (double *)(t + i * M), -1);
            orc_green_apply(n, k0, E, (const double *)t, (double *)t);
            for (int i = 0; i < 3; ++i) orc_fft3(n, (double *)(t + i * M), +1);
            /* multiplier step lam+ = lam + k0 (e+ - d); local step
             * d+ = (lam+ + k0 e+) / (k + k0); residual sqrt(<|e+ - d+|^2>);
             * flux <k d+> */
            double r2 = 0.0;
            for (int i = 0; i < 3; ++i) {
                double s = 0.0;
                for (size_t v = 0; v < M; ++v) {
                    double c = creal(t[i * M + v]) / (double)M;
                    lam[i * M + v] += k0 * (c - d[i * M + v]);
                    d[i * M + v] = (lam[i * M + v] + k0 * c) / (kvox[v] + k0);
                    double g = c - d[i * M + v];
                    r2 += g * g;
                    e[i * M + v] = c;
                    s += kvox[v] * d[i * M + v];
                }
                F[i] = s / (double)M;
            }
            r = sqrt(r2 / (double)M);
            if (hist && it < hist_cap) hist[lc * hist_cap + it] = r;
            ++it;
            if (!isfinite(r)) {
                st = ORC_ERR_NONFINITE;
                break;
            }
            if (r < tol) {
                st = ORC_OK;
                break;
            }
        }
        if (scheme == 3) /* the flux iterate starts at k0 E (divergence free) */
            for (int i = 0; i < 3; ++i)
                for (size_t v = 0; v < M; ++v) e[i * M + v] = k0 * E[i];
        while (scheme == 3 && it < max_iter) {
            /* e = phi / k; the dual Green operator on e - E */
            for (int i = 0; i < 3; ++i)
                for (size_t v = 0; v < M; ++v) t[i * M + v] = e[i * M + v] / kvox[v] - E[i];
            for (int i = 0; i < 3; ++i) orc_fft3(n, (double *)(t + i * M), -1);
            dual_green_apply(n, k0, t);
            for (int i = 0; i < 3; ++i) orc_fft3(n, (double *)(t + i * M), +1);
            /* phi+ = phi - Delta0 * (e - E); residual and mean flux */
            double r2 = 0.0;
            for (int i = 0; i < 3; ++i) {
                double sF = 0.0;
                for (size_t v = 0; v < M; ++v) {
                    double d = creal(t[i * M + v]) / (double)M;
                    r2 += d * d;
                    e[i * M + v] -= d;
                    sF += e[i * M + v];
                }
                F[i] = sF / (double)M;
            }
            r = sqrt(r2 / (double)M) / k0;
            if (hist && it < hist_cap) hist[lc * hist_cap + it] = r;
            ++it;
            if (!isfinite(r)) {
                st = ORC_ERR_NONFINITE;
                break;
            }
            if (r < tol) {
                st = ORC_OK;
                break;
            }
        }
        if (scheme == 4) /* the polarization of the start field */
            for (int i = 0; i < 3; ++i)
                for (size_t v = 0; v < M; ++v) e[i * M + v] *= kvox[v] - k0;
        while (scheme == 4 && it < max_iter) {
            /* c = E - Gamma0 tau (steps 3-5 on tau) */
            for (int i = 0; i < 3; ++i)
                for (size_t v = 0; v < M; ++v) t[i * M + v] = e[i * M + v];
            for (int i = 0; i < 3; ++i) orc_fft3(n, (double *)(t + i * M), -1);
            orc_green_apply(n, k0, E, (const double *)t, (double *)t);
            for (int i = 0; i < 3; ++i) orc_fft3(n, (double *)(t + i * M), +1);
            /* g = ((k - k0) c - tau) / (k + k0); tau+ = tau + alpha k0 g */
            double r2 = 0.0;
            for (int i = 0; i < 3; ++i) {
                double sF = 0.0;
                for (size_t v = 0; v < M; ++v) {
                    double c = creal(t[i * M + v]) / (double)M;
                    double g = ((kvox[v] - k0) * c - e[i * M + v]) / (kvox[v] + k0);
                    r2 += g * g;
                    e[i * M + v] += alpha * k0 * g;
                    sF += e[i * M + v] + k0 * c;
                }
                F[i] = sF / (double)M;
            }
            r = sqrt(r2 / (double)M);
            if (hist && it < hist_cap) hist[lc * hist_cap + it] = r;
            ++it;
            if (!isfinite(r)) {
                st = ORC_ERR_NONFINITE;
                break;
            }
            if (r < tol) {
                st = ORC_OK;
                break;
            }
        }
        while (scheme <= 1 && it < max_iter) {
            eq = -1.0;
            /* step 2: tau = (k - k0) e */
            for (int i = 0; i < 3; ++i)
                for (size_t v = 0; v < M; ++v)
                    t[i * M + v] = (kvox[v] - k0) * e[i * M + v];
            /* step 3: tau^ = FFT(tau) */
            for (int i = 0; i < 3; ++i) orc_fft3(n, (double *)(t + i * M), -1);
            /* step 4: Green operator, xi = 0 pinned to E */
            orc_green_apply(n, k0, E, (const double *)t, (double *)t);
            /* step 5: grad theta_comp = FFT^-1, real part (R3) */
            for (int i = 0; i < 3; ++i) orc_fft3(n, (double *)(t + i * M), +1);
            /* step 6: eps_comp = sqrt(<|e - c|^2>) / |E| */
            double r2 = 0.0;
            for (int i = 0; i < 3; ++i)
                for (size_t v = 0; v < M; ++v) {
                    double d = e[i * M + v] - creal(t[i * M + v]) / (double)M;
                    r2 += d * d;
                }
            r = sqrt(r2 / (double)M);
            /* step 7: e+ = e + 2 k0 / (k + k0) (c - e); basic scheme: e+ = c */
            for (int i = 0; i < 3; ++i)
                for (size_t v = 0; v < M; ++v) {
                    double c = creal(t[i * M + v]) / (double)M;
                    if (scheme == 1) {
                        e[i * M + v] = c;
                    } else {
                        double wgt = 2.0 * k0 / (kvox[v] + k0);
                        e[i * M + v] += wgt * (c - e[i * M + v]);
                    }
                }
            /* <phi> of the updated field (R5): F_i = <k e_i> */
            for (int i = 0; i < 3; ++i) {
                double s = 0.0;
                for (size_t v = 0; v < M; ++v) s += kvox[v] * e[i * M + v];
                F[i] = s / (double)M;
            }
            if (hist && it < hist_cap) hist[lc * hist_cap + it] = r;
            ++it;
            if (!isfinite(r)) {
                st = ORC_ERR_NONFINITE;
                break;
            }
            if (r < tol) {
                if (!eq_check) {
                    st = ORC_OK;
                    break;
                }
                /* step 1: second stage on the current iterate */
                eq = equilibrium_error(n, kvox, e, t);
                if (eq < tol) {
                    st = ORC_OK;
                    break;
                }
            }
        }
        for (int i = 0; i < 3; ++i) K[i * 3 + lc] = F[i];
        if (iters) iters[lc] = it;
        if (status) status[lc] = st;
        if (final_res) final_res[lc] = r;
        if (eps_eq)
            eps_eq[lc] = (eq >= 0.0) ? eq : (scheme >= 3 ? -1.0 : equilibrium_error(n, kvox, e, t));
        if (out_field && scheme == 2)
            for (int i = 0; i < 3; ++i)
                for (size_t v = 0; v < M; ++v)
                    out_field[(size_t)(lc * 3 + i) * M + v] = lam[i * M + v] - k0 * d[i * M + v];
        else if (out_field)
            memcpy(out_field + (size_t)lc * 3 * M, e, sizeof(double) * 3 * M);
    }
    free(kvox);
    free(e);
    free(t);
    free(d);
    free(lam);
    return ORC_OK;
}

/* ========================================================================
 * Elastic case.  Sec. 6 names linear elasticity as the extension of the
 * method; the scheme is the same accelerated iteration with isotropic phases
 * C = 3 kappa J + 2 mu K (J, K: the hydrostatic and deviatoric projectors)
 * and the isotropic reference C0 (kappa0, mu0):
 *   tau   = (C - C0) : e                                      (step 2)
 *   c^    = -Gamma0(xi) : tau^ for xi != 0, c^(0) = M E       (steps 3-5)
 *   eps   = sqrt(<|e - c|^2>) / |E|   (Frobenius norm of the full tensor)
 *   e+    = e + 2 (C + C0)^-1 C0 : (c - e), i.e. the hydrostatic part of
 *           c - e times 2 kappa0 / (kappa + kappa0), the deviatoric part
 *           times 2 mu0 / (mu + mu0)                          (step 7)
 *   column of C_hom: the mean stress <C : e+>
 * with the Green operator of the isotropic reference medium
 *   Gamma0_ijkh = (d_ki x_h x_j + d_hi x_k x_j + d_kj x_h x_i + d_hj x_k x_i)
 *                 / (4 mu0 |x|^2)
 *               - (lambda0 + mu0) / (mu0 (lambda0 + 2 mu0)) x_i x_j x_k x_h / |x|^4,
 * lambda0 = kappa0 - 2 mu0 / 3, averaged over the signs of the Nyquist
 * components as in R3, and kappa0 = sqrt(min kappa max kappa),
 * mu0 = sqrt(min mu max mu) (the Sec. 5 rule applied to each modulus).
 * Tensors are stored as the 6 components 11, 22, 33, 23, 13, 12 of the full
 * symmetric tensor (tensor shear components, not engineering ones).
 * The equations are not in the paper (they are in the cited elastic work):
 * parity unpinned against that work; pinned by closed forms and a dense
 * displacement solve in the tests.
 * ====================================================================== */

static const int EL_I[6] = {0, 1, 2, 1, 0, 0};
static const int EL_J[6] = {0, 1, 2, 2, 2, 1};

static int el_comp(int i, int j)
{
    if (i == j) return i;
    int a = i < j ? i : j, b = i < j ? j : i;
    return (a == 1 && b == 2) ? 3 : (a == 0 && b == 2) ? 4 : 5;
}

/* Gamma0_ijkh at mode kk, averaged over the Nyquist signs (R3). */
static void el_green_symbol(int n, const int kk[3], double mu0, double beta, double G[3][3][3][3])
{
    double xi[3];
    int flip = 0;
    for (int d = 0; d < 3; ++d) {
        xi[d] = wavenumber(kk[d], n);
        if (is_nyquist(kk[d], n)) flip |= 1 << d;
    }
    memset(G, 0, sizeof(double) * 81);
    int count = 0;
    for (int s = 0; s < 8; ++s) {
        if (s & ~flip) continue;
        double v[3];
        for (int d = 0; d < 3; ++d) v[d] = ((s >> d) & 1) ? -xi[d] : xi[d];
        double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                for (int k = 0; k < 3; ++k)
                    for (int h = 0; h < 3; ++h) {
                        double a = ((k == i) * v[h] * v[j] + (h == i) * v[k] * v[j] +
                                    (k == j) * v[h] * v[i] + (h == j) * v[k] * v[i]) / (4.0 * mu0 * v2);
                        double b = beta * v[i] * v[j] * v[k] * v[h] / (v2 * v2);
                        G[i][j][k][h] += a - b;
                    }
        ++count;
    }
    for (int i = 0; i < 81; ++i) ((double *)G)[i] /= (double)count;
}

int orc_homogenize_elastic(int n, const uint8_t *phase, const double moduli[6], int nlc,
                           const double *Elc, double tol, int max_iter, double *S, int *iters,
                           int *status, double *final_res, double *hist, int hist_cap,
                           double *out_field)
{
    if (n < 1 || nlc < 1 || !Elc || max_iter < 1 || !(tol >= 0.0) || !phase || !moduli || !S)
        return ORC_ERR_ARG;
    for (int q = 0; q < 6; ++q)
        if (!(moduli[q] > 0.0) || !isfinite(moduli[q])) return ORC_ERR_ARG;
    size_t M = (size_t)n * n * n;
    for (size_t v = 0; v < M; ++v)
        if (phase[v] > 2) return ORC_ERR_ARG;
    double kap[3], mu[3];
    for (int p = 0; p < 3; ++p) {
        kap[p] = moduli[2 * p];
        mu[p] = moduli[2 * p + 1];
    }
    double kmin = fmin(kap[0], fmin(kap[1], kap[2])), kmax = fmax(kap[0], fmax(kap[1], kap[2]));
    double mmin = fmin(mu[0], fmin(mu[1], mu[2])), mmax = fmax(mu[0], fmax(mu[1], mu[2]));
    double kap0 = sqrt(kmin * kmax), mu0 = sqrt(mmin * mmax);
    double lam0 = kap0 - 2.0 * mu0 / 3.0;
    double beta = (lam0 + mu0) / (mu0 * (lam0 + 2.0 * mu0));

    double *e = malloc(sizeof(double) * 6 * M);
    cplx *t = malloc(sizeof(cplx) * 6 * M);
    if (!e || !t) {
        free(e);
        free(t);
        return ORC_ERR_ARG;
    }
    for (int lc = 0; lc < nlc; ++lc) {
        const double *E = Elc + 6 * lc;
        double E2 = 0.0;
        for (int q = 0; q < 6; ++q) E2 += (q < 3 ? 1.0 : 2.0) * E[q] * E[q];
        double Enorm = sqrt(E2);
        for (int q = 0; q < 6; ++q)
            for (size_t v = 0; v < M; ++v) e[q * M + v] = E[q];
        double r = 0.0, Sm[6] = {0, 0, 0, 0, 0, 0};
        int st = ORC_NOT_CONVERGED, it = 0;
        while (it < max_iter) {
            /* tau = (C - C0) : e = 3 (kappa - kappa0) (tr e / 3) I + 2 (mu - mu0) dev e */
            for (size_t v = 0; v < M; ++v) {
                int p = phase[v];
                double tr3 = (e[v] + e[M + v] + e[2 * M + v]) / 3.0;
                for (int q = 0; q < 6; ++q) {
                    double dev = e[q * M + v] - (q < 3 ? tr3 : 0.0);
                    t[q * M + v] = 3.0 * (kap[p] - kap0) * (q < 3 ? tr3 : 0.0) + 2.0 * (mu[p] - mu0) * dev;
                }
            }
            for (int q = 0; q < 6; ++q) orc_fft3(n, (double *)(t + q * M), -1);
            /* c^ = -Gamma0 : tau^ (sum over the full k, h), c^(0) = M E */
            #pragma omp parallel for schedule(static)
            for (long idx = 0; idx < (long)M; ++idx) {
                int kk[3] = {(int)(idx % n), (int)((idx / n) % n), (int)(idx / ((long)n * n))};
                if (kk[0] == 0 && kk[1] == 0 && kk[2] == 0) {
                    for (int q = 0; q < 6; ++q) t[q * M + idx] = (double)M * E[q];
                    continue;
                }
                double G[3][3][3][3];
                el_green_symbol(n, kk, mu0, beta, G);
                cplx tv[6], cv[6];
                for (int q = 0; q < 6; ++q) tv[q] = t[q * M + idx];
                for (int q = 0; q < 6; ++q) {
                    cplx acc = 0;
                    for (int k = 0; k < 3; ++k)
                        for (int h = 0; h < 3; ++h) acc += G[EL_I[q]][EL_J[q]][k][h] * tv[el_comp(k, h)];
                    cv[q] = -acc;
                }
                for (int q = 0; q < 6; ++q) t[q * M + idx] = cv[q];
            }
            for (int q = 0; q < 6; ++q) orc_fft3(n, (double *)(t + q * M), +1);
            /* residual, update, mean stress */
            double r2 = 0.0;
            double acc[6] = {0, 0, 0, 0, 0, 0};
            for (size_t v = 0; v < M; ++v) {
                int p = phase[v];
                double d[6];
                for (int q = 0; q < 6; ++q) {
                    d[q] = creal(t[q * M + v]) / (double)M - e[q * M + v];
                    r2 += (q < 3 ? 1.0 : 2.0) * d[q] * d[q];
                }
                double dtr3 = (d[0] + d[1] + d[2]) / 3.0;
                double wk = 2.0 * kap0 / (kap[p] + kap0), wm = 2.0 * mu0 / (mu[p] + mu0);
                for (int q = 0; q < 6; ++q) {
                    double hyd = q < 3 ? dtr3 : 0.0;
                    e[q * M + v] += wk * hyd + wm * (d[q] - hyd);
                }
                double tr3 = (e[v] + e[M + v] + e[2 * M + v]) / 3.0;
                for (int q = 0; q < 6; ++q) {
                    double hyd = q < 3 ? tr3 : 0.0;
                    acc[q] += 3.0 * kap[p] * hyd + 2.0 * mu[p] * (e[q * M + v] - hyd);
                }
            }
            for (int q = 0; q < 6; ++q) Sm[q] = acc[q] / (double)M;
            r = sqrt(r2 / (double)M) / Enorm;
            if (hist && it < hist_cap) hist[lc * hist_cap + it] = r;
            ++it;
            if (!isfinite(r)) {
                st = ORC_ERR_NONFINITE;
                break;
            }
            if (r < tol) {
                st = ORC_OK;
                break;
            }
        }
        for (int q = 0; q < 6; ++q) S[6 * lc + q] = Sm[q];
        if (iters) iters[lc] = it;
        if (status) status[lc] = st;
        if (final_res) final_res[lc] = r;
        if (out_field) memcpy(out_field + (size_t)lc * 6 * M, e, sizeof(double) * 6 * M);
    }
    free(e);
    free(t);
    return ORC_OK;
}
