/*
 * rvehom.h -- C ABI of the MI355X library that computes the effective thermal
 * conductivity tensor of a periodic voxelized three-phase RVE with the
 * accelerated (Eyre-Milton) FFT scheme.
 *
 * Paper: S. Lemaitre, V. Salnikov, D. Choi, P. Karamian, arXiv:1504.07499.
 *   Sec. 2  RVE generation (RSA spheres, voxelization, coating layer l).
 *   Sec. 3  problem: periodic RVE V, phi = -L grad(theta), div(phi) = 0,
 *           <grad(theta)> = grad(Theta) imposed; polarization eq. (1);
 *           Lippmann-Schwinger eq. (3); Green operator Gamma^0; the
 *           Algorithm "FFT-based homogenization scheme for thermal
 *           conductivity case"; L_hom from <phi> = -L_hom grad(Theta).
 *   Sec. 5  phase tensors k I and the reference medium
 *           L0 = -sqrt(min k * max k) I.
 *
 * Conventions shared by every call:
 *  - phase images are N^3 bytes, [z][y][x] with x fastest; 0 = matrix,
 *    1 = inclusion, 2 = coating;
 *  - k_phases[3] are the conductivities of matrix, inclusion, coating
 *    (finite, > 0);
 *  - the three load cases are the unit gradients E = e_1, e_2, e_3; column j
 *    of K (K[i*3 + j], row-major) is <k e_i> for load case j, i.e. L_hom e_j;
 *  - fields exchanged with the host are FP64, [lc][comp][z][y][x] (9 N^3);
 *  - N must be one of the grid sizes the library was built for
 *    (rve_supported_n); every call validates its arguments and returns an
 *    rve_status; no call aborts or throws across the ABI;
 *  - handles are not thread-safe: do not use one handle from two threads at
 *    once.  Distinct handles may be used concurrently.
 */
#ifndef RVEHOM_H
#define RVEHOM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RVE_OK = 0,             /* converged: eps_comp < tol (and eps_eq < tol if asked) */
    RVE_NOT_CONVERGED = 1,  /* max_iter reached; K holds the last iterate */
    RVE_STALLED = 2,        /* no new residual minimum over stall_window iterations */
    RVE_PENDING = 3,        /* serving: request not finished yet */
    RVE_ERR_ARG = -1,       /* invalid argument; nothing was computed */
    RVE_ERR_JAMMED = -2,    /* spheres could not be placed */
    RVE_ERR_OOM = -3,       /* device or host allocation failed */
    RVE_ERR_DEVICE = -4,    /* a HIP runtime call failed */
    RVE_ERR_NONFINITE = -5  /* NaN/Inf met in the FP64 residual */
} rve_status;

typedef struct rve_s *rve_t;

/* Geometry of Sec. 2: N^3 voxels, n_spheres identical spheres of volume
 * fraction f (coating included), coating layer l = width / radius. */
typedef struct {
    int n;
    int n_spheres;
    double volume_fraction;
    double layer;
    uint64_t seed;
} rve_geom;

typedef struct {
    int max_iter;           /* iteration cap; 0 = default 10000 */
    int precision;          /* 0 = FP32 FFT/update with FP64 reductions, 1 = FP64 */
    int equilibrium_check;  /* 1 = two-stage stop of step 1 (eps_comp then eps_eq) */
    int stall_window;       /* -1 = default (50 in FP32, off in FP64), 0 = off */
    int lc_mask;            /* load cases to solve, bit j = e_(j+1); 0 = all three */
    int timing;             /* bitmask of kernels to time with HIP events: 1 fwd_plane,
                               2 zgreen, 4 inv_plane, 8 reduce (15 = all); the events are
                               recorded inside the replayed iteration graphs.  + 16
                               (sampled): only one batch of iterations in four is
                               timed, which keeps the events' own cost low */
    void *stream;           /* hipStream_t for all work, NULL = the handle's own */
    const double *init_field; /* host, 9 N^3 FP64 start field, NULL = E */
    double *out_field;      /* host, 9 N^3 FP64 final field, NULL = not returned */
    void *workspace;        /* device buffer of >= rve_workspace_size bytes, or NULL
                               (the library then allocates and caches its own) */
    size_t workspace_bytes;
    int scheme;             /* 0 = accelerated (Eyre-Milton, Sec. 3 Algorithm, k0 of Sec. 5);
                               1 = basic scheme named in Sec. 3 (e+ = c, the compatible
                               field, with k0 = (min k + max k) / 2);
                               2 = augmented-Lagrangian scheme named in Sec. 3 (k0 of
                               Sec. 5): local step d = (lam + k0 e) / (k + k0), compatible
                               step e+ = E - Gamma0 (lam - k0 d), multiplier step
                               lam+ = lam + k0 (e+ - d), from d = e = E (or init_field)
                               and lam = k d; final_residual is sqrt<|e+ - d+|^2>, K the
                               flux <k d+>, out_field the state lam - k0 d; with
                               equilibrium_check: RVE_ERR_ARG;
                               3 = dual scheme named in Sec. 3: the flux phi is the
                               iterate, phi+ = phi - Delta0 (phi / k - E) from phi = k0 E,
                               k0 = 2 min k max k / (min k + max k), Delta0 the dual Green
                               operator k0 P (P: projection on divergence-free fields; on an
                               even grid those whose divergence vanishes for every sign of
                               the Nyquist components) and k0 at xi = 0; final_residual is
                               sqrt<|phi+ - phi|^2> / k0, K the flux <phi+>, out_field phi;
                               with init_field or equilibrium_check: RVE_ERR_ARG;
                               4 = polarization scheme named in Sec. 3 (k0 of Sec. 5): on
                               tau = (k - k0) e, c = E - Gamma0 tau,
                               g = ((k - k0) c - tau) / (k + k0), tau+ = tau + alpha k0 g;
                               final_residual sqrt<g^2>, K <tau+ + k0 c>, out_field tau;
                               alpha = 1 is scheme 2, and with alpha = 2 the iterates are
                               (k - k0) times those of scheme 0; with equilibrium_check:
                               RVE_ERR_ARG.  eps_eq is -1 for schemes 3 and 4 */
    int fp32_refine;        /* FP32 only.  0 = default: a load case that the FP32 rounding
                               floor stops above tol (RVE_STALLED by the floor or stall rule)
                               is continued in FP64 from its FP32 field, with the same scheme
                               and tol, until eps_comp < tol (step 6); iters then counts both
                               parts and refine_iters the FP64 ones.  The FP64 workspace of the
                               grid is allocated on first use and cached on the handle.
                               -1 = off: the load case ends RVE_STALLED with the last FP32 K. */
    int path_flags;         /* measurement switches, 0 = the library's choice.  Results do not
                               depend on them (the same arithmetic in the same order) but
                               where noted for 64 / 128:
                               1 = launch kernel by kernel instead of replaying iteration graphs,
                               2 = separate inverse and forward plane passes instead of the
                                   fused one, 4 = the reduction as a launch of its own instead
                               of inside the next z pass, 8 = one stream for the three load
                               cases instead of three concurrent chains, 16 / 32 = the default /
                               the alternative z-pass tile width instead of the autotuned one;
                               64 / 128 = the default / the alternative thread count of the
                               fused plane pass instead of the autotuned one (the same
                               arithmetic per voxel, up to the compiler's instruction choice
                               for each shape, and another grouping of the FP64 partial sums
                               of eps_comp and the flux: results agree to rounding) */
    double alpha;           /* scheme 4: the relaxation alpha in (0, 2]; 0 = default 2 */
} rve_opts;

typedef struct {
    double K[9];               /* L_hom, row-major, column j = load case e_(j+1) */
    int iters[3];              /* FFT round trips per load case */
    int status[3];             /* rve_status per load case */
    double final_residual[3];  /* last eps_comp per load case */
    double eps_eq[3];          /* equilibrium error of the final field (-1 if not computed) */
    double solve_ms;           /* device time of the iteration phase (HIP events) */
    int refine_iters[3];       /* FP64 iterations of the fp32_refine continuation (0 if none) */
} rve_result;

/* Per-kernel device time of the last homogenize call with opts.timing != 0,
 * over the launches that did work (those of iterations before the last load
 * case finished).  names: "fwd_plane", "zgreen", "inv_plane", "reduce".
 * total_bytes: algorithmic HBM bytes of those launches (each pass reads and
 * writes its fields once; load cases already converged are not counted). */
typedef struct {
    const char *name[4];
    double total_ms[4];
    int launches[4];
    double total_bytes[4];
} rve_kernel_times;

/* Grid sizes N the library supports for a precision (0 FP32, 1 FP64): the
 * {2,3}-smooth N from 8 to 512 with N % 4 == 0 and at most two factors 3
 * that it instantiates (8, 12, 16, 24, 32, 36, 48, 64, 72, 96, 128, 144,
 * 192, 256, 288, 384, 512).  out: up to cap ints; count receives the
 * number. */
rve_status rve_supported_n(int precision, int *out, int cap, int *count);

/* The autotuner's choices.  The first solve of each (GPU architecture,
 * precision, N) in a process times the z pass at its two tile widths, and
 * the fused plane pass (grids whose whole xy-plane fits in LDS) at its two
 * thread counts per workgroup, and keeps the faster of each (path_flags 16
 * to 128 fix them instead).  The z-tile choice does not change a result;
 * the plane choice changes results at rounding level only.  The
 * choices are text lines "<gfx arch> <precision 0|1> <n> ztile <0|1>" and
 * "<gfx arch> <precision 0|1> <n> plane <0|1>" (1 = the other width or
 * thread count).
 * rve_tune_export: copies the choices made or imported in this process into
 *   buf (at most cap - 1 characters, then a terminating 0; buf may be null
 *   with cap 0) and returns the size needed including the terminating 0.
 * rve_tune_import: adds the choices of such text (blank lines ignored; a
 *   line for another architecture is kept but applies only to devices of
 *   that architecture); a malformed line gives RVE_ERR_ARG and imports
 *   nothing.  Imported choices replace the timing for their grids. */
size_t rve_tune_export(char *buf, size_t cap);
rve_status rve_tune_import(const char *text);

/* Sec. 2: RSA placement + voxelization of g, uploaded to the current HIP
 * device.  RVE_ERR_ARG for n unsupported, n_spheres < 1, f or l outside
 * (0, 1) or a sphere radius >= 0.5; RVE_ERR_JAMMED if the spheres do not
 * fit.  *out is owned by the caller (rve_destroy). */
rve_status rve_create(const rve_geom *g, rve_t *out);

/* Same, from a caller phase image (host, n^3 bytes, copied). */
rve_status rve_create_from_phases(int n, const uint8_t *phases, rve_t *out);

/* Copy the phase image back (cap >= n^3 bytes). */
rve_status rve_get_phases(rve_t rve, uint8_t *out, size_t cap);

/* Sphere list of Sec. 2 (centre x, y, z and radius per sphere; coating
 * included in the radius).  count = spheres written; layer may be NULL.
 * An RVE made from a phase image has no spheres (count = 0). */
rve_status rve_get_spheres(rve_t rve, double *xyzr, int cap, int *count, double *layer);

/* Grid size of an RVE. */
int rve_n(rve_t rve);

/* Device workspace bytes homogenize needs for this RVE and precision (one
 * workspace: a caller-provided one, or one solve of a single load case).  A
 * solve of all three load cases without a caller workspace, without the
 * two-stage stop and without a start or final field, on a grid whose
 * xy-planes fit in LDS (whole or split; not FP64 256^3 and up, nor FP32
 * 288^3 and up), runs the
 * load cases as three concurrent chains and allocates three such workspaces
 * (cached on the handle until rve_destroy); the results are the same. */
size_t rve_workspace_size(rve_t rve, int precision);

/* The Algorithm of Sec. 3 for the three load cases, on the GPU.
 * k_phases: host, 3 conductivities; tol: convergence criterion acc (> 0,
 * or 0 to run exactly max_iter iterations); opts may be NULL; out: host.
 * residual_history: host [3][hist_cap] eps_comp per iteration, or NULL.
 * Returns the worst per-load-case status (an error < 0 first, then
 * NONFINITE, STALLED, NOT_CONVERGED, OK).  Stream-ordered on opts->stream;
 * returns after the results are on the host. */
rve_status homogenize(rve_t rve, const double k_phases[3], double tol, const rve_opts *opts,
                      rve_result *out, double *residual_history, int hist_cap);

/* homogenize for callers that cannot allocate (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same kernels
 * in the same order and the same results as homogenize, with every device
 * buffer beyond the RVE's phase image in one fixed array of device memory
 * that belongs to the library image (64 MiB per GPU, held from the first
 * call on that GPU until the process ends).  No hipMalloc, hipFree, pinned
 * host allocation, stream, event or graph is created; parameters and
 * results pass through stack buffers and the call synchronises opts->stream
 * (NULL: the null stream) several times.
 * Limit: the workspace (rve_workspace_size) of the precision, plus for FP32
 * with fp32_refine the FP64 workspace of the continuation, must fit in
 * 64 MiB (N <= 64); larger grids give RVE_ERR_ARG with the bytes needed.
 * Honoured opts: precision, max_iter, stall_window, lc_mask, scheme,
 * fp32_refine, stream and the path_flags 2, 4 and 16 to 128 (without them the
 * z-tile width and the fused pass's thread count are the autotuner's choices
 * made or imported in this process for the grid, else the defaults: this
 * call times nothing); init_field, out_field,
 * workspace, timing or equilibrium_check give RVE_ERR_ARG.  solve_ms is
 * host wall time.  Calls on one GPU share its array: the library
 * serialises calls from threads of one process on a GPU (each call leaves
 * the array in use until it returns), and every solve initialises what it
 * reads; calls from different processes on one GPU each have their own
 * copy of the library image. */
rve_status homogenize_no_alloc(rve_t rve, const double k_phases[3], double tol, const rve_opts *opts,
                               rve_result *out, double *residual_history, int hist_cap);

/* Several RVEs (any mix of grid sizes) solved concurrently on the device.
 * k_phases: [3*count]; tol: [count]; opts applies to all (its fields and
 * workspace must be NULL); out: [count]. */
rve_status homogenize_batch(int count, const rve_t *rves, const double *k_phases,
                            const double *tol, const rve_opts *opts, rve_result *out);

/* Kernel timings of the last homogenize call on this handle. */
rve_status rve_get_kernel_times(rve_t rve, rve_kernel_times *out);

/* ---- Elastic case: linear elasticity with isotropic phases, which Sec. 6
 * names as the extension of the method.  The same accelerated iteration:
 * tau = (C - C0) : e, c^ = -Gamma0 : tau^ with the Green operator of the
 * isotropic reference medium (its Nyquist modes read as for conductivity),
 * e+ = e + 2 (C + C0)^-1 C0 : (c - e), the mean stress <C : e+> as the
 * column of C_hom.  Reference medium: kappa0 = sqrt(min kappa max kappa),
 * mu0 = sqrt(min mu max mu) (the Sec. 5 rule applied to each modulus).
 * The six load cases impose E = B_j, the orthonormal basis of symmetric
 * tensors
 *   B0 = I / sqrt3,  B1 = (e1e1 - e2e2) / sqrt2,
 *   B2 = (e1e1 + e2e2 - 2 e3e3) / sqrt6,  B3 = (e2e3 + e3e2) / sqrt2,
 *   B4 = (e1e3 + e3e1) / sqrt2,  B5 = (e1e2 + e2e1) / sqrt2,
 * in which an isotropic stiffness is diag(3 kappa, 2 mu, 2 mu, 2 mu, 2 mu,
 * 2 mu); the residual of load case j is sqrt<|e - c|^2> (|B_j| = 1). */
typedef struct {
    double C[36];              /* C_hom, Voigt, row-major: sigma_I = sum_J C[6 I + J] eps_J,
                                  I, J over 11, 22, 33, 23, 13, 12 with engineering shear
                                  strains (C[6 I + J] = C_ijkl) */
    double C_basis[36];        /* C_basis[6 k + l] = B_k : C_hom : B_l (column l: load case B_l) */
    int iters[6];              /* per load case B_j */
    int status[6];
    double final_residual[6];
    double solve_ms;           /* device time of the iteration phase */
} rve_elastic_result;

/* moduli: host, (kappa, mu) of matrix, inclusion, coating (bulk and shear
 * moduli, > 0, finite); tol as in homogenize.  opts may be NULL; honoured:
 * precision, max_iter, stall_window, stream, init_field and out_field (host,
 * 36 N^3 doubles, [load case j][component k][z][y][x] in the basis above).
 * equilibrium_check, scheme != 0, a workspace or a partial lc_mask give
 * RVE_ERR_ARG, as does a grid size not in rve_supported_n_elastic.
 * residual_history: host [6][hist_cap] or NULL.  Returns the worst
 * per-load-case status, as homogenize. */
rve_status homogenize_elastic(rve_t rve, const double moduli[6], double tol, const rve_opts *opts,
                              rve_elastic_result *out, double *residual_history, int hist_cap);

/* Grid sizes N the elastic case supports for a precision: 8, 12, 16, 24,
 * 32, 48, 64, 96, 128, 256 and 512 in both (FP64 from 256^3 on, and FP32
 * 512^3, in the five-pass form). */
rve_status rve_supported_n_elastic(int precision, int *out, int cap, int *count);

/* Serving: a request loop that keeps fields resident on the device,
 * admits requests by device-memory footprint and free slots, and advances
 * all admitted requests together (continuous batching: chunks of iterations
 * of every resident request are enqueued round-robin on per-slot streams,
 * and a request is admitted as soon as a slot and memory free up).
 * precision as in rve_opts; FP32 requests get the FP64 continuation of
 * rve_opts.fp32_refine.
 * rve_server_create reserves hbm_budget_bytes of device memory (one
 * allocation, freed by rve_server_destroy) and, per slot, a stream, events
 * and a pinned staging buffer for the largest phase image that fits the
 * budget.  A request occupies one block of that reservation, of
 * phase image + workspace (+ for FP32 the FP64 workspace of its
 * continuation) bytes, from admission to completion; nothing is allocated
 * or freed per request.  Requests are admitted in submission order while a
 * slot is free and their block fits.  RVE_ERR_ARG for max_slots outside
 * 1..256 or a budget below the smallest grid's footprint; RVE_ERR_OOM if
 * the reservation fails. */
typedef struct rve_server_s *rve_server_t;
rve_status rve_server_create(size_t hbm_budget_bytes, int max_slots, int precision,
                             rve_server_t *out);
typedef struct {
    size_t arena_bytes;       /* device memory reserved at creation */
    size_t peak_bytes;        /* largest sum of the blocks of resident requests */
    int resident_peak;        /* most requests resident at once */
    uint64_t admitted;        /* requests brought onto the device */
    uint64_t completed;       /* requests finished (including setup failures) */
    uint64_t refined;         /* requests that ran the FP64 continuation */
    uint64_t graph_hits;      /* solves that reused an instantiated iteration graph */
    uint64_t graph_misses;    /* graphs captured and instantiated */
} rve_server_stats;
/* Counters of a server since its creation. */
rve_status rve_server_get_stats(rve_server_t s, rve_server_stats *out);
/* Queue one solve; the geometry is generated on a host worker.  ticket out. */
rve_status rve_server_submit(rve_server_t s, const rve_geom *g, const double k_phases[3],
                             double tol, uint64_t *ticket);
/* RVE_PENDING until done; then the result and latency (seconds from submit
 * to completion).  A ticket can be collected once. */
rve_status rve_server_poll(rve_server_t s, uint64_t ticket, rve_result *out, double *latency_s);
/* Block until every submitted request has finished. */
rve_status rve_server_drain(rve_server_t s);
void rve_server_destroy(rve_server_t s);

void rve_destroy(rve_t rve);

/* Message of the last failed call on this thread ("" if none); valid until
 * the next call on this thread. */
const char *rve_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RVEHOM_H */
