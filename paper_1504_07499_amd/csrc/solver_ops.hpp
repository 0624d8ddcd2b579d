// solver_ops.hpp -- host-side table of launchers for one (precision, N).
// The kernel translation units (kernels_f32.hip, kernels_f64.hip) fill it;
// the C ABI (rvehom_api.hip) only sees these function pointers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace rvehom {

struct DevParams;
struct DevState;

struct LaunchArgs {
    void *e;
    const uint8_t *ph;
    void *spec;
    void *nyq;
    const void *tw;
    const DevParams *prm;
    DevState *st;
    double *part;
    double *hist;
    double *peq;  // equilibrium-error partials [3][eq_tiles][2]
    void *spec2;  // split planes: the parity-layout forward spectrum (or nullptr)
    void *nyq2;
};

struct SolverOps {
    int n;
    int precision;       // 0 FP32, 1 FP64
    int split;           // S: plane rows split in S parities
    int ztile;           // W: z-pencil tile width
    int nper;            // P3 partials per channel
    size_t real_bytes;   // sizeof(T)
    size_t spec_elems;   // complex elements of spec (9 N N N/2)
    size_t nyq_elems;    // complex elements of nyq (9 N N)
    int grid[3];         // blocks of P1, P2, P3
    int threads[3];      // threads per block of P1, P2, P3
    double bytes[3];     // algorithmic HBM field bytes of one launch of P1, P2, P3 (all load
                         // cases; the phase image is phase_bytes)
    int eq_tiles;        // k_zeq blocks per load case
    double bytes_fused;  // algorithmic bytes of one fused inverse + forward launch
    // fused inverse pass + next forward pass, or nullptr where planes are split
    // lc_sel: -1 = all three load cases, else the one load case to iterate
    void (*inv_fwd)(const LaunchArgs &, hipStream_t, int lc_sel);
    void (*fwd)(const LaunchArgs &, hipStream_t, int lc_sel);
    void (*fwd_phi)(const LaunchArgs &, hipStream_t);
    void (*zeq)(const LaunchArgs &, hipStream_t);
    void (*zgreen)(const LaunchArgs &, hipStream_t, int red_nper, int lc_sel);
    int ztile_alt;  // the other z-tile width the autotuner tries
    void (*zgreen_alt)(const LaunchArgs &, hipStream_t, int red_nper, int lc_sel);  // or nullptr
    void (*inv)(const LaunchArgs &, hipStream_t, int lc_sel);
    void (*init)(const LaunchArgs &, size_t M, hipStream_t);
    void (*from_f64)(void *e, const double *src, size_t count, hipStream_t);
    void (*to_f64)(double *dst, const void *e, size_t count, hipStream_t);
    // the augmented-Lagrangian update: fused pass (nullptr where there is no
    // fused pass), separate inverse pass, and the start field's conversion to
    // tau^0 = (k - k0) e^0
    void (*inv_fwd_al)(const LaunchArgs &, hipStream_t, int lc_sel);
    void (*inv_al)(const LaunchArgs &, hipStream_t, int lc_sel);
    void (*to_tau)(const LaunchArgs &, size_t M, hipStream_t);
    // components per load case = number of load cases: 3 (conductivity) or
    // 6 (elasticity); the fields hold nc * nc channels
    int nc;
    // the reduction of the per-block partials as a launch of its own
    void (*reduce)(const LaunchArgs &, int nper, hipStream_t);
    // the phase image (1 byte per voxel), counted once per launch of the
    // passes that read it (P1, P3, fused) whatever the number of load cases
    double phase_bytes;
    // split planes with the fused pass: the first forward pass and the z
    // pass of the parity layout (the fused pass writes it to spec2 / nyq2,
    // the z pass combines it into spec / nyq); nullptr elsewhere
    void (*fwd_par)(const LaunchArgs &, hipStream_t, int lc_sel);
    void (*zgreen_par)(const LaunchArgs &, hipStream_t, int red_nper, int lc_sel);
    // the dual scheme's update: fused pass (nullptr where there is none) and
    // separate inverse pass
    void (*inv_fwd_dual)(const LaunchArgs &, hipStream_t, int lc_sel);
    void (*inv_dual)(const LaunchArgs &, hipStream_t, int lc_sel);
    // the fused pass at the other thread count per workgroup that the
    // autotuner tries (0 / nullptr where there is none): the accelerated
    // and basic, augmented-Lagrangian and polarization, and dual updates
    int plane_threads_alt;
    void (*inv_fwd_alt[3])(const LaunchArgs &, hipStream_t, int lc_sel);
};

const SolverOps *ops_f32(int n);
const SolverOps *ops_f64(int n);
// the {2,3}-smooth sizes with a factor 3 beyond 96 and its divisors (their
// own translation units, compiled in parallel with the others)
const SolverOps *ops_f32_smooth(int n);
const SolverOps *ops_f64_smooth(int n);
const SolverOps *ops_el_f32(int n);
const SolverOps *ops_el_f64(int n);
void launch_reduce(const LaunchArgs &a, int nper, hipStream_t s);
void launch_eq_reduce(const LaunchArgs &a, int per_lc, int final, hipStream_t s);
void launch_eq_request(const LaunchArgs &a, hipStream_t s);

// Grid sizes compiled into the library (ascending), per precision; the
// elastic case's own list.
int supported_sizes(int precision, const int **list);
int supported_sizes_el(int precision, const int **list);

}  // namespace rvehom
