// solver_state.hpp -- parameter and state blocks shared by the kernels and
// the host side of the C ABI (device memory, plain structs).
#pragma once

namespace rvehom {

// Per-call parameters, in device memory (read by every kernel).
struct DevParams {
    double k[3];   // phase conductivities
    double dk[3];  // k - k0           (step 2)
    double w[3];   // 2 k0 / (k + k0)  (step 7)
    double k0;
    double inv_k0M;  // 1 / (k0 M): Green scale with the 1/M of the inverse folded in
    double tol;
    double invM;
    double prog10;  // 1 - rho^10: least progress of 10 iterations the scheme's contraction bound allows
    double gam[3];  // 1 / (k + k0) (augmented-Lagrangian local step)
    int max_iter;
    int stall_window;  // 0 = off
    int hist_cap;
    int eq_check;
    int lc_mask;  // bit lc set = solve that load case
    int scheme;   // 0 accelerated, 1 basic, 2 augmented Lagrangian
    int pad_[2];
};

// Solver state, in device memory; written only by k_reduce / k_init.
struct DevState {
    int iter;
    int all_done;
    int done[3];
    int status[3];
    int iters[3];
    int best_it[3];
    int eq_pending[3];
    int pad_;
    double K[9];
    double res[3];
    double best[3];
    double eps_eq[3];
    // per channel mean of tau = (k - k0) e for the next forward pass; it is
    // subtracted there (the mean mode of tau is replaced by E anyway), which
    // keeps the FFT's rounding error relative to the fluctuation only
    double tau_mean[9];
};

enum : int { ST_OK = 0, ST_NOT_CONVERGED = 1, ST_STALLED = 2, ST_NONFINITE = -5 };

}  // namespace rvehom
