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
    double relax;   // multiple of k0 g added to tau: 1 augmented Lagrangian, alpha polarization
    // elastic case: the channels of the hydrostatic basis tensor use k, dk,
    // w, k0 above (3 kappa, 3 (kappa - kappa0), 2 kappa0 / (kappa + kappa0),
    // 3 kappa0); the five deviatoric ones use these (2 mu, ...)
    double k_dev[3];
    double dk_dev[3];
    double w_dev[3];
    double k0_dev;
    double el_inv_mu0M;  // 1 / (mu0 M): Green operator scale, 1/M of the inverse folded in
    double el_betaM;     // (lambda0 + mu0) / (mu0 (lambda0 + 2 mu0)) / M
    int max_iter;
    int stall_window;  // 0 = off
    int hist_cap;
    int eq_check;
    int lc_mask;  // bit lc set = solve that load case
    int scheme;   // 0 accelerated, 1 basic, 2 augmented Lagrangian
    int nc;       // components per load case = load cases: 3 (conductivity) or 6 (elasticity)
    int pad_;
};

// Solver state, in device memory; written only by k_reduce / k_init.
// Arrays hold up to six load cases of six components (elasticity); the
// conductivity problem uses the first three and nine.
struct DevState {
    int iter;
    int all_done;
    int done[6];
    int status[6];
    int iters[6];
    int best_it[6];
    int eq_pending[6];
    double K[36];  // K[nc * comp + lc]
    double res[6];
    double best[6];
    double eps_eq[6];
    // per channel mean of tau = (k - k0) e for the next forward pass; it is
    // subtracted there (the mean mode of tau is replaced by E anyway), which
    // keeps the FFT's rounding error relative to the fluctuation only
    double tau_mean[36];
};

enum : int { ST_OK = 0, ST_NOT_CONVERGED = 1, ST_STALLED = 2, ST_NONFINITE = -5 };

}  // namespace rvehom
