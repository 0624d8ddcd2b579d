// FP64 instances of the solver kernels for the {2,3}-smooth grid sizes
// 36, 72, 144, 192, 288 and 384 (the radix-3 stages of the transforms).
#include "kernel_instances.hpp"

namespace rvehom {

const SolverOps *ops_f64_smooth(int n) {
    switch (n) {
    case 36: return Instance<double, 36>::ops(1);
    case 72: return Instance<double, 72>::ops(1);
    case 144: return Instance<double, 144>::ops(1);
    case 192: return Instance<double, 192>::ops(1);
    case 288: return Instance<double, 288>::ops(1);
    case 384: return Instance<double, 384>::ops(1);
    default: return nullptr;
    }
}

}  // namespace rvehom
