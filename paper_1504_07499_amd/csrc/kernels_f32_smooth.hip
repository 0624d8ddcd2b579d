// FP32 instances of the solver kernels for the {2,3}-smooth grid sizes
// 36, 72, 144, 192, 288 and 384 (the radix-3 stages of the transforms).
#include "kernel_instances.hpp"

namespace rvehom {

const SolverOps *ops_f32_smooth(int n) {
    switch (n) {
    case 36: return Instance<float, 36>::ops(0);
    case 72: return Instance<float, 72>::ops(0);
    case 144: return Instance<float, 144>::ops(0);
    case 192: return Instance<float, 192>::ops(0);
    case 288: return Instance<float, 288>::ops(0);
    case 384: return Instance<float, 384>::ops(0);
    default: return nullptr;
    }
}

}  // namespace rvehom
