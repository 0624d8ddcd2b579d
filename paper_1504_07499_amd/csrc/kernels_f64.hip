// FP64 instances of the solver kernels (the reference GPU path).
#include "kernel_instances.hpp"

namespace rvehom {

const SolverOps *ops_f64(int n) {
    switch (n) {
    case 8: return Instance<double, 8>::ops(1);
    case 12: return Instance<double, 12>::ops(1);
    case 16: return Instance<double, 16>::ops(1);
    case 24: return Instance<double, 24>::ops(1);
    case 32: return Instance<double, 32>::ops(1);
    case 48: return Instance<double, 48>::ops(1);
    case 64: return Instance<double, 64>::ops(1);
    case 96: return Instance<double, 96>::ops(1);
    case 128: return Instance<double, 128>::ops(1);
    case 256: return Instance<double, 256>::ops(1);
    case 512: return Instance<double, 512>::ops(1);
    default: return ops_f64_smooth(n);
    }
}

}  // namespace rvehom
