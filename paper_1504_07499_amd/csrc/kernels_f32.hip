// FP32 instances of the solver kernels (FFT and update in FP32, reductions in FP64).
#include "kernel_instances.hpp"

namespace rvehom {

const SolverOps *ops_f32(int n) {
    switch (n) {
    case 8: return Instance<float, 8>::ops(0);
    case 12: return Instance<float, 12>::ops(0);
    case 16: return Instance<float, 16>::ops(0);
    case 24: return Instance<float, 24>::ops(0);
    case 32: return Instance<float, 32>::ops(0);
    case 48: return Instance<float, 48>::ops(0);
    case 64: return Instance<float, 64>::ops(0);
    case 96: return Instance<float, 96>::ops(0);
    case 128: return Instance<float, 128>::ops(0);
    case 256: return Instance<float, 256>::ops(0);
    case 512: return Instance<float, 512>::ops(0);
    default: return ops_f32_smooth(n);
    }
}

}  // namespace rvehom
