// FP32 instances of the elastic-case kernels.
#include "elastic_kernels.hpp"

namespace rvehom {

const SolverOps *ops_el_f32(int n) {
    switch (n) {
    case 8: return ElasticInstance<float, 8>::ops(0);
    case 12: return ElasticInstance<float, 12>::ops(0);
    case 16: return ElasticInstance<float, 16>::ops(0);
    case 24: return ElasticInstance<float, 24>::ops(0);
    case 32: return ElasticInstance<float, 32>::ops(0);
    case 48: return ElasticInstance<float, 48>::ops(0);
    case 64: return ElasticInstance<float, 64>::ops(0);
    case 96: return ElasticInstance<float, 96>::ops(0);
    case 128: return ElasticInstance<float, 128>::ops(0);
    case 256: return ElasticInstance<float, 256>::ops(0);
    case 512: return ElasticInstance<float, 512>::ops(0);
    default: return nullptr;
    }
}

}  // namespace rvehom
