// FP64 instances of the elastic-case kernels.
#include "elastic_kernels.hpp"

namespace rvehom {

const SolverOps *ops_el_f64(int n) {
    switch (n) {
    case 8: return ElasticInstance<double, 8>::ops(1);
    case 12: return ElasticInstance<double, 12>::ops(1);
    case 16: return ElasticInstance<double, 16>::ops(1);
    case 24: return ElasticInstance<double, 24>::ops(1);
    case 32: return ElasticInstance<double, 32>::ops(1);
    case 48: return ElasticInstance<double, 48>::ops(1);
    case 64: return ElasticInstance<double, 64>::ops(1);
    case 96: return ElasticInstance<double, 96>::ops(1);
    case 128: return ElasticInstance<double, 128>::ops(1);
    case 256: return ElasticInstance<double, 256>::ops(1);
    case 512: return ElasticInstance<double, 512>::ops(1);
    default: return nullptr;
    }
}

}  // namespace rvehom
