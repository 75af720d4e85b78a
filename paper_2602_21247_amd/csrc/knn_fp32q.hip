// Leaf kernel instantiations for the float32 operand in the four-lane
// layout (knn_quad.hpp); the two-lane ones are in knn.hip.
#include "knn_quad.hpp"

namespace pipnn {

hipError_t launch_knn_fp32_quad(const KnnArgs &a, int ksel, int n_items, int n_cu,
                                hipStream_t s) {
  constexpr int P = PIPNN_PREC_FP32;
  switch (a.ldo) {
    case 32: return launch_knn_quad_k<P, 32>(a, ksel, n_items, n_cu, s);
    case 64: return launch_knn_quad_k<P, 64>(a, ksel, n_items, n_cu, s);
    case 96: return launch_knn_quad_k<P, 96>(a, ksel, n_items, n_cu, s);
    case 128: return launch_knn_quad_k<P, 128>(a, ksel, n_items, n_cu, s);
    case 192: return launch_knn_quad_k<P, 192>(a, ksel, n_items, n_cu, s);
    case 256: return launch_knn_quad_k<P, 256>(a, ksel, n_items, n_cu, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pipnn
