// Leaf kernel instantiations for the bf16 GEMM operand (FP32 accumulation).
#include "knn_quad.hpp"

namespace pipnn {

hipError_t launch_knn_bf16(const KnnArgs &a, int ksel, int n_items, int nw, bool quad, int n_cu,
                          hipStream_t s) {
  return launch_knn_lowp<PIPNN_PREC_BF16>(a, ksel, n_items, nw, quad, n_cu, s);
}

}  // namespace pipnn
