// Fused leaf distance GEMM + per-row k-nearest selection: the FP32
// instantiations and the dispatch over operand precisions. The kernel
// itself is in knn_kernel.hpp.
#include "knn_kernel.hpp"

namespace pipnn {

template <int DP>
static hipError_t launch_dp(const KnnArgs &args, int ksel, int n_items, int nw, int n_cu,
                           hipStream_t s) {
  if (ksel <= 4) return launch_knn_shape<PIPNN_PREC_FP32, DP, 4>(args, n_items, nw, n_cu, s);
  if (ksel <= 16) return launch_knn_shape<PIPNN_PREC_FP32, DP, 16>(args, n_items, nw, n_cu, s);
  return launch_knn_shape<PIPNN_PREC_FP32, DP, 32>(args, n_items, nw, n_cu, s);
}

int knn_operand_dim(int d, int prec) {
  if (prec != PIPNN_PREC_FP32) return lowp_padded_dim(d);
  return d <= 32 ? 32 : d <= 64 ? 64 : d <= 96 ? 96 : d <= 128 ? 128 : d <= 192 ? 192
       : d <= 256 ? 256 : 0;
}

bool knn_nw_available(int d, int prec, int nw) {
  const int dp = knn_operand_dim(d, prec);
  return dp != 0 && (nw == 4 || (nw == 2 && dp <= 256 && knn_has_nw2(dp)));
}

bool knn_quad_available(int d, int prec) {
  const int dp = knn_operand_dim(d, prec);
  const int eb = prec == PIPNN_PREC_FP32 ? 4 : prec == PIPNN_PREC_FP8 ? 1 : 2;
  return dp != 0 && (dp * eb) % 64 == 0;
}

bool knn_pair_available(int d, int prec) {
  const int dp = knn_operand_dim(d, prec);
  return dp != 0 && dp <= 256;
}

hipError_t launch_knn(const KnnLaunch &L, hipStream_t s) {
  const Index &I = *L.idx;
  if (L.n_items == 0) return hipSuccess;
  const bool lowp = L.prec != PIPNN_PREC_FP32;
  KnnArgs a;
  a.X = I.xf();
  a.Xop = lowp ? I.xlow.p : reinterpret_cast<const void *>(I.xop32());
  a.norms = lowp ? I.lnorms.as<float>() : I.norms.as<float>();
  a.scale = L.prec == PIPNN_PREC_FP8 ? I.xscale.as<float>() : nullptr;
  a.row_base = L.row_base;
  a.col_base = L.col_base;
  a.jobs = L.jobs;
  a.items = L.items;
  a.out_col = L.out_col;
  a.out_dist = L.out_dist;
  a.out_matrix = L.out_matrix;
  a.matrix_ld = L.matrix_ld;
  a.n_items = L.n_items;
  a.d = I.d;
  a.ldo = lowp ? I.ldo : I.ldf;
  a.metric = I.p.metric;
  a.k_out = L.k_out;
  a.out_ids = L.out_ids;
  a.recompute = L.recompute;
  a.rescore_k = L.rescore_k;
  a.work_counter = nullptr;
  a.items_per_xcd = 0;
  if (!knn_nw_available(I.d, L.prec, L.nw) || L.n_items % kNumXcd != 0) return hipErrorInvalidValue;
  // operands wider than 256 dimensions exist in the four-lane layout only
  const bool quad = L.quad || !knn_pair_available(I.d, L.prec);
  if (quad && (L.nw != 4 || !knn_quad_available(I.d, L.prec))) return hipErrorInvalidValue;
  if (L.persistent) {
    a.work_counter = I.s_counter.as<int32_t>();
    if (!a.work_counter) return hipErrorInvalidValue;
    hipError_t e = launch_fill_u32(I.s_counter.as<uint32_t>(), 0u, kNumXcd, s);
    if (e != hipSuccess) return e;
  }
  const int nw = L.nw, n_cu = I.n_cu;
  if (lowp) {
    if (!a.Xop || a.ldo != lowp_padded_dim(I.d) || L.prec != I.copy_prec)
      return hipErrorInvalidValue;
    if (L.prec == PIPNN_PREC_BF16) return launch_knn_bf16(a, L.ksel, L.n_items, nw, quad, n_cu, s);
    if (L.prec == PIPNN_PREC_FP16) return launch_knn_fp16(a, L.ksel, L.n_items, nw, quad, n_cu, s);
    if (L.prec == PIPNN_PREC_FP8) return launch_knn_fp8(a, L.ksel, L.n_items, nw, quad, n_cu, s);
    return hipErrorInvalidValue;
  }
  if (I.ldf != knn_operand_dim(I.d, PIPNN_PREC_FP32)) return hipErrorInvalidValue;
  if (quad) return launch_knn_fp32_quad(a, L.ksel, L.n_items, n_cu, s);
  switch (I.ldf) {
    case 32: return launch_dp<32>(a, L.ksel, L.n_items, nw, n_cu, s);
    case 64: return launch_dp<64>(a, L.ksel, L.n_items, nw, n_cu, s);
    case 96: return launch_dp<96>(a, L.ksel, L.n_items, nw, n_cu, s);
    case 128: return launch_dp<128>(a, L.ksel, L.n_items, nw, n_cu, s);
    case 192: return launch_dp<192>(a, L.ksel, L.n_items, nw, n_cu, s);
    case 256: return launch_dp<256>(a, L.ksel, L.n_items, nw, n_cu, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pipnn
