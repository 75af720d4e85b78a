// All-to-All Prune leaf picker (Supplement, "Picking within Leaves",
// All-to-All Prune): for every member x of a leaf, RobustPrune (Alg. 2) in
// its lazy form (Supplement, "Optimizing RobustPrune") with every other
// member of the leaf as a candidate.
//
// The leaf kernel first writes each leaf's GEMM distance matrix (row r of a
// batch at D + r * ld, column = position in the leaf). Then one wave per
// leaf row:
//  1. loads the row's distances to the other members as 64-bit keys
//     (order-preserving rank of the distance, column) -- E per lane, up to
//     2,048 members -- and sorts them (register bitonic sort);
//  2. takes them 64 at a time in (distance, column) order: a candidate c is
//     dropped if an already admitted y has alpha * d(y, c) < d(x, c) (the
//     sign of one fused multiply-add, as in the final prune; d(y, c) read
//     from y's row of the matrix); among the survivors of a chunk the first
//     is admitted (nothing before it can prune it), the rest are tested
//     against it, and so on: the sequential scan's admissions, one round per
//     admission;
//  3. stops at R admissions and writes the admitted ids in admission order
//     with their distances (the FP32 direct difference of the pair where the
//     GEMM form may differ from it).
// Columns are positions in the leaf, whose members are ascending ids, so
// column order is id order: ties go to the smaller id, as in the oracle.
#include "common.hpp"
#include "internal.hpp"
#include "wave_sort.hpp"

namespace pipnn {

namespace {

constexpr int kA2aWaves = 4;
constexpr uint64_t kNoKey = ~0ull;

__device__ __forceinline__ float a2a_rank_to_f32(uint32_t r) {
  return __uint_as_float((r & 0x80000000u) ? (r & 0x7FFFFFFFu) : ~r);
}

struct A2aArgs {
  const float *D;           // batch distance matrices
  int64_t ld;               // row stride of D
  const int64_t *leaf_off;  // absolute CSR offsets of the batch's leaves (n_leaves + 1)
  int64_t n_leaves;
  int64_t off0;             // absolute position of the batch's first row
  int64_t rows;             // rows of the batch
  const uint32_t *members;  // absolute CSR members
  const float *X;           // float32 points (for the direct-difference distances)
  int d, metric, recompute, R;
  float alpha;
  uint32_t *out_id;         // rows x R point ids
  float *out_dist;          // rows x R
};

template <int E>
__device__ void a2a_row(const A2aArgs &a, int64_t r, int64_t start, int s, int i, int lane,
                        uint32_t *sAdm, float *sAdmD) {
  const float *Dr = a.D + r * a.ld;
  uint64_t v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int j = e * 64 + lane;  // the j-th other member: position j, or j + 1 past the row's own
    uint64_t key = kNoKey;
    if (j < s - 1) {
      const int c = j + (j >= i ? 1 : 0);
      key = ((uint64_t)f32_rank(Dr[c]) << 32) | (uint32_t)c;
    }
    v[e] = key;
  }
  if constexpr (E <= 4) reg_bitonic_sort<E>(v, lane);
  else reg_bitonic_sort_loop<E>(v, lane);
  int nadm = 0;
  const float alpha = a.alpha;
  bool done = false;  // R admitted, or no candidate left
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if (!done && (nadm >= a.R || __ballot(v[e] != kNoKey) == 0)) done = true;
    if (done) continue;
    const bool valid = v[e] != kNoKey;
    const uint32_t c = (uint32_t)v[e];
    const float dxc = valid ? a2a_rank_to_f32((uint32_t)(v[e] >> 32)) : 0.f;
    bool alive = valid;
    // the admissions of earlier chunks
    for (int t = 0; t < nadm; ++t) {
      const uint32_t y = sAdm[t];
      if (alive) {
        const float dyc = a.D[(start + y) * a.ld + c];
        if (fmaf(alpha, dyc, -dxc) < 0.f) alive = false;
      }
    }
    // rounds: the first survivor is admitted, the later ones are tested against it
    for (;;) {
      const uint64_t m = __ballot(alive);
      if (m == 0 || nadm >= a.R) break;
      const int f = __ffsll((long long)m) - 1;
      const uint32_t cf = (uint32_t)__builtin_amdgcn_readlane((int)c, f);
      const float df = __uint_as_float(
          (uint32_t)__builtin_amdgcn_readlane((int)__float_as_uint(dxc), f));
      if (lane == 0) {
        sAdm[nadm] = cf;
        sAdmD[nadm] = df;
      }
      wave_sync();
      ++nadm;
      if (lane == f) alive = false;
      if (alive) {
        const float dyc = a.D[(start + cf) * a.ld + c];
        if (fmaf(alpha, dyc, -dxc) < 0.f) alive = false;
      }
    }
  }
  wave_sync();
  // output: ids in admission order, distances
  const int64_t abs_row = a.off0 + r;
  const uint32_t x = a.members[abs_row];
  for (int t = lane; t < a.R; t += 64) {
    uint32_t id = kEmptyId;
    float dist = INFINITY;
    if (t < nadm) {
      const uint32_t cl = sAdm[t];
      id = a.members[a.off0 + start + cl];
      dist = sAdmD[t];
      if (a.recompute) {
        // FP32 direct difference (or the FP32 inner product), index order
        const float *xv = a.X + (int64_t)x * a.d;
        const float *cv = a.X + (int64_t)id * a.d;
        float acc = 0.f;
        if (a.metric == PIPNN_METRIC_L2) {
          for (int q = 0; q < a.d; ++q) {
            const float df = xv[q] - cv[q];
            acc = fmaf(df, df, acc);
          }
        } else {
          for (int q = 0; q < a.d; ++q) acc = fmaf(xv[q], cv[q], acc);
          acc = -acc;
        }
        dist = acc;
      }
    }
    a.out_id[r * a.R + t] = id;
    a.out_dist[r * a.R + t] = dist;
  }
}

// One launch per size class: rows of leaves of 32 E + 1 .. 64 E members
// (1 .. 64 for E = 1); rows of other leaves return at once.
template <int E>
__global__ void __launch_bounds__(64 * kA2aWaves) a2a_prune_kernel(A2aArgs a) {
  __shared__ uint32_t sAdm[kA2aWaves][32];
  __shared__ float sAdmD[kA2aWaves][32];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r = (int64_t)blockIdx.x * kA2aWaves + wave;
  if (r >= a.rows) return;
  // the row's leaf: the last leaf whose first row is at or before it
  const int64_t ar = a.off0 + r;
  int64_t lo = 0, hi = a.n_leaves - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (a.leaf_off[mid] <= ar) lo = mid; else hi = mid - 1;
  }
  const int64_t start = a.leaf_off[lo] - a.off0;
  const int s = (int)(a.leaf_off[lo + 1] - a.leaf_off[lo]);
  if (s > 64 * E || (E > 1 && s <= 32 * E)) return;
  a2a_row<E>(a, r, start, s, (int)(r - start), lane, sAdm[wave], sAdmD[wave]);
}

}  // namespace

hipError_t launch_a2a_prune(const float *D, int64_t ld, const int64_t *leaf_off, int64_t n_leaves,
                            int64_t off0, int64_t rows, const uint32_t *members, const float *X,
                            int32_t d, int32_t metric, int32_t recompute, int32_t R, float alpha,
                            uint32_t *out_id, float *out_dist, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  if (R < 1 || R > 32 || n_leaves < 1) return hipErrorInvalidValue;
  A2aArgs a{D, ld, leaf_off, n_leaves, off0, rows, members, X, d, metric, recompute, R, alpha,
            out_id, out_dist};
  const dim3 g((unsigned)((rows + kA2aWaves - 1) / kA2aWaves)), b(64 * kA2aWaves);
  hipLaunchKernelGGL(a2a_prune_kernel<1>, g, b, 0, s, a);
  hipLaunchKernelGGL(a2a_prune_kernel<2>, g, b, 0, s, a);
  hipLaunchKernelGGL(a2a_prune_kernel<4>, g, b, 0, s, a);
  hipLaunchKernelGGL(a2a_prune_kernel<8>, g, b, 0, s, a);
  hipLaunchKernelGGL(a2a_prune_kernel<16>, g, b, 0, s, a);
  hipLaunchKernelGGL(a2a_prune_kernel<32>, g, b, 0, s, a);
  return hipGetLastError();
}

}  // namespace pipnn
