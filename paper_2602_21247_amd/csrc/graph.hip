// Final RobustPrune (Alg. 2, Sec. 4.3) and BeamSearch (Alg. 1) on gfx950.
#include "common.hpp"
#include "internal.hpp"

namespace pipnn {

constexpr uint64_t kNoKey = ~0ull;

__device__ __forceinline__ float rank_to_f32(uint32_t r) {
  const uint32_t u = (r & 0x80000000u) ? (r & 0x7FFFFFFFu) : ~r;
  return __uint_as_float(u);
}

// Distance of a wave-uniform row y to this lane's row z, by direct
// difference with the dimension index ascending.
__device__ __forceinline__ float row_dist(const float *__restrict__ X, int d, bool l2, uint32_t y,
                                          uint32_t z) {
  const float *ry = X + (int64_t)y * d;
  const float *rz = X + (int64_t)z * d;
  float s = 0.f;
  if ((d & 3) == 0) {
    for (int i = 0; i < d; i += 4) {
      const float4 a = *reinterpret_cast<const float4 *>(ry + i);
      const float4 b = *reinterpret_cast<const float4 *>(rz + i);
      if (l2) {
        float t = a.x - b.x; s = fmaf(t, t, s);
        t = a.y - b.y; s = fmaf(t, t, s);
        t = a.z - b.z; s = fmaf(t, t, s);
        t = a.w - b.w; s = fmaf(t, t, s);
      } else {
        s = fmaf(a.x, b.x, s); s = fmaf(a.y, b.y, s);
        s = fmaf(a.z, b.z, s); s = fmaf(a.w, b.w, s);
      }
    }
  } else {
    for (int i = 0; i < d; ++i) {
      if (l2) {
        const float t = ry[i] - rz[i];
        s = fmaf(t, t, s);
      } else {
        s = fmaf(ry[i], rz[i], s);
      }
    }
  }
  return l2 ? s : -s;
}

__device__ void wave_sort_u64(uint64_t *A, int P) {
  const int lane = lane_id();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = lane; t < P / 2; t += 64) {
        const int i = (t / j) * 2 * j + (t % j);
        const int l = i + j;
        const bool asc = (i & k) == 0;
        const uint64_t x = A[i], y = A[l];
        if ((x > y) == asc) {
          A[i] = y;
          A[l] = x;
        }
      }
      wave_sync();
    }
  }
}

// ---------------------------------------------------------------------
// RobustPrune. One wave per point x. Candidates are the reservoir ids; they
// are sorted by (d(x,c), id) and walked in that order: the first live
// candidate is admitted, then every live candidate z with
// alpha * d(y,z) < d(x,z) is removed (tested as the sign of one fused
// multiply-add, so the comparison is exact for the float32 inputs). This
// is the loop of Alg. 2; it admits exactly the candidates the lazy form
// admits. Lane j owns sorted positions j, j+64, j+128, j+192.
constexpr int kRpWaves = 4;

__global__ void __launch_bounds__(64 * kRpWaves) robustprune_kernel(
    const float *__restrict__ X, int64_t n, int d, int metric, const uint64_t *__restrict__ res,
    int l_max, float alpha, int R, uint32_t *__restrict__ graph, uint32_t *__restrict__ degree) {
  __shared__ uint64_t sK[kRpWaves][256];
  __shared__ uint32_t sE[kRpWaves][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t x = (int64_t)blockIdx.x * kRpWaves + wave;
  if (x >= n) return;
  const bool l2 = metric == PIPNN_METRIC_L2;
  uint64_t *K = sK[wave];
  uint32_t *E = sE[wave];
  int P = 2;
  while (P < l_max) P <<= 1;
  const uint32_t xu = (uint32_t)x;
  for (int i = lane; i < P; i += 64) {
    uint64_t key = kNoKey;
    if (i < l_max) {
      const uint32_t c = slot_id(res[x * l_max + i]);
      if (c != kEmptyId && c != xu && c < n) {
        const float dxc = row_dist(X, d, l2, xu, c);
        key = ((uint64_t)f32_rank(dxc) << 32) | c;
      }
    }
    K[i] = key;
  }
  wave_sync();
  wave_sort_u64(K, P);

  // per-lane live flags and distances of owned positions
  bool live[4];
  float dx[4];
  uint32_t cid[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = lane + 64 * q;
    const uint64_t key = (i < P) ? K[i] : kNoKey;
    live[q] = key != kNoKey;
    cid[q] = (uint32_t)key;
    dx[q] = live[q] ? rank_to_f32((uint32_t)(key >> 32)) : 0.f;
  }
  int ne = 0;
  while (ne < R) {
    int first = -1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint64_t m = __ballot(live[q]);
      if (first < 0 && m) first = 64 * q + __ffsll((long long)m) - 1;
    }
    if (first < 0) break;
    const uint32_t y = __builtin_amdgcn_readfirstlane((uint32_t)K[first]);
    if (lane == 0) E[ne] = y;
    ++ne;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (lane + 64 * q == first) live[q] = false;
      if (live[q]) {
        const float dyz = row_dist(X, d, l2, y, cid[q]);
        if (fmaf(alpha, dyz, -dx[q]) < 0.f) live[q] = false;
      }
    }
  }
  wave_sync();
  for (int i = lane; i < R; i += 64) graph[x * R + i] = i < ne ? E[i] : kEmptyId;
  if (lane == 0) degree[x] = (uint32_t)ne;
}

hipError_t launch_robustprune(const Index &I, const uint64_t *res, uint32_t *graph, uint32_t *degree,
                              hipStream_t s) {
  if (I.p.l_max > 256 || I.p.R > 256) return hipErrorInvalidValue;
  const int64_t blocks = (I.n + kRpWaves - 1) / kRpWaves;
  hipLaunchKernelGGL(robustprune_kernel, dim3((unsigned)blocks), dim3(64 * kRpWaves), 0, s, I.xf(),
                     I.n, I.d, I.p.metric, res, I.p.l_max, I.p.alpha, I.p.R, graph, degree);
  return hipGetLastError();
}

// ---------------------------------------------------------------------
// BeamSearch. One wave per query. The beam is a sorted array of keys
// (rank(distance), id) in LDS with a visited flag per entry; `seen` is a
// per-query bitmap over the n points in global memory (cleared by the
// caller). Each step visits the first unvisited entry, evaluates its
// neighbours that were never seen, sorts them, and merges them into the
// beam, which keeps its first L entries (Alg. 1).
constexpr int kMaxL = 1024;
constexpr int kMaxR = 256;
constexpr int kMaxQD = 1024;

__global__ void __launch_bounds__(64) search_kernel(const float *__restrict__ X, int64_t n, int d,
                                                    int metric, const uint32_t *__restrict__ graph,
                                                    int R, const float *__restrict__ Q, int k,
                                                    int L, uint32_t start,
                                                    uint32_t *__restrict__ out_ids,
                                                    float *__restrict__ out_dist,
                                                    uint32_t *__restrict__ out_cmps,
                                                    uint32_t *__restrict__ seen_bits,
                                                    int64_t words_per_query) {
  __shared__ uint64_t beam[kMaxL];
  __shared__ uint64_t tmp[kMaxL];
  __shared__ uint8_t vis[kMaxL];
  __shared__ uint8_t tvis[kMaxL];
  __shared__ uint64_t nw[kMaxR];
  __shared__ float qv[kMaxQD];
  const int lane = threadIdx.x;
  const int64_t qi = blockIdx.x;
  const bool l2 = metric == PIPNN_METRIC_L2;
  const float *q = Q + qi * d;
  for (int i = lane; i < d; i += 64) qv[i] = q[i];
  uint32_t *seen = seen_bits + qi * words_per_query;
  wave_sync();
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

  auto qdist = [&](uint32_t u) {
    const float *xu = X + (int64_t)u * d;
    float s = 0.f;
    for (int i = 0; i < d; ++i) {
      if (l2) {
        const float t = qv[i] - xu[i];
        s = fmaf(t, t, s);
      } else {
        s = fmaf(qv[i], xu[i], s);
      }
    }
    return l2 ? s : -s;
  };

  int nb = 1;
  uint32_t cmps = 1;
  if (lane == 0) {
    beam[0] = ((uint64_t)f32_rank(qdist(start)) << 32) | start;
    vis[0] = 0;
    atomicOr(&seen[start >> 5], 1u << (start & 31));
  }
  wave_sync();
  for (;;) {
    int cur = -1;
    for (int base = 0; base < nb; base += 64) {
      const int i = base + lane;
      const uint64_t m = __ballot(i < nb && vis[i] == 0);
      if (m) {
        cur = base + __ffsll((long long)m) - 1;
        break;
      }
    }
    if (cur < 0) break;
    const uint32_t p = __builtin_amdgcn_readfirstlane((uint32_t)beam[cur]);
    wave_sync();
    if (lane == 0) vis[cur] = 1;
    // unseen neighbours
    int nn = 0;
    for (int base = 0; base < R; base += 64) {
      const int e = base + lane;
      uint64_t key = kNoKey;
      bool fresh = false;
      if (e < R) {
        const uint32_t u = graph[(int64_t)p * R + e];
        if (u != kEmptyId && u < n) {
          const uint32_t bit = 1u << (u & 31);
          const uint32_t old = atomicOr(&seen[u >> 5], bit);
          if (!(old & bit)) {
            fresh = true;
            key = ((uint64_t)f32_rank(qdist(u)) << 32) | u;
          }
        }
      }
      const uint64_t m = __ballot(fresh);
      if (fresh) nw[nn + __popcll(m & below)] = key;
      nn += __popcll(m);
    }
    cmps += nn;
    if (nn == 0) {
      wave_sync();
      continue;
    }
    int P = 2;
    while (P < nn) P <<= 1;
    for (int i = nn + lane; i < P; i += 64) nw[i] = kNoKey;
    wave_sync();
    wave_sort_u64(nw, P);
    // merge: every key is unique, so ranks give final positions
    const int total = nb + nn < L ? nb + nn : L;
    for (int i = lane; i < nb; i += 64) {
      const uint64_t key = beam[i];
      int lo = 0, hi = nn;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (nw[mid] < key) lo = mid + 1; else hi = mid;
      }
      const int pos = i + lo;
      if (pos < total) {
        tmp[pos] = key;
        tvis[pos] = vis[i];
      }
    }
    for (int j = lane; j < nn; j += 64) {
      const uint64_t key = nw[j];
      int lo = 0, hi = nb;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (beam[mid] < key) lo = mid + 1; else hi = mid;
      }
      const int pos = j + lo;
      if (pos < total) {
        tmp[pos] = key;
        tvis[pos] = 0;
      }
    }
    wave_sync();
    for (int i = lane; i < total; i += 64) {
      beam[i] = tmp[i];
      vis[i] = tvis[i];
    }
    nb = total;
    wave_sync();
  }
  for (int i = lane; i < k; i += 64) {
    const bool ok = i < nb;
    out_ids[qi * k + i] = ok ? (uint32_t)beam[i] : kEmptyId;
    if (out_dist) out_dist[qi * k + i] = ok ? rank_to_f32((uint32_t)(beam[i] >> 32)) : INFINITY;
  }
  if (out_cmps && lane == 0) out_cmps[qi] = cmps;
}

hipError_t launch_search(const Index &I, const uint32_t *graph, const float *Q, int64_t nq,
                         int32_t k, int32_t L, uint32_t start, uint32_t *out_ids, float *out_dist,
                         uint32_t *out_cmps, uint32_t *visited_bits, int64_t words_per_query,
                         hipStream_t s) {
  if (nq == 0) return hipSuccess;
  if (L > kMaxL || I.p.R > kMaxR || I.d > kMaxQD) return hipErrorInvalidValue;
  hipLaunchKernelGGL(search_kernel, dim3((unsigned)nq), dim3(64), 0, s, I.xf(), I.n, I.d,
                     I.p.metric, graph, I.p.R, Q, k, L, start, out_ids, out_dist, out_cmps,
                     visited_bits, words_per_query);
  return hipGetLastError();
}

}  // namespace pipnn
