// Final RobustPrune (Alg. 2, Sec. 4.3) and BeamSearch (Alg. 1) on gfx950.
#include <cmath>

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

__device__ __forceinline__ void wave_sort_u64(uint64_t *A, int P) {
  const int lane = lane_id();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = lane; t < P / 2; t += 64) {
        const int i = 2 * t - (t & (j - 1));  // t = q*j + r -> q*2j + r (j is a power of two)
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
    int l_max, float alpha, int R, const uint32_t *__restrict__ order, int64_t n_items,
    uint32_t *__restrict__ graph, uint32_t *__restrict__ degree) {
  __shared__ uint64_t sK[kRpWaves][256];
  __shared__ uint32_t sE[kRpWaves][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t it = (int64_t)blockIdx.x * kRpWaves + wave;
  if (it >= n_items) return;
  const int64_t x = order ? (int64_t)order[it] : it;
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

typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ int acc_row32(int v, int h) { return (v & 3) + 8 * (v >> 2) + 4 * h; }

// RobustPrune with the candidate Gram on MFMA (up to 64 candidates,
// d <= DP <= 128). One wave per point x:
//  1. the valid reservoir candidates, compacted in slot order;
//  2. their rows loaded into MFMA operand fragments (lane l: candidate l%32
//     of a 32-block, the dims of its half); d(x,c) by direct difference
//     from those registers (each half summed in index order, the lower
//     half's sum plus the upper half's); the 64 x 64 Gram G = C C^T as four
//     32 x 32 blocks on MFMA;
//  3. d(y,z) = |y|^2 + |z|^2 - 2 G[y][z] (or -G for inner product), and y
//     prunes z when alpha*d(y,z) < d(x,z): the sign of one fused
//     multiply-add. A lane holds one column z of a block; the signs of its
//     16 rows are shifted into a word (v_alignbit), so z's set of pruners is
//     built with one instruction per pair, and the two halves of a column
//     meet in one cross-half lane swap;
//  4. for each candidate, the set of candidates ranked before it by
//     (d(x,c), id), by comparison with every key; then the lazy scan in
//     that order -- z is admitted iff no admitted candidate ranked before it
//     prunes it, the first R admitted kept -- run as rounds over the whole
//     wave on the pruner sets restricted to earlier candidates. This admits
//     exactly the candidates of Alg. 2.

// Column z of Gram block g (rows row0 + acc_row32(v, h), v = 0..15): bit
// 8*(v>>2) + (v&3) is set when row y prunes z. The lanes of the upper half
// hold rows 4 further on, so their word is the same pattern shifted by 4.
// ndx is 0 - d(x,z), never -0, so the fused multiply-add is never -0 and
// its sign bit is exactly (alpha*d(y,z) - d(x,z) < 0) for non-NaN inputs.
template <bool L2>
__device__ __forceinline__ uint32_t rp_sign_bits(const f32x16 &g, const float *sNw, int row0,
                                                 float nz, float ndx, float alpha) {
  const int h = (threadIdx.x >> 5) & 1;
  uint32_t b = 0u;
#pragma unroll
  for (int grp = 3; grp >= 0; --grp) {
    float ny[4] = {0.f, 0.f, 0.f, 0.f};
    if constexpr (L2) {
      const float4 q = *reinterpret_cast<const float4 *>(sNw + row0 + 8 * grp + 4 * h);
      ny[0] = q.x; ny[1] = q.y; ny[2] = q.z; ny[3] = q.w;
    }
#pragma unroll
    for (int j = 3; j >= 0; --j) {
      const float gv = g[4 * grp + j];
      const float dyz = L2 ? ny[j] + fmaf(-2.f, gv, nz) : -gv;
      b = __builtin_amdgcn_alignbit(b, __float_as_uint(fmaf(alpha, dyz, ndx)), 31);
    }
    if (grp) b <<= 4;
  }
  return b;
}

// Joins the half-column words of two blocks that share their rows: lane j
// (< 32) gets column j of block A whole, lane 32 + j column j of block B.
__device__ __forceinline__ uint32_t rp_join(uint32_t a, uint32_t b) {
  const auto s = __builtin_amdgcn_permlane32_swap(a, b, false, false);
  return s[0] | (s[1] << 4);
}

// Step 4: from the pruner sets by slot (lane j holds slot j's: bit y of
// mlo / mhi for slot y / 32 + y) and the ranking keys in LDS, the admitted
// neighbours of x in rank order.
__device__ __forceinline__ void rp_select(uint32_t mlo, uint32_t mhi, int nv, int R, uint32_t x,
                                          const uint64_t *sKw, const uint32_t *sIw,
                                          uint32_t *__restrict__ graph,
                                          uint32_t *__restrict__ degree) {
  const int lane = threadIdx.x & 63;
  const uint64_t valid = nv >= 64 ? ~0ull : ((1ull << nv) - 1ull);
  // slots ranked before this lane's: keys are distinct (distinct ids), so
  // this is a strict order; keys past nv are stale and masked off
  uint64_t before = 0ull;
  {
    const uint64_t kt = sKw[lane];
    // four keys per step, the highest slot first: slot u lands on bit u
    auto bits = [&](int u0) -> uint32_t {
      uint32_t b = 0u;
#pragma unroll 2
      for (int u = u0 + 28; u >= u0; u -= 4) {
        const ulonglong2 p = *reinterpret_cast<const ulonglong2 *>(sKw + u);
        const ulonglong2 q = *reinterpret_cast<const ulonglong2 *>(sKw + u + 2);
        b = b + b + (q.y < kt ? 1u : 0u);
        b = b + b + (q.x < kt ? 1u : 0u);
        b = b + b + (p.y < kt ? 1u : 0u);
        b = b + b + (p.x < kt ? 1u : 0u);
      }
      return b;
    };
    const uint32_t hi = nv > 32 ? bits(32) : 0u;
    const uint32_t lo = bits(0);
    if (lane < nv) before = ((((uint64_t)hi) << 32) | lo) & valid;
  }
  // the lazy scan of Alg. 2 in rounds: a candidate is admitted once none of
  // its earlier pruners is admitted or undecided, rejected once one of them
  // is admitted; each round decides at least the earliest undecided one, and
  // the outcome is the sequential scan's
  const uint64_t pr = ((((uint64_t)mhi) << 32) | mlo) & before;
  uint64_t adm = 0ull, und = valid;
  while (und != 0ull) {
    const bool u = (und >> lane) & 1ull;
    const bool rej = u && (pr & adm) != 0ull;
    const bool ok = u && !rej && (pr & und) == 0ull;
    const uint64_t ma = __ballot(ok), mr = __ballot(rej);
    adm |= ma;
    und &= ~(ma | mr);
  }
  // the first R admitted in rank order
  const int na = __popcll(adm);
  const int ne = na < R ? na : R;
  uint32_t *grow = graph + (int64_t)x * R;
  if (lane < nv && ((adm >> lane) & 1ull)) {
    const int pos = __popcll(adm & before);
    if (pos < R) grow[pos] = sIw[lane];
  }
  for (int i = ne + lane; i < R; i += 64) grow[i] = kEmptyId;
  if (lane == 0) degree[x] = (uint32_t)ne;
}

// Step 1, shared by the MFMA forms: the valid candidates (rv: this lane's
// reservoir word) compacted into sIw in slot order; returns their count.
__device__ __forceinline__ int rp_compact(uint64_t rv, int l_max, uint32_t x, int64_t n,
                                          uint32_t *sIw) {
  const int lane = threadIdx.x & 63;
  const uint32_t c = slot_id(rv);
  const bool ok = lane < l_max && c != kEmptyId && c != x && c < n;
  const uint64_t m = __ballot(ok);
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  if (ok) sIw[__popcll(m & below)] = c;
  return __popcll(m);
}

// d(x, slot) of this lane's two slots (lanes j and 32 + j hold the lower and
// upper half sums of slots j and 32 + j) into the per-slot records.
template <bool L2>
__device__ __forceinline__ void rp_records(float s0, float s1, int nv, float nrm, float *sDw,
                                           float *sNw, uint64_t *sKw, const uint32_t *sIw) {
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5;
  // lower half's sum plus upper half's
  const float o0 = __shfl_xor(s0, 32, 64), o1 = __shfl_xor(s1, 32, 64);
  const float t0 = h == 0 ? s0 + o0 : o0 + s0, t1 = h == 0 ? s1 + o1 : o1 + s1;
  // lane j < 32 records slot j, lane 32 + j records slot 32 + j
  const float t = h == 0 ? t0 : t1;
  const float dxm = L2 ? t : -t;
  if (lane < nv) {
    const uint32_t cid = sIw[lane];
    sDw[lane] = dxm;
    sNw[lane] = nrm;
    sKw[lane] = ((uint64_t)f32_rank(dxm) << 32) | cid;
  }
}

template <int DP, bool L2, bool FULL>
__global__ void __launch_bounds__(64 * kRpWaves, 4) robustprune_mfma_kernel(
    const float *__restrict__ X, const float *__restrict__ norms, int64_t n, int d,
    const uint64_t *__restrict__ res, int l_max, float alpha, int R,
    const uint32_t *__restrict__ order, int64_t n_items, uint32_t *__restrict__ graph,
    uint32_t *__restrict__ degree) {
  constexpr int HALF = DP / 2;
  __shared__ __align__(16) uint64_t sK[kRpWaves][64];
  __shared__ __align__(16) float sD[kRpWaves][64];
  __shared__ __align__(16) float sN[kRpWaves][64];
  __shared__ uint32_t sI[kRpWaves][64];
  __shared__ float sT[kRpWaves][32 * 33];  // block 01, transposed into block 10
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int h = lane >> 5, l32 = lane & 31;
  const int64_t item = (int64_t)xcd_item(blockIdx.x, gridDim.x) * kRpWaves + wave;
  if (item >= n_items) return;
  const uint32_t x = __builtin_amdgcn_readfirstlane(order ? order[item] : (uint32_t)item);
  const uint64_t rv = lane < l_max ? res[(int64_t)x * l_max + lane] : (uint64_t)kEmptyId;
  // 1. valid candidates in slot order (FULL: d == DP)
  const int nv = rp_compact(rv, l_max, x, n, sI[wave]);
  wave_sync();

  // 2. fragments F0 (slots 0..31) and F1 (slots 32..63), taken CH
  //    dimensions of each half at a time: each chunk's rows feed the direct
  //    sums for d(x, c) (continued in index order) and the Gram's MFMAs (in
  //    the same k order as whole rows would). The next chunk's rows are
  //    loaded into registers while the current chunk's MFMAs run, so two
  //    chunks are live.
  constexpr int CH = HALF < 8 ? HALF : 8;
  static_assert(HALF % CH == 0, "chunking");
  f32x16 g00, g01, g11;
#pragma unroll
  for (int v = 0; v < 16; ++v) { g00[v] = 0.f; g01[v] = 0.f; g11[v] = 0.f; }
  float s0 = 0.f, s1 = 0.f, nrm = 0.f;
  const bool both = nv > 32;
  {
    const int kb = h * HALF;
    // slots past nv read x's own row: finite values whose Gram rows and
    // columns no decision reads (the rank sets hold valid slots only)
    const bool v0 = l32 < nv, v1 = 32 + l32 < nv;
    const uint32_t c0 = v0 ? sI[wave][l32] : x, c1 = v1 ? sI[wave][32 + l32] : x;
    // the norm of this lane's record slot (lane j: slot j, lane 32 + j: slot
    // 32 + j), loaded with the rows
    nrm = (L2 && lane < nv) ? norms[h == 0 ? c0 : c1] : 0.f;
    const float *r0 = X + (int64_t)c0 * d + kb;
    const float *r1 = X + (int64_t)c1 * d + kb;
    const float *rx = X + (int64_t)x * d + kb;
    float n0[CH], n1[CH], nx[CH];
    auto load_chunk = [&](int k0) {
      if constexpr (FULL) {
#pragma unroll
        for (int j = 0; j < CH; j += 4) {
          const float4 q0 = *reinterpret_cast<const float4 *>(r0 + k0 + j);
          const float4 q1 = *reinterpret_cast<const float4 *>(r1 + k0 + j);
          const float4 qx = *reinterpret_cast<const float4 *>(rx + k0 + j);
          n0[j] = q0.x; n0[j + 1] = q0.y; n0[j + 2] = q0.z; n0[j + 3] = q0.w;
          n1[j] = q1.x; n1[j + 1] = q1.y; n1[j + 2] = q1.z; n1[j + 3] = q1.w;
          nx[j] = qx.x; nx[j + 1] = qx.y; nx[j + 2] = qx.z; nx[j + 3] = qx.w;
        }
      } else {
#pragma unroll
        for (int j = 0; j < CH; ++j) {
          const bool in = kb + k0 + j < d;
          n0[j] = in ? r0[k0 + j] : 0.f;
          n1[j] = in ? r1[k0 + j] : 0.f;
          nx[j] = in ? rx[k0 + j] : 0.f;
        }
      }
    };
    load_chunk(0);
#pragma unroll
    for (int k0 = 0; k0 < HALF; k0 += CH) {
      float f0[CH], f1[CH], fx[CH];
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        f0[j] = n0[j];
        f1[j] = n1[j];
        fx[j] = nx[j];
      }
      if (k0 + CH < HALF) load_chunk(k0 + CH);
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        if constexpr (L2) {
          const float t0 = f0[j] - fx[j], t1 = f1[j] - fx[j];
          s0 = fmaf(t0, t0, s0);
          s1 = fmaf(t1, t1, s1);
        } else {
          s0 = fmaf(f0[j], fx[j], s0);
          s1 = fmaf(f1[j], fx[j], s1);
        }
      }
#pragma unroll
      for (int j = 0; j < CH; ++j)
        g00 = __builtin_amdgcn_mfma_f32_32x32x2f32(f0[j], f0[j], g00, 0, 0, 0);
      if (both) {
#pragma unroll
        for (int j = 0; j < CH; ++j) {
          g01 = __builtin_amdgcn_mfma_f32_32x32x2f32(f0[j], f1[j], g01, 0, 0, 0);
          g11 = __builtin_amdgcn_mfma_f32_32x32x2f32(f1[j], f1[j], g11, 0, 0, 0);
        }
      }
      // the chunk's sums are taken here, with one chunk in flight ahead and
      // no more: the compiler would otherwise defer the sums past the loop
      // and keep every chunk's rows live
      asm volatile("" : "+v"(s0), "+v"(s1));
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  rp_records<L2>(s0, s1, nv, nrm, sD[wave], sN[wave], sK[wave], sI[wave]);
  // block 10 (rows 32..63, columns 0..31) is block 01 transposed: T[r][c] =
  // G[r][32 + c] is written from block 01's layout and read back in block
  // 10's, G[32 + r][c] = T[c][r] (rows padded to 33 words)
  f32x16 g10;
  float *T = sT[wave];
  if (both) {
#pragma unroll
    for (int v = 0; v < 16; ++v) T[acc_row32(v, h) * 33 + l32] = g01[v];
  }
  wave_sync();
  if (both) {
#pragma unroll
    for (int v = 0; v < 16; ++v) g10[v] = T[l32 * 33 + acc_row32(v, h)];
  }
  // 3. pruner sets by slot
  const float *sNw = sN[wave];
  const float nA = L2 ? sNw[l32] : 0.f, xA = 0.f - sD[wave][l32];
  const uint32_t c00 = rp_sign_bits<L2>(g00, sNw, 0, nA, xA, alpha);
  uint32_t mlo, mhi = 0u;
  if (both) {
    const float nB = L2 ? sNw[32 + l32] : 0.f, xB = 0.f - sD[wave][32 + l32];
    const uint32_t c10 = rp_sign_bits<L2>(g10, sNw, 32, nA, xA, alpha);
    const uint32_t c01 = rp_sign_bits<L2>(g01, sNw, 0, nB, xB, alpha);
    const uint32_t c11 = rp_sign_bits<L2>(g11, sNw, 32, nB, xB, alpha);
    mlo = rp_join(c00, c01);
    mhi = rp_join(c10, c11);
  } else {
    mlo = c00 | ((uint32_t)__shfl_xor((int)c00, 32, 64) << 4);
  }
  rp_select(mlo, mhi, nv, R, x, sK[wave], sI[wave], graph, degree);
}

// The same RobustPrune reading a 16-bit operand (the index's bf16 / fp16
// copy, n x DP, zero padded) when that copy holds X exactly: the rows are
// half the bytes, d(x,c) is the same FP32 direct difference (of the same
// values, in the same order), and the Gram runs on v_mfma_f32_32x32x16 with
// FP32 accumulation of exact products, so where those sums are exact
// (integer data) every decision is the float32 kernel's. IDIFF (fp16 copy
// of integer data of range <= 2048, every distance form exact in float32):
// the differences are taken two at a time in fp16 (exact integers) and
// squared and summed by v_dot2_f32_f16, whose every partial sum is an
// integer of at most 2^24, so d(x,c) is the float32 kernel's value with a
// quarter of the instructions.
template <int PREC, int DP, bool L2, bool IDIFF>
__global__ void __launch_bounds__(64 * kRpWaves, 4) robustprune_mfma16_kernel(
    const uint8_t *__restrict__ Xop, const float *__restrict__ norms, int64_t n,
    const uint64_t *__restrict__ res, int l_max, float alpha, int R,
    const uint32_t *__restrict__ order, int64_t n_items, uint32_t *__restrict__ graph,
    uint32_t *__restrict__ degree) {
  static_assert(!IDIFF || PREC == PIPNN_PREC_FP16, "packed differences are fp16");
  constexpr int HALF = DP / 2;
  constexpr int NA = HALF / 8;        // 16-byte vectors (8 values) per lane
  constexpr int CB = DP * 2;          // bytes per operand row
  __shared__ __align__(16) uint64_t sK[kRpWaves][64];
  __shared__ __align__(16) float sD[kRpWaves][64];
  __shared__ __align__(16) float sN[kRpWaves][64];
  __shared__ uint32_t sI[kRpWaves][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int h = lane >> 5, l32 = lane & 31;
  const int64_t item = (int64_t)xcd_item(blockIdx.x, gridDim.x) * kRpWaves + wave;
  if (item >= n_items) return;
  const uint32_t x = __builtin_amdgcn_readfirstlane(order ? order[item] : (uint32_t)item);
  const uint64_t rv = lane < l_max ? res[(int64_t)x * l_max + lane] : (uint64_t)kEmptyId;

  const int nv = rp_compact(rv, l_max, x, n, sI[wave]);
  wave_sync();

  auto val = [](uint32_t code) -> float {
    if constexpr (PREC == PIPNN_PREC_BF16) return __uint_as_float(code << 16);
    else return (float)__builtin_bit_cast(_Float16, (uint16_t)code);
  };
  typedef _Float16 h2_t __attribute__((ext_vector_type(2)));
  uint4 a0[NA], a1[NA];
  float s0 = 0.f, s1 = 0.f, nrm = 0.f;
  const bool both = nv > 32;
  {
    // slots past nv read x's own row: finite values whose Gram rows and
    // columns no decision reads (the rank sets hold valid slots only)
    const bool v0 = l32 < nv, v1 = 32 + l32 < nv;
    const uint32_t c0 = v0 ? sI[wave][l32] : x, c1 = v1 ? sI[wave][32 + l32] : x;
    // the norm of this lane's record slot (lane j: slot j, lane 32 + j: slot
    // 32 + j), loaded with the rows
    nrm = (L2 && lane < nv) ? norms[h == 0 ? c0 : c1] : 0.f;
    const uint4 *r0 = reinterpret_cast<const uint4 *>(Xop + (int64_t)c0 * CB + h * HALF * 2);
    const uint4 *r1 = reinterpret_cast<const uint4 *>(Xop + (int64_t)c1 * CB + h * HALF * 2);
    const uint4 *rx = reinterpret_cast<const uint4 *>(Xop + (int64_t)x * CB + h * HALF * 2);
#pragma unroll
    for (int sv = 0; sv < NA; ++sv) {
      a0[sv] = r0[sv];
      a1[sv] = r1[sv];
      const uint4 qx = rx[sv];
      const uint32_t w0[4] = {a0[sv].x, a0[sv].y, a0[sv].z, a0[sv].w};
      const uint32_t w1[4] = {a1[sv].x, a1[sv].y, a1[sv].z, a1[sv].w};
      const uint32_t wx[4] = {qx.x, qx.y, qx.z, qx.w};
      if constexpr (IDIFF) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const h2_t c0v = __builtin_bit_cast(h2_t, w0[e]), c1v = __builtin_bit_cast(h2_t, w1[e]);
          const h2_t xv = __builtin_bit_cast(h2_t, wx[e]);
          if constexpr (L2) {
            const h2_t t0 = c0v - xv, t1 = c1v - xv;
            s0 = __builtin_amdgcn_fdot2(t0, t0, s0, false);
            s1 = __builtin_amdgcn_fdot2(t1, t1, s1, false);
          } else {
            s0 = __builtin_amdgcn_fdot2(c0v, xv, s0, false);
            s1 = __builtin_amdgcn_fdot2(c1v, xv, s1, false);
          }
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float c0v = val((w0[e >> 1] >> (16 * (e & 1))) & 0xFFFFu);
          const float c1v = val((w1[e >> 1] >> (16 * (e & 1))) & 0xFFFFu);
          const float xv = val((wx[e >> 1] >> (16 * (e & 1))) & 0xFFFFu);
          if constexpr (L2) {
            const float t0 = c0v - xv, t1 = c1v - xv;
            s0 = fmaf(t0, t0, s0);
            s1 = fmaf(t1, t1, s1);
          } else {
            s0 = fmaf(c0v, xv, s0);
            s1 = fmaf(c1v, xv, s1);
          }
        }
      }
    }
  }
  rp_records<L2>(s0, s1, nv, nrm, sD[wave], sN[wave], sK[wave], sI[wave]);
  wave_sync();
  typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
  typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
  auto mm = [](uint4 p, uint4 q, f32x16 acc) -> f32x16 {
    if constexpr (PREC == PIPNN_PREC_BF16)
      return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, p),
                                                      __builtin_bit_cast(bf16x8_t, q), acc, 0, 0, 0);
    else
      return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8_t, p),
                                                     __builtin_bit_cast(f16x8_t, q), acc, 0, 0, 0);
  };
  auto gram = [&](const uint4 *p, const uint4 *q) -> f32x16 {
    f32x16 g;
#pragma unroll
    for (int v = 0; v < 16; ++v) g[v] = 0.f;
#pragma unroll
    for (int sv = 0; sv < NA; ++sv) g = mm(p[sv], q[sv], g);
    return g;
  };
  // 3. the four blocks, in the order that frees F0 after the third
  const float *sNw = sN[wave];
  const float nA = L2 ? sNw[l32] : 0.f, xA = 0.f - sD[wave][l32];
  uint32_t mlo, mhi = 0u;
  if (both) {
    const float nB = L2 ? sNw[32 + l32] : 0.f, xB = 0.f - sD[wave][32 + l32];
    // (the scheduling barriers keep at most two fragments and three blocks
    // live, so that the rows fit the registers of four waves per SIMD)
    const f32x16 g00 = gram(a0, a0);
    const f32x16 g01 = gram(a0, a1);
    __builtin_amdgcn_sched_barrier(0);
    const uint32_t c00 = rp_sign_bits<L2>(g00, sNw, 0, nA, xA, alpha);
    const f32x16 g10 = gram(a1, a0);
    __builtin_amdgcn_sched_barrier(0);
    const uint32_t c01 = rp_sign_bits<L2>(g01, sNw, 0, nB, xB, alpha);
    const f32x16 g11 = gram(a1, a1);
    __builtin_amdgcn_sched_barrier(0);
    const uint32_t c10 = rp_sign_bits<L2>(g10, sNw, 32, nA, xA, alpha);
    const uint32_t c11 = rp_sign_bits<L2>(g11, sNw, 32, nB, xB, alpha);
    mlo = rp_join(c00, c01);
    mhi = rp_join(c10, c11);
  } else {
    const f32x16 g00 = gram(a0, a0);
    const uint32_t c00 = rp_sign_bits<L2>(g00, sNw, 0, nA, xA, alpha);
    mlo = c00 | ((uint32_t)__shfl_xor((int)c00, 32, 64) << 4);
  }
  rp_select(mlo, mhi, nv, R, x, sK[wave], sI[wave], graph, degree);
}

typedef int i32x4_t __attribute__((ext_vector_type(4)));
typedef int i32x16_t __attribute__((ext_vector_type(16)));

// The same RobustPrune (L2) on the index's int8 rows (x - lo8 - 128 of an
// integral X whose coordinates span at most 256 values, DB bytes per row):
// the rows are a quarter of the float32 bytes and half the fp16 ones. Every
// distance is an integer below 2^24 and L2 is translation invariant, so
// d(x,c) = |x'|^2 + |c'|^2 - 2 x'.c' (x'.c' by v_dot4_i32_i8, each half
// wave's partial sum plus the other's) is the float32 direct difference's
// value, and the prune test becomes integer arithmetic: with alpha = am *
// 2^-ash exactly, fma(alpha, d(y,z), -d(x,z)) < 0 (one rounding of an exact
// multiple of 2^-ash, so its sign is exact) holds iff d(y,z) < t_z, t_z the
// least integer with am * t_z >= d(x,z) * 2^ash. So the Gram MFMA
// (v_mfma_i32_32x32x32_i8) starts from t_z - 1 - |z'|^2 - |y'|^2 and takes
// each k-step twice: entry (y,z) ends as t_z - 1 - d(y,z), >= 0 exactly when
// y prunes z, and its sign bit is the complement of the pruner bit.
template <int DB>
__global__ void __launch_bounds__(64 * kRpWaves, 4) robustprune_i8_kernel(
    const uint8_t *__restrict__ X8, const float *__restrict__ n8, int64_t n,
    const uint64_t *__restrict__ res, int l_max, float alpha, uint32_t am, int ash, int R,
    const uint32_t *__restrict__ order, int64_t n_items, uint32_t *__restrict__ graph,
    uint32_t *__restrict__ degree) {
  constexpr int HB = DB / 2;   // bytes of a row per half wave
  constexpr int NA = HB / 16;  // 16-byte vectors per lane
  __shared__ __align__(16) uint64_t sK[kRpWaves][64];
  __shared__ __align__(16) float sD[kRpWaves][64];
  __shared__ __align__(16) int sN[kRpWaves][64];  // |c'|^2
  __shared__ uint32_t sI[kRpWaves][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int h = lane >> 5, l32 = lane & 31;
  const int64_t item = (int64_t)xcd_item(blockIdx.x, gridDim.x) * kRpWaves + wave;
  if (item >= n_items) return;
  const uint32_t x = __builtin_amdgcn_readfirstlane(order ? order[item] : (uint32_t)item);
  const uint64_t rv = lane < l_max ? res[(int64_t)x * l_max + lane] : (uint64_t)kEmptyId;

  const int nv = rp_compact(rv, l_max, x, n, sI[wave]);
  wave_sync();

  uint4 a0[NA], a1[NA];
  const bool both = nv > 32;
  {
    // slots past nv read x's own row: finite values whose Gram rows and
    // columns no decision reads (the rank sets hold valid slots only)
    const bool v0 = l32 < nv, v1 = 32 + l32 < nv;
    const uint32_t c0 = v0 ? sI[wave][l32] : x, c1 = v1 ? sI[wave][32 + l32] : x;
    const int nrm = lane < nv ? (int)n8[h == 0 ? c0 : c1] : 0;
    const int nx = (int)n8[x];
    const uint4 *r0 = reinterpret_cast<const uint4 *>(X8 + (int64_t)c0 * DB + h * HB);
    const uint4 *r1 = reinterpret_cast<const uint4 *>(X8 + (int64_t)c1 * DB + h * HB);
    const uint4 *rx = reinterpret_cast<const uint4 *>(X8 + (int64_t)x * DB + h * HB);
    int p0 = 0, p1 = 0;
#pragma unroll
    for (int sv = 0; sv < NA; ++sv) {
      a0[sv] = r0[sv];
      a1[sv] = r1[sv];
      const uint4 qx = rx[sv];
      p0 = __builtin_amdgcn_sdot4((int)a0[sv].x, (int)qx.x, p0, false);
      p0 = __builtin_amdgcn_sdot4((int)a0[sv].y, (int)qx.y, p0, false);
      p0 = __builtin_amdgcn_sdot4((int)a0[sv].z, (int)qx.z, p0, false);
      p0 = __builtin_amdgcn_sdot4((int)a0[sv].w, (int)qx.w, p0, false);
      p1 = __builtin_amdgcn_sdot4((int)a1[sv].x, (int)qx.x, p1, false);
      p1 = __builtin_amdgcn_sdot4((int)a1[sv].y, (int)qx.y, p1, false);
      p1 = __builtin_amdgcn_sdot4((int)a1[sv].z, (int)qx.z, p1, false);
      p1 = __builtin_amdgcn_sdot4((int)a1[sv].w, (int)qx.w, p1, false);
    }
    // lane j < 32 records slot j, lane 32 + j records slot 32 + j
    const int o0 = __shfl_xor(p0, 32, 64), o1 = __shfl_xor(p1, 32, 64);
    const int xc = h == 0 ? p0 + o0 : p1 + o1;
    const float dxm = (float)(nx + nrm - 2 * xc);
    if (lane < nv) {
      const uint32_t cid = sI[wave][lane];
      sD[wave][lane] = dxm;
      sN[wave][lane] = nrm;
      sK[wave][lane] = ((uint64_t)f32_rank(dxm) << 32) | cid;
    }
  }
  wave_sync();
  // t_z - 1 - |z'|^2 for column slot z (d(x,z) < 2^24: the float estimate
  // of t_z is off by at most one; two exact 48-bit tests settle it)
  auto col_term = [&](int z) -> int {
    const float dx = sD[wave][z];
    const uint64_t num = (uint64_t)(uint32_t)(int)dx << ash;
    int t = (int)ceilf(dx / alpha);
    t = t < 1 ? 1 : t;
    if ((uint64_t)(uint32_t)(t - 1) * am >= num) --t;
    if ((uint64_t)(uint32_t)t * am < num) ++t;
    return t - 1 - sN[wave][z];
  };
  // pruner bits of column z of block (rows row0 + acc_row32(v, h)), laid out
  // as rp_sign_bits lays them out
  auto pruners = [&](const uint4 *p, const uint4 *q, int row0, int cz) -> uint32_t {
    i32x16_t g;
#pragma unroll
    for (int grp = 0; grp < 4; ++grp) {
      const int4 ny = *reinterpret_cast<const int4 *>(&sN[wave][row0 + 8 * grp + 4 * h]);
      g[4 * grp] = cz - ny.x; g[4 * grp + 1] = cz - ny.y;
      g[4 * grp + 2] = cz - ny.z; g[4 * grp + 3] = cz - ny.w;
    }
#pragma unroll
    for (int sv = 0; sv < NA; ++sv) {
      const i32x4_t pa = __builtin_bit_cast(i32x4_t, p[sv]), qb = __builtin_bit_cast(i32x4_t, q[sv]);
      g = __builtin_amdgcn_mfma_i32_32x32x32_i8(pa, qb, g, 0, 0, 0);
      g = __builtin_amdgcn_mfma_i32_32x32x32_i8(pa, qb, g, 0, 0, 0);
    }
    uint32_t b = 0u;
#pragma unroll
    for (int grp = 3; grp >= 0; --grp) {
#pragma unroll
      for (int j = 3; j >= 0; --j) b = __builtin_amdgcn_alignbit(b, (uint32_t)g[4 * grp + j], 31);
      if (grp) b <<= 4;
    }
    return ~b & 0x0F0F0F0Fu;
  };
  const int czA = col_term(l32);
  uint32_t mlo, mhi = 0u;
  if (both) {
    const int czB = col_term(32 + l32);
    const uint32_t c00 = pruners(a0, a0, 0, czA);
    const uint32_t c01 = pruners(a0, a1, 0, czB);
    const uint32_t c10 = pruners(a1, a0, 32, czA);
    const uint32_t c11 = pruners(a1, a1, 32, czB);
    mlo = rp_join(c00, c01);
    mhi = rp_join(c10, c11);
  } else {
    const uint32_t c00 = pruners(a0, a0, 0, czA);
    mlo = c00 | ((uint32_t)__shfl_xor((int)c00, 32, 64) << 4);
  }
  rp_select(mlo, mhi, nv, R, x, sK[wave], sI[wave], graph, degree);
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

template <int PREC>
__device__ __forceinline__ f32x4 rp_mfma16(uint4 a, uint4 b, f32x4 acc) {
  if constexpr (PREC == PIPNN_PREC_BF16)
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                    __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                   __builtin_bit_cast(f16x8, b), acc, 0, 0, 0);
}

// Upper-triangle index of the candidate Gram, y <= z, packed by column.
__device__ __forceinline__ int tri_idx(int y, int z) {
  return y <= z ? z * (z + 1) / 2 + y : y * (y + 1) / 2 + z;
}

// RobustPrune for wide operands (512 or 768 dimensions, the index's bf16 /
// fp16 GEMM operand; up to 111 reservoir candidates, R <= 64). One wave per
// point x. Rows are x and its candidates (reservoir order); their Gram
// G = C C^T is accumulated on 16x16x32 MFMAs, all block pairs i <= j, with
// the rows staged through LDS 64 dimensions at a time; the upper triangle
// of G is kept in LDS. Distances are the GEMM form of the operand:
// d(y,z) = G[y][y] + G[z][z] - 2 G[y][z] (squared L2) or -G[y][z] (inner
// product). The candidates are ranked by (d(x,c), id) by counting, then
// walked in that order: z is admitted unless an admitted y has
// alpha * d(y,z) < d(x,z) (the sign of a fused multiply-add), until R are
// admitted -- the lazy form of Alg. 2.
constexpr int kRpwRows = 112;  // x + up to 111 candidates: 7 blocks of 16
constexpr int kRpwKC = 64;     // dimensions per staged chunk
constexpr int kRpwTri = kRpwRows * (kRpwRows + 1) / 2;

template <int PREC, int DP, bool L2>
__global__ void __launch_bounds__(256, 1) robustprune_wide_kernel(
    const uint8_t *__restrict__ Xop, int64_t op_ld, int64_t n, const uint64_t *__restrict__ res,
    int l_max, float alpha, int R, const uint32_t *__restrict__ order, int64_t n_items,
    uint32_t *__restrict__ graph, uint32_t *__restrict__ degree) {
  constexpr int LROW = kRpwKC + 8;  // staged row stride (16-bit elements)
  constexpr int NCHUNK = DP / kRpwKC;
  static_assert(kRpwRows * LROW / 2 <= kRpwTri, "staging fits in the Gram region");
  __shared__ uint32_t sW[kRpWaves][kRpwTri];
  __shared__ uint32_t sId[kRpWaves][kRpwRows];
  __shared__ uint32_t sPos[kRpWaves][kRpwRows];
  __shared__ uint64_t sKey[kRpWaves][kRpwRows];
  __shared__ float sDx[kRpWaves][kRpwRows];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t item = (int64_t)xcd_item(blockIdx.x, gridDim.x) * kRpWaves + wave;
  if (item >= n_items) return;
  const uint32_t x = __builtin_amdgcn_readfirstlane(order ? order[item] : (uint32_t)item);
  uint32_t *W = sW[wave];
  uint32_t *ids = sId[wave];

  // 1. rows: x, then the valid reservoir candidates in slot order
  if (lane == 0) ids[0] = x;
  int M = 0;
  for (int b = 0; b < l_max; b += 64) {
    const int i = b + lane;
    uint32_t c = kEmptyId;
    if (i < l_max) c = slot_id(res[(int64_t)x * l_max + i]);
    const bool ok = i < l_max && c != kEmptyId && c != x && c < n;
    const uint64_t m = __ballot(ok);
    const int pos = __popcll(m & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
    if (ok && 1 + M + pos < kRpwRows) ids[1 + M + pos] = c;
    M += __popcll(m);
  }
  if (M > kRpwRows - 1) M = kRpwRows - 1;
  const int rows = M + 1;
  const int NB = (rows + 15) >> 4;
  wave_sync();

  // 2. Gram on MFMA: acc[p] for block pair p = (i, j), i <= j < NB
  constexpr int NP = 28;  // pairs of 7 blocks
  f32x4 acc[NP];
#pragma unroll
  for (int p2 = 0; p2 < NP; ++p2) acc[p2] = f32x4{0.f, 0.f, 0.f, 0.f};
  uint16_t *stg = reinterpret_cast<uint16_t *>(W);
  const int q = lane >> 4, l16 = lane & 15;
  // Staging of rows [0, 16*NB) x dims [ch*KC, ch*KC + KC), 8 pieces of 16
  // bytes per row, lane-strided: piece pc = lane + 64 i. The pieces of chunk
  // ch + 1 are loaded into registers while chunk ch's MFMAs run.
  constexpr int NPC = kRpwRows * 8 / 64;  // pieces per lane at most (14)
  const int npc = 16 * NB * 8;
  uint4 nxt[NPC];
  auto load_chunk = [&](int ch) {
#pragma unroll
    for (int i = 0; i < NPC; ++i) {
      const int pc = lane + 64 * i;
      const int r = pc >> 3, part = pc & 7;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (pc < npc && r < rows)
        v = *reinterpret_cast<const uint4 *>(Xop + (int64_t)ids[r] * op_ld +
                                             (int64_t)(ch * kRpwKC + part * 8) * 2);
      nxt[i] = v;
    }
  };
  load_chunk(0);
  for (int ch = 0; ch < NCHUNK; ++ch) {
#pragma unroll
    for (int i = 0; i < NPC; ++i) {
      const int pc = lane + 64 * i;
      const int r = pc >> 3, part = pc & 7;
      if (pc < npc) *reinterpret_cast<uint4 *>(&stg[r * LROW + part * 8]) = nxt[i];
    }
    wave_sync();
    if (ch + 1 < NCHUNK) load_chunk(ch + 1);
#pragma unroll
    for (int st = 0; st < kRpwKC / 32; ++st) {
      uint4 f[7];
#pragma unroll
      for (int i = 0; i < 7; ++i)
        f[i] = (i < NB) ? *reinterpret_cast<const uint4 *>(&stg[(16 * i + l16) * LROW + st * 32 + q * 8])
                        : make_uint4(0u, 0u, 0u, 0u);
      int p2 = 0;
#pragma unroll
      for (int i = 0; i < 7; ++i)
#pragma unroll
        for (int j = i; j < 7; ++j, ++p2)
          if (j < NB) acc[p2] = rp_mfma16<PREC>(f[i], f[j], acc[p2]);
    }
    wave_sync();
  }
  // 3. upper triangle of G into LDS (over the staging area)
  {
    int p2 = 0;
#pragma unroll
    for (int i = 0; i < 7; ++i)
#pragma unroll
      for (int j = i; j < 7; ++j, ++p2) {
        if (j < NB) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int y = 16 * i + 4 * q + r, z = 16 * j + l16;
            if (y <= z) W[z * (z + 1) / 2 + y] = __float_as_uint(acc[p2][r]);
          }
        }
      }
  }
  wave_sync();
  auto G = [&](int y, int z) { return __uint_as_float(W[tri_idx(y, z)]); };

  // 4. d(x, c) and the rank of (d, id) among the candidates
  const float g00 = G(0, 0);
  for (int t = lane; t < M; t += 64) {
    const int r = t + 1;
    const float gxz = G(0, r);
    const float dxz = L2 ? g00 + fmaf(-2.f, gxz, G(r, r)) : -gxz;
    sDx[wave][r] = dxz;
    sKey[wave][r] = ((uint64_t)f32_rank(dxz) << 32) | ids[r];
  }
  wave_sync();
  for (int t = lane; t < M; t += 64) {
    const uint64_t kt = sKey[wave][t + 1];
    int rank = 0;
    for (int u = 1; u <= M; ++u) rank += sKey[wave][u] < kt ? 1 : 0;
    sPos[wave][rank] = (uint32_t)(t + 1);
  }
  wave_sync();

  // 5. lazy admission: lane a holds the a-th admitted row
  int ne = 0;
  int my_row = 0;
  for (int p = 0; p < M && ne < R; ++p) {
    const int z = (int)sPos[wave][p];
    const float dxz = sDx[wave][z];
    bool prune = false;
    if (lane < ne) {
      const float gyz = G(my_row, z);
      const float dyz = L2 ? G(my_row, my_row) + fmaf(-2.f, gyz, G(z, z)) : -gyz;
      prune = fmaf(alpha, dyz, -dxz) < 0.f;
    }
    if (__ballot(prune) == 0ull) {
      if (lane == ne) my_row = z;
      ++ne;
    }
  }
  uint32_t *grow = graph + (int64_t)x * R;
  if (lane < R) grow[lane] = lane < ne ? ids[my_row] : kEmptyId;
  if (lane == 0) degree[x] = (uint32_t)ne;
}

int rp_row_bits(const Index &I) {
  if (I.p.l_max > 64) return I.p.l_max <= kRpwRows - 1 && I.p.R <= 64 && I.xlow.p &&
                             (I.p.gemm_prec == PIPNN_PREC_FP16 || I.p.gemm_prec == PIPNN_PREC_BF16) &&
                             (I.ldo == 512 || I.ldo == 768) ? 16 : 32;
  if (I.p.metric == PIPNN_METRIC_L2 && I.i8_ok && I.x8.p && (I.ld8 == 64 || I.ld8 == 128) &&
      I.p.alpha < 8388608.f)
    return 8;
  if (I.copy16_exact() && (I.ldo == 64 || I.ldo == 96 || I.ldo == 128)) return 16;
  if (I.d <= 128) return 32;
  const bool wide_op = (I.p.gemm_prec == PIPNN_PREC_FP16 || I.p.gemm_prec == PIPNN_PREC_BF16) &&
                       (I.ldo == 512 || I.ldo == 768) && I.xlow.p;
  return wide_op && I.p.R <= 64 ? 16 : 32;
}

hipError_t launch_robustprune(const Index &I, const uint64_t *res, uint32_t *graph, uint32_t *degree,
                              const uint32_t *subset, int64_t n_subset, hipStream_t s) {
  if (I.p.l_max > 256 || I.p.R > 256) return hipErrorInvalidValue;
  const uint32_t *order =
      subset ? subset : (I.rp_order_valid ? I.rp_order.as<uint32_t>() : nullptr);
  const int64_t n_items = subset ? n_subset : I.n;
  if (n_items <= 0) return hipSuccess;
  const bool op16 = I.copy16_exact();
  const bool l2 = I.p.metric == PIPNN_METRIC_L2;
  if (rp_row_bits(I) == 8) {
    const int64_t blocks = xcd_grid((n_items + kRpWaves - 1) / kRpWaves);
    // alpha = am * 2^-ash exactly (1 <= alpha < 2^23: ash in 1..23)
    int ex = 0;
    const float fr = std::frexp(I.p.alpha, &ex);
    const uint32_t am = (uint32_t)std::ldexp(fr, 24);
    const int ash = 24 - ex;
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64 * kRpWaves), 0, s,
                         I.x8.as<uint8_t>(), I.n8.as<float>(), I.n, res, I.p.l_max, I.p.alpha, am,
                         ash, I.p.R, order, n_items, graph, degree);
    };
    I.ld8 == 64 ? go(robustprune_i8_kernel<64>) : go(robustprune_i8_kernel<128>);
    return hipGetLastError();
  }
  if (I.p.l_max <= 64 && op16 && (I.ldo == 64 || I.ldo == 96 || I.ldo == 128)) {
    const int64_t blocks = xcd_grid((n_items + kRpWaves - 1) / kRpWaves);
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64 * kRpWaves), 0, s,
                         I.xlow.as<uint8_t>(), I.norms.as<float>(), I.n, res, I.p.l_max,
                         I.p.alpha, I.p.R, order, n_items, graph, degree);
    };
    // packed fp16 differences: integer data (every distance form exact in
    // float32) whose differences are fp16 integers (range <= 2048)
    const bool idiff = I.copy_prec == PIPNN_PREC_FP16 && I.int_exact &&
                       (!l2 || I.int_hi - I.int_lo <= 2048);
    auto pick = [&](auto dp) {
      constexpr int DP = decltype(dp)::value;
      if (I.copy_prec == PIPNN_PREC_BF16)
        l2 ? go(robustprune_mfma16_kernel<PIPNN_PREC_BF16, DP, true, false>)
           : go(robustprune_mfma16_kernel<PIPNN_PREC_BF16, DP, false, false>);
      else if (idiff)
        l2 ? go(robustprune_mfma16_kernel<PIPNN_PREC_FP16, DP, true, true>)
           : go(robustprune_mfma16_kernel<PIPNN_PREC_FP16, DP, false, true>);
      else
        l2 ? go(robustprune_mfma16_kernel<PIPNN_PREC_FP16, DP, true, false>)
           : go(robustprune_mfma16_kernel<PIPNN_PREC_FP16, DP, false, false>);
    };
    if (I.ldo == 64) pick(std::integral_constant<int, 64>());
    else if (I.ldo == 96) pick(std::integral_constant<int, 96>());
    else pick(std::integral_constant<int, 128>());
    return hipGetLastError();
  }
  if (I.p.l_max <= 64 && I.d <= 128) {
    const int64_t blocks = xcd_grid((n_items + kRpWaves - 1) / kRpWaves);
    auto args = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64 * kRpWaves), 0, s, I.xf(),
                         I.norms.as<float>(), I.n, I.d, res, I.p.l_max, I.p.alpha, I.p.R, order,
                         n_items, graph, degree);
    };
    auto pick = [&](auto dp) {
      constexpr int DP = decltype(dp)::value;
      if (I.d == DP)
        l2 ? args(robustprune_mfma_kernel<DP, true, true>)
           : args(robustprune_mfma_kernel<DP, false, true>);
      else
        l2 ? args(robustprune_mfma_kernel<DP, true, false>)
           : args(robustprune_mfma_kernel<DP, false, false>);
    };
    if (I.d <= 32) pick(std::integral_constant<int, 32>());
    else if (I.d <= 64) pick(std::integral_constant<int, 64>());
    else if (I.d <= 96) pick(std::integral_constant<int, 96>());
    else pick(std::integral_constant<int, 128>());
    return hipGetLastError();
  }
  const int dp = I.ldo;
  const bool wide_op = (I.p.gemm_prec == PIPNN_PREC_FP16 || I.p.gemm_prec == PIPNN_PREC_BF16) &&
                       (dp == 512 || dp == 768) && I.xlow.p;
  if (wide_op && I.p.l_max <= kRpwRows - 1 && I.p.R <= 64) {
    const int64_t blocks = xcd_grid((n_items + kRpWaves - 1) / kRpWaves);
    const uint8_t *xop = I.xlow.as<uint8_t>();
    const int64_t op_ld = (int64_t)dp * 2;
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64 * kRpWaves), 0, s, xop, op_ld, I.n,
                         res, I.p.l_max, I.p.alpha, I.p.R, order, n_items, graph, degree);
    };
    if (I.p.gemm_prec == PIPNN_PREC_FP16) {
      if (dp == 512) l2 ? go(robustprune_wide_kernel<PIPNN_PREC_FP16, 512, true>)
                        : go(robustprune_wide_kernel<PIPNN_PREC_FP16, 512, false>);
      else l2 ? go(robustprune_wide_kernel<PIPNN_PREC_FP16, 768, true>)
              : go(robustprune_wide_kernel<PIPNN_PREC_FP16, 768, false>);
    } else {
      if (dp == 512) l2 ? go(robustprune_wide_kernel<PIPNN_PREC_BF16, 512, true>)
                        : go(robustprune_wide_kernel<PIPNN_PREC_BF16, 512, false>);
      else l2 ? go(robustprune_wide_kernel<PIPNN_PREC_BF16, 768, true>)
              : go(robustprune_wide_kernel<PIPNN_PREC_BF16, 768, false>);
    }
    return hipGetLastError();
  }
  const int64_t blocks = (n_items + kRpWaves - 1) / kRpWaves;
  hipLaunchKernelGGL(robustprune_kernel, dim3((unsigned)blocks), dim3(64 * kRpWaves), 0, s, I.xf(),
                     I.n, I.d, I.p.metric, res, I.p.l_max, I.p.alpha, I.p.R, order, n_items, graph,
                     degree);
  return hipGetLastError();
}

// ---------------------------------------------------------------------
// Processing order for RobustPrune: points in the order of their first
// appearance in the leaf CSR (so that a point's candidates, which come from
// its own leaves, are read while those leaves are hot in L2), then every
// point that no leaf holds, ascending.
__global__ void first_pos_kernel(const uint32_t *mem, int64_t cnt, int64_t n, uint32_t *first) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < cnt && mem[p] < n) atomicMin(&first[mem[p]], (uint32_t)p);
}
__global__ void first_flag_kernel(const uint32_t *mem, int64_t cnt, int64_t n,
                                  const uint32_t *first, uint32_t *flag) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < cnt) flag[p] = (mem[p] < n && first[mem[p]] == (uint32_t)p) ? 1u : 0u;
}
__global__ void order_seen_kernel(const uint32_t *mem, int64_t cnt, const uint32_t *flag,
                                  const int64_t *pos, uint32_t *order) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < cnt && flag[p]) order[pos[p]] = mem[p];
}
__global__ void unseen_flag_kernel(const uint32_t *first, int64_t n, uint32_t *flag) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x < n) flag[x] = first[x] == 0xFFFFFFFFu ? 1u : 0u;
}
__global__ void order_unseen_kernel(const uint32_t *flag, const int64_t *pos, int64_t n,
                                    const int64_t *n_seen, uint32_t *order) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x < n && flag[x]) order[*n_seen + pos[x]] = (uint32_t)x;
}

// first/flag: n and max(n, cnt) uint32; pos: max(n, cnt)+1 int64; tmp: scan scratch
hipError_t launch_leaf_order(const uint32_t *mem, int64_t cnt, int64_t n, uint32_t *first,
                             uint32_t *flag, int64_t *pos, int64_t *pos2, int64_t *tmp,
                             uint32_t *order, hipStream_t s) {
  const unsigned gc = (unsigned)((cnt + 255) / 256), gn = (unsigned)((n + 255) / 256);
  hipError_t e = launch_fill_u32(first, 0xFFFFFFFFu, n, s);
  if (e != hipSuccess) return e;
  if (cnt > 0) {
    hipLaunchKernelGGL(first_pos_kernel, dim3(gc), dim3(256), 0, s, mem, cnt, n, first);
    hipLaunchKernelGGL(first_flag_kernel, dim3(gc), dim3(256), 0, s, mem, cnt, n, first, flag);
    if ((e = launch_scan_u32(flag, pos, cnt, tmp, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(order_seen_kernel, dim3(gc), dim3(256), 0, s, mem, cnt, flag, pos, order);
  } else {
    if ((e = launch_fill_u64(reinterpret_cast<uint64_t *>(pos), 0ull, 1, s)) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(unseen_flag_kernel, dim3(gn), dim3(256), 0, s, first, n, flag);
  if ((e = launch_scan_u32(flag, pos2, n, tmp, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(order_unseen_kernel, dim3(gn), dim3(256), 0, s, flag, pos2, n, pos + cnt,
                     order);
  return hipGetLastError();
}

// ---------------------------------------------------------------------
// BeamSearch. One wave per query. The beam is a sorted array of keys
// (rank(distance), id) in LDS with a visited flag per entry; `seen` is a
// per-query bitmap over the n points in global memory (cleared by the
// caller). Each step visits the first unvisited entry, evaluates its
// neighbours that were never seen, sorts them, and merges them into the
// beam, which keeps its first L entries (Alg. 1).
//
// LDS is sized per launch for the beam width L, the degree bound R and the
// dimension d (beam and merge buffer: 2 x 8 L bytes, visited flags 2 L,
// sorted new keys 8 x pow2(R), the query 4 d), so that narrow beams keep
// many queries resident per compute unit. A lane evaluates one neighbour:
// with VEC its row is read as 16-byte vectors (d a multiple of 4, rows 16-byte
// aligned); the products are summed in index order either way.
constexpr int kMaxL = 1024;
constexpr int kMaxR = 256;
constexpr int kMaxQD = 1024;

struct SearchLds {
  int beam, tmp, vis, tvis, nw, qv, bytes;
};
static SearchLds search_lds(int L, int R, int d) {
  int P = 2;
  while (P < R) P <<= 1;
  auto up = [](int b) { return (b + 15) & ~15; };
  SearchLds o;
  o.beam = 0;
  o.tmp = o.beam + up(8 * L);
  o.nw = o.tmp + up(8 * L);
  o.qv = o.nw + up(8 * P);
  o.vis = o.qv + up(4 * d);
  o.tvis = o.vis + up(L);
  o.bytes = o.tvis + up(L);
  return o;
}

template <bool VEC>
__global__ void __launch_bounds__(64) search_kernel(const float *__restrict__ X, int64_t n, int d,
                                                    int metric, const uint32_t *__restrict__ graph,
                                                    int R, const float *__restrict__ Q, int k,
                                                    int L, uint32_t start,
                                                    uint32_t *__restrict__ out_ids,
                                                    float *__restrict__ out_dist,
                                                    uint32_t *__restrict__ out_cmps,
                                                    uint32_t *__restrict__ seen_bits,
                                                    int64_t words_per_query, SearchLds lo) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  uint64_t *beam = reinterpret_cast<uint64_t *>(smem + lo.beam);
  uint64_t *tmp = reinterpret_cast<uint64_t *>(smem + lo.tmp);
  uint8_t *vis = smem + lo.vis;
  uint8_t *tvis = smem + lo.tvis;
  uint64_t *nw = reinterpret_cast<uint64_t *>(smem + lo.nw);
  float *qv = reinterpret_cast<float *>(smem + lo.qv);
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
    if constexpr (VEC) {
      const float4 *xv = reinterpret_cast<const float4 *>(xu);
      const float4 *qq = reinterpret_cast<const float4 *>(qv);
#pragma unroll 4
      for (int i = 0; i < d / 4; ++i) {
        const float4 x = xv[i], c = qq[i];
        if (l2) {
          float t = c.x - x.x; s = fmaf(t, t, s);
          t = c.y - x.y; s = fmaf(t, t, s);
          t = c.z - x.z; s = fmaf(t, t, s);
          t = c.w - x.w; s = fmaf(t, t, s);
        } else {
          s = fmaf(c.x, x.x, s); s = fmaf(c.y, x.y, s);
          s = fmaf(c.z, x.z, s); s = fmaf(c.w, x.w, s);
        }
      }
    } else {
      for (int i = 0; i < d; ++i) {
        if (l2) {
          const float t = qv[i] - xu[i];
          s = fmaf(t, t, s);
        } else {
          s = fmaf(qv[i], xu[i], s);
        }
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
      int lo2 = 0, hi = nn;
      while (lo2 < hi) {
        const int mid = (lo2 + hi) >> 1;
        if (nw[mid] < key) lo2 = mid + 1; else hi = mid;
      }
      const int pos = i + lo2;
      if (pos < total) {
        tmp[pos] = key;
        tvis[pos] = vis[i];
      }
    }
    for (int j = lane; j < nn; j += 64) {
      const uint64_t key = nw[j];
      int lo2 = 0, hi = nb;
      while (lo2 < hi) {
        const int mid = (lo2 + hi) >> 1;
        if (beam[mid] < key) lo2 = mid + 1; else hi = mid;
      }
      const int pos = j + lo2;
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

hipError_t launch_search(const Index &I, int64_t n, const uint32_t *graph, const float *Q,
                         int64_t nq, int32_t k, int32_t L, uint32_t start, uint32_t *out_ids,
                         float *out_dist, uint32_t *out_cmps, uint32_t *visited_bits,
                         int64_t words_per_query, hipStream_t s) {
  if (nq == 0) return hipSuccess;
  if (L < 1 || L > kMaxL || I.p.R > kMaxR || I.d > kMaxQD || words_per_query * 32 < n)
    return hipErrorInvalidValue;
  const SearchLds lo = search_lds(L, I.p.R, I.d);
  const float *X = I.xf();
  const bool vec = I.d % 4 == 0 && (reinterpret_cast<uintptr_t>(X) & 15u) == 0;
  if (vec)
    hipLaunchKernelGGL(search_kernel<true>, dim3((unsigned)nq), dim3(64), (size_t)lo.bytes, s, X, n,
                       I.d, I.p.metric, graph, I.p.R, Q, k, L, start, out_ids, out_dist, out_cmps,
                       visited_bits, words_per_query, lo);
  else
    hipLaunchKernelGGL(search_kernel<false>, dim3((unsigned)nq), dim3(64), (size_t)lo.bytes, s, X,
                       n, I.d, I.p.metric, graph, I.p.R, Q, k, L, start, out_ids, out_dist,
                       out_cmps, visited_bits, words_per_query, lo);
  return hipGetLastError();
}

// Rows of k + 1 search results of the points q0 .. q0 + nq - 1 searched as
// queries: each row's own id is dropped (its first occurrence), or, when it
// is not among the k + 1, the last entry; k entries per point remain.
__global__ void drop_self_kernel(const uint32_t *__restrict__ ids, const float *__restrict__ dist,
                                 int64_t nq, int k1, int64_t q0, uint32_t *__restrict__ out_ids,
                                 float *__restrict__ out_dist) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nq) return;
  const uint32_t self = (uint32_t)(q0 + r);
  const int k = k1 - 1;
  const uint32_t *in = ids + r * k1;
  const float *din = dist + r * k1;
  uint32_t *o = out_ids + (q0 + r) * k;
  float *od = out_dist ? out_dist + (q0 + r) * k : nullptr;
  bool dropped = false;
  int j = 0;
  for (int i = 0; i < k1 && j < k; ++i) {
    const uint32_t id = in[i];
    if (!dropped && id == self) {
      dropped = true;
      continue;
    }
    o[j] = id;
    if (od) od[j] = din[i];
    ++j;
  }
}

hipError_t launch_drop_self(const uint32_t *ids, const float *dist, int64_t nq, int32_t k1,
                            int64_t q0, uint32_t *out_ids, float *out_dist, hipStream_t s) {
  if (nq == 0) return hipSuccess;
  hipLaunchKernelGGL(drop_self_kernel, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, s, ids,
                     dist, nq, k1, q0, out_ids, out_dist);
  return hipGetLastError();
}

}  // namespace pipnn
