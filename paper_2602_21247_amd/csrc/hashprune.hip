// HashPrune on gfx950 (Sec. 3, Alg. 3).
//
// Candidate records are first binned by destination point (a counting sort:
// per-point counts, an exclusive scan, then a scatter). Each binned record
// is already a reservoir slot: candidate id, the residualized hash h_p(c)
// (bit b set iff Sketch(c)_b >= Sketch(p)_b) and the bf16 distance.
//
// One wave then merges a point's reservoir with its bin. By the
// history-independence lemma the result is the l_max smallest keys among
// the per-bucket minimum keys of (reservoir U bin), where a key is
// (bf16 distance, id). The merge computes exactly that: the bucket minima
// in an LDS hash table (compare-and-swap to claim a bucket's slot, atomic
// min to keep its smallest key), a bitonic sort of the minima by key, and
// the first l_max. Large bins are taken
// in chunks; since dropped bucket minima can never re-enter (every kept key
// is smaller and sits in a different bucket), merging chunk by chunk gives
// the same reservoir as one merge. Atomics decide only record positions
// inside a bin, never reservoir contents, so the result is deterministic.
#include "common.hpp"
#include "internal.hpp"
#include "wave_sort.hpp"

namespace pipnn {

__device__ __forceinline__ uint32_t hash_of(const float *__restrict__ S, int m, uint32_t p,
                                            uint32_t c) {
  const float *sp = S + (int64_t)p * m;
  const float *sc = S + (int64_t)c * m;
  uint32_t h = 0;
  for (int b = 0; b < m; ++b) h |= (sc[b] >= sp[b] ? 1u : 0u) << b;
  return h;
}

// Both hashes of a pair from one read of each sketch: bit b of h_p(c) is
// Sketch(c)_b >= Sketch(p)_b and bit b of h_c(p) is Sketch(p)_b >= Sketch(c)_b.
__device__ __forceinline__ void hash_pair(const float *__restrict__ S, int m, uint32_t p,
                                          uint32_t c, uint32_t &hpc, uint32_t &hcp) {
  const float *sp = S + (int64_t)p * m;
  const float *sc = S + (int64_t)c * m;
  uint32_t a = 0, b = 0;
  for (int i = 0; i < m; ++i) {
    const float x = sp[i], y = sc[i];
    a |= (y >= x ? 1u : 0u) << i;
    b |= (x >= y ? 1u : 0u) << i;
  }
  hpc = a;
  hcp = b;
}

// picks: n_rows x k candidate ids (0xFFFFFFFF unused); row g belongs to
// point row_ids[g]. Each pick (i -> j) yields the records (i, j) and (j, i).
// One thread per pick, so the k picks of a row are k consecutive lanes; when
// k is a power of two that group is aligned inside a wave and the row's
// forward records are counted and placed with one atomic (AGG).
template <bool AGG, bool BIDIR = true>
__global__ void __launch_bounds__(256) bin_count_kernel(const uint32_t *row_ids,
                                                        const uint32_t *picks, int64_t n_rows,
                                                        int k, uint32_t *cnt, int64_t n,
                                                        int32_t *flag) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = t < n_rows * k;
  const uint32_t j = in ? picks[t] : kEmptyId;
  const uint32_t i = in ? row_ids[t / k] : kEmptyId;
  if (in && j != kEmptyId && (i >= n || j >= n)) atomicOr(flag, 1);
  const bool ok = in && j != kEmptyId && i < n && j < n && i != j;
  if (AGG) {
    const int lane = threadIdx.x & 63;
    const int g0 = lane & ~(k - 1);
    const uint64_t m = __ballot(ok);
    const uint64_t gm = (k == 64) ? m : ((m >> g0) & ((1ull << k) - 1));
    if (lane == g0 && gm) atomicAdd(&cnt[i], (uint32_t)__popcll(gm));
  } else if (ok) {
    atomicAdd(&cnt[i], 1u);
  }
  if (BIDIR && ok) atomicAdd(&cnt[j], 1u);
}

template <bool AGG, bool BIDIR = true>
__global__ void __launch_bounds__(256) bin_scatter_kernel(const uint32_t *row_ids,
                                                          const uint32_t *picks, const float *dist,
                                                          int64_t n_rows, int k, const float *S,
                                                          int m, const int64_t *off,
                                                          uint32_t *cursor, uint64_t *bins,
                                                          int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = t < n_rows * k;
  const uint32_t j = in ? picks[t] : kEmptyId;
  const uint32_t i = in ? row_ids[t / k] : kEmptyId;
  const bool ok = in && j != kEmptyId && i < n && j < n && i != j;
  uint32_t hij = 0, hji = 0, bf = 0;
  if (ok) {
    bf = bf16_rne(dist[t]);
    hash_pair(S, m, i, j, hij, hji);
  }
  int64_t pi = 0;
  if (AGG) {
    const int lane = threadIdx.x & 63;
    const int g0 = lane & ~(k - 1);
    const uint64_t msk = __ballot(ok);
    const uint64_t gm = (k == 64) ? msk : ((msk >> g0) & ((1ull << k) - 1));
    uint32_t base = 0;
    if (lane == g0 && gm) base = atomicAdd(&cursor[i], (uint32_t)__popcll(gm));
    base = __shfl(base, g0, 64);
    const uint64_t below = (lane == g0) ? 0ull : ((~0ull >> (64 - (lane - g0))));
    pi = off[i] + base + __popcll(gm & below);
  } else if (ok) {
    pi = off[i] + atomicAdd(&cursor[i], 1u);
  }
  if (!ok) return;
  bins[pi] = slot_pack(j, hij, bf);
  if (BIDIR) {
    const int64_t pj = off[j] + atomicAdd(&cursor[j], 1u);
    bins[pj] = slot_pack(i, hji, bf);
  }
}

// Leaf-local binning. Every record of a leaf pick joins two members of the
// same leaf, so one workgroup per leaf can group them in LDS: the forward
// records of row r are its valid picks, its reverse records the picks of the
// leaf's other rows that name r. The count pass adds each row's total to its
// point's count with one global atomic; the scatter pass reserves the row's
// run of its point's bin with one atomic and writes the run (reverse records
// first, then forward) at positions taken from LDS counters. Picks are local
// column indices (kEmptyId or any value >= the leaf size marks an unused
// pick). The records and their bins are those of the global scheme; only
// their order inside a bin differs, which the merge does not see.

// The scatter pass stages the leaf's member sketches in LDS when they fit
// beside the row counters (about 1,200 rows at m = 12), so each record's two
// hashes compare LDS copies instead of gathering two sketches from memory;
// larger leaves read the sketches from memory. The compares are the same.
constexpr int kLeafBinLds = kLeafBinMaxRows * 20;  // bytes: int64 base + 3 uint32 counters per row
// The scatter of leaves whose counters and sketches need more than
// kLeafBinLds runs in a second launch with one workgroup per CU and this
// much LDS (leaves of up to ~2,100 rows at m = 12), so that their hashes
// also compare LDS copies.
constexpr int kLeafBinLdsBig = 144 * 1024;
constexpr int kLeafBinThreads = 1024;  // 16 waves: the LDS admits two workgroups per CU

// LDSB: LDS bytes of the scatter. A leaf is scattered by the instance that
// stages its sketches with the least LDS: the small one unless only the big
// one fits them; leaves that fit neither read the sketches from memory in
// the small instance.
template <bool SCATTER, int LDSB = kLeafBinLds>
__global__ void __launch_bounds__(kLeafBinThreads) leaf_bin_kernel(
    const int64_t *__restrict__ leaf_off, int64_t off0, const uint32_t *__restrict__ members,
    const uint32_t *__restrict__ picks, const float *__restrict__ dist, int k,
    const float *__restrict__ S, int m, const int64_t *__restrict__ bin_off,
    uint32_t *__restrict__ cnt, uint64_t *__restrict__ bins) {
  // per row: sB (the row's first bin position), sF / sR (forward / reverse
  // records: count, then cursor), sRn (reverse total); then the sketches
  __shared__ __attribute__((aligned(16))) uint8_t sMem[SCATTER ? LDSB : kLeafBinMaxRows * 8];
  const int64_t r0 = leaf_off[blockIdx.x] - off0;
  const int mm = (int)(leaf_off[blockIdx.x + 1] - off0 - r0);
  const int64_t need = (int64_t)mm * (20 + 4 * m);
  if (SCATTER) {
    const bool big_only = need > kLeafBinLds && need <= kLeafBinLdsBig;
    if (big_only != (LDSB == kLeafBinLdsBig)) return;
  }
  const bool lds_sk = SCATTER && need <= LDSB;
  const int cap = lds_sk ? mm : kLeafBinMaxRows;
  int64_t *sB = reinterpret_cast<int64_t *>(sMem);
  uint32_t *sF = reinterpret_cast<uint32_t *>(sMem + (SCATTER ? (size_t)cap * 8 : 0));
  uint32_t *sR = sF + cap;
  uint32_t *sRn = sR + cap;
  float *sS = reinterpret_cast<float *>(sRn + cap);
  const int tid = threadIdx.x;
  for (int r = tid; r < mm; r += kLeafBinThreads) {
    sF[r] = 0u;
    sR[r] = 0u;
  }
  if (lds_sk) {
    for (int t = tid; t < mm * m; t += kLeafBinThreads) {
      const int r = t / m;
      sS[t] = S[(int64_t)members[r0 + r] * m + (t - r * m)];
    }
  }
  __syncthreads();
  const int tot = mm * k;
  for (int t = tid; t < tot; t += kLeafBinThreads) {
    const int r = t / k;
    const uint32_t c = picks[(r0 + r) * k + (t - r * k)];
    if (c < (uint32_t)mm && c != (uint32_t)r) {
      atomicAdd(&sF[r], 1u);
      atomicAdd(&sR[c], 1u);
    }
  }
  __syncthreads();
  if constexpr (!SCATTER) {
    for (int r = tid; r < mm; r += kLeafBinThreads) {
      const uint32_t n_r = sF[r] + sR[r];
      if (n_r) atomicAdd(&cnt[members[r0 + r]], n_r);
    }
  } else {
    for (int r = tid; r < mm; r += kLeafBinThreads) {
      const uint32_t n_r = sF[r] + sR[r];
      const uint32_t p = members[r0 + r];
      sRn[r] = sR[r];
      sB[r] = n_r ? bin_off[p] + atomicAdd(&cnt[p], n_r) : 0;
    }
    __syncthreads();
    for (int t = tid; t < tot; t += kLeafBinThreads) {
      const int r = t / k;
      const int64_t g = (r0 + r) * k + (t - r * k);
      const uint32_t c = picks[g];
      if (c < (uint32_t)mm && c != (uint32_t)r) {
        const uint32_t i = members[r0 + r], j = members[r0 + c];
        uint32_t hij, hji;
        if (lds_sk) {
          // bit b of h_i(j): Sketch(j)_b >= Sketch(i)_b; of h_j(i): the reverse
          const float *si = sS + r * m, *sj = sS + c * m;
          uint32_t a = 0, b = 0;
          for (int e = 0; e < m; ++e) {
            const float x = si[e], y = sj[e];
            a |= (y >= x ? 1u : 0u) << e;
            b |= (x >= y ? 1u : 0u) << e;
          }
          hij = a;
          hji = b;
        } else {
          hash_pair(S, m, i, j, hij, hji);
        }
        const uint32_t bf = bf16_rne(dist[g]);
        const uint32_t pf = atomicSub(&sF[r], 1u) - 1u;
        bins[sB[r] + sRn[r] + pf] = slot_pack(j, hij, bf);
        const uint32_t pr = atomicSub(&sR[c], 1u) - 1u;
        bins[sB[c] + pr] = slot_pack(i, hji, bf);
      }
    }
  }
}

hipError_t launch_leaf_bin(bool scatter, const int64_t *leaf_off, int64_t off0, int64_t n_leaves,
                           const uint32_t *members, const uint32_t *picks, const float *dist,
                           int32_t k, const float *sketch, int32_t m, const int64_t *bin_off,
                           uint32_t *cnt, uint64_t *bins, hipStream_t s) {
  if (n_leaves <= 0) return hipSuccess;
  if (scatter) {
    hipLaunchKernelGGL(leaf_bin_kernel<true>, dim3((unsigned)n_leaves), dim3(kLeafBinThreads), 0, s, leaf_off,
                       off0, members, picks, dist, k, sketch, m, bin_off, cnt, bins);
    hipLaunchKernelGGL((leaf_bin_kernel<true, kLeafBinLdsBig>), dim3((unsigned)n_leaves),
                       dim3(kLeafBinThreads), 0, s, leaf_off, off0, members, picks, dist, k, sketch,
                       m, bin_off, cnt, bins);
  } else
    hipLaunchKernelGGL(leaf_bin_kernel<false>, dim3((unsigned)n_leaves), dim3(kLeafBinThreads), 0, s, leaf_off,
                       off0, members, picks, dist, k, sketch, m, bin_off, cnt, bins);
  return hipGetLastError();
}

hipError_t launch_bin_count(const uint32_t *row_ids, const uint32_t *picks, int64_t n_rows,
                            int32_t k, uint32_t *cnt, int64_t n, int32_t *flag, hipStream_t s,
                            bool bidir) {
  const int64_t tot = n_rows * k;
  if (tot == 0) return hipSuccess;
  const bool agg = k <= 64 && (k & (k - 1)) == 0;
  const dim3 g((unsigned)((tot + 255) / 256)), b(256);
  if (agg && bidir)
    hipLaunchKernelGGL((bin_count_kernel<true, true>), g, b, 0, s, row_ids, picks, n_rows, k, cnt, n, flag);
  else if (agg)
    hipLaunchKernelGGL((bin_count_kernel<true, false>), g, b, 0, s, row_ids, picks, n_rows, k, cnt, n, flag);
  else if (bidir)
    hipLaunchKernelGGL((bin_count_kernel<false, true>), g, b, 0, s, row_ids, picks, n_rows, k, cnt, n, flag);
  else
    hipLaunchKernelGGL((bin_count_kernel<false, false>), g, b, 0, s, row_ids, picks, n_rows, k, cnt, n, flag);
  return hipGetLastError();
}

hipError_t launch_bin_scatter(const uint32_t *row_ids, const uint32_t *picks, const float *dist,
                              int64_t n_rows, int32_t k, const float *sketch, int32_t m,
                              const int64_t *off, uint32_t *cursor, uint64_t *bins, int64_t n,
                              hipStream_t s, bool bidir) {
  const int64_t tot = n_rows * k;
  if (tot == 0) return hipSuccess;
  const bool agg = k <= 64 && (k & (k - 1)) == 0;
  const dim3 g((unsigned)((tot + 255) / 256)), b(256);
  if (agg && bidir)
    hipLaunchKernelGGL((bin_scatter_kernel<true, true>), g, b, 0, s, row_ids, picks, dist, n_rows,
                       k, sketch, m, off, cursor, bins, n);
  else if (agg)
    hipLaunchKernelGGL((bin_scatter_kernel<true, false>), g, b, 0, s, row_ids, picks, dist, n_rows,
                       k, sketch, m, off, cursor, bins, n);
  else if (bidir)
    hipLaunchKernelGGL((bin_scatter_kernel<false, true>), g, b, 0, s, row_ids, picks, dist,
                       n_rows, k, sketch, m, off, cursor, bins, n);
  else
    hipLaunchKernelGGL((bin_scatter_kernel<false, false>), g, b, 0, s, row_ids, picks, dist,
                       n_rows, k, sketch, m, off, cursor, bins, n);
  return hipGetLastError();
}

// Explicit records (p = dst, c = cand, dist) for pipnn_hashprune_insert.
__global__ void rec_count_kernel(const uint32_t *dst, const uint32_t *cand, int64_t cnt_rec,
                                 uint32_t *cnt, int64_t n, int32_t *flag) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cnt_rec) return;
  const uint32_t p = dst[t], c = cand[t];
  if (p >= n || c >= n) {
    atomicOr(flag, 1);
    return;
  }
  if (p == c) return;
  atomicAdd(&cnt[p], 1u);
}

__global__ void rec_scatter_kernel(const uint32_t *dst, const uint32_t *cand, const float *dist,
                                   int64_t cnt_rec, const float *S, int m, const int64_t *off,
                                   uint32_t *cursor, uint64_t *bins, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cnt_rec) return;
  const uint32_t p = dst[t], c = cand[t];
  if (p >= n || c >= n || p == c) return;
  const int64_t pos = off[p] + atomicAdd(&cursor[p], 1u);
  bins[pos] = slot_pack(c, hash_of(S, m, p, c), bf16_rne(dist[t]));
}

hipError_t launch_rec_count(const uint32_t *dst, const uint32_t *cand, int64_t cnt_rec,
                            uint32_t *cnt, int64_t n, int32_t *flag, hipStream_t s) {
  if (cnt_rec == 0) return hipSuccess;
  hipLaunchKernelGGL(rec_count_kernel, dim3((unsigned)((cnt_rec + 255) / 256)), dim3(256), 0, s,
                     dst, cand, cnt_rec, cnt, n, flag);
  return hipGetLastError();
}

hipError_t launch_rec_scatter(const uint32_t *dst, const uint32_t *cand, const float *dist,
                              int64_t cnt_rec, const float *sketch, int32_t m, const int64_t *off,
                              uint32_t *cursor, uint64_t *bins, int64_t n, hipStream_t s) {
  if (cnt_rec == 0) return hipSuccess;
  hipLaunchKernelGGL(rec_scatter_kernel, dim3((unsigned)((cnt_rec + 255) / 256)), dim3(256), 0, s,
                     dst, cand, dist, cnt_rec, sketch, m, off, cursor, bins, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------
constexpr int kMergeWaves = 4;
constexpr uint64_t kNone = ~0ull;

// key1 = (hash, rank16(bf16), id): groups buckets, minimum first.
// key2 = (rank16(bf16), id, hash): the reservoir order.
__device__ __forceinline__ uint64_t key1_of_slot(uint64_t s) {
  return ((uint64_t)slot_hash(s) << 48) | ((uint64_t)bf16_rank(slot_bf(s)) << 32) | slot_id(s);
}
__device__ __forceinline__ uint64_t key2_of_key1(uint64_t k1) {
  const uint64_t hash = k1 >> 48, rank = (k1 >> 32) & 0xFFFFu, id = k1 & 0xFFFFFFFFu;
  return (rank << 48) | (id << 16) | hash;
}
__device__ __forceinline__ uint64_t key1_of_key2(uint64_t k2) {
  const uint64_t rank = k2 >> 48, id = (k2 >> 16) & 0xFFFFFFFFu, hash = k2 & 0xFFFFu;
  return (hash << 48) | (rank << 32) | id;
}
__device__ __forceinline__ uint64_t slot_of_key2(uint64_t k2) {
  const uint32_t rank = (uint32_t)(k2 >> 48), id = (uint32_t)((k2 >> 16) & 0xFFFFFFFFu),
                 hash = (uint32_t)(k2 & 0xFFFFu);
  return slot_pack(id, hash, rank_to_bf16(rank));
}

__device__ void wave_bitonic_sort(uint64_t *A, int P) {
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

__device__ __forceinline__ int pow2_at_least(int v) {
  int P = 2;
  while (P < v) P <<= 1;
  return P;
}

// ARR: LDS entries per wave for the reservoir plus one chunk of records
// (the table has 2 ARR); a point's records are taken ARR - l_max at a time.
// The smaller arrays (l_max <= 128) keep twice the waves resident.
template <int ARR>
__global__ void __launch_bounds__(64 * kMergeWaves) hashprune_merge_kernel(
    uint64_t *__restrict__ res, int64_t n, int l_max, const uint64_t *__restrict__ bins,
    const int64_t *__restrict__ off) {
  // sT: open-addressing table of bucket minima (key1, hashed by bucket);
  // sB: the reservoir in key2 order
  __shared__ uint64_t sT[kMergeWaves][2 * ARR];
  __shared__ uint64_t sB[kMergeWaves][ARR];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t p = (int64_t)blockIdx.x * kMergeWaves + wave;
  if (p >= n) return;
  const int64_t b0 = off[p], b1 = off[p + 1];
  if (b1 == b0) return;
  uint64_t *T = sT[wave];
  uint64_t *B = sB[wave];
  uint64_t *r = res + p * l_max;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

  // current reservoir -> B as key2, compacted
  int nres = 0;
  for (int base = 0; base < l_max; base += 64) {
    const int i = base + lane;
    const uint64_t s = i < l_max ? r[i] : empty_slot();
    const bool ok = slot_id(s) != kEmptyId;
    const uint64_t mask = __ballot(ok);
    if (ok) B[nres + __popcll(mask & below)] = key2_of_key1(key1_of_slot(s));
    nres += __popcll(mask);
  }
  wave_sync();

  const int chunk_cap = ARR - l_max;
  for (int64_t c0 = b0; c0 < b1; c0 += chunk_cap) {
    const int nc = (int)min((int64_t)chunk_cap, b1 - c0);
    const int tot = nres + nc;
    // a table of twice the entries' power of two, so probes stay short
    const int TS = 2 * pow2_at_least(tot);
    const int tbits = 31 - __clz(TS);
    for (int i = lane; i < TS; i += 64) T[i] = kNone;
    wave_sync();
    // each entry's bucket keeps its minimum key1: a slot is claimed for a
    // bucket by compare-and-swap from empty, and keys of the same bucket
    // meet there by atomic min (they share the hash in the top 16 bits, so
    // the minimum keeps it)
    for (int i = lane; i < tot; i += 64) {
      const uint64_t k1 = i < nres ? key1_of_key2(B[i]) : key1_of_slot(bins[c0 + (i - nres)]);
      const uint32_t h = (uint32_t)(k1 >> 48);
      uint32_t slot = (h * 2654435761u) >> (32 - tbits);
      for (;;) {
        const uint64_t prev = atomicCAS((unsigned long long *)&T[slot], (unsigned long long)kNone,
                                        (unsigned long long)k1);
        if (prev == kNone) break;
        if ((uint32_t)(prev >> 48) == h) {
          atomicMin((unsigned long long *)&T[slot], (unsigned long long)k1);
          break;
        }
        slot = (slot + 1) & (TS - 1);
      }
    }
    wave_sync();
    // the bucket minima, compacted into B as key2
    int nk = 0;
    for (int base = 0; base < TS; base += 64) {
      const int i = base + lane;
      const uint64_t k1 = i < TS ? T[i] : kNone;
      const bool keep = k1 != kNone;
      const uint64_t mask = __ballot(keep);
      if (keep) B[nk + __popcll(mask & below)] = key2_of_key1(k1);
      nk += __popcll(mask);
    }
    wave_sync();
    const int P2 = pow2_at_least(nk);
    for (int i = nk + lane; i < P2; i += 64) B[i] = kNone;
    wave_sync();
    wave_bitonic_sort(B, P2);
    nres = nk < l_max ? nk : l_max;
  }
  for (int i = lane; i < l_max; i += 64) r[i] = i < nres ? slot_of_key2(B[i]) : empty_slot();
}

// ---------------------------------------------------------------------
// Register merge (l_max <= 128): a wave holds the point's reservoir and up
// to 64 * E - l_max of its records as 64-bit keys, E per lane (element
// i = e * 64 + lane). A bitonic sort by key1 = (hash, rank, id) puts every
// bucket's minimum first in its run, so an element is a bucket minimum iff
// its hash differs from the previous element's; a second sort of the minima
// by key2 = (rank, id, hash) gives the reservoir order, whose first l_max
// entries are the new reservoir. Larger bins are taken in chunks (the kept
// minima stay in the first elements). No LDS is used.
__device__ __forceinline__ uint64_t shfl_up1_u64(uint64_t v) {
  const uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)v, 1, 64);
  const uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(v >> 32), 1, 64);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t readlane63_u64(uint64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
  return ((uint64_t)hi << 32) | lo;
}

// Merge of one point with E keys per lane, writing its reservoir r. s0/s1:
// the reservoir's slots lane and 64 + lane (as loaded); `used`: the elements
// the reservoir occupies (its valid prefix, or all l_max slots when the
// valid slots are not a prefix), so records start at element `used`.
template <int E>
__device__ void merge_point_reg(uint64_t *__restrict__ r, int l_max, uint64_t s0, uint64_t s1,
                                int used, const uint64_t *__restrict__ bins, int64_t b0,
                                int64_t b1, int lane) {
  constexpr int N = 64 * E;
  uint64_t v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint64_t sl = e == 0 ? s0 : e == 1 ? s1 : empty_slot();
    v[e] = slot_id(sl) != kEmptyId ? key1_of_slot(sl) : kNone;
  }
  int nres = 0;
  int64_t c0 = b0;
  for (;;) {
    const int nc = (int)min((int64_t)(N - used), b1 - c0);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i = e * 64 + lane;
      if (i >= used && i < used + nc) v[e] = key1_of_slot(bins[c0 + (i - used)]);
    }
    c0 += nc;
    reg_bitonic_sort<E>(v, lane);
    // bucket minima: the first element of every run of equal hash
    uint64_t last = kNone;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const uint64_t up = shfl_up1_u64(v[e]);
      const uint64_t prev = lane == 0 ? last : up;
      const bool first = (e == 0 && lane == 0) || (prev >> 48) != (v[e] >> 48);
      last = readlane63_u64(v[e]);
      v[e] = (v[e] != kNone && first) ? key2_of_key1(v[e]) : kNone;
    }
    int nk = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) nk += __popcll(__ballot(v[e] != kNone));
    reg_bitonic_sort<E>(v, lane);
    nres = nk < l_max ? nk : l_max;
    if (c0 >= b1) break;
    // keep the first nres minima (as key1) for the next chunk
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i = e * 64 + lane;
      v[e] = i < nres ? key1_of_key2(v[e]) : kNone;
    }
    used = nres;
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = e * 64 + lane;
    if (i < l_max) r[i] = i < nres ? slot_of_key2(v[e]) : empty_slot();
  }
  for (int i = N + lane; i < l_max; i += 64) r[i] = empty_slot();
}

__global__ void __launch_bounds__(64 * kMergeWaves) hashprune_merge_reg_kernel(
    uint64_t *__restrict__ res, int64_t n, int l_max, const uint64_t *__restrict__ bins,
    const int64_t *__restrict__ off) {
  const int lane = threadIdx.x & 63;
  const int64_t p = (int64_t)blockIdx.x * kMergeWaves + (threadIdx.x >> 6);
  if (p >= n) return;
  const int64_t b0 = off[p], b1 = off[p + 1];
  if (b1 == b0) return;
  uint64_t *r = res + p * l_max;
  // the reservoir (l_max <= 128: two slots per lane)
  const uint64_t s0 = lane < l_max ? r[lane] : empty_slot();
  const uint64_t s1 = 64 + lane < l_max ? r[64 + lane] : empty_slot();
  const uint64_t m0 = __ballot(slot_id(s0) != kEmptyId);
  const uint64_t m1 = __ballot(slot_id(s1) != kEmptyId);
  const int nres = __popcll(m0) + __popcll(m1);
  // reservoirs this library writes keep their valid slots first
  const bool prefix = m1 == 0 ? (m0 & (m0 + 1)) == 0 : (m0 == ~0ull && (m1 & (m1 + 1)) == 0);
  const int used = prefix ? nres : l_max;
  const int64_t tot = (int64_t)used + (b1 - b0);
  if (tot <= 64) merge_point_reg<1>(r, l_max, s0, s1, used, bins, b0, b1, lane);
  else if (tot <= 128) merge_point_reg<2>(r, l_max, s0, s1, used, bins, b0, b1, lane);
  else merge_point_reg<4>(r, l_max, s0, s1, used, bins, b0, b1, lane);
}

hipError_t launch_hashprune_merge(uint64_t *res, int64_t n, int32_t l_max, const uint64_t *bins,
                                  const int64_t *off, hipStream_t s) {
  if (l_max > 256) return hipErrorInvalidValue;
  const int64_t blocks = (n + kMergeWaves - 1) / kMergeWaves;
  if (l_max <= 128)
    hipLaunchKernelGGL(hashprune_merge_reg_kernel, dim3((unsigned)blocks), dim3(64 * kMergeWaves),
                       0, s, res, n, l_max, bins, off);
  else
    hipLaunchKernelGGL(hashprune_merge_kernel<512>, dim3((unsigned)blocks), dim3(64 * kMergeWaves),
                       0, s, res, n, l_max, bins, off);
  return hipGetLastError();
}

// Canonical layout: per point, valid slots by (bf16 distance, id), empties last.
__global__ void __launch_bounds__(64 * kMergeWaves) canonical_kernel(const uint64_t *in,
                                                                     uint64_t *out, int64_t n,
                                                                     int l_max) {
  __shared__ uint64_t sA[kMergeWaves][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t p = (int64_t)blockIdx.x * kMergeWaves + wave;
  if (p >= n) return;
  uint64_t *A = sA[wave];
  const int P = pow2_at_least(l_max);
  for (int i = lane; i < P; i += 64) {
    uint64_t k2 = kNone;
    if (i < l_max) {
      const uint64_t s = in[p * l_max + i];
      if (slot_id(s) != kEmptyId) k2 = key2_of_key1(key1_of_slot(s));
    }
    A[i] = k2;
  }
  wave_sync();
  wave_bitonic_sort(A, P);
  for (int i = lane; i < l_max; i += 64)
    out[p * l_max + i] = A[i] != kNone ? slot_of_key2(A[i]) : empty_slot();
}

hipError_t launch_reservoir_canonical(const uint64_t *in, uint64_t *out, int64_t n, int32_t l_max,
                                      hipStream_t s) {
  if (l_max > 256) return hipErrorInvalidValue;
  const int64_t blocks = (n + kMergeWaves - 1) / kMergeWaves;
  hipLaunchKernelGGL(canonical_kernel, dim3((unsigned)blocks), dim3(64 * kMergeWaves), 0, s, in, out,
                     n, l_max);
  return hipGetLastError();
}

}  // namespace pipnn
