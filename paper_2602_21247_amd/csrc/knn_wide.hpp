// Fused leaf distance GEMM + per-row k-nearest selection for wide
// reduced-precision operands (512 or 768 dimensions; bf16, fp16 or e4m3).
//
// Same contract as knn_item in knn_kernel.hpp (same arguments, work items of
// 128 rows, same selection order and outputs); what changes is the register
// layout, so that a row's operand fits in registers at this width. The
// 16x16x32 MFMAs spread a row over four lanes (lane group q = lane / 16
// holds the quarter [q*DP/4, (q+1)*DP/4) of the dimensions) instead of two,
// which halves the A fragment (96 VGPRs for 768 fp16 dimensions). A
// workgroup of 8 waves owns 128 rows, 16 per wave; column tiles of 32 points
// are staged in LDS and shared by the 8 waves, one workgroup per CU.
//
// Selection follows knn_item: survivors of each tile are appended at their
// ballot rank and drained into a descending list of 64-bit (distance rank,
// column) keys; here the list of a row is split over the row's four lanes
// (part p holds positions [p*KSEL/4, (p+1)*KSEL/4)), and each part needs
// only the first key of the next part for the branch-free insertion. The
// FP32 direct-difference recompute sums each quarter of the dimensions in
// index order on one of the four lanes and adds the quarters as
// (q0 + q1) + (q2 + q3), the same value whichever row a pair is found from.
#pragma once
#include "knn_kernel.hpp"

namespace pipnn {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// x.y of 16 bytes of each operand per lane for the 16x16x32 shapes: 8 bf16 /
// fp16 values (one MFMA) or 16 e4m3 values (two).
template <int PREC>
__device__ __forceinline__ f32x4 mfma16x16(uint4 a, uint4 b, f32x4 acc) {
  if constexpr (PREC == PIPNN_PREC_BF16) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                    __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
  } else if constexpr (PREC == PIPNN_PREC_FP16) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                   __builtin_bit_cast(f16x8, b), acc, 0, 0, 0);
  } else {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(pack64(a.x, a.y), pack64(b.x, b.y), acc, 0, 0,
                                                     0);
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(pack64(a.z, a.w), pack64(b.z, b.w), acc, 0, 0,
                                                      0);
  }
}

// The value of lane (lane & ~3) + ((lane & 3) + 1), i.e. the next lane of
// the same group of four (lane 3 of a group reads itself), by a DPP
// quad permutation.
__device__ __forceinline__ uint32_t quad_next_u32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xF9, 0xF, 0xF, false);  // [1,2,3,3]
}
__device__ __forceinline__ float quad_xor1(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ float quad_xor2(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x4E, 0xF, 0xF, false));
}
__device__ __forceinline__ int quad_sum(int x) {
  x += __builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false);  // [1,0,3,2]
  x += __builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, false);  // [2,3,0,1]
  return x;
}

template <int PREC, int DP, int KSEL, bool L2>
__device__ __forceinline__ void knn_wide_item(const KnnArgs &a, const int item) {
  constexpr bool F8 = PREC == PIPNN_PREC_FP8;
  constexpr int EB = OpBytes<PREC>::v;
  constexpr int NW = 8;           // waves per workgroup
  constexpr int RW = 16;          // rows per wave
  constexpr int BM = NW * RW;     // 128 rows per workgroup
  constexpr int BN = 32;          // columns per tile
  constexpr int Q4 = DP / 4;      // dimensions per lane group
  constexpr int NA = Q4 * EB / 16;         // 16-byte operand vectors per lane
  constexpr int LDW = DP * EB / 4 + 4;     // LDS stride of a staged column (32-bit words)
  constexpr int CPC = DP * EB / 16;        // 16-byte chunks per column
  constexpr int NTH = NW * 64;
  constexpr int CH_PER_TILE = BN * CPC;
  constexpr int NPRE = (CH_PER_TILE + NTH - 1) / NTH;
  constexpr int PR = NPRE < 4 ? NPRE : 4;
  constexpr int CAP = BN;         // a tile appends at most BN survivors per row
  constexpr int BUFD = CAP + 1;
  constexpr int BUFC = CAP + 2;
  constexpr int KQ = KSEL / 4;    // kept-list entries per lane of a row's group
  constexpr int KST = KSEL + 1;
  static_assert(KSEL % 4 == 0 && Q4 % 8 == 0, "wide kernel shape");

  __shared__ __attribute__((aligned(16))) uint32_t sBw[BN * LDW];
  __shared__ float sBufD[BM * BUFD];
  __shared__ uint16_t sBufC[BM * BUFC];
  __shared__ uint64_t sKeep[BM * KST];
  __shared__ float sTau[BM];
  __shared__ int sBufN[BM];
  __shared__ float sColN[BN];
  __shared__ float sNr[BM];
  __shared__ float sColS[F8 ? BN : 1];
  __shared__ float sRs[F8 ? BM : 1];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int q = lane >> 4, l16 = lane & 15;  // MFMA lane group and column
  if (item >= a.n_items || a.items[item].job < 0) return;
  const KnnItem it = a.items[item];
  const KnnJob J = a.jobs[it.job];
  const int rbase = it.rb * BM;
  const int wrow = rbase + wave * RW;  // first row of this wave
  const uint32_t *rows = a.row_base + J.row_off;
  const uint32_t *cols = a.col_base + J.col_off;
  const int d = a.d;
  constexpr bool l2 = L2;
  const bool excl = (J.flags & 1) != 0;
  const bool full_d = (d == DP);
  const int n_rows = J.n_rows, n_cols = J.n_cols;
  const uint8_t *xop = reinterpret_cast<const uint8_t *>(a.Xop);
  const int64_t op_ld = (int64_t)a.ldo * EB;

  for (int i = tid; i < BM * KST; i += NTH) sKeep[i] = kEmptyKey;
  for (int r = tid; r < BM; r += NTH) {
    const bool ok = rbase + r < n_rows;
    sTau[r] = ok ? INFINITY : -INFINITY;
    sBufN[r] = 0;
    sNr[r] = (ok && l2) ? a.norms[rows[rbase + r]] : 0.f;
    if constexpr (F8) sRs[r] = ok ? a.scale[rows[rbase + r]] : 0.f;
  }

  // A operand: lane holds row wrow + l16, dimensions [q*Q4, q*Q4 + Q4)
  uint4 aw[NA];
  {
    const int r = wrow + l16;
    if (r < n_rows) {
      const uint4 *src = reinterpret_cast<const uint4 *>(xop + (int64_t)rows[r] * op_ld + q * Q4 * EB);
#pragma unroll
      for (int s = 0; s < NA; ++s) aw[s] = src[s];
    } else {
#pragma unroll
      for (int s = 0; s < NA; ++s) aw[s] = make_uint4(0u, 0u, 0u, 0u);
    }
  }

  // accumulator entry j of group g: row wrow + 4q + j, column 16g + l16
  uint4 pre[PR];
  float pre_n = 0.f, pre_s = 0.f;

  // drain lanes: row dr = lane / 4 of the wave, part p = lane % 4
  const int dr = lane >> 2, part = lane & 3;
  const int drow = wave * RW + dr;  // LDS row index
  auto drain = [&]() {
    const int nb = (wrow + dr < n_rows) ? sBufN[drow] : 0;
    if (nb > 0) {
      uint64_t ks[KQ];
#pragma unroll
      for (int i = 0; i < KQ; ++i) ks[i] = sKeep[drow * KST + part * KQ + i];
      float nd = sBufD[drow * BUFD];
      uint32_t ncv = sBufC[drow * BUFC];
      for (int e = 0; e < nb; ++e) {
        const uint64_t x = sel_key(nd, ncv);
        if (e + 1 < nb) {
          nd = sBufD[drow * BUFD + e + 1];
          ncv = sBufC[drow * BUFC + e + 1];
        }
        const uint32_t nlo = quad_next_u32((uint32_t)ks[0]);
        const uint32_t nhi = quad_next_u32((uint32_t)(ks[0] >> 32));
        const uint64_t below = part < 3 ? (((uint64_t)nhi << 32) | nlo) : 0ull;
#pragma unroll
        for (int i = 0; i < KQ; ++i) {
          const uint64_t nxt = (i + 1 < KQ) ? ks[i + 1] : below;
          ks[i] = kmax(nxt, kmin(ks[i], x));
        }
      }
#pragma unroll
      for (int i = 0; i < KQ; ++i) sKeep[drow * KST + part * KQ + i] = ks[i];
      if (part == 0) {
        sBufN[drow] = 0;
        sTau[drow] = ks[0] == kEmptyKey ? INFINITY : key_dist(ks[0]);
      }
    }
  };

  for (int c0 = 0; c0 < n_cols; c0 += BN) {
#pragma unroll
    for (int r0 = 0; r0 < NPRE; r0 += PR) {
      if (r0 == 0 && tid < BN) {
        pre_n = (l2 && c0 + tid < n_cols) ? a.norms[cols[c0 + tid]] : 0.f;
        if constexpr (F8) pre_s = c0 + tid < n_cols ? a.scale[cols[c0 + tid]] : 0.f;
      }
#pragma unroll
      for (int i = 0; i < PR; ++i) {
        const int qq = tid + (r0 + i) * NTH;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (qq < CH_PER_TILE) {
          const int c = qq / CPC, kq = qq % CPC;
          if (c0 + c < n_cols)
            v = *reinterpret_cast<const uint4 *>(xop + (int64_t)cols[c0 + c] * op_ld + kq * 16);
        }
        pre[i] = v;
      }
      if (r0 == 0 && tid < BN) {
        sColN[tid] = pre_n;
        if constexpr (F8) sColS[tid] = pre_s;
      }
#pragma unroll
      for (int i = 0; i < PR; ++i) {
        const int qq = tid + (r0 + i) * NTH;
        if (qq < CH_PER_TILE) {
          const int c = qq / CPC, kq = qq % CPC;
          *reinterpret_cast<uint4 *>(&sBw[c * LDW + kq * 4]) = pre[i];
        }
      }
    }
    __syncthreads();

    f32x4 acc[2];
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      acc[g] = f32x4{0.f, 0.f, 0.f, 0.f};
      const uint32_t *bw = &sBw[(16 * g + l16) * LDW + q * (Q4 * EB / 4)];
#pragma unroll
      for (int g0 = 0; g0 < NA; g0 += 8) {
#pragma unroll
        for (int s2 = g0; s2 < g0 + 8 && s2 < NA; ++s2)
          acc[g] = mfma16x16<PREC>(aw[s2], *reinterpret_cast<const uint4 *>(bw + 4 * s2), acc[g]);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    float dv[2][4];
    uint32_t pass = 0;  // bit 4g + j
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      const int cc = c0 + 16 * g + l16;
      const bool vc = cc < n_cols;
      const float nc = sColN[16 * g + l16];
      const float cs = F8 ? sColS[16 * g + l16] : 1.f;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int rl = wave * RW + 4 * q + j;
        float x = acc[g][j];
        if constexpr (F8) x = x * sRs[rl] * cs;
        dv[g][j] = l2 ? sNr[rl] + fmaf(-2.f, x, nc) : -x;
        if (a.out_matrix && vc && wrow + 4 * q + j < n_rows)
          a.out_matrix[(J.out_off + wrow + 4 * q + j) * a.matrix_ld + cc] = dv[g][j];
        const bool ok = vc && dv[g][j] <= sTau[rl] && !(excl && wrow + 4 * q + j + J.self_off == cc);
        pass |= (ok ? 1u : 0u) << (4 * g + j);
      }
    }
    if (__ballot(pass != 0) != 0ull) {
      // append at the rank among the row's survivors of this tile (group 0's
      // columns first, then group 1's)
      const uint32_t below = (1u << l16) - 1u;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint64_t m0 = __ballot((pass >> j) & 1u);
        const uint64_t m1 = __ballot((pass >> (4 + j)) & 1u);
        if ((m0 | m1) == 0ull) continue;
        const uint32_t g0m = (uint32_t)(m0 >> (16 * q)) & 0xFFFFu;
        const uint32_t g1m = (uint32_t)(m1 >> (16 * q)) & 0xFFFFu;
        const int rl = wave * RW + 4 * q + j;
        const int c0n = __popc(g0m);
        if ((pass >> j) & 1u) {
          const int pos = __popc(g0m & below);
          sBufD[rl * BUFD + pos] = dv[0][j];
          sBufC[rl * BUFC + pos] = (uint16_t)(c0 + l16);
        }
        if ((pass >> (4 + j)) & 1u) {
          const int pos = c0n + __popc(g1m & below);
          sBufD[rl * BUFD + pos] = dv[1][j];
          sBufC[rl * BUFC + pos] = (uint16_t)(c0 + 16 + l16);
        }
        if (l16 == 0) sBufN[rl] = c0n + __popc(g1m);
      }
      wave_sync();
      drain();
      wave_sync();
    }
    __syncthreads();  // every wave is done with sBw
  }

  // ---- epilogue: this wave's 16 rows, four lanes per row ----
  int tn = 0;
  const bool rvalid = wrow + dr < n_rows;
  if (rvalid) {
    int empty = 0;
#pragma unroll
    for (int i = 0; i < KQ; ++i) {
      const uint64_t k = sKeep[drow * KST + part * KQ + i];
      const int qpos = KSEL - 1 - (part * KQ + i);
      empty += k == kEmptyKey ? 1 : 0;
      sBufD[drow * BUFD + qpos] = k == kEmptyKey ? INFINITY : key_dist(k);
      sBufC[drow * BUFC + qpos] = (uint16_t)k;
    }
    tn = KSEL - quad_sum(empty);
  }
  wave_sync();

  const int ksel_job = J.k_sel < KSEL ? J.k_sel : KSEL;
  const int cnt_r = rvalid ? (tn < ksel_job ? tn : ksel_job) : 0;
  if (a.recompute) {
    // FP32 direct difference: lane `part` sums quarter `part` of the
    // dimensions in index order; the quarters are added as (q0+q1)+(q2+q3)
    constexpr int QD = DP / 4;
    const int kb = part * QD;
    const float *xrow = a.X + (int64_t)rows[rvalid ? wrow + dr : 0] * d + kb;
    for (int i = 0; i < KSEL; ++i) {
      if (!__any(i < cnt_r)) break;
      const uint32_t cr = i < cnt_r ? sBufC[drow * BUFC + i] : 0u;
      const uint32_t c = cr < (uint32_t)n_cols ? cr : 0u;
      const float *xc = a.X + (int64_t)cols[c] * d + kb;
      float s = 0.f;
      if (full_d) {
#pragma unroll 4
        for (int kk = 0; kk < QD; kk += 4) {
          const float4 u = *reinterpret_cast<const float4 *>(xrow + kk);
          const float4 v = *reinterpret_cast<const float4 *>(xc + kk);
          if (l2) {
            float t = u.x - v.x; s = fmaf(t, t, s);
            t = u.y - v.y; s = fmaf(t, t, s);
            t = u.z - v.z; s = fmaf(t, t, s);
            t = u.w - v.w; s = fmaf(t, t, s);
          } else {
            s = fmaf(u.x, v.x, s); s = fmaf(u.y, v.y, s);
            s = fmaf(u.z, v.z, s); s = fmaf(u.w, v.w, s);
          }
        }
      } else {
        for (int kk = 0; kk < QD; ++kk) {
          const bool in = kb + kk < d;
          const float u = in ? xrow[kk] : 0.f, v = in ? xc[kk] : 0.f;
          if (l2) {
            const float t = u - v;
            s = fmaf(t, t, s);
          } else {
            s = fmaf(u, v, s);
          }
        }
      }
      // pair sums in a fixed order, then the two pairs
      const float o1 = quad_xor1(s);
      const float pr = (part & 1) ? o1 + s : s + o1;   // q_even + q_odd of the pair
      const float o2 = quad_xor2(pr);
      const float tot = (part & 2) ? o2 + pr : pr + o2;  // (q0+q1) + (q2+q3)
      if (part == 0 && i < cnt_r) sBufD[drow * BUFD + i] = l2 ? tot : -tot;
    }
  }
  wave_sync();

  if (part == 0 && rvalid) {
    const int rr = wrow + dr;
    int cnt = cnt_r;
    float *dd = &sBufD[drow * BUFD];
    uint16_t *cc = &sBufC[drow * BUFC];
    if (a.rescore_k > 0) {
      for (int i = 1; i < cnt; ++i) {
        const float di = dd[i];
        const uint16_t ci = cc[i];
        int j = i - 1;
        while (j >= 0 && (dd[j] > di || (dd[j] == di && cc[j] > ci))) {
          dd[j + 1] = dd[j];
          cc[j + 1] = cc[j];
          --j;
        }
        dd[j + 1] = di;
        cc[j + 1] = ci;
      }
      if (cnt > a.rescore_k) cnt = a.rescore_k;
    }
    const int64_t o = (J.out_off + rr) * (int64_t)a.k_out;
    for (int i = 0; i < a.k_out; ++i) {
      const uint32_t c = i < cnt ? cc[i] : 0xFFFFu;
      if (c < (uint32_t)n_cols) {
        a.out_col[o + i] = a.out_ids ? cols[c] : c;
        if (a.out_dist) a.out_dist[o + i] = dd[i];
      } else {
        a.out_col[o + i] = kEmptyId;
        if (a.out_dist) a.out_dist[o + i] = INFINITY;
      }
    }
  }
}

template <int PREC, int DP, int KSEL, bool L2>
__global__ void __launch_bounds__(512, 2) knn_wide_kernel(KnnArgs a) {
  knn_wide_item<PREC, DP, KSEL, L2>(a, (int)blockIdx.x);
}

template <int PREC, int DP, int KSEL, bool L2>
__global__ void __launch_bounds__(512, 2) knn_wide_kernel_persistent(KnnArgs a) {
  __shared__ int sNext;
  const int x = (int)(blockIdx.x % kNumXcd);
  for (;;) {
    if (threadIdx.x == 0) sNext = atomicAdd(&a.work_counter[x], 1);
    __syncthreads();
    const int i = sNext;
    __syncthreads();
    if (i >= a.items_per_xcd) break;
    knn_wide_item<PREC, DP, KSEL, L2>(a, i * kNumXcd + x);
    __syncthreads();
  }
}

// One launch of the wide kernel: one workgroup (8 waves) per CU.
template <int PREC, int DP, int KSEL>
static hipError_t launch_knn_wide(KnnArgs args, int n_items, int n_cu, hipStream_t s) {
  unsigned grid = (unsigned)n_items;
  if (args.work_counter) {
    const int resident = n_cu / kNumXcd * kNumXcd;
    args.items_per_xcd = n_items / kNumXcd;
    grid = (unsigned)(n_items < resident ? n_items : resident);
  }
  const bool l2 = args.metric == PIPNN_METRIC_L2;
  if (args.work_counter) {
    if (l2)
      hipLaunchKernelGGL((knn_wide_kernel_persistent<PREC, DP, KSEL, true>), dim3(grid), dim3(512),
                         0, s, args);
    else
      hipLaunchKernelGGL((knn_wide_kernel_persistent<PREC, DP, KSEL, false>), dim3(grid),
                         dim3(512), 0, s, args);
  } else if (l2) {
    hipLaunchKernelGGL((knn_wide_kernel<PREC, DP, KSEL, true>), dim3(grid), dim3(512), 0, s, args);
  } else {
    hipLaunchKernelGGL((knn_wide_kernel<PREC, DP, KSEL, false>), dim3(grid), dim3(512), 0, s,
                       args);
  }
  return hipGetLastError();
}

// Dispatch of a reduced-precision operand over the instantiated widths
// (the operand row stride a.ldo is one of them).
template <int PREC>
static hipError_t launch_knn_lowp(const KnnArgs &a, int ksel, int n_items, int nw, int n_cu,
                                  hipStream_t s) {
  const bool k32 = ksel > 16;
#define PIPNN_KNN_CASE(DPV)                                                           \
  case DPV:                                                                           \
    return k32 ? launch_knn_shape<PREC, DPV, 32>(a, n_items, nw, n_cu, s)             \
               : launch_knn_shape<PREC, DPV, 16>(a, n_items, nw, n_cu, s);
  switch (a.ldo) {
    PIPNN_KNN_CASE(64)
    PIPNN_KNN_CASE(96)
    PIPNN_KNN_CASE(128)
    PIPNN_KNN_CASE(256)
    case 512:
      return k32 ? launch_knn_wide<PREC, 512, 32>(a, n_items, n_cu, s)
                 : launch_knn_wide<PREC, 512, 16>(a, n_items, n_cu, s);
    case 768:
      return k32 ? launch_knn_wide<PREC, 768, 32>(a, n_items, n_cu, s)
                 : launch_knn_wide<PREC, 768, 16>(a, n_items, n_cu, s);
    default: return hipErrorInvalidValue;
  }
#undef PIPNN_KNN_CASE
}

}  // namespace pipnn
