// Fused leaf distance GEMM + per-row k-nearest selection, four lanes per
// row (16x16 MFMA shapes), for every operand precision.
//
// Same contract as knn_item in knn_kernel.hpp (same arguments, work items of
// 128 rows, same selection order, same outputs and the same FP32 distance
// values); what changes is the register layout. The 16x16 MFMAs spread a row
// over four lanes (lane group q = lane / 16 holds the quarter
// [q*DP/4, (q+1)*DP/4) of the dimensions) instead of two, which halves the A
// fragment, and a wave owns 16 rows instead of 32. A workgroup of 8 waves
// owns 128 rows; column tiles of 32 points are staged by global-to-LDS
// transfers into two buffers exactly as in knn_item, the transfer of the
// next tile overlapping the MFMAs and selection of the current one. With the
// smaller register footprint two workgroups (16 waves) fit on a CU for
// operand rows up to 512 bytes, so one wave's selection overlaps three
// others' MFMA work; wider operands (the 512- and 768-dimension fp16 / bf16
// vectors) run one workgroup per CU.
//
// Selection follows knn_item: survivors of each tile are appended at their
// ballot rank and drained into a descending list of 64-bit (distance rank,
// column) keys, here split over the row's four lanes (part p holds
// positions [p*KSEL/4, (p+1)*KSEL/4)) and kept in registers. A key x enters
// with one comparison per entry: with g_i = (a_i > x), which is true on a
// prefix of the descending list, the new entry i is a_(i+1) where g_(i+1)
// holds, x where g_i holds but g_(i+1) does not, and a_i otherwise; each
// part needs only the first key of the next part.
//
// The FP32 direct-difference recompute sums each half of the dimensions in
// index order and adds the lower half's sum to the upper's, as knn_item
// does, so the value of a pair depends neither on the layout nor on the
// row it is found from; here each half runs as a chain through two lanes.
#pragma once
#include "knn_kernel.hpp"

namespace pipnn {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// x.y of 16 bytes of each operand per lane for the 16x16 shapes: 4 float32
// values (four 16x16x4 MFMAs), 8 bf16 / fp16 values (one 16x16x32 MFMA) or
// 16 e4m3 values (two).
template <int PREC>
__device__ __forceinline__ f32x4 mfma16x16(uint4 a, uint4 b, f32x4 acc) {
  if constexpr (PREC == PIPNN_PREC_FP32) {
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.x), __uint_as_float(b.x), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.y), __uint_as_float(b.y), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.z), __uint_as_float(b.z), acc, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.w), __uint_as_float(b.w), acc, 0, 0, 0);
  } else if constexpr (PREC == PIPNN_PREC_BF16) {
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

// Lane-mask compares (one v_cmp writing a wave mask; the predicates are
// LLVM's CmpInst codes: ordered <=, signed <, ==).
constexpr int kFcmpOle = 5, kIcmpEq = 32, kIcmpSlt = 40;

// The value of lane (lane & ~3) + ((lane & 3) + 1), i.e. the next lane of
// the same group of four (lane 3 of a group reads itself), by a DPP
// quad permutation.
__device__ __forceinline__ uint32_t quad_next_u32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xF9, 0xF, 0xF, false);  // [1,2,3,3]
}
__device__ __forceinline__ int quad_sum(int x) {
  x += __builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false);  // [1,0,3,2]
  x += __builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, false);  // [2,3,0,1]
  return x;
}

// The four-lane layout exists for operand rows that split into four whole
// 16-byte vectors (every width but the 96-dimension e4m3 operand).
constexpr bool knn_quad_shape(int dp, int eb) { return (dp * eb) % 64 == 0; }

// Resident waves per SIMD (the second launch bound): two workgroups of 8
// waves per CU for operand rows up to 512 bytes, one above.
template <int PREC, int DP> struct QuadOcc {
  static constexpr int v = DP * OpBytes<PREC>::v <= 512 ? 4 : 2;
};

template <int PREC, int DP, int KSEL, bool L2>
__device__ __forceinline__ void knn_quad_item(const KnnArgs &a, const int item) {
  constexpr bool F8 = PREC == PIPNN_PREC_FP8;
  constexpr int EB = OpBytes<PREC>::v;
  constexpr int NW = 8;           // waves per workgroup
  constexpr int RW = 16;          // rows per wave
  constexpr int BM = NW * RW;     // 128 rows per workgroup
  constexpr int BN = 32;          // columns per staged tile
  constexpr int CB = DP * EB;     // bytes per operand row
  constexpr int CPC = CB / 16;    // 16-byte chunks per operand row
  constexpr int NQ = CPC / 4;     // 16-byte operand vectors per lane (one quarter)
  constexpr int TB = BN * CB;     // bytes per staged tile
  constexpr int NI = TB / 1024;   // 1 KiB wave transfers per tile
  constexpr int HALF = DP / 2;
  // Survivors accumulate in the row buffers over several tiles: the
  // workgroup drains all its rows at once, after the first tile that leaves
  // some row with more than CAP - BN buffered (a tile appends at most BN).
  // Fewer, larger drains cost fewer insertion rounds (a round waits for the
  // row with the most entries); the thresholds stay a little stale between
  // drains, which lets somewhat more survivors through.
  constexpr int CAP = BN + 16;
  constexpr int BUFD = CAP + 1;
  constexpr int BUFC = CAP + 2;
  constexpr int KQ = KSEL / 4;    // kept-list entries per lane of a row's group
  constexpr int NTH = NW * 64;
  static_assert(KSEL % 4 == 0 && knn_quad_shape(DP, EB) && TB % 1024 == 0, "quad kernel shape");

  __shared__ __attribute__((aligned(16))) uint8_t sT[2 * TB];
  __shared__ float sColN[2 * BN];
  __shared__ float sColS[F8 ? 2 * BN : 1];
  __shared__ float sBufD[BM * BUFD];
  __shared__ uint16_t sBufC[BM * BUFC];
  __shared__ __attribute__((aligned(16))) float sTau[BM];
  __shared__ int sBufN[BM];
  __shared__ __attribute__((aligned(16))) int sWmax[2][NW];  // per tile parity: each wave's largest buffer count
  __shared__ __attribute__((aligned(16))) float sNr[BM];
  __shared__ __attribute__((aligned(16))) float sRs[F8 ? BM : 4];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform over the wave
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

  for (int r = tid; r < BM; r += NTH) {
    const bool ok = rbase + r < n_rows;
    sTau[r] = ok ? INFINITY : -INFINITY;
    sBufN[r] = 0;
    sNr[r] = (ok && l2) ? a.norms[rows[rbase + r]] : 0.f;
    if constexpr (F8) sRs[r] = ok ? a.scale[rows[rbase + r]] : 0.f;
  }

  // A operand: lane holds row wrow + l16, quarter q of the padded operand
  uint4 aw[NQ];
  {
    const int r = wrow + l16;
    if (r < n_rows) {
      const uint4 *src = reinterpret_cast<const uint4 *>(xop + (int64_t)rows[r] * CB + q * (CB / 4));
#pragma unroll
      for (int s = 0; s < NQ; ++s) aw[s] = src[s];
    } else {
#pragma unroll
      for (int s = 0; s < NQ; ++s) aw[s] = make_uint4(0u, 0u, 0u, 0u);
    }
  }

  // tile staging, as in knn_item: lanes < BN hold the ids of the tile being
  // fetched; transfer g moves the tile's chunks [64g, 64g + 64)
  auto col_id = [&](int c0) -> uint32_t {
    const int c = c0 + (lane & (BN - 1));
    return cols[c < n_cols ? c : 0];
  };
  float pre_n = 0.f, pre_s = 0.f;
  auto fetch = [&](int buf, uint32_t cid, int c0) {
    uint8_t *dst = sT + buf * TB;
#pragma unroll
    for (int j = 0; j < (NI + NW - 1) / NW; ++j) {
      const int g = wave + j * NW;
      if (NI % NW == 0 || g < NI) {
        const int t = g * 64 + lane;
        const int c = t / CPC, p = t - c * CPC;
        const uint32_t id = (uint32_t)__shfl((int)cid, c, 64);
        const int qq = p ^ chunk_swz<CPC>(c);
        lds_dma16(xop + (int64_t)id * CB + qq * 16, dst + g * 1024);
      }
    }
    if (tid < BN) {
      pre_n = (l2 && c0 + tid < n_cols) ? a.norms[cid] : 0.f;
      if constexpr (F8) pre_s = c0 + tid < n_cols ? a.scale[cid] : 0.f;
    }
  };
  auto put_norms = [&](int buf) {
    if (tid < BN) {
      sColN[buf * BN + tid] = pre_n;
      if constexpr (F8) sColS[buf * BN + tid] = pre_s;
    }
  };

  // drain lanes: row dr = lane / 4 of the wave, part p = lane % 4
  const int dr = lane >> 2, part = lane & 3;
  const int drow = wave * RW + dr;  // LDS row index
  uint64_t ks[KQ];
#pragma unroll
  for (int i = 0; i < KQ; ++i) ks[i] = kEmptyKey;
  // The filter's threshold is the job's k_sel-th smallest kept key: a key
  // above it can no longer reach the output, even where the list keeps more
  // (k_sel < KSEL: the partition's top-f, a smaller k). In the descending
  // list that is position KSEL - k_sel, entry tidx of part tpart.
  const int tpos = KSEL - (J.k_sel < KSEL ? J.k_sel : KSEL);
  const int tpart = tpos / KQ, tidx = tpos - tpart * KQ;
  auto drain = [&]() {
    const int nb = (wrow + dr < n_rows) ? sBufN[drow] : 0;
    if (nb > 0) {
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
        const uint64_t below = ((uint64_t)nhi << 32) | nlo;
        bool gt[KQ + 1];
#pragma unroll
        for (int i = 0; i < KQ; ++i) gt[i] = ks[i] > x;
        gt[KQ] = part < 3 && below > x;
#pragma unroll
        for (int i = 0; i < KQ; ++i) {
          const uint64_t nxt = (i + 1 < KQ) ? ks[i + 1] : below;
          ks[i] = gt[i + 1] ? nxt : (gt[i] ? x : ks[i]);
        }
      }
      if (part == 0) sBufN[drow] = 0;
      if (part == tpart) {
        uint64_t kt = ks[0];
#pragma unroll
        for (int i = 1; i < KQ; ++i) kt = i == tidx ? ks[i] : kt;
        sTau[drow] = kt == kEmptyKey ? INFINITY : key_dist(kt);
      }
    }
  };

  const bool active = wrow < n_rows;
  int cntj[4] = {0, 0, 0, 0};  // buffered survivors of rows rb + j (uniform over the lane group)
  uint32_t cid = 0;
  if (n_cols > 0) {
    cid = col_id(0);
    fetch(0, cid, 0);
    cid = col_id(BN);
    put_norms(0);
  }
  __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
  __syncthreads();

  // The filter's per-row operands live in registers: accumulator entry j of
  // a lane belongs to row wave * RW + 4q + j, whose norm (and e4m3 scale)
  // never changes and whose threshold changes only when the rows are drained.
  const int rq = wave * RW + 4 * q;
  const f32x4 nr4 = *reinterpret_cast<const f32x4 *>(sNr + rq);
  const f32x4 rs4 = F8 ? *reinterpret_cast<const f32x4 *>(sRs + rq) : f32x4{1.f, 1.f, 1.f, 1.f};
  f32x4 tau4 = *reinterpret_cast<const f32x4 *>(sTau + rq);
  // the wave's own columns (leaf self-joins) fall in the tiles holding
  // columns [diag0, diag0 + RW)
  const int diag0 = excl ? J.self_off + wrow : -(1 << 30);

  // B-fragment addresses without per-read arithmetic: when the row and the
  // per-lane vector count are powers of two, column l16's chunk qn + s sits
  // at (buffer + l16 CB + ((qn ^ swz) << 4)) ^ (s << 4) (the terms occupy
  // disjoint bits), and both column groups share the swizzle (the second
  // group adds 16 CB, a constant offset).
  constexpr bool PRE = (CB & (CB - 1)) == 0 && (NQ & (NQ - 1)) == 0 && TB % CB == 0;
  const int bbase = l16 * CB + (((q * NQ) ^ chunk_swz<CPC>(l16)) << 4);

  for (int t = 0, c0 = 0; c0 < n_cols; ++t, c0 += BN) {
    const int buf = t & 1;
    const bool more = c0 + BN < n_cols;
    if (more) {
      fetch(buf ^ 1, cid, c0 + BN);
      cid = col_id(c0 + 2 * BN);
    }
    if (t > 0) {
      // drain every row of the workgroup if the last tile left some row's
      // buffer too full for another tile (the decision is the same on every
      // wave: all read the counts published before the barrier)
      int wm = 0;
#pragma unroll
      for (int w = 0; w < NW; ++w) wm = max(wm, sWmax[buf ^ 1][w]);
      if (wm > CAP - BN) {
        drain();
#pragma unroll
        for (int j = 0; j < 4; ++j) cntj[j] = 0;
        wave_sync();
        tau4 = *reinterpret_cast<const f32x4 *>(sTau + rq);
      }
    }
    if (active) {
      // per-tile bases, opaque to the compiler (see knn_item)
      int rb = wave * RW + 4 * q;   // LDS row of accumulator entry 0
      int qn = q * NQ;              // this lane's first chunk
      int sw0 = chunk_swz<CPC>(l16), sw1 = chunk_swz<CPC>(16 + l16);
      int tb = buf * TB + l16 * CB;  // column l16 of the tile (16 + l16: + 16 CB)
      asm volatile("" : "+v"(rb), "+v"(qn), "+v"(sw0), "+v"(sw1), "+v"(tb));
      // accumulator entry j of group g: row wrow + 4q + j, column c0 + 16g + l16
      f32x4 acc0 = f32x4{0.f, 0.f, 0.f, 0.f}, acc1 = f32x4{0.f, 0.f, 0.f, 0.f};
      if constexpr (PRE) {
        int tbase = buf * TB + bbase;
        asm volatile("" : "+v"(tbase));
#pragma unroll
        for (int s = 0; s < NQ; ++s) {
          const uint8_t *a = sT + (tbase ^ (s << 4));
          const uint4 b0 = *reinterpret_cast<const uint4 *>(a);
          const uint4 b1 = *reinterpret_cast<const uint4 *>(a + 16 * CB);
          acc0 = mfma16x16<PREC>(aw[s], b0, acc0);
          acc1 = mfma16x16<PREC>(aw[s], b1, acc1);
        }
      } else {
#pragma unroll
        for (int s = 0; s < NQ; ++s) {
          const uint4 b0 = *reinterpret_cast<const uint4 *>(sT + tb + (((qn + s) ^ sw0) << 4));
          const uint4 b1 = *reinterpret_cast<const uint4 *>(sT + tb + 16 * CB + (((qn + s) ^ sw1) << 4));
          acc0 = mfma16x16<PREC>(aw[s], b0, acc0);
          acc1 = mfma16x16<PREC>(aw[s], b1, acc1);
        }
      }
      // survivors as wave masks: bit l of mk[g][j] is lane l's entry j of
      // group g (no branch per entry; the masks are the append's ranks)
      float dv[2][4];
      uint64_t mk[2][4];
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        const f32x4 acc = g ? acc1 : acc0;
        const int cc = c0 + 16 * g + l16;
        const bool vc = cc < n_cols;
        const uint64_t vcm = __builtin_amdgcn_sicmpl((int64_t)cc, (int64_t)n_cols, kIcmpSlt);
        const float nc = sColN[buf * BN + 16 * g + l16];
        const float cs = F8 ? sColS[buf * BN + 16 * g + l16] : 1.f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          float x = acc[j];
          if constexpr (F8) x = x * rs4[j] * cs;
          dv[g][j] = l2 ? nr4[j] + fmaf(-2.f, x, nc) : -x;
          mk[g][j] = vcm & __builtin_amdgcn_fcmpf(dv[g][j], tau4[j], kFcmpOle);
        }
        if (a.out_matrix) {
          // test-only: the GEMM distance of every pair
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (vc && wrow + 4 * q + j < n_rows)
              a.out_matrix[(J.out_off + wrow + 4 * q + j) * a.matrix_ld + cc] = dv[g][j];
        }
      }
      if (c0 < diag0 + RW && c0 + BN > diag0) {
        // drop each row's own column: entry j of group g at column
        // c0 + 16g + l16 is row wrow + 4q + j's own when the two coincide
        const int self = c0 + l16 - diag0 - 4 * q;
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
          for (int j = 0; j < 4; ++j) mk[g][j] &= ~__builtin_amdgcn_sicmp(self + 16 * g, j, kIcmpEq);
      }
      uint64_t any = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) any |= mk[0][j] | mk[1][j];
      if (any != 0ull) {
        // append at the rank among the row's survivors of this tile (group
        // 0's columns first, then group 1's)
        const uint32_t below = (1u << l16) - 1u;
        float *bd = sBufD + rb * BUFD;
        uint16_t *bc = sBufC + rb * BUFC;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint64_t m0 = mk[0][j], m1 = mk[1][j];
          if ((m0 | m1) == 0ull) continue;
          const uint32_t g0m = (uint32_t)(m0 >> (16 * q)) & 0xFFFFu;
          const uint32_t g1m = (uint32_t)(m1 >> (16 * q)) & 0xFFFFu;
          const int c0n = cntj[j] + __popc(g0m);
          if ((g0m >> l16) & 1u) {
            const int pos = cntj[j] + __popc(g0m & below);
            bd[j * BUFD + pos] = dv[0][j];
            bc[j * BUFC + pos] = (uint16_t)(c0 + l16);
          }
          if ((g1m >> l16) & 1u) {
            const int pos = c0n + __popc(g1m & below);
            bd[j * BUFD + pos] = dv[1][j];
            bc[j * BUFC + pos] = (uint16_t)(c0 + 16 + l16);
          }
          cntj[j] = c0n + __popc(g1m);
          if (l16 == 0) sBufN[rb + j] = cntj[j];
        }
      }
    }
    {
      // publish this wave's largest buffer count for the drain decision
      int wm = max(max(cntj[0], cntj[1]), max(cntj[2], cntj[3]));
      wm = max(wm, __shfl_xor(wm, 16, 64));
      wm = max(wm, __shfl_xor(wm, 32, 64));
      if (lane == 0) sWmax[buf][wave] = wm;
    }
    if (more) put_norms(buf ^ 1);
    // the next tile has landed and every wave is done with this one
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    __syncthreads();
  }

  // what is still buffered
  wave_sync();
  drain();
  wave_sync();

  // ---- epilogue: this wave's 16 rows, four lanes per row ----
  int tn = 0;
  const bool rvalid = wrow + dr < n_rows;
  if (rvalid) {
    int empty = 0;
#pragma unroll
    for (int i = 0; i < KQ; ++i) {
      const uint64_t k = ks[i];
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
    // FP32 direct difference, in the MFMA lane mapping: lane (l16, q) holds
    // quarter q of row l16's float32 values. Each half of the dimensions is
    // summed in index order by a chain through its two quarters: at step s
    // the lanes of quarters 0 and 2 start winner s and hand their partial
    // sums to the lanes of quarters 1 and 3, which finish winner s - 1 from
    // the partials handed over at the previous step; the lane of quarter 1
    // then adds the upper half's sum (from quarter 3) to the lower half's.
    constexpr int Q4 = DP / 4;
    const int rl = wave * RW + l16;   // LDS row of the MFMA row
    const int rrow = wrow + l16;
    const int cnt_m = rrow < n_rows ? (J.k_sel < KSEL ? J.k_sel : KSEL) : 0;
    // the row's count of winners, from its drain group (lane 4 * l16)
    const int cnt_l = min(cnt_m, __shfl(cnt_r, 4 * l16, 64));
    const int kb = q * Q4;
    // the row's quarter: the FP32 A operand itself; for a reduced-precision
    // operand its float32 values in registers (up to 32 of them), else read
    // again at every step (cache resident)
    constexpr bool FP = PREC == PIPNN_PREC_FP32;
    constexpr bool XREG = !FP && Q4 <= 32;
    const float *xsrc = a.X + (int64_t)rows[rrow < n_rows ? rrow : 0] * d + kb;
    float xr[XREG ? Q4 : 1];
    if constexpr (XREG) {
#pragma unroll
      for (int kk = 0; kk < Q4; ++kk) xr[kk] = (rrow < n_rows && kb + kk < d) ? xsrc[kk] : 0.f;
    }
    auto rowv = [&](int kk) -> float {
      if constexpr (FP) {
        const uint4 w = aw[kk >> 2];
        return __uint_as_float((kk & 3) == 0 ? w.x : (kk & 3) == 1 ? w.y : (kk & 3) == 2 ? w.z : w.w);
      } else if constexpr (XREG) {
        return xr[kk];
      } else {
        return 0.f;  // not used: the wide path streams the row
      }
    };
    const bool first = (q & 1) == 0;  // quarters 0 and 2 start a half
    float hand = 0.f;                 // partial handed over at the previous step
    for (int st = 0; st <= KSEL; ++st) {
      if (!__any(st - 1 < cnt_l)) break;
      const int i = first ? st : st - 1;   // the winner this lane works on
      const bool live = i >= 0 && i < cnt_l;
      const uint32_t cr = live ? sBufC[rl * BUFC + i] : 0u;
      const uint32_t c = cr < (uint32_t)n_cols ? cr : 0u;
      const float *xc = a.X + (int64_t)cols[c] * d + kb;
      float sum = first ? 0.f : hand;
      if constexpr (!FP && !XREG) {
        // wide operand: row and column quarters streamed from memory
        const float *xs = xsrc;
        asm volatile("" : "+v"(xs));
#pragma unroll 4
        for (int kk = 0; kk < Q4; ++kk) {
          const bool in = rrow < n_rows && kb + kk < d;
          const float r = in ? xs[kk] : 0.f;
          const float v = kb + kk < d ? xc[kk] : 0.f;
          if (l2) {
            const float t = r - v;
            sum = fmaf(t, t, sum);
          } else {
            sum = fmaf(r, v, sum);
          }
        }
      } else if (full_d) {
#pragma unroll
        for (int kk = 0; kk < Q4; kk += 4) {
          const float4 v = *reinterpret_cast<const float4 *>(xc + kk);
          const float r0 = rowv(kk), r1 = rowv(kk + 1), r2 = rowv(kk + 2), r3 = rowv(kk + 3);
          if (l2) {
            float t = r0 - v.x; sum = fmaf(t, t, sum);
            t = r1 - v.y; sum = fmaf(t, t, sum);
            t = r2 - v.z; sum = fmaf(t, t, sum);
            t = r3 - v.w; sum = fmaf(t, t, sum);
          } else {
            sum = fmaf(r0, v.x, sum); sum = fmaf(r1, v.y, sum);
            sum = fmaf(r2, v.z, sum); sum = fmaf(r3, v.w, sum);
          }
        }
      } else {
#pragma unroll
        for (int kk = 0; kk < Q4; ++kk) {
          const float v = kb + kk < d ? xc[kk] : 0.f;
          const float r = rowv(kk);
          if (l2) {
            const float t = r - v;
            sum = fmaf(t, t, sum);
          } else {
            sum = fmaf(r, v, sum);
          }
        }
      }
      // quarters 0, 2 -> 1, 3: the partial of winner st
      hand = __shfl_xor(sum, 16, 64);
      // quarter 1 holds the lower half of winner st - 1, quarter 3 the upper
      const float upper = __shfl_xor(sum, 32, 64);
      if (q == 1 && live) {
        const float tot = sum + upper;
        sBufD[rl * BUFD + i] = l2 ? tot : -tot;
      }
    }
  }
  wave_sync();

  if (part == 0 && rvalid) {
    const int rr = wrow + dr;
    int cnt = cnt_r;
    float *dd = &sBufD[drow * BUFD];
    uint16_t *cc = &sBufC[drow * BUFC];
    if (a.rescore_k > 0) {
      // re-rank the GEMM winners by (direct distance, column)
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
__global__ void __launch_bounds__(512, (QuadOcc<PREC, DP>::v)) knn_quad_kernel(KnnArgs a) {
  knn_quad_item<PREC, DP, KSEL, L2>(a, (int)blockIdx.x);
}

template <int PREC, int DP, int KSEL, bool L2>
__global__ void __launch_bounds__(512, (QuadOcc<PREC, DP>::v)) knn_quad_kernel_persistent(KnnArgs a) {
  __shared__ int sNext;
  const int x = (int)(blockIdx.x % kNumXcd);
  for (;;) {
    if (threadIdx.x == 0) sNext = atomicAdd(&a.work_counter[x], 1);
    __syncthreads();
    const int i = sNext;
    __syncthreads();
    if (i >= a.items_per_xcd) break;
    knn_quad_item<PREC, DP, KSEL, L2>(a, i * kNumXcd + x);
    __syncthreads();
  }
}

// One launch of the four-lane kernel on work items of 128 rows.
template <int PREC, int DP, int KSEL>
static hipError_t launch_knn_quad(KnnArgs args, int n_items, int n_cu, hipStream_t s) {
  unsigned grid = (unsigned)n_items;
  if (args.work_counter) {
    constexpr int per_cu = QuadOcc<PREC, DP>::v * 4 / 8;  // workgroups resident per CU
    const int resident = (n_cu * per_cu) / kNumXcd * kNumXcd;
    args.items_per_xcd = n_items / kNumXcd;
    grid = (unsigned)(n_items < resident ? n_items : resident);
  }
  const bool l2 = args.metric == PIPNN_METRIC_L2;
  if (args.work_counter) {
    if (l2)
      hipLaunchKernelGGL((knn_quad_kernel_persistent<PREC, DP, KSEL, true>), dim3(grid), dim3(512),
                         0, s, args);
    else
      hipLaunchKernelGGL((knn_quad_kernel_persistent<PREC, DP, KSEL, false>), dim3(grid),
                         dim3(512), 0, s, args);
  } else if (l2) {
    hipLaunchKernelGGL((knn_quad_kernel<PREC, DP, KSEL, true>), dim3(grid), dim3(512), 0, s, args);
  } else {
    hipLaunchKernelGGL((knn_quad_kernel<PREC, DP, KSEL, false>), dim3(grid), dim3(512), 0, s,
                       args);
  }
  return hipGetLastError();
}

// Selection sizes built: 4 (the partition's nearest leaders), 16, 20 and 24
// (rows of up to 256 dimensions) and 32. A selection costs about its list
// length times its survivor count (k (1 + ln(s / k)) over a random column
// order), so a size between 16 and 32 pays only for what it keeps.
template <int PREC, int DP>
static hipError_t launch_knn_quad_k(const KnnArgs &a, int ksel, int n_items, int n_cu,
                                    hipStream_t s) {
  if constexpr (PREC == PIPNN_PREC_FP32 || DP <= 256) {
    if (ksel <= 4) return launch_knn_quad<PREC, DP, 4>(a, n_items, n_cu, s);
  }
  if (ksel <= 16) return launch_knn_quad<PREC, DP, 16>(a, n_items, n_cu, s);
  if constexpr (PREC == PIPNN_PREC_FP32 || DP <= 256) {
    if (ksel <= 20) return launch_knn_quad<PREC, DP, 20>(a, n_items, n_cu, s);
    if (ksel <= 24) return launch_knn_quad<PREC, DP, 24>(a, n_items, n_cu, s);
  }
  return launch_knn_quad<PREC, DP, 32>(a, n_items, n_cu, s);
}

// Dispatch of a reduced-precision operand over the instantiated widths (the
// operand row stride a.ldo is one of them): the two-lane layout for 128-
// and 64-row items where it is built and not overridden, else four lanes.
template <int PREC>
static hipError_t launch_knn_lowp(const KnnArgs &a, int ksel, int n_items, int nw, bool quad,
                                  int n_cu, hipStream_t s) {
  const bool k32 = ksel > 16;
  constexpr int EB = OpBytes<PREC>::v;
#define PIPNN_KNN_CASE(DPV)                                                              \
  case DPV:                                                                              \
    if constexpr (knn_quad_shape(DPV, EB)) {                                             \
      if (quad && nw == 4) return launch_knn_quad_k<PREC, DPV>(a, ksel, n_items, n_cu, s); \
    }                                                                                    \
    if (quad) return hipErrorInvalidValue;                                               \
    if (ksel <= 4) return launch_knn_shape<PREC, DPV, 4>(a, n_items, nw, n_cu, s);       \
    return k32 ? launch_knn_shape<PREC, DPV, 32>(a, n_items, nw, n_cu, s)                \
               : launch_knn_shape<PREC, DPV, 16>(a, n_items, nw, n_cu, s);
  switch (a.ldo) {
    PIPNN_KNN_CASE(64)
    PIPNN_KNN_CASE(96)
    PIPNN_KNN_CASE(128)
    PIPNN_KNN_CASE(256)
    case 512:
      if (nw != 4) return hipErrorInvalidValue;
      return launch_knn_quad_k<PREC, 512>(a, ksel, n_items, n_cu, s);
    case 768:
      if (nw != 4) return hipErrorInvalidValue;
      return launch_knn_quad_k<PREC, 768>(a, ksel, n_items, n_cu, s);
    default: return hipErrorInvalidValue;
  }
#undef PIPNN_KNN_CASE
}

}  // namespace pipnn
