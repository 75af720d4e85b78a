// Fused leaf distance GEMM + per-row k-nearest selection for gfx950.
//
// One kernel serves every dense "rows x columns -> k nearest columns per
// row" step of PiPNN:
//   - the leaf pick (Sec. 4.2): rows = columns = the members of a leaf, the
//     own column excluded, k nearest by (distance, column);
//   - the ball-carving assignment (Alg. 5): rows = the points of a
//     subproblem, columns = its leaders, f nearest leaders per point.
// The distance of a pair is the GEMM form ||x||^2 + ||y||^2 - 2 x.y
// (squared L2) or -x.y (negated inner product), with x.y on MFMA.
//
// Work decomposition: a work item is (job, block of 32*NW rows). A
// workgroup of NW waves owns one item; wave w owns 32 rows and keeps their
// A operand (the row vectors) in registers for the whole item. Column
// tiles of 32 points are staged in LDS by direct global-to-LDS transfers
// into two buffers: the transfer of tile t+1 is in flight while the MFMAs
// and the selection of tile t run, and one barrier per tile hands the
// buffers over. The columns of a tile sit back to back with their 16-byte
// chunks permuted per column (chunk_swz), so the fragment reads are free
// of bank conflicts. The host lists the work items in launch order (block b
// runs on XCD b % 8): whole small jobs go to one XCD so that their column
// vectors stay in that XCD's L2, and jobs are dealt to XCDs largest first
// by work so that the eight XCDs finish together. Two workgroups fit on a
// CU, so one's selection and epilogue overlap the other's MFMA work.
//
// Selection: each row keeps its KSEL best (distance, column) pairs in
// registers (split over its two lanes) and a threshold tau in LDS (the
// worst kept pair once KSEL are kept). After each 32x32 MFMA block, every
// lane tests its 16 accumulator entries against the tau of their rows and
// appends the survivors to the row's LDS buffer; the row's lane pair then
// drains the buffer into the kept set. The filter uses <= so that equal
// distances with a smaller column are not lost; the drain applies the exact
// (distance, column) order.
//
// Epilogue: the kept pairs are sorted by (GEMM distance, column); when
// asked, each winner's FP32 distance is recomputed by direct difference,
// sum_i (x_i - y_i)^2 (or -sum x_i y_i): each half of the dimensions is
// summed in index order and the halves are added, so a pair always gets the
// same value whichever row it is found from. With rescoring, the k_sel GEMM
// winners are re-ranked by (direct distance, column) and the first k kept.
//
// Operand precision: the FP32 form runs v_mfma_f32_32x32x2_f32 on the
// float32 vectors (zero padded to DP when d is not DP). The reduced-precision forms (bf16, fp16, OCP e4m3 with a
// per-point scale) read a copy of the vectors in that format, made once per
// index and zero padded to DP, and run the 32x32x16 MFMAs with FP32
// accumulation; their squared norms are those of the decoded operand, so the
// GEMM form approximates the distance between the decoded vectors. The
// direct-difference recompute always reads the float32 vectors.
//
// This header holds the kernel template; each operand precision is
// instantiated in a translation unit of its own (knn.hip: FP32 and the
// dispatch; knn_bf16.hip, knn_fp16.hip, knn_fp8.hip).
#pragma once
#include "common.hpp"
#include "internal.hpp"

namespace pipnn {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

struct KnnArgs {
  const float *X;        // float32 vectors (n x d): FP32 operand and direct-difference rescoring
  const float *norms;    // squared norms of the GEMM operand
  const uint32_t *row_base;
  const uint32_t *col_base;
  const KnnJob *jobs;
  const KnnItem *items;
  uint32_t *out_col;
  float *out_dist;
  float *out_matrix;
  int64_t matrix_ld;
  int32_t n_items;
  int32_t d;
  int32_t metric;
  int32_t k_out;
  int32_t out_ids;
  int32_t recompute;
  int32_t rescore_k;
  int32_t ldo;           // operand row stride (elements): the padded width DP
  const void *Xop;       // GEMM operand (n x ldo, zero padded, 16-byte aligned rows)
  const float *scale;    // fp8 operand: per-point decode scale, else NULL
  // persistent schedule: NULL, or 8 per-XCD counters (zero at launch); the
  // workgroups of XCD x then take items[i * 8 + x] for i = 0, 1, ... in
  // turn until i reaches items_per_xcd
  int32_t *work_counter;
  int32_t items_per_xcd;
};

// Row (0..31) of accumulator entry v held by a lane in the upper (h=1) or
// lower (h=0) half of the wave; the 32x32 MFMA forms share this layout.
__device__ __forceinline__ int acc_row(int v, int h) { return (v & 3) + 8 * (v >> 2) + 4 * h; }

template <int PREC> struct OpBytes { static constexpr int v = 4; };
template <> struct OpBytes<PIPNN_PREC_BF16> { static constexpr int v = 2; };
template <> struct OpBytes<PIPNN_PREC_FP16> { static constexpr int v = 2; };
template <> struct OpBytes<PIPNN_PREC_FP8> { static constexpr int v = 1; };

__device__ __forceinline__ long pack64(uint32_t lo, uint32_t hi) {
  return (long)(((uint64_t)hi << 32) | lo);
}

// x.y of 16 bytes of each operand per lane: 8 bf16 / 8 fp16 values (one
// 32x32x16 MFMA) or 16 e4m3 values (two). Lane half h and the vector's
// position fix which dimensions it holds; A and B use the same mapping, so
// the sum covers every dimension once.
template <int PREC>
__device__ __forceinline__ f32x16 mfma16(uint4 a, uint4 b, f32x16 acc) {
  if constexpr (PREC == PIPNN_PREC_BF16) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                    __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
  } else if constexpr (PREC == PIPNN_PREC_FP16) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                   __builtin_bit_cast(f16x8, b), acc, 0, 0, 0);
  } else {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(pack64(a.x, a.y), pack64(b.x, b.y), acc, 0, 0,
                                                     0);
    return __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(pack64(a.z, a.w), pack64(b.z, b.w), acc, 0, 0,
                                                      0);
  }
}

// Selection key of a (distance, column) pair: the order-preserving rank of
// the float32 distance above the column, so that unsigned 64-bit order is
// the (distance, column) order. All ones marks an empty slot.
__device__ __forceinline__ uint64_t sel_key(float d, uint32_t c) {
  return ((uint64_t)f32_rank(d) << 32) | c;
}
__device__ __forceinline__ float key_dist(uint64_t k) {
  const uint32_t r = (uint32_t)(k >> 32);
  return __uint_as_float((r & 0x80000000u) ? (r & 0x7FFFFFFFu) : ~r);
}
constexpr uint64_t kEmptyKey = ~0ull;

// The value lane l ^ 32 holds (the same lane of the other half-wave), by a
// VALU swap of the two halves (v_permlane32_swap) instead of an LDS route.
__device__ __forceinline__ uint32_t other_half_u32(uint32_t x) {
  const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
  return (__lane_id() < 32) ? r[1] : r[0];
}
__device__ __forceinline__ float other_half(float x) {
  return __uint_as_float(other_half_u32(__float_as_uint(x)));
}
__device__ __forceinline__ uint64_t kmin(uint64_t a, uint64_t b) { return a < b ? a : b; }
__device__ __forceinline__ uint64_t kmax(uint64_t a, uint64_t b) { return a < b ? b : a; }

// Resident waves per SIMD the kernel is built for (the second launch bound
// is waves per execution unit): operand rows wider than 768 bytes take one
// (their A fragments and double-buffered tiles are large), narrower ones two.
template <int PREC, int DP> struct KnnOcc {
  static constexpr int v = DP * OpBytes<PREC>::v > 768 ? 1 : 2;
};

// 16-byte chunk q of staged column c sits at LDS chunk position
// q ^ swz(c) of the column's row: consecutive columns then spread the same
// chunk over different banks, so the B-fragment reads (lane l32 reads
// column l32) are free of bank conflicts although the columns are staged
// back to back, as the 1 KiB global-to-LDS transfers require. The mask stays
// below the largest power of two dividing CPC, so the map is a permutation
// of each column's chunks.
template <int CPC> __device__ __forceinline__ int chunk_swz(int c) {
  if constexpr (CPC % 16 == 0) return c & 15;
  else if constexpr (CPC % 8 == 0) return (c >> 1) & 7;
  else if constexpr (CPC % 4 == 0) return (c >> 2) & 3;
  else if constexpr (CPC % 2 == 0) return (c >> 3) & 1;
  else return 0;
}

typedef __attribute__((address_space(3))) void lds_void_t;

// s_waitcnt with vmcnt(0) and the other counters unconstrained (gfx9
// encoding: vmcnt bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8). As a
// builtin the compiler's own wait tracking sees it.
constexpr int kWaitVmcnt0 = 0x0F70;

// 16 bytes per lane from global memory straight into LDS: lane i of the
// wave writes LDS bytes [lds + 16 i, lds + 16 i + 16). Written as asm so that
// the compiler does not order every later LDS read behind the transfer (it
// cannot tell the two tile buffers apart); the caller waits for the transfer
// with s_waitcnt vmcnt(0) before the barrier that publishes the tile. The
// instruction has no register result, and M0 is set right before it.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
__device__ __forceinline__ void lds_dma16(const void *src, const void *lds) {
  const uint32_t base = __builtin_amdgcn_readfirstlane(
      (uint32_t)(uintptr_t)reinterpret_cast<const __attribute__((address_space(3))) char *>(
          (const __attribute__((address_space(3))) char *)lds));
  asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off"
               :
               : "v"(src), "s"(base)
               : "memory", "m0");
}
#pragma clang diagnostic pop

template <int PREC, int DP, int KSEL, int NW, bool L2>
__device__ __forceinline__ void knn_item(const KnnArgs &a, const int item) {
  constexpr bool LP = PREC != PIPNN_PREC_FP32;  // reduced-precision operand
  constexpr bool F8 = PREC == PIPNN_PREC_FP8;
  constexpr int EB = OpBytes<PREC>::v;          // bytes per operand element
  constexpr int BM = 32 * NW;     // rows per workgroup
  constexpr int BN = 32;          // columns per staged tile
  constexpr int CB = DP * EB;     // bytes per operand row
  constexpr int CPC = CB / 16;    // 16-byte chunks per operand row
  constexpr int TB = BN * CB;     // bytes per staged tile
  constexpr int NI = TB / 1024;   // 1 KiB wave transfers per tile
  constexpr int HALF = DP / 2;    // k-range owned by each half of the wave
  constexpr int NA = CPC / 2;     // 16-byte operand vectors per lane
  constexpr int CAP = 32;         // per-row buffer: a 32-column block appends at most 32
  constexpr int BUFD = CAP + 1;
  constexpr int BUFC = CAP + 2;
  constexpr int KH = KSEL / 2;    // kept-list entries held by each lane of a row's pair
  constexpr int NTH = NW * 64;
  constexpr bool ROW_REG = !LP || HALF <= 64;   // recompute row half in registers
  static_assert(TB % 1024 == 0 && KSEL <= CAP, "tile shape");

  __shared__ __attribute__((aligned(16))) uint8_t sT[2 * TB];
  __shared__ float sColN[2 * BN];
  __shared__ float sColS[F8 ? 2 * BN : 1];
  __shared__ float sBufD[BM * BUFD];
  __shared__ uint16_t sBufC[BM * BUFC];
  __shared__ float sTau[BM];
  __shared__ int sBufN[BM];
  __shared__ float sNr[BM];
  __shared__ float sRs[F8 ? BM : 1];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 5, l32 = lane & 31;
  if (item >= a.n_items || a.items[item].job < 0) return;
  const KnnItem it = a.items[item];
  const KnnJob J = a.jobs[it.job];
  const int rbase = it.rb * BM;
  const int wrow = rbase + wave * 32;
  const uint32_t *rows = a.row_base + J.row_off;
  const uint32_t *cols = a.col_base + J.col_off;
  const int d = a.d;
  constexpr bool l2 = L2;
  const bool excl = (J.flags & 1) != 0;
  const bool full_d = (d == DP);
  const int n_rows = J.n_rows, n_cols = J.n_cols;
  const uint8_t *xop = reinterpret_cast<const uint8_t *>(a.Xop);

  // per-row squared norm and selection threshold (-inf past the last row)
  for (int r = tid; r < BM; r += NTH) {
    const bool ok = rbase + r < n_rows;
    sTau[r] = ok ? INFINITY : -INFINITY;
    sBufN[r] = 0;
    sNr[r] = (ok && l2) ? a.norms[rows[rbase + r]] : 0.f;
    if constexpr (F8) { sRs[r] = ok ? a.scale[rows[rbase + r]] : 0.f; }
  }
  uint32_t rowmask = 0;
#pragma unroll
  for (int v = 0; v < 16; ++v) rowmask |= (wrow + acc_row(v, h) < n_rows ? 1u : 0u) << v;

  // A operand: lane holds row l32 of this wave, dims [h*HALF, h*HALF+HALF)
  // of the zero-padded operand, as NA 16-byte vectors
  uint4 aw[NA];
  {
    const int r = wrow + l32;
    if (r < n_rows) {
      const uint4 *src = reinterpret_cast<const uint4 *>(xop + (int64_t)rows[r] * CB + h * (CB / 2));
#pragma unroll
      for (int s = 0; s < NA; ++s) aw[s] = src[s];
    } else {
#pragma unroll
      for (int s = 0; s < NA; ++s) aw[s] = make_uint4(0u, 0u, 0u, 0u);
    }
  }
  // FP32 operand: element kk of this lane's half
  auto afl = [&](int kk) -> float {
    const uint4 q = aw[kk >> 2];
    const uint32_t w = (kk & 3) == 0 ? q.x : (kk & 3) == 1 ? q.y : (kk & 3) == 2 ? q.z : q.w;
    return __uint_as_float(w);
  };

  // lanes l32 and l32 + 32 own row wrow + l32 together
  const int orow = wave * 32 + l32;  // LDS row index

  // Column tiles are staged by global-to-LDS transfers (no register
  // round trip), one tile ahead of the MFMA work: transfer g of a tile moves
  // its 16-byte chunks [64g, 64g+64); lane i of the wave lands at LDS
  // position 64g + i and fetches the chunk that the swizzle puts there.
  // Lanes < BN hold the column ids of the tile being fetched (cid); the
  // column norms (and fp8 scales) travel through a register.
  auto col_id = [&](int c0) -> uint32_t {
    const int c = c0 + l32;
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
        const int q = p ^ chunk_swz<CPC>(c);
        lds_dma16(xop + (int64_t)id * CB + q * 16, dst + g * 1024);
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

  // the row's kept list, sorted in descending key order and split between
  // its two lanes (lane h holds positions [h*KH, h*KH+KH))
  uint64_t ks[KH];
#pragma unroll
  for (int i = 0; i < KH; ++i) ks[i] = kEmptyKey;
  // The filter's threshold is the job's k_sel-th smallest kept key (a key
  // above it can no longer reach the output, even where the list keeps
  // more): position KSEL - k_sel of the descending list, entry tidx of
  // half thalf.
  const int tpos = KSEL - (J.k_sel < KSEL ? J.k_sel : KSEL);
  const int thalf = tpos / KH, tidx = tpos - thalf * KH;

  // Drain: a key x enters by b[i] = max(a[i+1], min(a[i], x)): the largest
  // entry drops out when x is smaller, and nothing changes otherwise. Every
  // entry is independent of the others, so the update has no select chain
  // and no rescan; the lane holding the upper half needs only the first
  // entry of the lower half.
  auto drain = [&]() {
    const int nb = (wrow + l32 < n_rows) ? sBufN[orow] : 0;
    if (nb > 0) {
      float nd = sBufD[orow * BUFD];
      uint32_t ncv = sBufC[orow * BUFC];
      for (int e = 0; e < nb; ++e) {
        const uint64_t x = sel_key(nd, ncv);
        if (e + 1 < nb) {
          nd = sBufD[orow * BUFD + e + 1];
          ncv = sBufC[orow * BUFC + e + 1];
        }
        const uint32_t lo = (uint32_t)ks[0], hi = (uint32_t)(ks[0] >> 32);
        const uint32_t olo = other_half_u32(lo), ohi = other_half_u32(hi);
        const uint64_t below = h == 0 ? (((uint64_t)ohi << 32) | olo) : 0ull;
#pragma unroll
        for (int i = 0; i < KH; ++i) {
          const uint64_t nxt = (i + 1 < KH) ? ks[i + 1] : below;
          ks[i] = kmax(nxt, kmin(ks[i], x));
        }
      }
      if (h == 0) sBufN[orow] = 0;
      if (h == thalf) {
        uint64_t kt = ks[0];
#pragma unroll
        for (int i = 1; i < KH; ++i) kt = i == tidx ? ks[i] : kt;
        sTau[orow] = kt == kEmptyKey ? INFINITY : key_dist(kt);
      }
    }
  };

  // waves whose 32 rows all lie past the job's last row only stage tiles
  const bool active = wrow < n_rows;
  uint32_t cid = 0;
  if (n_cols > 0) {
    cid = col_id(0);
    fetch(0, cid, 0);
    cid = col_id(BN);
    put_norms(0);
  }
  __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
  __syncthreads();

  for (int t = 0, c0 = 0; c0 < n_cols; ++t, c0 += BN) {
    const int buf = t & 1;
    const bool more = c0 + BN < n_cols;
    if (more) {
      fetch(buf ^ 1, cid, c0 + BN);
      cid = col_id(c0 + 2 * BN);
    }
    if (active) {
      // Per-tile bases of the LDS and output addressing. They are passed
      // through an empty asm so that the compiler forms each access as one
      // base plus a constant offset inside the tile, instead of holding
      // dozens of precomputed addresses live across the whole loop.
      int rb = wave * 32 + 4 * h;             // LDS row of accumulator entry 0
      int hn = h * NA;                        // this lane's first chunk
      int sw = chunk_swz<CPC>(l32);           // the column's chunk permutation
      int tb = buf * TB + l32 * CB;           // this lane's column in the tile
      asm volatile("" : "+v"(rb), "+v"(hn), "+v"(sw), "+v"(tb));
      // MFMA: this wave's 32 rows against columns c0 + [0, 32)
      f32x16 acc;
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[v] = 0.f;
#pragma unroll
      for (int s = 0; s < NA; ++s) {
        const uint4 b = *reinterpret_cast<const uint4 *>(sT + tb + (((hn + s) ^ sw) << 4));
        if constexpr (LP) {
          acc = mfma16<PREC>(aw[s], b, acc);
        } else {
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(aw[s].x), __uint_as_float(b.x), acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(aw[s].y), __uint_as_float(b.y), acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(aw[s].z), __uint_as_float(b.z), acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(aw[s].w), __uint_as_float(b.w), acc, 0, 0, 0);
        }
      }
      constexpr auto accr = [](int v) { return (v & 3) + 8 * (v >> 2); };  // acc_row(v, 0)
      const int cc = c0 + l32;
      const bool vc = cc < n_cols;
      const float nc = sColN[buf * BN + l32];
      float nr[16], tau[16];
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        nr[v] = sNr[rb + accr(v)];
        tau[v] = sTau[rb + accr(v)];
      }
      if constexpr (F8) {
        // decode scales: x.y = (codes_x . codes_y) * scale_x * scale_y
        const float cs = sColS[buf * BN + l32];
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[v] = acc[v] * sRs[rb + accr(v)] * cs;
      }
      float dv[16];
#pragma unroll
      for (int v = 0; v < 16; ++v) dv[v] = l2 ? nr[v] + fmaf(-2.f, acc[v], nc) : -acc[v];
      if (a.out_matrix && vc) {
        // test-only: the GEMM distance of every pair
        int64_t mrow = J.out_off + wrow + 4 * h;
        asm volatile("" : "+v"(mrow));
        float *mo = a.out_matrix + mrow * a.matrix_ld + cc;
#pragma unroll
        for (int v = 0; v < 16; ++v)
          if ((rowmask >> v) & 1u) mo[accr(v) * a.matrix_ld] = dv[v];
      }
      // branch-free pass test; a block without any survivor costs one ballot
      uint32_t pass = 0;
      const int self = excl ? cc - J.self_off - (wrow + 4 * h) : -1;  // accr(v) of the own column
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const bool ok = vc && dv[v] <= tau[v] && self != accr(v);
        pass |= (ok ? 1u : 0u) << v;
      }
      if (__ballot(pass != 0) != 0ull) {
        // append: a row's survivors go to its buffer (empty after every
        // drain) at their rank among the row's survivors, from one ballot
        float *bd = sBufD + rb * BUFD;
        uint16_t *bc = sBufC + rb * BUFC;
        int *bn = sBufN + rb;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const uint64_t m = __ballot((pass >> v) & 1u);
          if (m == 0ull) continue;
          if ((pass >> v) & 1u) {
            const uint32_t hm = h ? (uint32_t)(m >> 32) : (uint32_t)m;
            const int pos = __popc(hm & ((1u << l32) - 1u));
            bd[accr(v) * BUFD + pos] = dv[v];
            bc[accr(v) * BUFC + pos] = (uint16_t)cc;
            if (pos == __popc(hm) - 1) bn[accr(v)] = pos + 1;
          }
        }
        wave_sync();
        drain();
        wave_sync();
      }
    }
    if (more) put_norms(buf ^ 1);
    // the next tile has landed and every wave is done with this one
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    __syncthreads();
  }

  // ---- epilogue: this wave's 32 rows ----
  // unpack each kept list into ascending (GEMM distance, column) order in
  // the row's buffer; empty slots sort last
  int tn = 0;
  if (wrow + l32 < n_rows) {
    int empty = 0;
#pragma unroll
    for (int i = 0; i < KH; ++i) {
      const uint64_t k = ks[i];
      const int q = KSEL - 1 - (h * KH + i);
      empty += k == kEmptyKey ? 1 : 0;
      sBufD[orow * BUFD + q] = k == kEmptyKey ? INFINITY : key_dist(k);
      sBufC[orow * BUFC + q] = (uint16_t)k;
    }
    tn = KSEL - empty - (int)other_half_u32((uint32_t)empty);
  }
  wave_sync();

  const int ksel_job = J.k_sel < KSEL ? J.k_sel : KSEL;
  if (a.recompute) {
    // FP32 direct-difference distance of each winner of row l32, into
    // sBufD[row][i]. Lane (l32, h) holds its row's dims [h*HALF, h*HALF+HALF)
    // in registers; it sums (x_r - x_c)^2 over that half in index order, and the
    // two halves are added, so a pair gets the same value from either row.
    const int rr = wrow + l32;
    const int cnt = rr < n_rows ? (tn < ksel_job ? tn : ksel_job) : 0;
    const int lrow = wave * 32 + l32;
    const int kbase = h * HALF;
    // the row's FP32 half: the A operand already holds it on the FP32 path
    float xr[(LP && ROW_REG) ? HALF : 1];
    // wide operands: the row half is re-read from memory (cache resident)
    const float *xrow = a.X + (int64_t)rows[rr < n_rows ? rr : 0] * d + kbase;
    if constexpr (LP && ROW_REG) {
      if (rr < n_rows) {
        const float *src = a.X + (int64_t)rows[rr] * d + kbase;
        if (full_d) {
#pragma unroll
          for (int kk = 0; kk < HALF; kk += 4) {
            const float4 q = *reinterpret_cast<const float4 *>(src + kk);
            xr[kk] = q.x; xr[kk + 1] = q.y; xr[kk + 2] = q.z; xr[kk + 3] = q.w;
          }
        } else {
#pragma unroll
          for (int kk = 0; kk < HALF; ++kk) xr[kk] = (kbase + kk < d) ? src[kk] : 0.f;
        }
      } else {
#pragma unroll
        for (int kk = 0; kk < HALF; ++kk) xr[kk] = 0.f;
      }
    }
    auto rv = [&](int kk) -> float {
      if constexpr (LP && ROW_REG) return xr[kk];
      else if constexpr (LP) return 0.f;
      else return afl(kk);
    };
    // sum over this lane's half of the dimensions for column c
    auto half_dist = [&](uint32_t c) -> float {
      const float *xc = a.X + (int64_t)cols[c] * d + kbase;
      float s = 0.f;
      if (full_d) {
#pragma unroll
        for (int kk = 0; kk < HALF; kk += 4) {
          const float4 q = *reinterpret_cast<const float4 *>(xc + kk);
          float r0, r1, r2, r3;
          if constexpr (ROW_REG) {
            r0 = rv(kk); r1 = rv(kk + 1); r2 = rv(kk + 2); r3 = rv(kk + 3);
          } else {
            const float4 rq = *reinterpret_cast<const float4 *>(xrow + kk);
            r0 = rq.x; r1 = rq.y; r2 = rq.z; r3 = rq.w;
          }
          if (l2) {
            float t = r0 - q.x; s = fmaf(t, t, s);
            t = r1 - q.y; s = fmaf(t, t, s);
            t = r2 - q.z; s = fmaf(t, t, s);
            t = r3 - q.w; s = fmaf(t, t, s);
          } else {
            s = fmaf(r0, q.x, s); s = fmaf(r1, q.y, s);
            s = fmaf(r2, q.z, s); s = fmaf(r3, q.w, s);
          }
        }
      } else {
#pragma unroll
        for (int kk = 0; kk < HALF; ++kk) {
          const bool in = kbase + kk < d;
          const float v = in ? xc[kk] : 0.f;
          float r;
          if constexpr (ROW_REG) r = rv(kk);
          else r = in ? xrow[kk] : 0.f;
          if (l2) {
            const float t = r - v;
            s = fmaf(t, t, s);
          } else {
            s = fmaf(r, v, s);
          }
        }
      }
      return s;
    };
    // two winners per pass, so that both columns' loads are in flight
    // together; a slot past the row's count reads column 0 and is dropped
    for (int i = 0; i < KSEL; i += 2) {
      if (!__any(i < cnt)) break;
      const uint32_t c0 = i < cnt ? sBufC[lrow * BUFC + i] : 0u;
      const uint32_t c1 = i + 1 < cnt ? sBufC[lrow * BUFC + i + 1] : 0u;
      const float s0 = half_dist(c0 < (uint32_t)n_cols ? c0 : 0u);
      const float s1 = half_dist(c1 < (uint32_t)n_cols ? c1 : 0u);
      const float o0 = other_half(s0), o1 = other_half(s1);
      // the lower half's sum first, then the upper half's
      const float t0 = h == 0 ? s0 + o0 : o0 + s0;
      const float t1 = h == 0 ? s1 + o1 : o1 + s1;
      if (h == 0) {
        if (i < cnt) sBufD[lrow * BUFD + i] = l2 ? t0 : -t0;
        if (i + 1 < cnt) sBufD[lrow * BUFD + i + 1] = l2 ? t1 : -t1;
      }
    }
  }
  wave_sync();

  if (l32 == lane && wrow + l32 < n_rows) {
    const int rr = wrow + l32;
    int cnt = tn < ksel_job ? tn : ksel_job;
    float *dd = &sBufD[orow * BUFD];
    uint16_t *cc = &sBufC[orow * BUFC];
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

// Static schedule: workgroup b takes item b.
template <int PREC, int DP, int KSEL, int NW, bool L2>
__global__ void __launch_bounds__(NW * 64, (KnnOcc<PREC, DP>::v)) knn_kernel(KnnArgs a) {
  knn_item<PREC, DP, KSEL, NW, L2>(a, (int)blockIdx.x);
}

// Persistent schedule: block b runs on XCD b % 8 and serves that XCD's item
// list from its counter until the list is exhausted.
template <int PREC, int DP, int KSEL, int NW, bool L2>
__global__ void __launch_bounds__(NW * 64, (KnnOcc<PREC, DP>::v)) knn_kernel_persistent(KnnArgs a) {
  __shared__ int sNext;
  const int x = (int)(blockIdx.x % kNumXcd);
  for (;;) {
    if (threadIdx.x == 0) sNext = atomicAdd(&a.work_counter[x], 1);
    __syncthreads();
    const int i = sNext;
    __syncthreads();
    if (i >= a.items_per_xcd) break;
    knn_item<PREC, DP, KSEL, NW, L2>(a, i * kNumXcd + x);
    __syncthreads();
  }
}

// One launch of a kernel shape. Static schedule: one workgroup per item.
// Persistent schedule: as many workgroups as stay resident (n_cu CUs times
// the workgroups per CU the shape is built for, a multiple of 8), each
// serving its XCD's item list.
template <int PREC, int DP, int KSEL, int NW>
static hipError_t launch_knn_nw(KnnArgs args, int n_items, int n_cu, hipStream_t s) {
  unsigned grid = (unsigned)n_items;
  if (args.work_counter) {
    constexpr int per_cu = KnnOcc<PREC, DP>::v * 4 / NW;  // workgroups resident per CU
    const int resident = (n_cu * per_cu) / kNumXcd * kNumXcd;
    args.items_per_xcd = n_items / kNumXcd;
    grid = (unsigned)(n_items < resident ? n_items : resident);
  }
  const bool l2 = args.metric == PIPNN_METRIC_L2;
  if (args.work_counter) {
    if (l2)
      hipLaunchKernelGGL((knn_kernel_persistent<PREC, DP, KSEL, NW, true>), dim3(grid),
                         dim3(NW * 64), 0, s, args);
    else
      hipLaunchKernelGGL((knn_kernel_persistent<PREC, DP, KSEL, NW, false>), dim3(grid),
                         dim3(NW * 64), 0, s, args);
  } else if (l2) {
    hipLaunchKernelGGL((knn_kernel<PREC, DP, KSEL, NW, true>), dim3(grid), dim3(NW * 64), 0, s,
                       args);
  } else {
    hipLaunchKernelGGL((knn_kernel<PREC, DP, KSEL, NW, false>), dim3(grid), dim3(NW * 64), 0, s,
                       args);
  }
  return hipGetLastError();
}

// Work items of 64 rows (two waves) are built for operands of 65..128
// dimensions; every shape has items of 128 rows (four waves).
constexpr bool knn_has_nw2(int dp) { return dp == 96 || dp == 128; }

template <int PREC, int DP, int KSEL>
static hipError_t launch_knn_shape(const KnnArgs &args, int n_items, int nw, int n_cu,
                                   hipStream_t s) {
  if constexpr (knn_has_nw2(DP)) {
    if (nw == 2) return launch_knn_nw<PREC, DP, KSEL, 2>(args, n_items, n_cu, s);
  }
  return launch_knn_nw<PREC, DP, KSEL, 4>(args, n_items, n_cu, s);
}

// Launches of the reduced-precision operands (nw: rows per item / 32; quad:
// the four-lane layout of knn_quad.hpp, on 128-row items) and of the
// float32 operand in the four-lane layout.
hipError_t launch_knn_bf16(const KnnArgs &a, int ksel, int n_items, int nw, bool quad, int n_cu,
                           hipStream_t s);
hipError_t launch_knn_fp16(const KnnArgs &a, int ksel, int n_items, int nw, bool quad, int n_cu,
                           hipStream_t s);
hipError_t launch_knn_fp8(const KnnArgs &a, int ksel, int n_items, int nw, bool quad, int n_cu,
                          hipStream_t s);
hipError_t launch_knn_fp32_quad(const KnnArgs &a, int ksel, int n_items, int n_cu, hipStream_t s);

}  // namespace pipnn
