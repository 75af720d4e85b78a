// Wave-level bitonic sort of 64-bit keys held in registers (E per lane,
// element e * 64 + lane), with cross-lane exchanges by VALU lane moves.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pipnn {

// x of lane ^ J, by VALU lane moves: DPP quad permutations (J = 1, 2), a
// half-row mirror then a quad reversal (J = 4: 7 - (i ^ 3) = i ^ 4 within 8
// lanes), a row rotation by 8 (J = 8), and the gfx950 row / half-wave swaps
// (J = 16, 32).
template <int J>
__device__ __forceinline__ uint32_t xor_lane_u32(uint32_t x) {
  if constexpr (J == 1) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, false);  // [1,0,3,2]
  } else if constexpr (J == 2) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4E, 0xF, 0xF, false);  // [2,3,0,1]
  } else if constexpr (J == 4) {
    const int m = __builtin_amdgcn_mov_dpp((int)x, 0x141, 0xF, 0xF, false);   // row_half_mirror
    return (uint32_t)__builtin_amdgcn_mov_dpp(m, 0x1B, 0xF, 0xF, false);      // [3,2,1,0]
  } else if constexpr (J == 8) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x128, 0xF, 0xF, false);  // row_ror:8
  } else if constexpr (J == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    return (__lane_id() & 16) ? r[0] : r[1];
  } else {
    static_assert(J == 32, "lane xor of 1..32");
    const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    return (__lane_id() & 32) ? r[0] : r[1];
  }
}
template <int J>
__device__ __forceinline__ uint64_t xor_lane_u64(uint64_t v) {
  const uint32_t lo = xor_lane_u32<J>((uint32_t)v);
  const uint32_t hi = xor_lane_u32<J>((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int j) {
  switch (j) {
    case 1: return xor_lane_u64<1>(v);
    case 2: return xor_lane_u64<2>(v);
    case 4: return xor_lane_u64<4>(v);
    case 8: return xor_lane_u64<8>(v);
    case 16: return xor_lane_u64<16>(v);
    default: return xor_lane_u64<32>(v);
  }
}
// Ascending bitonic sort of the 64 * E keys of the wave.
template <int E>
__device__ __forceinline__ void reg_bitonic_sort(uint64_t (&v)[E], int lane) {
  constexpr int N = 64 * E;
#pragma unroll
  for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j >= 64) {
        const int je = j >> 6;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          if ((e & je) == 0) {
            const bool asc = ((e * 64 + lane) & k) == 0;
            const uint64_t x = v[e], y = v[e | je];
            const bool sw = (x > y) == asc;
            v[e] = sw ? y : x;
            v[e | je] = sw ? x : y;
          }
        }
      } else {
        const bool lower = (lane & j) == 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          // the lower lane of a pair keeps the minimum in an ascending block,
          // the upper lane in a descending one: one compare and one select
          const bool keep_min = lower == (((e * 64 + lane) & k) == 0);
          const uint64_t y = shfl_xor_u64(v[e], j);
          v[e] = ((v[e] < y) == keep_min) ? v[e] : y;
        }
      }
    }
  }
}

// The same sort for large E with the stage loops kept as loops: each stage
// runs a body fixed by its exchange distance (in-lane swaps of registers e
// and e | J/64, or a cross-lane exchange at lane distance J), chosen by a
// switch, so the register array is indexed statically while the code stays
// small.
template <int E, int JE>
__device__ __forceinline__ void stage_in_lane(uint64_t (&v)[E], int lane, int k) {
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if ((e & JE) == 0) {
      const bool asc = ((e * 64 + lane) & k) == 0;
      const uint64_t x = v[e], y = v[e | JE];
      const bool sw = (x > y) == asc;
      v[e] = sw ? y : x;
      v[e | JE] = sw ? x : y;
    }
  }
}
template <int E, int J>
__device__ __forceinline__ void stage_cross_lane(uint64_t (&v)[E], int lane, int k) {
  const bool lower = (lane & J) == 0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const bool keep_min = lower == (((e * 64 + lane) & k) == 0);
    const uint64_t y = xor_lane_u64<J>(v[e]);
    v[e] = ((v[e] < y) == keep_min) ? v[e] : y;
  }
}
template <int E>
__device__ __forceinline__ void reg_bitonic_sort_loop(uint64_t (&v)[E], int lane) {
  constexpr int N = 64 * E;
  for (int k = 2; k <= N; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      switch (j) {
        case 1: stage_cross_lane<E, 1>(v, lane, k); break;
        case 2: stage_cross_lane<E, 2>(v, lane, k); break;
        case 4: stage_cross_lane<E, 4>(v, lane, k); break;
        case 8: stage_cross_lane<E, 8>(v, lane, k); break;
        case 16: stage_cross_lane<E, 16>(v, lane, k); break;
        case 32: stage_cross_lane<E, 32>(v, lane, k); break;
        default:
          if constexpr (E >= 2) if (j == 64) stage_in_lane<E, 1>(v, lane, k);
          if constexpr (E >= 4) if (j == 128) stage_in_lane<E, 2>(v, lane, k);
          if constexpr (E >= 8) if (j == 256) stage_in_lane<E, 4>(v, lane, k);
          if constexpr (E >= 16) if (j == 512) stage_in_lane<E, 8>(v, lane, k);
          if constexpr (E >= 32) if (j == 1024) stage_in_lane<E, 16>(v, lane, k);
          break;
      }
    }
  }
}

}  // namespace pipnn
