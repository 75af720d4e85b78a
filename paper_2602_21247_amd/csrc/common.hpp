// Device-side helpers shared by the PiPNN gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pipnn {

constexpr uint32_t kEmptyId = 0xFFFFFFFFu;
constexpr uint16_t kBf16Inf = 0x7F80u;
constexpr int kNumXcd = 8;

// Reservoir slot (Sec. 3, Implementation): 4-byte id, 2-byte hash, bf16
// distance, packed as bits 0..31 / 32..47 / 48..63.
__host__ __device__ __forceinline__ uint64_t slot_pack(uint32_t id, uint32_t hash, uint32_t bf) {
  return (uint64_t)id | ((uint64_t)(hash & 0xFFFFu) << 32) | ((uint64_t)(bf & 0xFFFFu) << 48);
}
__host__ __device__ __forceinline__ uint32_t slot_id(uint64_t s) { return (uint32_t)s; }
__host__ __device__ __forceinline__ uint32_t slot_hash(uint64_t s) { return (uint32_t)(s >> 32) & 0xFFFFu; }
__host__ __device__ __forceinline__ uint32_t slot_bf(uint64_t s) { return (uint32_t)(s >> 48); }
__host__ __device__ __forceinline__ uint64_t empty_slot() { return slot_pack(kEmptyId, 0, kBf16Inf); }

// float32 -> bf16 bits, round to nearest even on the 16 dropped bits; -0
// becomes +0 and NaN becomes the canonical quiet NaN.
__device__ __forceinline__ uint32_t bf16_rne(float f) {
  if (f == 0.0f) return 0u;
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return 0x7FC0u;
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}

// bf16 bits -> unsigned rank that follows the numeric order.
__host__ __device__ __forceinline__ uint32_t bf16_rank(uint32_t b) {
  return (b & 0x8000u) ? (~b & 0xFFFFu) : (b | 0x8000u);
}
__host__ __device__ __forceinline__ uint32_t rank_to_bf16(uint32_t r) {
  return (r & 0x8000u) ? (r & 0x7FFFu) : (~r & 0xFFFFu);
}

// float32 -> unsigned rank that follows the numeric order (no NaN).
__device__ __forceinline__ uint32_t f32_rank(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Orders LDS traffic between the lanes of one wave (a compiler and memory
// fence at wavefront scope; lanes of a wave execute in lockstep).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Workgroups are dealt to the 8 XCDs round robin (block b runs on XCD b % 8).
// This remaps block ids so that consecutive work items land on one XCD and
// share its L2. The grid must hold 8 * ceil(n_items / 8) blocks.
__device__ __forceinline__ int xcd_item(int block, int nblocks) {
  const int per = nblocks / kNumXcd;
  return (block % kNumXcd) * per + block / kNumXcd;
}
__host__ __forceinline__ int xcd_grid(int64_t n_items) {
  return (int)(((n_items + kNumXcd - 1) / kNumXcd) * kNumXcd);
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Inclusive wave-wide prefix sum of an int.
__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = lane_id();
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int t = __shfl_up(v, off, 64);
    if (lane >= off) v += t;
  }
  return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace pipnn
