// Supporting kernels: norms and sketches, conversions, fills, prefix sums,
// and the stable group-by, merge and copy steps of randomized ball carving.
#include "common.hpp"
#include "internal.hpp"

namespace pipnn {

// ---------------------------------------------------------------------
// Squared norms (for the GEMM distance form) and sketches
// Sketch(v)_b = H_b . v (Sec. 3, Implementation). One thread per point
// accumulates every output in dimension order; the rows and the matching
// columns of the hyperplanes are staged through LDS. The same pass
// takes the integer check: chk[0] is set when a coordinate is not an
// integer of magnitude <= 2^20, chk[1] / chk[2] collect the smallest and
// largest coordinate (one atomic per wave, only when it would change them).
// A coordinate is flagged here when it is not an integer (NaN included);
// infinities and magnitudes above 2^20 show in the wave's lo / hi.
__device__ __forceinline__ void coord_check(float v, bool &bad, float &lo, float &hi) {
  bad |= v != rintf(v);
  lo = fminf(lo, v);
  hi = fmaxf(hi, v);
}

__global__ void __launch_bounds__(256) norms_sketches_kernel(const float *__restrict__ X, int64_t n,
                                                             int d, const float *__restrict__ H,
                                                             int m, float *__restrict__ norms,
                                                             float *__restrict__ S,
                                                             int *__restrict__ chk) {
  // The block's 256 rows pass through LDS 16 dimensions at a time: the slab
  // is loaded with consecutive lanes on consecutive 16-byte pieces of the
  // rows (coalesced), then each thread continues its own row's sums in
  // dimension order from LDS.
  constexpr int KD = 16;
  __shared__ float sX[256][KD + 1];             // the slab (+1: conflict-free row reads)
  __shared__ float sHk[16][KD];                 // the slab's columns of the hyperplanes (m <= 16)
  const int64_t p0 = (int64_t)blockIdx.x * 256;
  const int64_t p = p0 + threadIdx.x;
  const int rows = (int)min<int64_t>(256, n - p0);
  bool bad = false;
  float lo = INFINITY, hi = -INFINITY;
  float nn = 0.f;
  float sk[16];
#pragma unroll
  for (int b = 0; b < 16; ++b) sk[b] = 0.f;
  for (int k0 = 0; k0 < d; k0 += KD) {
    const int kw = min(KD, d - k0);
    __syncthreads();  // the previous slab is consumed
    for (int t = threadIdx.x; t < m * kw; t += 256) {
      const int b = t / kw, c = t - b * kw;
      sHk[b][c] = H[b * d + k0 + c];
    }
    if ((d & 3) == 0) {
      // kw is a multiple of 4: 4-float pieces, kw / 4 per row
      const int pr = kw >> 2;
      for (int t = threadIdx.x; t < rows * pr; t += 256) {
        const int r = t / pr, c = (t - r * pr) * 4;
        const float4 v = *reinterpret_cast<const float4 *>(X + (p0 + r) * d + k0 + c);
        sX[r][c] = v.x; sX[r][c + 1] = v.y; sX[r][c + 2] = v.z; sX[r][c + 3] = v.w;
      }
    } else {
      for (int t = threadIdx.x; t < rows * kw; t += 256) {
        const int r = t / kw, c = t - r * kw;
        sX[r][c] = X[(p0 + r) * d + k0 + c];
      }
    }
    __syncthreads();
    if (p < n) {
      for (int j = 0; j < kw; ++j) {
        const float v = sX[threadIdx.x][j];
        nn = fmaf(v, v, nn);
        coord_check(v, bad, lo, hi);
#pragma unroll
        for (int b = 0; b < 16; ++b)
          if (b < m) sk[b] = fmaf(sHk[b][j], v, sk[b]);
      }
    }
  }
  if (p < n) {
    norms[p] = nn;
#pragma unroll
    for (int b = 0; b < 16; ++b)
      if (b < m) S[p * m + b] = sk[b];
  }
  // the wave's check (lanes past n hold the neutral +inf / -inf)
  bool wbad = __ballot(bad) != 0ull;
  if (!wbad) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      lo = fminf(lo, __shfl_xor(lo, off, 64));
      hi = fmaxf(hi, __shfl_xor(hi, off, 64));
    }
    wbad = lo <= hi && (lo < -1048576.f || hi > 1048576.f);
  }
  if ((threadIdx.x & 63) == 0 && chk) {
    if (wbad) {
      if (*(volatile int *)chk == 0) atomicOr(chk, 1);
    } else if (lo <= hi) {  // some lane of the wave holds a point
      const int ilo = (int)lo, ihi = (int)hi;
      if (*(volatile int *)(chk + 1) > ilo) atomicMin(chk + 1, ilo);
      if (*(volatile int *)(chk + 2) < ihi) atomicMax(chk + 2, ihi);
    }
  }
}

hipError_t launch_norms_sketches(const Index &I, hipStream_t s) {
  return launch_norms_sketches_range(I, 0, I.n, s);
}

hipError_t launch_norms_sketches_range(const Index &I, int64_t p0, int64_t cnt, hipStream_t s) {
  if (cnt <= 0) return hipSuccess;
  const int64_t blocks = (cnt + 255) / 256;
  hipLaunchKernelGGL(norms_sketches_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                     I.xf() + p0 * I.d, cnt, I.d, I.H, I.m, I.norms.as<float>() + p0,
                     I.sketches.as<float>() + p0 * I.m, I.int_chk.as<int>());
  return hipGetLastError();
}

__global__ void int_check_init_kernel(int *chk) {
  if (threadIdx.x == 0) {
    chk[0] = 0;
    chk[1] = 0x7FFFFFFF;
    chk[2] = (int)0x80000000;
  }
}

hipError_t clear_int_check(Index &I, hipStream_t s) {
  hipLaunchKernelGGL(int_check_init_kernel, dim3(1), dim3(64), 0, s, I.int_chk.as<int>());
  return hipGetLastError();
}

// Every distance form is exact in float32 when the coordinates are integers
// whose squared norms sum to at most 2^24 for any pair (d * A^2 <= 2^23,
// A = the largest magnitude) and whose squared differences sum to at most
// 2^24 (d * W^2 <= 2^24, W = the range): every product, partial sum and
// result of the direct difference, the norms and the norm expansion is then
// an integer of magnitude <= 2^24.
hipError_t read_int_check(Index &I, bool reset, hipStream_t s) {
  int32_t h[3] = {1, 0, 0};
  hipError_t e = hipMemcpyAsync(h, I.int_chk.p, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  const bool had = !reset && I.int_exact;
  if (h[0] != 0 || (!reset && !I.int_exact)) {
    I.int_exact = false;
    return hipSuccess;
  }
  int64_t lo = h[1], hi = h[2];
  if (lo > hi) {  // no points were checked
    I.int_exact = had;
    return hipSuccess;
  }
  if (had) {
    lo = std::min(lo, I.int_lo);
    hi = std::max(hi, I.int_hi);
  }
  const int64_t A = std::max(-lo, hi), W = hi - lo;
  const int64_t d = I.d;
  I.int_lo = lo;
  I.int_hi = hi;
  I.int_exact = d * A * A <= (int64_t(1) << 23) && d * W * W <= (int64_t(1) << 24);
  return hipSuccess;
}

// ---- reduced-precision GEMM operand -------------------------------------
// bf16: upper half of the binary32 after round-to-nearest-even.
__device__ __forceinline__ uint32_t enc_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (u >> 16) | 0x40u;
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
// OCP E4M3 ("e4m3fn": bias 7, 3 fraction bits, subnormals, no infinities,
// S.1111.111 = NaN, largest finite 448), round-to-nearest-even on the
// dropped fraction bits, saturating at +-448.
__device__ __forceinline__ uint32_t enc_e4m3(float f) {
  const uint32_t u = __float_as_uint(f);
  const uint32_t sign = (u >> 24) & 0x80u;
  const uint32_t a = u & 0x7FFFFFFFu;
  if (a > 0x7F800000u) return sign | 0x7Fu;        // NaN
  if (a >= 0x43E00000u) return sign | 0x7Eu;       // |f| >= 448
  if (a < 0x3C800000u) {                           // |f| < 2^-6: subnormal step 2^-9
    return sign | (uint32_t)rintf(__uint_as_float(a) * 512.f);  // 8 is the smallest normal
  }
  const uint32_t e = (a >> 23) - 120u;             // biased E4M3 exponent, 1..15
  const uint32_t m = a & 0x7FFFFFu;
  const uint32_t r = (m + 0x7FFFFu + ((m >> 20) & 1u)) >> 20;  // 0..8, 8 carries
  return sign | ((e << 3) + r);
}
__device__ __forceinline__ float dec_e4m3(uint32_t c) {
  const uint32_t e = (c >> 3) & 15u, m = c & 7u;
  const float v = e == 0 ? (float)m * 0.001953125f : __uint_as_float(((e + 120u) << 23) | (m << 20));
  return (c & 0x80u) ? -v : v;
}

// One wave per point: encode its d values (zero padded to ldo), and the
// squared norm of the decoded vector, summed per lane and then across the
// wave. fp8 scales each point by 448 / max|x_i| first.
__global__ void __launch_bounds__(256) quantize_kernel(const float *__restrict__ X, int64_t n, int d,
                                                       int ldo, int prec, void *out,
                                                       float *__restrict__ scale,
                                                       float *__restrict__ norms,
                                                       int *__restrict__ inexact) {
  const int lane = threadIdx.x & 63;
  const int64_t p = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (p >= n) return;
  const float *x = X + p * d;
  float s = 1.f, inv = 1.f;
  if (prec == PIPNN_PREC_FP8) {
    float mx = 0.f;
    for (int i = lane; i < d; i += 64) mx = fmaxf(mx, fabsf(x[i]));
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
    if (mx > 0.f) {
      s = 448.f / mx;
      inv = mx / 448.f;
    }
    if (lane == 0) scale[p] = inv;
  }
  float nn = 0.f;
  bool lossy = false;
  for (int i = lane; i < ldo; i += 64) {
    const float v = i < d ? x[i] : 0.f;
    float q;
    if (prec == PIPNN_PREC_BF16) {
      const uint32_t c = enc_bf16(v);
      reinterpret_cast<uint16_t *>(out)[p * ldo + i] = (uint16_t)c;
      q = __uint_as_float(c << 16);
    } else if (prec == PIPNN_PREC_FP16) {
      const _Float16 c = (_Float16)v;
      reinterpret_cast<_Float16 *>(out)[p * ldo + i] = c;
      q = (float)c;
    } else {
      const uint32_t c = enc_e4m3(v * s);
      reinterpret_cast<uint8_t *>(out)[p * ldo + i] = (uint8_t)c;
      q = dec_e4m3(c) * inv;
    }
    nn = fmaf(q, q, nn);
    lossy |= q != v;
  }
  nn = wave_sum(nn);
  if (lane == 0) norms[p] = nn;
  // every writer stores the same 1, so no read-modify-write is needed; a
  // wave that already sees the flag set skips the store
  if (__ballot(lossy) != 0ull && lane == 0 && *(volatile int *)inexact == 0) *inexact = 1;
}

// The two-byte codes (bf16, fp16) of rows whose padded width ldo is 64, 128,
// 256 or 512 and whose width d is a multiple of 4: one lane per 8 values
// (two 16-byte loads, one 16-byte store), the G = ldo / 8 lanes of a point
// consecutive in the wave; the squared norm of the decoded values is summed
// per lane in index order, then over the point's lanes.
// With I8 the same pass also writes the int8 rows (x - base, base = lo8 +
// 128; 8 bytes per lane) and their exact squared norms.
template <int PREC, bool I8>
__global__ void __launch_bounds__(256) quantize16_kernel(const float *__restrict__ X, int64_t n,
                                                         int d, int lg, uint4 *__restrict__ out,
                                                         float *__restrict__ norms,
                                                         int *__restrict__ inexact, float base,
                                                         uint2 *__restrict__ out8,
                                                         float *__restrict__ norms8) {
  const int G = 1 << lg;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t p = t >> lg;
  const int c = (int)(t & (G - 1));
  float nn = 0.f;
  int n8 = 0;
  bool lossy = false;
  if (p < n) {
    const float *x = X + p * d + 8 * c;
    float v[8];
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
      if (8 * c + 4 * hh < d) q = *reinterpret_cast<const float4 *>(x + 4 * hh);
      v[4 * hh] = q.x; v[4 * hh + 1] = q.y; v[4 * hh + 2] = q.z; v[4 * hh + 3] = q.w;
    }
    if constexpr (I8) {
      uint32_t b[2] = {0u, 0u};
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int q = 8 * c + j < d ? (int)(v[j] - base) : 0;  // padding gives 0
        n8 += q * q;
        b[j >> 2] |= ((uint32_t)q & 0xFFu) << (8 * (j & 3));
      }
      out8[t] = make_uint2(b[0], b[1]);
    }
    uint32_t w[4];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      uint32_t code;
      float q;
      if constexpr (PREC == PIPNN_PREC_BF16) {
        code = enc_bf16(v[j]);
        q = __uint_as_float(code << 16);
      } else {
        const _Float16 hv = (_Float16)v[j];
        code = __builtin_bit_cast(uint16_t, hv);
        q = (float)hv;
      }
      if (j & 1) w[j >> 1] |= code << 16;
      else w[j >> 1] = code;
      nn = fmaf(q, q, nn);
      lossy |= q != v[j];
    }
    out[t] = make_uint4(w[0], w[1], w[2], w[3]);
  }
  for (int off = G >> 1; off >= 1; off >>= 1) nn += __shfl_xor(nn, off, 64);
  if (p < n && c == 0) norms[p] = nn;
  if constexpr (I8) {
    for (int off = G >> 1; off >= 1; off >>= 1) n8 += __shfl_xor(n8, off, 64);
    if (p < n && c == 0) norms8[p] = (float)n8;
  }
  if (__ballot(lossy) != 0ull && (threadIdx.x & 63) == 0 && *(volatile int *)inexact == 0)
    *inexact = 1;
}

// The int8 rows of an integral float32 X whose coordinates lie in
// [lo8, lo8 + 255]: value x - lo8 - 128 (exact), zero past d (a zero
// coordinate adds nothing to any dot product or norm), one lane per 16
// values (one 16-byte store), the G = ld8 / 16 lanes of a point consecutive
// in the wave; the squared norm is an exact integer sum.
__global__ void __launch_bounds__(256) quantize8_kernel(const float *__restrict__ X, int64_t n,
                                                        int d, int lg, float base, bool vec,
                                                        uint4 *__restrict__ out,
                                                        float *__restrict__ norms) {
  const int G = 1 << lg;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t p = t >> lg;
  const int c = (int)(t & (G - 1));
  int nn = 0;
  if (p < n) {
    const float *x = X + p * d + 16 * c;
    float v[16];
    if (vec) {
#pragma unroll
      for (int j4 = 0; j4 < 4; ++j4) {
        float4 q = make_float4(base, base, base, base);
        if (16 * c + 4 * j4 < d) q = *reinterpret_cast<const float4 *>(x + 4 * j4);
        v[4 * j4] = q.x; v[4 * j4 + 1] = q.y; v[4 * j4 + 2] = q.z; v[4 * j4 + 3] = q.w;
      }
    } else {
#pragma unroll
      for (int j = 0; j < 16; ++j) v[j] = 16 * c + j < d ? x[j] : base;
    }
    uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int q = (int)(v[j] - base);  // base = lo8 + 128; padding gives 0
      nn += q * q;
      w[j >> 2] |= ((uint32_t)q & 0xFFu) << (8 * (j & 3));
    }
    out[t] = make_uint4(w[0], w[1], w[2], w[3]);
  }
  for (int off = G >> 1; off >= 1; off >>= 1) nn += __shfl_xor(nn, off, 64);
  if (p < n && c == 0) norms[p] = (float)nn;
}

hipError_t launch_quantize8_range(const Index &I, int64_t p0, int64_t cnt, hipStream_t s) {
  if (cnt <= 0) return hipSuccess;
  if (!I.x8.p || !I.n8.p || (I.ld8 != 64 && I.ld8 != 128)) return hipErrorInvalidValue;
  const int lg = I.ld8 == 64 ? 2 : 3;
  const int64_t threads = cnt << lg;
  const bool vec = I.d % 4 == 0 && (reinterpret_cast<uintptr_t>(I.xf()) & 15u) == 0;
  hipLaunchKernelGGL(quantize8_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s,
                     I.xf() + p0 * I.d, cnt, I.d, lg, (float)(I.lo8 + 128), vec,
                     reinterpret_cast<uint4 *>(I.x8.as<uint8_t>() + p0 * I.ld8),
                     I.n8.as<float>() + p0);
  return hipGetLastError();
}

// One thread per 16-byte chunk of the padded rows: float32 values, zeros
// past d.
__global__ void __launch_bounds__(256) pad_kernel(const float *__restrict__ X, int64_t n, int d,
                                                  int ldf, float4 *__restrict__ out) {
  const int cpr = ldf / 4;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * cpr) return;
  const int64_t p = i / cpr;
  const int k = (int)(i - p * cpr) * 4;
  const float *x = X + p * d;
  float4 v;
  v.x = k < d ? x[k] : 0.f;
  v.y = k + 1 < d ? x[k + 1] : 0.f;
  v.z = k + 2 < d ? x[k + 2] : 0.f;
  v.w = k + 3 < d ? x[k + 3] : 0.f;
  out[i] = v;
}

hipError_t launch_pad_range(const Index &I, int64_t p0, int64_t cnt, hipStream_t s) {
  if (cnt <= 0 || !I.xpad.p) return hipSuccess;
  const int64_t chunks = cnt * (I.ldf / 4);
  hipLaunchKernelGGL(pad_kernel, dim3((unsigned)((chunks + 255) / 256)), dim3(256), 0, s,
                     I.xf() + p0 * I.d, cnt, I.d, I.ldf,
                     reinterpret_cast<float4 *>(I.xpad.as<float>() + p0 * I.ldf));
  return hipGetLastError();
}

hipError_t launch_quantize(const Index &I, hipStream_t s) {
  return launch_quantize_range(I, 0, I.n, s, false);
}

hipError_t launch_quantize_range(const Index &I, int64_t p0, int64_t cnt, hipStream_t s,
                                 bool with8) {
  if (cnt <= 0) return hipSuccess;
  const int64_t blocks = (cnt + 3) / 4;
  if (!I.xlow.p || I.copy_prec == PIPNN_PREC_FP32) return hipErrorInvalidValue;
  const size_t eb = I.copy_prec == PIPNN_PREC_FP8 ? 1 : 2;
  const int lg = I.ldo == 64 ? 3 : I.ldo == 128 ? 4 : I.ldo == 256 ? 5 : I.ldo == 512 ? 6 : 0;
  if (eb == 2 && lg && I.d % 4 == 0 && (reinterpret_cast<uintptr_t>(I.xf()) & 15u) == 0) {
    // the int8 rows in the same pass where their width is the copy's
    const bool fuse8 = with8 && I.copy_prec == PIPNN_PREC_FP16 && I.x8.p && I.ld8 == I.ldo;
    const int64_t threads = cnt << lg;
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s,
                         I.xf() + p0 * I.d, cnt, I.d, lg,
                         reinterpret_cast<uint4 *>(I.xlow.as<uint8_t>() + p0 * I.ldo * eb),
                         I.lnorms.as<float>() + p0, I.op_flag.as<int>(), (float)(I.lo8 + 128),
                         fuse8 ? reinterpret_cast<uint2 *>(I.x8.as<uint8_t>() + p0 * I.ld8)
                               : nullptr,
                         fuse8 ? I.n8.as<float>() + p0 : nullptr);
    };
    if (I.copy_prec == PIPNN_PREC_BF16) go(quantize16_kernel<PIPNN_PREC_BF16, false>);
    else if (fuse8) go(quantize16_kernel<PIPNN_PREC_FP16, true>);
    else go(quantize16_kernel<PIPNN_PREC_FP16, false>);
    if (with8 && !fuse8) {
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      return launch_quantize8_range(I, p0, cnt, s);
    }
    return hipGetLastError();
  }
  if (with8) {
    hipError_t e = launch_quantize8_range(I, p0, cnt, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(quantize_kernel, dim3((unsigned)blocks), dim3(256), 0, s, I.xf() + p0 * I.d,
                     cnt, I.d, I.ldo, I.copy_prec,
                     reinterpret_cast<void *>(I.xlow.as<uint8_t>() + p0 * I.ldo * eb),
                     I.xscale.as<float>() + p0, I.lnorms.as<float>() + p0, I.op_flag.as<int>());
  return hipGetLastError();
}

hipError_t clear_op_flag(Index &I, hipStream_t s) {
  return launch_fill_u32(I.op_flag.as<uint32_t>(), 0u, 1, s);
}

hipError_t read_op_flag(Index &I, bool reset, hipStream_t s) {
  if (reset) I.op_exact = false;
  int32_t f = 1;
  hipError_t e = hipMemcpyAsync(&f, I.op_flag.p, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  if (reset) I.op_exact = f == 0;
  else if (f != 0) I.op_exact = false;
  return hipSuccess;
}

// ---- leaf table of an index (kept for insertion) ------------------------
__global__ void rebase_i64_kernel(const int64_t *in, int64_t n, int64_t *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i] - in[0];
}
__global__ void copy_u32_kernel(const uint32_t *in, int64_t n, uint32_t *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i];
}
hipError_t launch_rebase_i64(const int64_t *in, int64_t n, int64_t *out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(rebase_i64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, n,
                     out);
  return hipGetLastError();
}
hipError_t launch_copy_u32(const uint32_t *in, int64_t n, uint32_t *out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, n,
                     out);
  return hipGetLastError();
}

// Representative of each leaf: the member m with the smallest
// (sum_i (s * x_mi - S_i)^2, id), S_i = sum of the leaf's members in
// dimension i and s the leaf size -- s^2 times m's squared distance to the
// leaf mean, without a division -- in FP64 (exact for integer-valued data).
// One workgroup per leaf.
__global__ void __launch_bounds__(256) leaf_rep_kernel(const float *__restrict__ X, int d,
                                                       const int64_t *__restrict__ off,
                                                       const uint32_t *__restrict__ mem,
                                                       uint32_t *__restrict__ rep) {
  extern __shared__ double sS[];  // d doubles
  __shared__ double sBd[256];
  __shared__ uint32_t sBi[256];
  const int64_t L = blockIdx.x;
  const int64_t o = off[L], s = off[L + 1] - off[L];
  if (s <= 0) {
    if (threadIdx.x == 0) rep[L] = 0u;  // any valid id: an empty leaf adds no members
    return;
  }
  for (int i = threadIdx.x; i < d; i += blockDim.x) {
    double acc = 0.0;
    for (int64_t j = 0; j < s; ++j) acc += (double)X[(int64_t)mem[o + j] * d + i];
    sS[i] = acc;
  }
  __syncthreads();
  double bd = INFINITY;
  uint32_t bi = 0xFFFFFFFFu;
  const double sd = (double)s;
  for (int64_t j = threadIdx.x; j < s; j += blockDim.x) {
    const uint32_t id = mem[o + j];
    const float *x = X + (int64_t)id * d;
    double dd = 0.0;
    for (int i = 0; i < d; ++i) {
      const double t = sd * (double)x[i] - sS[i];
      dd = fma(t, t, dd);
    }
    if (dd < bd || (dd == bd && id < bi)) {
      bd = dd;
      bi = id;
    }
  }
  sBd[threadIdx.x] = bd;
  sBi[threadIdx.x] = bi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double od = sBd[threadIdx.x + w];
      const uint32_t oi = sBi[threadIdx.x + w];
      if (od < sBd[threadIdx.x] || (od == sBd[threadIdx.x] && oi < sBi[threadIdx.x])) {
        sBd[threadIdx.x] = od;
        sBi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) rep[L] = sBi[0];
}
hipError_t launch_leaf_reps(const float *X, int d, const int64_t *off, const uint32_t *mem,
                            int64_t n_leaves, uint32_t *rep, hipStream_t s) {
  if (n_leaves <= 0) return hipSuccess;
  hipLaunchKernelGGL(leaf_rep_kernel, dim3((unsigned)n_leaves), dim3(256), (size_t)d * 8, s, X, d,
                     off, mem, rep);
  return hipGetLastError();
}

// ---- touched-set compaction -----------------------------------------------
__global__ void mark_ids_kernel(const uint32_t *ids, int64_t cnt, int64_t n, uint32_t *flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) {
    const uint32_t v = ids[i];
    if (v < n) flag[v] = 1u;
  }
}
__global__ void compact_flags_kernel(const uint32_t *flag, const int64_t *pos, int64_t n,
                                     uint32_t *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && flag[i]) out[pos[i]] = (uint32_t)i;
}
hipError_t launch_mark_ids(const uint32_t *ids, int64_t cnt, int64_t n, uint32_t *flag,
                           hipStream_t s) {
  if (cnt <= 0) return hipSuccess;
  hipLaunchKernelGGL(mark_ids_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, ids,
                     cnt, n, flag);
  return hipGetLastError();
}
hipError_t launch_compact_flags(const uint32_t *flag, const int64_t *pos, int64_t n, uint32_t *out,
                                hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(compact_flags_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     flag, pos, n, out);
  return hipGetLastError();
}

__global__ void to_f32_kernel(const void *src, int dtype, float *dst, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  if (dtype == PIPNN_DTYPE_F16) {
    dst[i] = (float)reinterpret_cast<const _Float16 *>(src)[i];
  } else if (dtype == PIPNN_DTYPE_BF16) {
    const uint16_t b = reinterpret_cast<const uint16_t *>(src)[i];
    dst[i] = __uint_as_float((uint32_t)b << 16);
  } else {
    dst[i] = reinterpret_cast<const float *>(src)[i];
  }
}

// Eight 16-bit values per thread: one 16-byte load, two 16-byte stores
// (16-byte aligned source and destination; the conversions are exact).
__global__ void to_f32_x8_kernel(const uint4 *__restrict__ src, int dtype, float4 *__restrict__ dst,
                                 int64_t n8) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n8) return;
  const uint4 v = src[i];
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
  float f[8];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t lo = w[j] & 0xFFFFu, hi = w[j] >> 16;
    if (dtype == PIPNN_DTYPE_F16) {
      f[2 * j] = (float)__builtin_bit_cast(_Float16, (uint16_t)lo);
      f[2 * j + 1] = (float)__builtin_bit_cast(_Float16, (uint16_t)hi);
    } else {
      f[2 * j] = __uint_as_float(lo << 16);
      f[2 * j + 1] = __uint_as_float(hi << 16);
    }
  }
  dst[2 * i] = make_float4(f[0], f[1], f[2], f[3]);
  dst[2 * i + 1] = make_float4(f[4], f[5], f[6], f[7]);
}

hipError_t launch_to_f32(const void *src, int dtype, float *dst, int64_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  int64_t head = 0;
  if (dtype != PIPNN_DTYPE_F32 && ((uintptr_t)src & 15) == 0 && ((uintptr_t)dst & 15) == 0) {
    const int64_t n8 = count / 8;
    if (n8 > 0)
      hipLaunchKernelGGL(to_f32_x8_kernel, dim3((unsigned)((n8 + 255) / 256)), dim3(256), 0, s,
                         reinterpret_cast<const uint4 *>(src), dtype,
                         reinterpret_cast<float4 *>(dst), n8);
    head = n8 * 8;
  }
  if (head < count) {
    const int64_t rest = count - head;
    const size_t eb = dtype == PIPNN_DTYPE_F32 ? 4 : 2;
    hipLaunchKernelGGL(to_f32_kernel, dim3((unsigned)((rest + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<const void *>(reinterpret_cast<const uint8_t *>(src) + head * eb),
                       dtype, dst + head, rest);
  }
  return hipGetLastError();
}

__global__ void iota_kernel(uint32_t *dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (uint32_t)i;
}
hipError_t launch_iota(uint32_t *dst, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(iota_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dst, n);
  return hipGetLastError();
}

__global__ void fill_u32_kernel(uint32_t *dst, uint32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = v;
}
hipError_t launch_fill_u32(uint32_t *dst, uint32_t v, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dst, v,
                     n);
  return hipGetLastError();
}
__global__ void fill_u64_kernel(uint64_t *dst, uint64_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = v;
}
hipError_t launch_fill_u64(uint64_t *dst, uint64_t v, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dst, v,
                     n);
  return hipGetLastError();
}

__global__ void gather_u32_kernel(const uint32_t *src, const int64_t *idx, uint32_t *dst,
                                  int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[idx[i]];
}
hipError_t launch_gather_u32(const uint32_t *src, const int64_t *idx, uint32_t *dst, int64_t n,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src,
                     idx, dst, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------
// Exclusive prefix sum. Tiles of 4096 values (256 threads x 16); tile sums
// are scanned by one workgroup (up to 4096 tiles), then added back.
constexpr int kScanThreads = 256;
constexpr int kScanPer = 16;
constexpr int kScanTile = kScanThreads * kScanPer;

template <class T>
__device__ int64_t block_excl_scan(int64_t v, int64_t *sh, int64_t *total) {
  // v: this thread's value; returns the exclusive prefix across the block
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int64_t t = __shfl_up(x, off, 64);
    if (lane >= off) x += t;
  }
  if (lane == 63) sh[wave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t acc = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) {
      int64_t t = sh[w];
      sh[w] = acc;
      acc += t;
    }
    *total = acc;
  }
  __syncthreads();
  return x - v + sh[wave];
}

template <class T>
__global__ void __launch_bounds__(kScanThreads) scan_tiles_kernel(const T *in, int64_t *out,
                                                                  int64_t n, int64_t *tile_sums) {
  __shared__ int64_t sh[kScanThreads / 64];
  __shared__ int64_t tot;
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
  int64_t v[kScanPer];
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    v[i] = (base + i < n) ? (int64_t)in[base + i] : 0;
    s += v[i];
  }
  int64_t pre = block_excl_scan<T>(s, sh, &tot);
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    if (base + i < n) out[base + i] = pre;
    pre += v[i];
  }
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kScanThreads) scan_sums_kernel(int64_t *sums, int64_t nt,
                                                                 int64_t *total_out) {
  __shared__ int64_t sh[kScanThreads / 64];
  __shared__ int64_t tot;
  const int64_t base = (int64_t)threadIdx.x * kScanPer;
  int64_t v[kScanPer];
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    v[i] = (base + i < nt) ? sums[base + i] : 0;
    s += v[i];
  }
  int64_t pre = block_excl_scan<int64_t>(s, sh, &tot);
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    if (base + i < nt) sums[base + i] = pre;
    pre += v[i];
  }
  if (threadIdx.x == 0) *total_out = tot;
}

__global__ void scan_add_kernel(int64_t *out, int64_t n, const int64_t *tile_pre) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += tile_pre[i / kScanTile];
}

int64_t scan_tmp_elems(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

template <class T>
static hipError_t scan_impl(const T *in, int64_t *out, int64_t n, int64_t *tmp, hipStream_t s) {
  const int64_t nt = (n + kScanTile - 1) / kScanTile;
  if (nt > kScanTile) return hipErrorInvalidValue;
  if (n == 0) {
    return launch_fill_u64(reinterpret_cast<uint64_t *>(out), 0ull, 1, s);
  }
  hipLaunchKernelGGL((scan_tiles_kernel<T>), dim3((unsigned)nt), dim3(kScanThreads), 0, s, in, out,
                     n, tmp);
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(kScanThreads), 0, s, tmp, nt, out + n);
  hipLaunchKernelGGL(scan_add_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, n,
                     tmp);
  return hipGetLastError();
}

hipError_t launch_scan_u32(const uint32_t *in, int64_t *out, int64_t n, int64_t *tmp,
                           hipStream_t s) {
  return scan_impl<uint32_t>(in, out, n, tmp, s);
}
hipError_t launch_scan_i64_inplace(int64_t *data, int64_t n, int64_t *tmp, hipStream_t s) {
  // out[i] may alias in[i]: each tile reads its values before writing them
  return scan_impl<int64_t>(data, data, n, tmp, s);
}

// ---------------------------------------------------------------------
// Stable group-by of ball-carving assignments into buckets.
//
// Elements of subproblem s are (instance r, fanout slot j) for r over its
// points in ascending id order; asg_col[e] is the leader index t of element
// e (or 0xFFFFFFFF for an unused slot). The counts of every (bucket t,
// tile) pair are laid out subproblem by subproblem, bucket-major, so that
// one exclusive scan gives each (bucket, tile) its output position, and a
// stable scatter then leaves every bucket in ascending id order.
constexpr int kGroupTile = 1024;  // elements per tile (one wave)
constexpr int kMaxLeaders = 4096;

__global__ void __launch_bounds__(64) group_hist_kernel(const uint32_t *asg, const GroupSub *subs,
                                                        const GroupTile *tiles, int64_t *cm) {
  __shared__ int hist[kMaxLeaders];
  const GroupTile tl = tiles[blockIdx.x];
  const GroupSub sb = subs[tl.sub];
  const int lane = threadIdx.x;
  for (int t = lane; t < sb.n_buckets; t += 64) hist[t] = 0;
  wave_sync();
  const int64_t e0 = sb.elem_off + (int64_t)tl.tile * kGroupTile;
  const int64_t e1 = min(e0 + kGroupTile, sb.elem_off + sb.n_elems);
  for (int64_t e = e0 + lane; e < e1; e += 64) {
    const uint32_t t = asg[e];
    if (t != kEmptyId) atomicAdd(&hist[t], 1);
  }
  wave_sync();
  for (int t = lane; t < sb.n_buckets; t += 64)
    cm[sb.cm_off + (int64_t)t * sb.n_tiles + tl.tile] = hist[t];
}

// The scatter of a tile, 64 elements at a time: each element ORs its lane
// bit into its bucket's LDS mask; an element's rank among the chunk's
// elements of its bucket is the count of lower lanes in that mask, so the
// elements keep their order, and the bucket's first element advances the
// bucket's position by the count and clears the mask. LDS: the buckets'
// positions, then their masks (max_buckets of each).
__global__ void __launch_bounds__(64) group_scatter_kernel(const uint32_t *asg,
                                                           const uint32_t *src_ids, int32_t fmax,
                                                           const GroupSub *subs,
                                                           const GroupTile *tiles,
                                                           const int64_t *cm, uint32_t *out,
                                                           int32_t max_buckets) {
  extern __shared__ int64_t gs_lds[];
  int64_t *pos = gs_lds;
  unsigned long long *mask = reinterpret_cast<unsigned long long *>(gs_lds + max_buckets);
  const GroupTile tl = tiles[blockIdx.x];
  const GroupSub sb = subs[tl.sub];
  const int lane = threadIdx.x;
  for (int t = lane; t < sb.n_buckets; t += 64) {
    pos[t] = cm[sb.cm_off + (int64_t)t * sb.n_tiles + tl.tile];
    mask[t] = 0ull;
  }
  wave_sync();
  const int64_t e0 = sb.elem_off + (int64_t)tl.tile * kGroupTile;
  const int64_t e1 = min(e0 + kGroupTile, sb.elem_off + sb.n_elems);
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int64_t c = e0; c < e1; c += 64) {
    const int64_t e = c + lane;
    const uint32_t t = e < e1 ? asg[e] : kEmptyId;
    const bool live = t != kEmptyId;
    if (live) atomicOr(&mask[t], 1ull << lane);
    wave_sync();
    int64_t mypos = -1;
    int cnt = 0;
    if (live) {
      const unsigned long long m = mask[t];
      const int rank = __popcll(m & below);
      mypos = pos[t] + rank;
      cnt = rank == 0 ? __popcll(m) : 0;
    }
    wave_sync();
    if (cnt > 0) {
      pos[t] += cnt;
      mask[t] = 0ull;
    }
    wave_sync();
    if (mypos >= 0) out[mypos] = src_ids[e / fmax];
  }
}

__global__ void bucket_start_kernel(const int64_t *cm, const int64_t *bucket_cm_idx,
                                    int64_t n_buckets, int64_t *bucket_start) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b < n_buckets) bucket_start[b] = cm[bucket_cm_idx[b]];
}

hipError_t launch_groupby(const uint32_t *asg_col, const uint32_t *src_ids, int32_t *fan,
                          const GroupSub *subs, const GroupTile *tiles, int32_t n_tiles,
                          int32_t tile_elems, int64_t *cm, int64_t cm_len, int64_t *tmp,
                          uint32_t *out, int64_t *bucket_start, int64_t n_buckets_total,
                          int32_t max_buckets, hipStream_t s) {
  (void)tile_elems;
  const int32_t fmax = *fan;
  if (n_tiles == 0) return hipSuccess;
  if (max_buckets < 1 || max_buckets > kMaxLeaders) return hipErrorInvalidValue;
  hipLaunchKernelGGL(group_hist_kernel, dim3(n_tiles), dim3(64), 0, s, asg_col, subs, tiles, cm);
  hipError_t e = launch_scan_i64_inplace(cm, cm_len, tmp, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(group_scatter_kernel, dim3(n_tiles), dim3(64), (size_t)max_buckets * 16, s,
                     asg_col, src_ids, fmax, subs, tiles, cm, out, max_buckets);
  // bucket_start holds, on entry, the cm index of every bucket's first tile
  hipLaunchKernelGGL(bucket_start_kernel, dim3((unsigned)((n_buckets_total + 255) / 256)),
                     dim3(256), 0, s, cm, bucket_start, n_buckets_total, bucket_start);
  return hipGetLastError();
}

// ---------------------------------------------------------------------
// Merge of small buckets: each group's buckets are concatenated, sorted and
// deduplicated (a point may sit in two small buckets of one subproblem).
constexpr int kMergeMax = 16384;

__global__ void __launch_bounds__(1024) merge_dedup_kernel(const uint32_t *const *seg_ptr,
                                                           const int32_t *seg_len,
                                                           const int32_t *grp_first_seg,
                                                           uint32_t *out, const int64_t *out_off,
                                                           int32_t *out_size) {
  __shared__ uint32_t buf[kMergeMax];
  const int g = blockIdx.x;
  const int s0 = grp_first_seg[g], s1 = grp_first_seg[g + 1];
  int total = 0;
  for (int sg = s0; sg < s1; ++sg) {
    const int len = seg_len[sg];
    const uint32_t *src = seg_ptr[sg];
    for (int i = threadIdx.x; i < len; i += blockDim.x) buf[total + i] = src[i];
    total += len;
  }
  int P = 1;
  while (P < total) P <<= 1;
  for (int i = total + threadIdx.x; i < P; i += blockDim.x) buf[i] = kEmptyId;
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < P / 2; t += blockDim.x) {
        const int i = 2 * t - (t & (j - 1));  // t = q*j + r -> q*2j + r (j is a power of two)
        const int l = i + j;
        const bool asc = (i & k) == 0;
        const uint32_t x = buf[i], y = buf[l];
        if ((x > y) == asc) { buf[i] = y; buf[l] = x; }
      }
      __syncthreads();
    }
  }
  // keep the first of every run; ranks via a block scan of keep flags
  __shared__ int wsum[16];
  int base = 0;
  for (int c = 0; c < total; c += blockDim.x) {
    const int i = c + threadIdx.x;
    const int keep = (i < total && (i == 0 || buf[i] != buf[i - 1])) ? 1 : 0;
    const int incl = wave_incl_scan(keep);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int wpre = 0, tot = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      if (w < wave) wpre += wsum[w];
      tot += wsum[w];
    }
    if (keep) out[out_off[g] + base + wpre + incl - 1] = buf[i];
    base += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) out_size[g] = base;
}

hipError_t launch_merge_dedup(const uint32_t *const *seg_ptr, const int32_t *seg_len,
                              const int32_t *grp_first_seg, int32_t n_groups, int32_t max_sum,
                              uint32_t *out, const int64_t *out_off, int32_t *out_size,
                              hipStream_t s) {
  if (n_groups == 0) return hipSuccess;
  if (max_sum > kMergeMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(merge_dedup_kernel, dim3(n_groups), dim3(1024), 0, s, seg_ptr, seg_len,
                     grp_first_seg, out, out_off, out_size);
  return hipGetLastError();
}

__global__ void copy_segments_kernel(const uint32_t *const *src, const int64_t *dst_off,
                                     const int32_t *len, uint32_t *dst) {
  const int g = blockIdx.x;
  const uint32_t *s = src[g];
  uint32_t *o = dst + dst_off[g];
  const int L = len[g];
  for (int i = threadIdx.x; i < L; i += blockDim.x) o[i] = s[i];
}

hipError_t launch_copy_segments(const uint32_t *const *src, const int64_t *dst_off,
                                const int32_t *len, int32_t n_segs, uint32_t *dst, hipStream_t s) {
  if (n_segs == 0) return hipSuccess;
  hipLaunchKernelGGL(copy_segments_kernel, dim3(n_segs), dim3(256), 0, s, src, dst_off, len, dst);
  return hipGetLastError();
}

// ---------------------------------------------------------------------
// Start point: nearest to the mean of X by (squared L2 in FP64, id).
__global__ void colsum_kernel(const float *X, int64_t n, int d, double *sum) {
  const int64_t p0 = (int64_t)blockIdx.x * 1024;
  const int64_t p1 = min(p0 + 1024, n);
  for (int j = threadIdx.x; j < d; j += blockDim.x) {
    double s = 0.0;
    for (int64_t p = p0; p < p1; ++p) s += (double)X[p * d + j];
    atomicAdd(&sum[j], s);
  }
}

__global__ void __launch_bounds__(256) center_dist_kernel(const float *X, int64_t n, int d,
                                                          const double *sum, double *bd,
                                                          uint32_t *bi) {
  __shared__ double sd[256];
  __shared__ uint32_t si[256];
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double best = INFINITY;
  uint32_t bid = kEmptyId;
  if (p < n) {
    double s = 0.0;
    for (int j = 0; j < d; ++j) {
      const double t = (double)X[p * d + j] - sum[j] / (double)n;
      s += t * t;
    }
    best = s;
    bid = (uint32_t)p;
  }
  sd[threadIdx.x] = best;
  si[threadIdx.x] = bid;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double o = sd[threadIdx.x + w];
      const uint32_t oi = si[threadIdx.x + w];
      if (o < sd[threadIdx.x] || (o == sd[threadIdx.x] && oi < si[threadIdx.x])) {
        sd[threadIdx.x] = o;
        si[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    bd[blockIdx.x] = sd[0];
    bi[blockIdx.x] = si[0];
  }
}

__global__ void __launch_bounds__(256) argmin_kernel(const double *bd, const uint32_t *bi,
                                                     int64_t nb, uint32_t *out) {
  __shared__ double sd[256];
  __shared__ uint32_t si[256];
  double best = INFINITY;
  uint32_t bid = kEmptyId;
  for (int64_t i = threadIdx.x; i < nb; i += 256) {
    if (bd[i] < best || (bd[i] == best && bi[i] < bid)) {
      best = bd[i];
      bid = bi[i];
    }
  }
  sd[threadIdx.x] = best;
  si[threadIdx.x] = bid;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double o = sd[threadIdx.x + w];
      const uint32_t oi = si[threadIdx.x + w];
      if (o < sd[threadIdx.x] || (o == sd[threadIdx.x] && oi < si[threadIdx.x])) {
        sd[threadIdx.x] = o;
        si[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = si[0];
}

// tmp: d + 2 * ceil(n/256) doubles
hipError_t launch_start_node(const Index &I, double *tmp, uint32_t *out, hipStream_t s) {
  const int64_t nb = (I.n + 255) / 256;
  double *sum = tmp;
  double *bd = tmp + I.d;
  uint32_t *bi = reinterpret_cast<uint32_t *>(bd + nb);
  hipError_t e = hipMemsetAsync(sum, 0, sizeof(double) * I.d, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)((I.n + 1023) / 1024)), dim3(256), 0, s, I.xf(),
                     I.n, I.d, sum);
  hipLaunchKernelGGL(center_dist_kernel, dim3((unsigned)nb), dim3(256), 0, s, I.xf(), I.n, I.d, sum,
                     bd, bi);
  hipLaunchKernelGGL(argmin_kernel, dim3(1), dim3(256), 0, s, bd, bi, nb, out);
  return hipGetLastError();
}

}  // namespace pipnn
