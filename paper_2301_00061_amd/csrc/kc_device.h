// kc_device.h -- device helpers for the gfx950 kernels: median-of-three,
// order-preserving float keys and wavefront (64-lane) reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace kcd {

constexpr int WAVE = 64;

// v_med3_f32: the clamp mid{lo, x, hi} of the closed form for beta_s^k.
__device__ __forceinline__ float med3(float a, float b, float c) {
  return __builtin_amdgcn_fmed3f(a, b, c);
}

// Order-preserving map float -> uint32 (total order of non-NaN floats), so
// integer min/max atomics give float min/max.
__device__ __forceinline__ uint32_t ford(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float fdec(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}
constexpr uint32_t FORD_POS_INF = 0xFF800000u;  // ford(+inf)
constexpr uint32_t FORD_NEG_INF = 0x007FFFFFu;  // ford(-inf)

// Packed (value, index) keys. For a non-negative float v the bit pattern is
// monotone in v, so max over (bits(v) << 32 | ~idx) gives the largest value
// and, among equal values, the lowest index; min over (bits(v) << 32 | idx)
// gives the smallest value and the lowest index.
__device__ __forceinline__ uint64_t key_max(float v, uint32_t idx) {
  return v < 0.0f ? 0ull : ((uint64_t)__float_as_uint(v) << 32) | (uint64_t)(~idx);
}
__device__ __forceinline__ uint64_t key_min(float v, uint32_t idx) {
  return idx == 0xffffffffu ? ~0ull : ((uint64_t)__float_as_uint(v) << 32) | (uint64_t)idx;
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
  uint32_t lo = __shfl_xor((unsigned)(v & 0xffffffffu), m);
  uint32_t hi = __shfl_xor((unsigned)(v >> 32), m);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    uint64_t w = shfl_xor_u64(v, m);
    v = w > v ? w : v;
  }
  return v;
}
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    uint64_t w = shfl_xor_u64(v, m);
    v = w < v ? w : v;
  }
  return v;
}
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    uint32_t w = __shfl_xor(v, m);
    v = w < v ? w : v;
  }
  return v;
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    uint32_t w = __shfl_xor(v, m);
    v = w > v ? w : v;
  }
  return v;
}
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
  return v;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

// Workgroup index remapped so that consecutive logical units land on the same
// XCD (the dispatcher assigns workgroup b to XCD b % 8): units that read the
// same samples then share that XCD's L2.
__device__ __forceinline__ int xcd_unit(int b, int nb) {
  if ((nb & 7) != 0) return b;
  return (b & 7) * (nb >> 3) + (b >> 3);
}

}  // namespace kcd
