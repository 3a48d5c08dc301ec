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

// Wavefront reductions on VALU lane exchanges instead of LDS permutes
// (callers run them with all 64 lanes active). DPP controls of the GFX9
// encoding: quad_perm [1,0,3,2] and [2,3,0,1] exchange lanes 1 and 2 apart;
// row_half_mirror and row_mirror then pair the two uniform halves of each
// group of 8 and 16 lanes; row_bcast:15 / row_bcast:31 carry lane 15 of a
// row into the next row (rows 1 and 3) and lane 31 into rows 2 and 3, so
// lane 63 ends with the whole wavefront's value.
constexpr int DPP_XOR1 = 0xB1, DPP_XOR2 = 0x4E, DPP_HALF_MIRROR = 0x141, DPP_MIRROR = 0x140,
              DPP_BCAST15 = 0x142, DPP_BCAST31 = 0x143;

// v moved by DPP control CTRL; rows outside ROW_MASK receive `old`.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t old, uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROW_MASK, 0xf, false);
}

template <class Op>
__device__ __forceinline__ uint32_t wave_reduce_u32(uint32_t v, uint32_t ident, Op op) {
  v = op(v, dpp_u32<DPP_XOR1>(ident, v));
  v = op(v, dpp_u32<DPP_XOR2>(ident, v));
  v = op(v, dpp_u32<DPP_HALF_MIRROR>(ident, v));
  v = op(v, dpp_u32<DPP_MIRROR>(ident, v));
  v = op(v, dpp_u32<DPP_BCAST15, 0xa>(ident, v));
  v = op(v, dpp_u32<DPP_BCAST31, 0xc>(ident, v));
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
  return wave_reduce_u32(v, 0xffffffffu, [](uint32_t a, uint32_t b) { return b < a ? b : a; });
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  return wave_reduce_u32(v, 0u, [](uint32_t a, uint32_t b) { return b > a ? b : a; });
}
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
  return wave_reduce_u32(v, 0u, [](uint32_t a, uint32_t b) { return a + b; });
}
// 64-bit keys: the extreme high word first, then the extreme low word among
// the lanes holding it
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
  const uint32_t hi = (uint32_t)(v >> 32), mh = wave_max_u32(hi);
  const uint32_t ml = wave_max_u32(hi == mh ? (uint32_t)v : 0u);
  return ((uint64_t)mh << 32) | ml;
}
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
  const uint32_t hi = (uint32_t)(v >> 32), mh = wave_min_u32(hi);
  const uint32_t ml = wave_min_u32(hi == mh ? (uint32_t)v : 0xffffffffu);
  return ((uint64_t)mh << 32) | ml;
}

// Minimum over aligned groups of kp lanes (kp a power of two, the same on
// every lane), every lane of a group receiving it: a butterfly whose steps of
// 4 and 8 lanes use the mirrors (the halves they pair are uniform by then)
// and whose steps of 16 and 32 lanes swap rows between two registers.
__device__ __forceinline__ float group_min(float v, int kp) {
  auto fmin_dpp = [](float x, uint32_t y) { return fminf(x, __uint_as_float(y)); };
  if (kp > 1) v = fmin_dpp(v, dpp_u32<DPP_XOR1>(__float_as_uint(v), __float_as_uint(v)));
  if (kp > 2) v = fmin_dpp(v, dpp_u32<DPP_XOR2>(__float_as_uint(v), __float_as_uint(v)));
  if (kp > 4) v = fmin_dpp(v, dpp_u32<DPP_HALF_MIRROR>(__float_as_uint(v), __float_as_uint(v)));
  if (kp > 8) v = fmin_dpp(v, dpp_u32<DPP_MIRROR>(__float_as_uint(v), __float_as_uint(v)));
  if (kp > 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = fminf(__uint_as_float(r[0]), __uint_as_float(r[1]));
  }
  if (kp > 32) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = fminf(__uint_as_float(r[0]), __uint_as_float(r[1]));
  }
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
