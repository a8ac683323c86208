// Device helpers shared by the kmx kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kmx {

// float -> bfloat16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  uint32_t r = 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)((u + r) >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t b) {
  return __uint_as_float(((uint32_t)b) << 16);
}

// Non-negative double -> float rounded toward +inf.
__device__ __forceinline__ float f64_to_f32_up(double x) {
  float f = (float)x;
  if ((double)f < x) f = __uint_as_float(__float_as_uint(f) + 1u);
  return f;
}

// Non-negative double -> float rounded toward zero (a lower bound).
__device__ __forceinline__ float f64_to_f32_down(double x) {
  if (!(x > 0.0)) return 0.0f;
  float f = (float)x;
  if ((double)f > x) f = __uint_as_float(__float_as_uint(f) - 1u);
  return f;
}

// Distance bounds from squared-distance bounds computed in FP64: sqrt of an
// upper (lower) bound, rounded up (down), with a relative margin of 2^-40 for
// the FP64 roundings of the bound's own arithmetic.
__device__ __forceinline__ float dist_up(double s2) {
  if (!(s2 > 0.0)) return 0.0f;
  if (!(s2 < 1e300)) return __builtin_inff();
  return f64_to_f32_up(sqrt(s2 * (1.0 + 0x1p-40)) * (1.0 + 0x1p-40));
}
__device__ __forceinline__ float dist_down(double s2) {
  if (!(s2 > 0.0)) return 0.0f;
  if (!(s2 < 1e300)) return __builtin_inff();
  return f64_to_f32_down(sqrt(s2 * (1.0 - 0x1p-40)) * (1.0 - 0x1p-40));
}

// Butterfly sums over the 64 lanes of a wave.  IEEE addition commutes, so
// every lane ends with the same bits and the order is fixed.
__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

__device__ __forceinline__ float wave_sum_f32(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Reductions over the 16 lanes of a DPP row (lanes 16r .. 16r + 15) with
// data-parallel-primitive moves: swaps of neighbours (quad permutations
// [1,0,3,2] and [2,3,0,1]), then the half-row and row mirrors.  Every lane
// of the row ends with the same bits (each step adds a value to its partner's
// value; addition and max are commutative).
__device__ __forceinline__ int dpp_xor1(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);
}
__device__ __forceinline__ int dpp_xor2(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);
}
__device__ __forceinline__ int dpp_half_mirror(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false);
}
__device__ __forceinline__ int dpp_mirror(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, false);
}
__device__ __forceinline__ float row16_sum(float v) {
  v += __int_as_float(dpp_xor1(__float_as_int(v)));
  v += __int_as_float(dpp_xor2(__float_as_int(v)));
  v += __int_as_float(dpp_half_mirror(__float_as_int(v)));
  v += __int_as_float(dpp_mirror(__float_as_int(v)));
  return v;
}
__device__ __forceinline__ unsigned row16_max(unsigned v) {
  v = max(v, (unsigned)dpp_xor1((int)v));
  v = max(v, (unsigned)dpp_xor2((int)v));
  v = max(v, (unsigned)dpp_half_mirror((int)v));
  v = max(v, (unsigned)dpp_mirror((int)v));
  return v;
}

// Error-free transformations (Knuth's TwoSum; FMA-based product).
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void two_prod(float a, float b, float& p, float& e) {
  p = a * b;
  e = __builtin_fmaf(a, b, -p);
}

// Accumulates the exact square of (x - c) into the double-float pair (s, e):
// the difference is split exactly by TwoSum, its square by TwoProd.
__device__ __forceinline__ void df_acc_sqdiff(float x, float c, float& s, float& e) {
  float dh, dl;
  two_sum(x, -c, dh, dl);
  float p, pe;
  two_prod(dh, dh, p, pe);
  pe = __builtin_fmaf(2.0f * dh, dl, pe);
  float t, te;
  two_sum(s, p, t, te);
  s = t;
  e += te + pe;
}

// Combines double-float partials across groups of G lanes (G = 64: the whole
// wave), fixed order, the same bits on every lane of a group.
template <int G = 64>
__device__ __forceinline__ void wave_sum_df(float& s, float& e) {
#pragma unroll
  for (int m = G / 2; m >= 1; m >>= 1) {
    float so = __shfl_xor(s, m, 64);
    float eo = __shfl_xor(e, m, 64);
    // symmetric in (self, other) so both partners hold identical bits
    float lo_s = fminf(s, so), hi_s = fmaxf(s, so);
    float t, te;
    two_sum(hi_s, lo_s, t, te);
    float el = fminf(e, eo), eh = fmaxf(e, eo);
    s = t;
    e = (eh + el) + te;
  }
}

// Normalizes a double-float so that (hi, lo) compare lexicographically.
__device__ __forceinline__ void df_norm(float s, float e, float& hi, float& lo) {
  hi = s + e;
  lo = e - (hi - s);
}

__device__ __forceinline__ bool df_less(float h1, float l1, float h2, float l2) {
  return h1 < h2 || (h1 == h2 && l1 < l2);
}

}  // namespace kmx
