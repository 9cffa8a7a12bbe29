// Value storage types: how a stored value is read into the accumulation type,
// and how an FP64 input value is rounded into storage (nearest, ties to even,
// directly from FP64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "argcsr.h"

namespace argcsr {

template <int DT> struct Val;

template <> struct Val<ARGCSR_F64> {
  using storage = double;
  using acc = double;
  __device__ static acc load(storage v) { return v; }
  __device__ static storage from_f64(double d) { return d; }
};

template <> struct Val<ARGCSR_F32> {
  using storage = float;
  using acc = float;
  __device__ static acc load(storage v) { return v; }
  __device__ static storage from_f64(double d) { return (float)d; }  // v_cvt_f32_f64, RNE
};

// FP64 -> FP32 rounded to odd: truncate toward zero, then set the last bit
// if the truncation was inexact.  A second rounding to nearest-even into a
// format with at least two fewer significand bits then equals the direct
// nearest-even rounding of the FP64 value (Boldo & Melquiond, "When double
// rounding is odd", 2005).
__device__ __forceinline__ uint32_t f64_to_f32_round_odd_bits(double d) {
  float f = (float)d;
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return u;            // NaN
  if (__builtin_fabs((double)f) > __builtin_fabs(d)) u -= 1u; // round-to-nearest overshot: step toward 0
  const float t = __builtin_bit_cast(float, u);
  if ((double)t != d) u |= 1u;                                // sticky bit
  return u;
}

template <> struct Val<ARGCSR_BF16> {
  using storage = uint16_t;
  using acc = float;
  __device__ static acc load(storage v) {
    return __builtin_bit_cast(float, uint32_t(v) << 16);
  }
  __device__ static storage from_f64(double d) {
    const uint32_t u = f64_to_f32_round_odd_bits(d);
    if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x0040u);  // quiet NaN
    const uint32_t lsb = (u >> 16) & 1u;
    return uint16_t((u + 0x7fffu + lsb) >> 16);                                // nearest-even
  }
};

template <> struct Val<ARGCSR_F16> {
  using storage = uint16_t;
  using acc = float;
  __device__ static acc load(storage v) {
    return (float)__builtin_bit_cast(_Float16, v);
  }
  __device__ static storage from_f64(double d) {
    const float f = __builtin_bit_cast(float, f64_to_f32_round_odd_bits(d));
    return __builtin_bit_cast(uint16_t, (_Float16)f);   // v_cvt_f16_f32, nearest-even
  }
};

}  // namespace argcsr
