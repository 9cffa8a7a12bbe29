// Shared helpers of libargcsr: status/error reporting, HIP call checking,
// and wave-level device primitives.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "argcsr.h"

namespace argcsr {

// Records a message for argcsr_last_error() and returns `code`.
int fail(int code, const char* fmt, ...);
void clear_error();

#define ARGCSR_HIP(call)                                                       \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess)                                                      \
      return ::argcsr::fail(ARGCSR_EHIP, "%s failed: %s (%s:%d)", #call,       \
                            hipGetErrorString(e_), __FILE__, __LINE__);        \
  } while (0)

// XCD-aware block remap: hardware dispatches consecutive workgroups round-robin
// over the 8 XCDs; give every XCD a contiguous range of logical blocks so that
// neighbouring groups (which gather neighbouring x lines) share one L2.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t nb) {
  constexpr uint32_t kXcd = 8;
  const uint32_t q = nb / kXcd, r = nb % kXcd;
  const uint32_t x = b % kXcd, i = b / kXcd;
  return x * q + (x < r ? x : r) + i;
}

// Orders this wave's LDS accesses (a wave executes its LDS operations in
// issue order; the fences stop the compiler from moving accesses across).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

template <typename T>
__device__ __forceinline__ T wave_uniform(T v) {
  return __builtin_amdgcn_readfirstlane(v);
}

// Inclusive wave-wide prefix sum of an int (Hillis-Steele over 64 lanes).
__device__ __forceinline__ int wave_inclusive_scan(int v) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const int t = __shfl_xor(v, d, 64);
    v = t > v ? t : v;
  }
  return v;
}

}  // namespace argcsr
