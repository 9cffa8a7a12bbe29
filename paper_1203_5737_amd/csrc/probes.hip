// Measurement probes: the ceilings an SpMV on this GPU is held against.
// They are not part of the SpMV path; the benchmark times them beside it.
//   argcsr_probe_read    streams a buffer once (16-byte non-temporal loads,
//                        contiguous per wave) -- the achievable read
//                        bandwidth for the format bytes of a matrix;
//   argcsr_probe_gather  reads an index stream (e.g. the column array of a
//                        converted matrix) and gathers x[index] for every
//                        index >= 0 -- the rate of the random x gathers
//                        alone, with all of a tile's gathers in flight.
// Each wave folds what it read into one value so that no load is dead, and
// writes it to sink[wave].
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.hpp"

namespace argcsr {
namespace {

constexpr int kProbeBlock = 256;
constexpr int kProbeWaves = kProbeBlock / 64;
constexpr int kReadUnroll = 4;          // 16-byte loads in flight per lane
constexpr int kGatherSteps = 8;         // indices per lane per tile
constexpr int32_t kBufferWord3 = 0x00020000;
typedef int32_t v4i __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kProbeBlock) void probe_read_kernel(const v4i* __restrict__ p,
                                                                 int64_t n16,
                                                                 double* __restrict__ sink) {
  const int64_t lanes = int64_t(gridDim.x) * kProbeBlock;
  const int64_t t = int64_t(blockIdx.x) * kProbeBlock + threadIdx.x;
  uint32_t acc = 0;
  for (int64_t i = t; i < n16; i += lanes * kReadUnroll) {
    v4i v[kReadUnroll];
#pragma unroll
    for (int u = 0; u < kReadUnroll; ++u) {
      const int64_t k = i + u * lanes;
      v[u] = k < n16 ? __builtin_nontemporal_load(p + k) : v4i{0, 0, 0, 0};
    }
#pragma unroll
    for (int u = 0; u < kReadUnroll; ++u) acc ^= uint32_t(v[u].x ^ v[u].y ^ v[u].z ^ v[u].w);
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) acc ^= uint32_t(__shfl_xor(int(acc), d, 64));
  if ((threadIdx.x & 63) == 0) sink[blockIdx.x * kProbeWaves + (threadIdx.x >> 6)] = double(acc);
}

template <typename A>
__global__ __launch_bounds__(kProbeBlock) void probe_gather_kernel(const int32_t* __restrict__ idx,
                                                                   int64_t n, const A* __restrict__ x,
                                                                   int32_t n_x,
                                                                   double* __restrict__ sink) {
  const int lane = lane_id();
  const int64_t wave = (int64_t(blockIdx.x) * kProbeBlock + threadIdx.x) >> 6;
  const int64_t n_waves = int64_t(gridDim.x) * kProbeWaves;
  const auto rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<A*>(x), int16_t(0),
                                                      int32_t(uint32_t(n_x) * sizeof(A)),
                                                      kBufferWord3);
  const int64_t tiles = (n + 64 * kGatherSteps - 1) / (64 * kGatherSteps);
  double acc = 0.0;
  for (int64_t tl = wave; tl < tiles; tl += n_waves) {
    const int64_t base = tl * 64 * kGatherSteps + lane;
    int32_t c[kGatherSteps];
#pragma unroll
    for (int u = 0; u < kGatherSteps; ++u) {
      const int64_t k = base + int64_t(u) * 64;
      c[u] = k < n ? __builtin_nontemporal_load(idx + k) : -1;
    }
    A v[kGatherSteps];
#pragma unroll
    for (int u = 0; u < kGatherSteps; ++u) {
      // an index < 0 asks past the end of x: the buffer range check gives 0
      const uint32_t off = uint32_t(c[u]) * uint32_t(sizeof(A));
      if constexpr (sizeof(A) == 8)
        v[u] = __builtin_bit_cast(A, __builtin_amdgcn_raw_buffer_load_b64(rsrc, off, 0, 0));
      else
        v[u] = __builtin_bit_cast(A, __builtin_amdgcn_raw_buffer_load_b32(rsrc, off, 0, 0));
    }
#pragma unroll
    for (int u = 0; u < kGatherSteps; ++u) acc += double(v[u]);
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
  if (lane == 0) sink[blockIdx.x * kProbeWaves + (threadIdx.x >> 6)] = acc;
}

uint32_t probe_blocks(int64_t work_per_block) {
  return uint32_t(std::max<int64_t>(1, std::min<int64_t>(ARGCSR_PROBE_SINK / kProbeWaves,
                                                         work_per_block)));
}

}  // namespace
}  // namespace argcsr

extern "C" int argcsr_probe_read(const void* buf, int64_t bytes, double* sink, void* stream) {
  using namespace argcsr;
  clear_error();
  if (bytes < 0 || (bytes > 0 && (!buf || !sink)))
    return fail(ARGCSR_EINVAL, "bad probe arguments");
  if ((reinterpret_cast<uintptr_t>(buf) & 15) != 0)
    return fail(ARGCSR_EINVAL, "buffer must be 16-byte aligned");
  const int64_t n16 = bytes / 16;                  // a tail of < 16 bytes is not read
  if (n16 == 0) return ARGCSR_OK;
  const uint32_t blocks = probe_blocks((n16 + kProbeBlock * kReadUnroll - 1) /
                                       (kProbeBlock * kReadUnroll));
  probe_read_kernel<<<blocks, kProbeBlock, 0, static_cast<hipStream_t>(stream)>>>(
      static_cast<const v4i*>(buf), n16, sink);
  ARGCSR_HIP(hipGetLastError());
  return ARGCSR_OK;
}

extern "C" int argcsr_probe_gather(const int32_t* idx, int64_t n, const void* x, int32_t n_x,
                                   int32_t x_bytes, double* sink, void* stream) {
  using namespace argcsr;
  clear_error();
  if (n < 0 || n_x < 0 || (x_bytes != 4 && x_bytes != 8) ||
      (n > 0 && (!idx || !x || !sink)))
    return fail(ARGCSR_EINVAL, "bad probe arguments");
  if (int64_t(n_x) * x_bytes > 0xFFFFFFF0ll)
    return fail(ARGCSR_EUNSUPPORTED, "x exceeds the 32-bit gather range");
  if (n == 0) return ARGCSR_OK;
  const int64_t tiles = (n + 64 * kGatherSteps - 1) / (64 * kGatherSteps);
  const uint32_t blocks = probe_blocks((tiles + kProbeWaves - 1) / kProbeWaves);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (x_bytes == 8)
    probe_gather_kernel<double><<<blocks, kProbeBlock, 0, s>>>(idx, n, static_cast<const double*>(x),
                                                               n_x, sink);
  else
    probe_gather_kernel<float><<<blocks, kProbeBlock, 0, s>>>(idx, n, static_cast<const float*>(x),
                                                              n_x, sink);
  ARGCSR_HIP(hipGetLastError());
  return ARGCSR_OK;
}
