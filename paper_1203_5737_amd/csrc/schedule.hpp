// Launch-schedule constants shared by host planning and the SpMV kernels.
#pragma once

#include <cstdint>

namespace argcsr {

constexpr int kSpmvWaves = 4;   // waves per SpMV workgroup
// x is gathered through 32-bit buffer offsets; a column -1 must land past the end
constexpr int64_t kMaxVectorBytes = 0xFFFFFFF0ll;
constexpr int kLoadSteps = 8;   // chunk steps loaded ahead per lane (U * W)

// A group is "heavy" when one wave would need many more rounds of loads for
// it than the matrix's typical group: at least kHeavyRounds rounds of
// kLoadSteps steps, and more than kHeavyMeanFactor times the mean chunk size.
// Heavy groups are listed at conversion time, dispatched first and processed
// by all waves of a workgroup, each taking a contiguous share of the chunk
// steps; on regular matrices no group is heavy.  Block dims without a GPU
// kernel get no heavy groups.
constexpr int kHeavyRounds = 4;
constexpr int kHeavyMeanFactor = 4;
__host__ __device__ constexpr int32_t heavy_chunk_for(int32_t block_dim, int64_t n_slots,
                                                      int32_t n_groups) {
  const int32_t by_rounds = block_dim == 64 ? kHeavyRounds * kLoadSteps
                          : block_dim == 128 ? kHeavyRounds * kLoadSteps / 2
                          : block_dim == 256 ? kHeavyRounds * kLoadSteps / 4
                          : INT32_MAX;
  if (by_rounds == INT32_MAX || n_groups <= 0) return by_rounds;
  const int64_t mean_chunk = (n_slots + int64_t(n_groups) * block_dim - 1) /
                             (int64_t(n_groups) * block_dim);
  const int64_t by_mean = kHeavyMeanFactor * mean_chunk;
  return by_rounds > by_mean ? by_rounds : int32_t(by_mean < INT32_MAX ? by_mean : INT32_MAX);
}

// Gather mode of the chunk loop: serial (one gather at a time, each FMA
// right after it) for 8-byte values when the mean chunk loop spans at least
// two load batches -- there the value stream is the limit and the paced
// gathers measured faster (27-point stencil, FP64: 140 vs 149 us) -- and
// batched (all gathers of a batch in flight) otherwise (power-law rows,
// FP64: 81 vs 86 us; every FP32 case).
__host__ __device__ constexpr bool serial_gathers(int32_t value_bytes, int32_t block_dim,
                                                  int64_t n_slots, int32_t n_groups) {
  if (value_bytes != 8 || n_groups <= 0 || block_dim <= 0) return false;
  const int64_t steps_per_batch = block_dim >= kLoadSteps * 64 ? 1 : kLoadSteps * 64 / block_dim;
  const int64_t mean_chunk = n_slots / (int64_t(n_groups) * block_dim);
  return mean_chunk >= 2 * steps_per_batch;
}

}  // namespace argcsr
