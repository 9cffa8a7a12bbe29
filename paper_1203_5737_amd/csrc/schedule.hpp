// Launch-schedule constants shared by host planning and the SpMV kernels.
#pragma once

#include <cstdint>

#include "argcsr.h"

namespace argcsr {

constexpr int kSpmvWaves = 4;   // waves per SpMV workgroup
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

// Runs (argcsr_run_info): group g opens a run iff it is the first group, it
// or its predecessor is heavy, or its offset lies in another window of
// ARGCSR_RUN_SLOTS slots than its predecessor's.  One wave takes a run: its
// slots are contiguous, so its chunk loads cover several short groups at once.
constexpr int32_t kRunSlots = ARGCSR_RUN_SLOTS;
static_assert(kRunSlots == kLoadSteps * 64, "a run window is one batch of loads");
__host__ __device__ constexpr bool opens_run(int32_t g, int32_t offset_prev, int32_t chunk_prev,
                                             int32_t offset, int32_t chunk, int32_t heavy_chunk) {
  return g == 0 || chunk > heavy_chunk || chunk_prev > heavy_chunk ||
         offset / kRunSlots != offset_prev / kRunSlots;
}

}  // namespace argcsr
