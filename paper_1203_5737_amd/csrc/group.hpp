// Conversion step 1 (grouping) on the GPU: binary lifting over the
// next-group-start function of the rows (group.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "argcsr.h"

namespace argcsr {

// The grouping of one matrix while its jump tables live (stream-ordered
// scratch on the stream given to build).  build() validates row_ptr on the
// device and counts the groups (synchronous: it reads the count back);
// write() enqueues the group table (first_row, size; offset and chunk size
// 0) into `groups`, which holds n_groups entries; release() frees the
// tables in stream order.
struct DeviceGrouping {
  int32_t n_rows = 0;
  int32_t n_groups = 0;
  int32_t levels_n = 0;
  int64_t stride = 0;
  int32_t* levels = nullptr;
  hipStream_t stream = nullptr;

  // format ARGCSR_FORMAT_RG: groups of block_dim rows (no nonzero budget);
  // region_desired (host, checked by the caller): a desiredChunkSize per
  // region of region_rows rows, taken from the region of a group's first row
  int build(int32_t n, const int32_t* row_ptr, int32_t block_dim, int32_t desired,
            int32_t format, hipStream_t s, int32_t region_rows = 0,
            const int32_t* region_desired = nullptr);
  int write(argcsr_group_info* groups) const;
  void release();
  ~DeviceGrouping() { release(); }
};

// Stream-ordered device allocation from the library's own memory pool on
// the current device (created on first use, one per device, with a release
// threshold that keeps freed memory in the pool: repeated conversions reuse
// their scratch instead of mapping it again at every synchronisation).  The
// pool holds at most the largest scratch any call needed until the process
// ends.  Free with hipFreeAsync.
int scratch_alloc_async(void** p, size_t bytes, hipStream_t s);

// Device scratch allocated and freed in stream order (scratch_alloc_async /
// hipFreeAsync): work queued on the stream may still use it after the
// owner goes out of scope, and concurrent conversions never share it.
struct StreamScratch {
  void* ptr = nullptr;
  hipStream_t stream = nullptr;
  int alloc(size_t bytes, hipStream_t s);
  ~StreamScratch() {
    if (ptr) (void)hipFreeAsync(ptr, stream);
  }
};

}  // namespace argcsr
