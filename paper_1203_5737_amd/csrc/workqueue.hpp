// Global work queues of the persistent multi-matrix SpMV kernels.
//
// Device-scope atomics on one address serialise far from the CUs, so the
// normal items are split into kQueues contiguous segments with a counter
// each (on separate 256-byte lines).  A wave starts on the segment of its
// own XCD (workgroups are dispatched round-robin over the 8 XCDs, so this
// also keeps neighbouring items -- and their x vectors -- on one L2) and
// moves on to the following segments once its own is drained.  Heavy items
// (whole workgroups) use one more counter.  Which wave takes which item never
// changes a result.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"

namespace argcsr {

constexpr int kQueues = 8;

struct alignas(256) QueueCounter {
  int32_t next;
  int32_t pad[63];
};

struct WorkQueues {
  QueueCounter heavy;
  QueueCounter normal[kQueues];
};

static __global__ void reset_work_queues_kernel(WorkQueues* q, int32_t count) {
  const int32_t i = int32_t(threadIdx.x);
  for (int32_t k = 0; k < count; ++k) {
    if (i == 0) q[k].heavy.next = 0;
    if (i < kQueues) q[k].normal[i].next = 0;
  }
}

// Per-wave cursor over the segments.  take() returns the first of up to
// `grab` consecutive items in [0, total) and their end, or false when every
// segment is drained.  Call with all lanes of the wave active.
struct QueueCursor {
  int home;
  int visited;
  __device__ bool take(WorkQueues* q, int32_t total, int32_t grab, int32_t* begin, int32_t* end) {
    while (visited < kQueues) {
      const int x = (home + visited) % kQueues;
      const int32_t seg_begin = int32_t(int64_t(total) * x / kQueues);
      const int32_t seg_end = int32_t(int64_t(total) * (x + 1) / kQueues);
      int32_t old = 0;
      if (lane_id() == 0) old = atomicAdd(&q->normal[x].next, grab);
      old = wave_uniform(__shfl(old, 0, 64));
      if (seg_begin + old < seg_end) {
        *begin = seg_begin + old;
        *end = seg_begin + old + grab < seg_end ? seg_begin + old + grab : seg_end;
        return true;
      }
      ++visited;
    }
    return false;
  }
};

}  // namespace argcsr
