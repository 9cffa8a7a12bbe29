// Batched SpMV state (the opaque argcsr_batch of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "argcsr.h"

namespace argcsr {

// One matrix of a batch as the persistent kernel sees it.
struct BatchMat {
  const argcsr_group_info* groups;
  const int32_t* tm;
  const int32_t* columns;
  const void* values;
  const void* x;
  void* y;
  int32_t block_dim;
  int32_t n_groups;
  int32_t n_cols;
  int32_t serial;            // gather mode (serial_gathers)
};

}  // namespace argcsr

struct argcsr_batch {
  int32_t n_mats = 0;
  int32_t dtype = 0;
  int32_t n_items = 0;       // groups processed by one wave
  int32_t n_heavy = 0;       // groups processed by a whole workgroup
  int32_t grid = 0;          // persistent workgroups
  argcsr::BatchMat* d_mats = nullptr;
  int2* d_items = nullptr;   // (matrix, group), longest first
  int2* d_heavy = nullptr;
  void* queue = nullptr;     // two int32 counters
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hipEvent_t last = nullptr;  // recorded after every launch; destroy waits for it
  bool launched = false;
};
