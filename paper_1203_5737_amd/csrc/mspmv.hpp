// y_m = A_m x_m for a set of matrices in ONE launch, driven by per-matrix
// prefix tables instead of a per-group work list: the first total_heavy
// workgroups take heavy item h = heavy_groups_m[h - heavy_begin[m]] each,
// and then wave i of the rest takes group i - group_begin[m] of the matrix m
// with group_begin[m] <= i < group_begin[m+1].  The prefix tables are staged
// in LDS once per workgroup and searched there.  Used by the serving loop,
// whose set of matrices changes from step to step: the grid is sized on the
// host for each step, so no wave takes work from a shared counter.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"
#include "schedule.hpp"
#include "spmv_kernels.hpp"

namespace argcsr {

constexpr int kMaxLaunchMats = 512;   // matrices per multi-matrix launch

struct MatWork {
  const argcsr_group_info* groups;
  const int32_t* tm;
  const int32_t* columns;
  const void* values;
  const int32_t* heavy;               // heavy group indices (may be NULL if n_heavy == 0)
  const void* x;
  void* y;
  int32_t block_dim;
  int32_t n_cols;
  int32_t serial;                     // gather mode (serial_gathers)
  int32_t heavy_chunk;                // groups with chunk_size above are in `heavy`
  int32_t group_begin;                // prefix over the launch's matrices
  int32_t heavy_begin;
};

// largest m in [0, n) with begin[m] <= i (begin[0] == 0, begin non-decreasing)
__device__ __forceinline__ int32_t find_owner(const int32_t* begin, int32_t n, int32_t i) {
  int32_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (begin[mid] <= i) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// All matrices of a launch share T = 64*W (the server converts with one
// block size), so each kernel instance holds one group routine only.
template <int DT, int W, int U>
__global__ __launch_bounds__(kSpmvWaves * 64) void mspmv_kernel(
    const MatWork* __restrict__ mw, int32_t n_mats, int32_t total_groups, int32_t total_heavy) {
  using Vt = Val<DT>;
  using S = typename Vt::storage;
  using A = typename Vt::acc;
  __shared__ int32_t gbeg[kMaxLaunchMats];
  __shared__ int32_t hbeg[kMaxLaunchMats];
  __shared__ int32_t ends[kSpmvWaves][64 * W];
  __shared__ A part_mem[kSpmvWaves - 1][64 * W];
  for (int32_t m = threadIdx.x; m < n_mats; m += blockDim.x) {
    gbeg[m] = mw[m].group_begin;
    hbeg[m] = mw[m].heavy_begin;
  }
  __syncthreads();
  const int wv = wave_uniform(int(threadIdx.x >> 6));
  const int32_t b = int32_t(blockIdx.x);

  if (b < total_heavy) {                            // a heavy group, the whole workgroup
    const int32_t m = find_owner(hbeg, n_mats, b);
    const MatWork& w = mw[m];
    const argcsr_group_info gi = w.groups[w.heavy[b - hbeg[m]]];
    spmv_group_split<DT, W, U>(gi.first_row, gi.size, gi.offset, gi.chunk_size, w.tm, w.columns,
                               static_cast<const S*>(w.values),
                               XGather<A>(static_cast<const A*>(w.x), w.n_cols), w.serial != 0,
                               static_cast<A*>(w.y), ends[0], part_mem, wv);
    return;
  }
  // the other groups, one wave each, every XCD a contiguous range of them
  const uint32_t nb = gridDim.x - uint32_t(total_heavy);
  const int32_t i = int32_t(xcd_remap(uint32_t(b - total_heavy), nb)) * kSpmvWaves + wv;
  if (i >= total_groups) return;
  const int32_t m = find_owner(gbeg, n_mats, i);
  const MatWork& w = mw[m];
  const argcsr_group_info gi = w.groups[i - gbeg[m]];
  if (gi.chunk_size > w.heavy_chunk) return;        // done by a heavy workgroup
  spmv_group<DT, W, U>(gi.first_row, gi.size, gi.offset, gi.chunk_size, w.tm, w.columns,
                       static_cast<const S*>(w.values),
                       XGather<A>(static_cast<const A*>(w.x), w.n_cols), w.serial != 0,
                       static_cast<A*>(w.y), ends[wv]);
}

}  // namespace argcsr
