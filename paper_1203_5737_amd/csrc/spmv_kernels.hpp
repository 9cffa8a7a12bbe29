// Device routine for one ARG-CSR group, shared by the single-matrix kernel
// and the batched work-queue kernel.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"
#include "values.hpp"

namespace argcsr {

constexpr int kSpmvWaves = 4;   // waves per workgroup; each wave owns one group at a time

// Computes the rows of one group with the calling wave (Sec. 4 semantics).
//   W      sub-blocks per lane: the group has T = 64*W chunks
//   U      steps j loaded ahead per sub-block (memory-level parallelism)
//   ends   this wave's LDS table of T ints (reused group after group)
template <int DT, int W, int U>
__device__ __forceinline__ void spmv_group(
    int32_t first, int32_t size, int32_t offset, int32_t c,
    const int32_t* __restrict__ tm, const int32_t* __restrict__ columns,
    const typename Val<DT>::storage* __restrict__ values,
    const typename Val<DT>::acc* __restrict__ x, typename Val<DT>::acc* __restrict__ y,
    int32_t* ends) {
  using Vt = Val<DT>;
  using S = typename Vt::storage;
  using A = typename Vt::acc;
  constexpr int T = 64 * W;
  const int lane = lane_id();

  // ---- row-end mask: chunk tm[l]-1 closes row l --------------------------
  wave_lds_sync();
#pragma unroll
  for (int w = 0; w < W; ++w) ends[w * 64 + lane] = 0;
  wave_lds_sync();
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const int l = w * 64 + lane;
    if (l < size) {
      const uint32_t e = uint32_t(tm[first + l] - 1);
      if (e < uint32_t(T)) ends[e] = 1;
    }
  }
  wave_lds_sync();
  uint64_t emask[W];
#pragma unroll
  for (int w = 0; w < W; ++w) emask[w] = __ballot(ends[w * 64 + lane] != 0);
  const int n_mapped = tm[first + size - 1];    // chunks in use; the rest are free

  // ---- chunk partial sums ---------------------------------------------------
  A acc[W];
  bool alive[W];
#pragma unroll
  for (int w = 0; w < W; ++w) { acc[w] = A(0); alive[w] = true; }
  const int32_t* cb = columns + offset + lane;
  const S* vb = values + offset + lane;
  for (int j = 0; j < c; j += U) {
    int32_t cc[U][W];
    S vv[U][W];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int w = 0; w < W; ++w) {
        if (j + u < c) {
          cc[u][w] = cb[(j + u) * T + w * 64];
          vv[u][w] = vb[(j + u) * T + w * 64];
        } else {
          cc[u][w] = -1;
          vv[u][w] = S(0);
        }
      }
    }
    bool any = false;
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int w = 0; w < W; ++w) {
        alive[w] = alive[w] && (cc[u][w] >= 0);
        if (alive[w]) acc[w] = __builtin_fma(Vt::load(vv[u][w]), x[cc[u][w]], acc[w]);
      }
    }
#pragma unroll
    for (int w = 0; w < W; ++w) any |= alive[w];
    if (__ballot(any) == 0) break;                // every chunk reached its padding
  }

  // ---- row sums: segmented scan over lanes, carried across sub-blocks ------
  int rows_before = 0;
  A carry = A(0);
  bool carry_on = false;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const uint64_t E = emask[w];
    const uint64_t below = E & ((uint64_t(1) << lane) - 1);
    const int seg_start = below ? 64 - __clzll((long long)below) : 0;
    const int dist = (w * 64 + lane < n_mapped) ? lane - seg_start : 0;
    A v = acc[w];
    for (int d = 1; d < 64; d <<= 1) {
      if (__ballot(dist >= d) == 0) break;
      const A t = __shfl_up(v, d, 64);
      if (dist >= d) v += t;
    }
    if (carry_on && below == 0) v = carry + v;
    if ((E >> lane) & 1) {
      const int row = rows_before + __popcll(below);
      if (row < size) y[first + row] = v;
    }
    rows_before += __popcll(E);
    carry = __shfl(v, 63, 64);
    carry_on = ((E >> 63) & 1) == 0;
  }
}

template <int DT, int W, int U>
__global__ __launch_bounds__(kSpmvWaves * 64) void argcsr_spmv_kernel(
    const argcsr_group_info* __restrict__ groups, int32_t n_groups,
    const int32_t* __restrict__ tm, const int32_t* __restrict__ columns,
    const typename Val<DT>::storage* __restrict__ values,
    const typename Val<DT>::acc* __restrict__ x, typename Val<DT>::acc* __restrict__ y) {
  __shared__ int32_t ends[kSpmvWaves][64 * W];
  const int wv = wave_uniform(int(threadIdx.x >> 6));
  const int g = int(xcd_remap(blockIdx.x, gridDim.x)) * kSpmvWaves + wv;
  if (g >= n_groups) return;
  const argcsr_group_info gi = groups[g];
  spmv_group<DT, W, U>(gi.first_row, gi.size, gi.offset, gi.chunk_size, tm, columns, values,
                       x, y, ends[wv]);
}

int check_matrix(const argcsr_matrix* A);

}  // namespace argcsr
