// Device routines for ARG-CSR SpMV, shared by the single-matrix kernel and
// the batched work-queue kernel (Sec. 4 semantics: chunk partial sums, then
// per-row sums of the partial sums).
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"
#include "schedule.hpp"
#include "values.hpp"

namespace argcsr {

// This lane's threads-mapping entries (rows l = 64*w + lane of the group).
template <int W>
__device__ __forceinline__ void load_mapping(int32_t first, int32_t size,
                                             const int32_t* __restrict__ tm, int32_t (&tmv)[W]) {
  const int lane = lane_id();
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const int l = w * 64 + lane;
    tmv[w] = l < size ? __builtin_nontemporal_load(tm + first + l) : 0;
  }
}

// Row-end bitmask of a group: bit k of word w is set iff chunk 64*w + k is
// the last chunk of a row, i.e. k+1 == threadsMapping[l] for some row l.
// Built through this wave's LDS table `ends` (T ints) and a ballot.
template <int W>
__device__ __forceinline__ void row_end_mask(const int32_t (&tmv)[W], int32_t* ends,
                                             uint64_t (&emask)[W]) {
  constexpr int T = 64 * W;
  const int lane = lane_id();
  wave_lds_sync();
#pragma unroll
  for (int w = 0; w < W; ++w) ends[w * 64 + lane] = 0;
  wave_lds_sync();
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const uint32_t e = uint32_t(tmv[w] - 1);        // rows beyond `size` hold 0 -> skipped
    if (e < uint32_t(T)) ends[e] = 1;
  }
  wave_lds_sync();
#pragma unroll
  for (int w = 0; w < W; ++w) emask[w] = __ballot(ends[w * 64 + lane] != 0);
}

// Partial sums of this lane's W chunks over steps j in [j0, j1): value *
// x[column], stopping at a chunk's first artificial zero (column -1).
template <int DT, int W, int U>
__device__ __forceinline__ void chunk_partials(
    int32_t offset, int32_t j0, int32_t j1, const int32_t* __restrict__ columns,
    const typename Val<DT>::storage* __restrict__ values,
    const typename Val<DT>::acc* __restrict__ x, typename Val<DT>::acc (&acc)[W]) {
  using Vt = Val<DT>;
  using S = typename Vt::storage;
  constexpr int T = 64 * W;
  const int lane = lane_id();
  bool alive[W];
#pragma unroll
  for (int w = 0; w < W; ++w) { acc[w] = 0; alive[w] = true; }
  const int32_t* cb = columns + offset + lane;
  const S* vb = values + offset + lane;
  if constexpr (sizeof(S) < 8) {
    // 4- and 2-byte values: the next U steps are loaded before this batch's x
    // gathers are issued (double buffering fits the register budget)
    int32_t cc[U][W];
    S vv[U][W];
    auto load = [&](int j, int32_t (&c)[U][W], S (&v)[U][W]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
          if (j + u < j1) {   // streamed once: keep L2 for the x gathers
            c[u][w] = __builtin_nontemporal_load(cb + (j + u) * T + w * 64);
            v[u][w] = __builtin_nontemporal_load(vb + (j + u) * T + w * 64);
          } else {
            c[u][w] = -1;
            v[u][w] = S(0);
          }
        }
      }
    };
    if (j0 < j1) load(j0, cc, vv);
    for (int j = j0; j < j1; j += U) {
      int32_t nc[U][W];
      S nv[U][W];
      const bool more = j + U < j1;
      if (more) load(j + U, nc, nv);
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
      if (__ballot(any) == 0 || !more) break;     // every chunk reached its padding
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int w = 0; w < W; ++w) { cc[u][w] = nc[u][w]; vv[u][w] = nv[u][w]; }
      }
    }
  } else {
    // 8-byte values: one batch of U steps at a time (double buffering would
    // cost occupancy)
    for (int j = j0; j < j1; j += U) {
      int32_t cc[U][W];
      S vv[U][W];
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
          if (j + u < j1) {   // streamed once: keep L2 for the x gathers
            cc[u][w] = __builtin_nontemporal_load(cb + (j + u) * T + w * 64);
            vv[u][w] = __builtin_nontemporal_load(vb + (j + u) * T + w * 64);
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
      if (__ballot(any) == 0) break;              // every chunk reached its padding
    }
  }
}

// Row sums from the chunk partial sums: a segmented inclusive scan across
// lanes (segments = rows, delimited by the row-end mask), carried from one
// sub-block of 64 chunks to the next; the lane holding a row's last chunk
// writes y[first + row].  Free chunks (beyond n_mapped) take no part.
template <int DT, int W>
__device__ __forceinline__ void row_sums(int32_t first, int32_t size, int32_t n_mapped,
                                         const uint64_t (&emask)[W],
                                         const typename Val<DT>::acc (&acc)[W],
                                         typename Val<DT>::acc* __restrict__ y) {
  using A = typename Val<DT>::acc;
  const int lane = lane_id();
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
      if (row < size) __builtin_nontemporal_store(v, y + first + row);
    }
    rows_before += __popcll(E);
    carry = __shfl(v, 63, 64);
    carry_on = ((E >> 63) & 1) == 0;
  }
}

// One whole group with the calling wave.
template <int DT, int W, int U>
__device__ __forceinline__ void spmv_group(
    int32_t first, int32_t size, int32_t offset, int32_t c,
    const int32_t* __restrict__ tm, const int32_t* __restrict__ columns,
    const typename Val<DT>::storage* __restrict__ values,
    const typename Val<DT>::acc* __restrict__ x, typename Val<DT>::acc* __restrict__ y,
    int32_t* ends) {
  using A = typename Val<DT>::acc;
  int32_t tmv[W];
  load_mapping<W>(first, size, tm, tmv);           // in flight with the first chunk loads
  const int32_t n_mapped = tm[first + size - 1];    // chunks in use; the rest are free
  A acc[W];
  chunk_partials<DT, W, U>(offset, 0, c, columns, values, x, acc);
  uint64_t emask[W];
  row_end_mask<W>(tmv, ends, emask);
  row_sums<DT, W>(first, size, n_mapped, emask, acc, y);
}

// One run of groups (argcsr_run_info) with the calling wave.  The run's
// slots are contiguous, so its steps are loaded U at a time whatever group
// they belong to: one batch of loads covers several short groups instead of
// one wave per short group waiting on its own few loads.  Each chunk's
// partial sum still runs over its own group's steps in order, stopping at
// its first artificial zero, and each group's row sums are formed as in
// spmv_group, so the results are bitwise those of spmv_group.  `stage` is
// this wave's LDS copy of the run's threads mapping (kRunSlots ints).
template <int DT, int W, int U>
__device__ __forceinline__ void spmv_run(
    const argcsr_run_info& run, const argcsr_run_info& next,
    const argcsr_group_info* __restrict__ groups, const int32_t* __restrict__ tm,
    const int32_t* __restrict__ columns, const typename Val<DT>::storage* __restrict__ values,
    const typename Val<DT>::acc* __restrict__ x, typename Val<DT>::acc* __restrict__ y,
    int32_t* ends, int32_t* stage) {
  using Vt = Val<DT>;
  using S = typename Vt::storage;
  using A = typename Vt::acc;
  constexpr int T = 64 * W;
  constexpr int kStage = kRunSlots / 64;
  static_assert(kRunSlots % T == 0 && kRunSlots / T <= 64, "run window");
  const int lane = lane_id();
  const int32_t n_groups = next.first_group - run.first_group;   // <= kRunSlots / T
  const int32_t row0 = run.first_row, n_rows = next.first_row - run.first_row;   // <= kRunSlots
  const int32_t n_steps = (next.offset - run.offset) / T;

  // the run's group table, group i in lane i; lanes beyond hold zeros
  int32_t g_first = 0, g_size = 0, g_chunk = 0;
  if (lane < n_groups) {
    const argcsr_group_info gi = groups[run.first_group + lane];
    g_first = gi.first_row;
    g_size = gi.size;
    g_chunk = gi.chunk_size;
  }
  int32_t tmr[kStage];
#pragma unroll
  for (int m = 0; m < kStage; ++m) {
    const int32_t i = m * 64 + lane;
    tmr[m] = i < n_rows ? __builtin_nontemporal_load(tm + row0 + i) : 0;
  }

  const int32_t* cb = columns + run.offset + lane;
  const S* vb = values + run.offset + lane;
  int32_t cc[U][W];
  S vv[U][W];
  auto load = [&](int32_t j, int32_t (&c)[U][W], S (&v)[U][W]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int w = 0; w < W; ++w) {
        if (j + u < n_steps) {   // streamed once: keep L2 for the x gathers
          c[u][w] = __builtin_nontemporal_load(cb + (j + u) * T + w * 64);
          v[u][w] = __builtin_nontemporal_load(vb + (j + u) * T + w * 64);
        } else {
          c[u][w] = -1;
          v[u][w] = S(0);
        }
      }
    }
  };
  // 4- and 2-byte values: the next batch is loaded before this batch's
  // products are summed (double buffering fits the register budget; for
  // 8-byte values it would cost occupancy)
  constexpr bool kDouble = sizeof(S) < 8;
  load(0, cc, vv);
#pragma unroll
  for (int m = 0; m < kStage; ++m)
    if (m * 64 + lane < n_rows) stage[m * 64 + lane] = tmr[m];
  wave_lds_sync();

  // row sums of run group g from the chunk partial sums in acc
  auto finish = [&](int32_t g, const A (&acc)[W]) {
    const int32_t first = __builtin_amdgcn_readlane(g_first, g);
    const int32_t size = __builtin_amdgcn_readlane(g_size, g);
    const int32_t base = first - row0;
    int32_t tmv[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const int l = w * 64 + lane;
      tmv[w] = l < size ? stage[base + l] : 0;
    }
    const int32_t n_mapped = stage[base + size - 1];
    uint64_t emask[W];
    row_end_mask<W>(tmv, ends, emask);
    row_sums<DT, W>(first, size, n_mapped, emask, acc, y);
  };

  A acc[W];
  bool alive[W];                 // state before the next step of the current group
#pragma unroll
  for (int w = 0; w < W; ++w) { acc[w] = A(0); alive[w] = true; }
  int32_t g = 0;                                            // current group of the run
  int32_t g_end = __builtin_amdgcn_readlane(g_chunk, 0);    // its end step
  for (int32_t j = 0;;) {
    // which slots of the batch a chunk still sums (up to its first -1)
    bool live[U][W];
    {
      int32_t end = g_end, h = g;
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
          alive[w] = alive[w] && (cc[u][w] >= 0);
          live[u][w] = alive[w];
        }
        if (j + u + 1 == end) {                             // group h ends at this step
#pragma unroll
          for (int w = 0; w < W; ++w) alive[w] = true;
          ++h;
          end += __builtin_amdgcn_readlane(g_chunk, h);
        }
      }
    }
    A xv[U][W];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int w = 0; w < W; ++w) xv[u][w] = live[u][w] ? x[cc[u][w]] : A(0);
    }
    int32_t nc[U][W];
    S nv[U][W];
    if constexpr (kDouble) {
      if (j + U < n_steps) load(j + U, nc, nv);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (j + u < n_steps) {
#pragma unroll
        for (int w = 0; w < W; ++w)
          if (live[u][w]) acc[w] = __builtin_fma(Vt::load(vv[u][w]), xv[u][w], acc[w]);
        if (j + u + 1 == g_end) {
          finish(g, acc);
#pragma unroll
          for (int w = 0; w < W; ++w) acc[w] = A(0);
          ++g;
          g_end += __builtin_amdgcn_readlane(g_chunk, g);
        }
      }
    }
    j += U;
    if (j >= n_steps) break;
    // every chunk of the unfinished group reached its padding: skip its rest
    bool any = false;
#pragma unroll
    for (int w = 0; w < W; ++w) any |= alive[w];
    if (__ballot(any) == 0) {
      finish(g, acc);
#pragma unroll
      for (int w = 0; w < W; ++w) { acc[w] = A(0); alive[w] = true; }
      j = g_end;
      ++g;
      g_end += __builtin_amdgcn_readlane(g_chunk, g);
      if (j >= n_steps) break;
      load(j, cc, vv);            // (a prefetched batch is dropped)
      continue;
    }
    if constexpr (kDouble) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int w = 0; w < W; ++w) { cc[u][w] = nc[u][w]; vv[u][w] = nv[u][w]; }
      }
    } else {
      load(j, cc, vv);
    }
  }
}

// One heavy group with all kSpmvWaves waves of the workgroup: wave q sums
// steps [q*share, (q+1)*share); waves 1.. leave their partials in LDS and
// wave 0 adds them in wave order (a fixed order: results are deterministic),
// then forms the row sums.  Every wave of the block must call this.
template <int DT, int W, int U>
__device__ __forceinline__ void spmv_group_split(
    int32_t first, int32_t size, int32_t offset, int32_t c,
    const int32_t* __restrict__ tm, const int32_t* __restrict__ columns,
    const typename Val<DT>::storage* __restrict__ values,
    const typename Val<DT>::acc* __restrict__ x, typename Val<DT>::acc* __restrict__ y,
    int32_t* ends, typename Val<DT>::acc (*part)[64 * W], int wv) {
  using A = typename Val<DT>::acc;
  const int lane = lane_id();
  const int32_t share = (c + kSpmvWaves - 1) / kSpmvWaves;
  const int32_t j0 = min(c, wv * share), j1 = min(c, j0 + share);
  int32_t tmv[W];
  load_mapping<W>(first, size, tm, tmv);
  A acc[W];
  chunk_partials<DT, W, U>(offset, j0, j1, columns, values, x, acc);
  if (wv > 0) {
#pragma unroll
    for (int w = 0; w < W; ++w) part[wv - 1][w * 64 + lane] = acc[w];
  }
  __syncthreads();
  if (wv == 0) {
#pragma unroll
    for (int q = 0; q < kSpmvWaves - 1; ++q) {
#pragma unroll
      for (int w = 0; w < W; ++w) acc[w] += part[q][w * 64 + lane];
    }
    uint64_t emask[W];
    row_end_mask<W>(tmv, ends, emask);
    row_sums<DT, W>(first, size, tm[first + size - 1], emask, acc, y);
  }
}

// Single-matrix launch: blocks [0, n_heavy) take one heavy group each (in
// the order of `heavy`, dispatched first); the remaining blocks take
// kSpmvWaves consecutive groups, one per wave, skipping heavy ones.
template <int DT, int W, int U>
__global__ __launch_bounds__(kSpmvWaves * 64) void argcsr_spmv_kernel(
    const argcsr_group_info* __restrict__ groups, int32_t n_groups,
    const int32_t* __restrict__ tm, const int32_t* __restrict__ columns,
    const typename Val<DT>::storage* __restrict__ values,
    const typename Val<DT>::acc* __restrict__ x, typename Val<DT>::acc* __restrict__ y,
    const int32_t* __restrict__ heavy, int32_t n_heavy, int32_t heavy_chunk) {
  using A = typename Val<DT>::acc;
  __shared__ int32_t ends[kSpmvWaves][64 * W];
  __shared__ A part[kSpmvWaves - 1][64 * W];
  const int wv = wave_uniform(int(threadIdx.x >> 6));
  const int32_t b = int32_t(blockIdx.x);
  if (b < n_heavy) {
    const argcsr_group_info gi = groups[heavy[b]];
    spmv_group_split<DT, W, U>(gi.first_row, gi.size, gi.offset, gi.chunk_size, tm, columns,
                               values, x, y, ends[0], part, wv);
    return;
  }
  const uint32_t nb = gridDim.x - uint32_t(n_heavy);
  const int g = int(xcd_remap(uint32_t(b - n_heavy), nb)) * kSpmvWaves + wv;
  if (g >= n_groups) return;
  const argcsr_group_info gi = groups[g];
  if (gi.chunk_size > heavy_chunk) return;          // processed by a heavy block
  spmv_group<DT, W, U>(gi.first_row, gi.size, gi.offset, gi.chunk_size, tm, columns, values,
                       x, y, ends[wv]);
}

// Single-matrix launch over runs: blocks [0, n_heavy) as above; the other
// blocks take kSpmvWaves consecutive runs, one per wave (heavy runs are left
// to the heavy blocks when there are any).
template <int DT, int W, int U>
__global__ __launch_bounds__(kSpmvWaves * 64) void argcsr_spmv_runs_kernel(
    const argcsr_group_info* __restrict__ groups, const argcsr_run_info* __restrict__ runs,
    int32_t n_runs, const int32_t* __restrict__ tm, const int32_t* __restrict__ columns,
    const typename Val<DT>::storage* __restrict__ values,
    const typename Val<DT>::acc* __restrict__ x, typename Val<DT>::acc* __restrict__ y,
    const int32_t* __restrict__ heavy, int32_t n_heavy) {
  using A = typename Val<DT>::acc;
  __shared__ int32_t ends[kSpmvWaves][64 * W];
  __shared__ int32_t stage[kSpmvWaves][kRunSlots];
  __shared__ A part[kSpmvWaves - 1][64 * W];
  const int wv = wave_uniform(int(threadIdx.x >> 6));
  const int32_t b = int32_t(blockIdx.x);
  if (b < n_heavy) {
    const argcsr_group_info gi = groups[heavy[b]];
    spmv_group_split<DT, W, U>(gi.first_row, gi.size, gi.offset, gi.chunk_size, tm, columns,
                               values, x, y, ends[0], part, wv);
    return;
  }
  const uint32_t nb = gridDim.x - uint32_t(n_heavy);
  const int k = int(xcd_remap(uint32_t(b - n_heavy), nb)) * kSpmvWaves + wv;
  if (k >= n_runs) return;
  const argcsr_run_info run = runs[k], next = runs[k + 1];
  if ((run.flags & ARGCSR_RUN_HEAVY) && n_heavy > 0) return;   // processed by a heavy block
  spmv_run<DT, W, U>(run, next, groups, tm, columns, values, x, y, ends[wv], stage[wv]);
}

int check_matrix(const argcsr_matrix* A);

}  // namespace argcsr
