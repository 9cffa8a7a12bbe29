// Device routines for ARG-CSR SpMV, shared by the single-matrix kernel and
// the batched work-queue kernel (Sec. 4 semantics: chunk partial sums, then
// per-row sums of the partial sums).
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"
#include "schedule.hpp"
#include "values.hpp"

namespace argcsr {

// Word 3 of a gfx9 buffer descriptor: 32-bit data format, no swizzle.  With
// stride 0 the hardware range check returns 0 for any load at or past
// num_records bytes, so out-of-range lanes need no branch.
constexpr int32_t kBufferWord3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), int16_t(0), int32_t(bytes),
                                           kBufferWord3);
}

// Gathers x[c] as raw buffer loads: a lane that must not gather asks for
// column -1, whose byte offset (uint32)(-1)*sizeof(A) lies past the end of
// x, and reads 0.  No branch guards the loads, so all gathers of a batch are
// in flight before the first wait.  Requires n_cols * sizeof(A) < 2^32 - 16
// (checked on the host).
template <typename A>
struct XGather {
  __amdgpu_buffer_rsrc_t rsrc;
  const A* xp;
  __device__ __forceinline__ XGather(const A* x, int32_t n_cols)
      : rsrc(buffer_rsrc(x, uint32_t(n_cols) * uint32_t(sizeof(A)))), xp(x) {}
  __device__ __forceinline__ A operator()(int32_t c, bool live) const {
    const uint32_t off = uint32_t(live ? c : -1) * uint32_t(sizeof(A));
    if constexpr (sizeof(A) == 8)
      return __builtin_bit_cast(A, __builtin_amdgcn_raw_buffer_load_b64(rsrc, off, 0, 0));
    else
      return __builtin_bit_cast(A, __builtin_amdgcn_raw_buffer_load_b32(rsrc, off, 0, 0));
  }
};

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
// x[column], stopping at a chunk's first artificial zero (column -1).  A
// batch of U steps is loaded at once.  Its gathers are either all put in
// flight before the FMAs (the default), or, with `serial` (wave-uniform),
// issued one at a time, each followed by its FMA: measured faster for
// 8-byte values with long chunk loops, where the stream, not the gathers,
// is the limit (see gather_mode).  The sums are the same in both modes.
template <int DT, int W, int U>
__device__ __forceinline__ void chunk_partials(
    int32_t offset, int32_t j0, int32_t j1, const int32_t* __restrict__ columns,
    const typename Val<DT>::storage* __restrict__ values,
    const XGather<typename Val<DT>::acc>& gx, bool serial, typename Val<DT>::acc (&acc)[W]) {
  using Vt = Val<DT>;
  using S = typename Vt::storage;
  using A = typename Vt::acc;
  constexpr int T = 64 * W;
  const int lane = lane_id();
  bool alive[W];
#pragma unroll
  for (int w = 0; w < W; ++w) { acc[w] = A(0); alive[w] = true; }
  const int32_t* cb = columns + offset + lane;
  const S* vb = values + offset + lane;
  // steps j .. j+U-1 (steps past j1 read as padding); streamed once:
  // non-temporal, keeping L2 for the x gathers
  auto load = [&](int32_t j, int32_t (&c)[U][W], S (&v)[U][W]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int w = 0; w < W; ++w) {
        if (j + u < j1) {
          c[u][w] = __builtin_nontemporal_load(cb + (j + u) * T + w * 64);
          v[u][w] = __builtin_nontemporal_load(vb + (j + u) * T + w * 64);
        } else {
          c[u][w] = -1;
          v[u][w] = S(0);
        }
      }
    }
  };
  // returns whether some chunk has not reached its padding yet
  auto consume = [&](const int32_t (&c)[U][W], const S (&v)[U][W]) {
    if (serial) {
      // one gather at a time, each FMA right after its load
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
          alive[w] = alive[w] && (c[u][w] >= 0);
          if (alive[w]) acc[w] = __builtin_fma(Vt::load(v[u][w]), gx.xp[c[u][w]], acc[w]);
        }
      }
    } else {
      // which slots are live, then all gathers of the batch, then the FMAs
      // in step order
      bool live[U][W];
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
          alive[w] = alive[w] && (c[u][w] >= 0);
          live[u][w] = alive[w];
        }
      }
      A xv[U][W];
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int w = 0; w < W; ++w) xv[u][w] = gx(c[u][w], live[u][w]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
          const A p = __builtin_fma(Vt::load(v[u][w]), xv[u][w], acc[w]);
          acc[w] = live[u][w] ? p : acc[w];
        }
      }
    }
    bool any = false;
#pragma unroll
    for (int w = 0; w < W; ++w) any |= alive[w];
    return __ballot(any) != 0;
  };
  int32_t cc[U][W];
  S vv[U][W];
  if constexpr (sizeof(S) < 8) {
    // 4- and 2-byte values: the next U steps are loaded before this batch's x
    // gathers are issued (double buffering fits the register budget)
    if (j0 < j1) load(j0, cc, vv);
    for (int j = j0; j < j1; j += U) {
      int32_t nc[U][W];
      S nv[U][W];
      const bool more = j + U < j1;
      if (more) load(j + U, nc, nv);
      if (!consume(cc, vv) || !more) break;      // every chunk reached its padding
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
      load(j, cc, vv);
      if (!consume(cc, vv)) break;               // every chunk reached its padding
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
    const XGather<typename Val<DT>::acc>& gx, bool serial, typename Val<DT>::acc* __restrict__ y,
    int32_t* ends) {
  using A = typename Val<DT>::acc;
  int32_t tmv[W];
  load_mapping<W>(first, size, tm, tmv);           // in flight with the first chunk loads
  const int32_t n_mapped = tm[first + size - 1];    // chunks in use; the rest are free
  A acc[W];
  chunk_partials<DT, W, U>(offset, 0, c, columns, values, gx, serial, acc);
  uint64_t emask[W];
  row_end_mask<W>(tmv, ends, emask);
  row_sums<DT, W>(first, size, n_mapped, emask, acc, y);
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
    const XGather<typename Val<DT>::acc>& gx, bool serial, typename Val<DT>::acc* __restrict__ y,
    int32_t* ends, typename Val<DT>::acc (*part)[64 * W], int wv) {
  using A = typename Val<DT>::acc;
  const int lane = lane_id();
  const int32_t share = (c + kSpmvWaves - 1) / kSpmvWaves;
  const int32_t j0 = min(c, wv * share), j1 = min(c, j0 + share);
  int32_t tmv[W];
  load_mapping<W>(first, size, tm, tmv);
  A acc[W];
  chunk_partials<DT, W, U>(offset, j0, j1, columns, values, gx, serial, acc);
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
    const typename Val<DT>::acc* __restrict__ x, int32_t n_cols,
    typename Val<DT>::acc* __restrict__ y,
    const int32_t* __restrict__ heavy, int32_t n_heavy, int32_t heavy_chunk, int32_t serial) {
  using A = typename Val<DT>::acc;
  __shared__ int32_t ends[kSpmvWaves][64 * W];
  __shared__ A part[kSpmvWaves - 1][64 * W];
  const int wv = wave_uniform(int(threadIdx.x >> 6));
  const XGather<A> gx(x, n_cols);
  const int32_t b = int32_t(blockIdx.x);
  if (b < n_heavy) {
    const argcsr_group_info gi = groups[heavy[b]];
    spmv_group_split<DT, W, U>(gi.first_row, gi.size, gi.offset, gi.chunk_size, tm, columns,
                               values, gx, serial != 0, y, ends[0], part, wv);
    return;
  }
  const uint32_t nb = gridDim.x - uint32_t(n_heavy);
  const int g = int(xcd_remap(uint32_t(b - n_heavy), nb)) * kSpmvWaves + wv;
  if (g >= n_groups) return;
  const argcsr_group_info gi = groups[g];
  if (gi.chunk_size > heavy_chunk) return;          // processed by a heavy block
  spmv_group<DT, W, U>(gi.first_row, gi.size, gi.offset, gi.chunk_size, tm, columns, values,
                       gx, serial != 0, y, ends[wv]);
}

int check_matrix(const argcsr_matrix* A);

}  // namespace argcsr
