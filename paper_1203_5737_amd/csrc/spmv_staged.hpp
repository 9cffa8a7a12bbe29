// ARG-CSR SpMV over a matrix whose x is staged per group (an extension of
// the storage for banded matrices; the staging is made in stage.hip).
//
// The chunk loop and the row sums are those of spmv_kernels.hpp; only where
// a slot's x value comes from differs.  Each slot holds a 16-bit position
// 64*q + i in its group's tiles of x (0xFFFF for an artificial zero), and
// the group's tile table (first column, length) is one entry per lane
// (a group has at most 64 tiles).  Two ways to read x:
//   XLDS = true   the group's tiles are loaded into this wave's LDS first,
//                 straight from memory into LDS (buffer loads with the lds
//                 flag, one 64-element tile per instruction for 4-byte x, two
//                 for FP64 x), and every slot reads x from LDS at its
//                 position: Sec. 4's staging of reused data in shared memory;
//   XLDS = false  x is gathered from memory at tile_start[q] + i, the tile
//                 start taken from lane q by a cross-lane permute: only the
//                 index stream shrinks (2 instead of 4 bytes per slot).
// The products and their order are the same as in the unstaged kernel, so y
// is bitwise the unstaged result.
#pragma once

#include <hip/hip_runtime.h>

#include "spmv_kernels.hpp"
#include "stage.hpp"

namespace argcsr {

typedef __attribute__((address_space(3))) void* lds_void_ptr;

// This wave's copy of a group's tile table: lane q holds tile q.
struct TileTable {
  int32_t start;
  int32_t len;
};

__device__ __forceinline__ TileTable load_tile_table(const int32_t* __restrict__ tile_start,
                                                     const int32_t* __restrict__ tile_len,
                                                     int32_t tp, int32_t nt) {
  const int lane = lane_id();
  TileTable t{0, 0};
  if (lane < nt) {
    t.start = tile_start[tp + lane];
    t.len = tile_len[tp + lane];
  }
  return t;
}

// Loads the group's nt tiles into xs[64*q + i] (this wave's LDS region),
// straight from memory into LDS; positions past a tile's length read 0
// through the buffer range check.  Waits for the loads before returning.
template <typename A>
__device__ __forceinline__ void stage_tiles(const A* __restrict__ x, int32_t n_cols,
                                            const TileTable& tt, int32_t nt, A* xs) {
  const int lane = lane_id();
  const __amdgpu_buffer_rsrc_t rsrc = buffer_rsrc(x, uint32_t(n_cols) * uint32_t(sizeof(A)));
  constexpr uint32_t kOut = 0xFFFFFFF0u;           // at or past the end of any x
  for (int q = 0; q < nt; ++q) {
    const int32_t s = __builtin_amdgcn_readlane(tt.start, q);
    const int32_t l = __builtin_amdgcn_readlane(tt.len, q);
    if constexpr (sizeof(A) == 8) {
      // 128 dwords per tile: lane k of half h moves dword k of elements
      // 32h .. 32h+31
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int e = 32 * h + (lane >> 1);
        const uint32_t off = e < l ? uint32_t(s + e) * 8u + uint32_t(lane & 1) * 4u : kOut;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rsrc, (lds_void_ptr)(reinterpret_cast<char*>(xs + 64 * q) + 256 * h), 4, off, 0, 0, 0);
      }
    } else {
      const uint32_t off = lane < l ? uint32_t(s + lane) * 4u : kOut;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (lds_void_ptr)(xs + 64 * q), 4, off, 0, 0, 0);
    }
  }
  // the compiler does not track these LDS writes: wait for them here
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  wave_lds_sync();
}

// Partial sums of this lane's W chunks over steps [j0, j1) of a staged
// group: as chunk_partials, with positions instead of columns.
template <int DT, int W, int U, bool XLDS>
__device__ __forceinline__ void chunk_partials_staged(
    int32_t offset, int32_t j0, int32_t j1, const uint16_t* __restrict__ local,
    const typename Val<DT>::storage* __restrict__ values, const typename Val<DT>::acc* xs,
    const TileTable& tt, const XGather<typename Val<DT>::acc>& gx,
    typename Val<DT>::acc (&acc)[W]) {
  using Vt = Val<DT>;
  using S = typename Vt::storage;
  using A = typename Vt::acc;
  constexpr int T = 64 * W;
  const int lane = lane_id();
  bool alive[W];
#pragma unroll
  for (int w = 0; w < W; ++w) { acc[w] = A(0); alive[w] = true; }
  const uint16_t* pb = local + offset + lane;
  const S* vb = values + offset + lane;
  auto load = [&](int32_t j, uint16_t (&p)[U][W], S (&v)[U][W]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int w = 0; w < W; ++w) {
        if (j + u < j1) {
          p[u][w] = __builtin_nontemporal_load(pb + (j + u) * T + w * 64);
          v[u][w] = __builtin_nontemporal_load(vb + (j + u) * T + w * 64);
        } else {
          p[u][w] = kStagePad;
          v[u][w] = S(0);
        }
      }
    }
  };
  auto consume = [&](const uint16_t (&p)[U][W], const S (&v)[U][W]) {
    bool live[U][W];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int w = 0; w < W; ++w) {
        alive[w] = alive[w] && (p[u][w] != kStagePad);
        live[u][w] = alive[w];
      }
    }
    A xv[U][W];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const uint32_t pos = p[u][w];
        if constexpr (XLDS) {
          xv[u][w] = xs[live[u][w] ? pos : 0u];
        } else {
          const int32_t start = __shfl(tt.start, int(pos >> 6), 64);
          xv[u][w] = gx(start + int32_t(pos & 63u), live[u][w]);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const A prod = __builtin_fma(Vt::load(v[u][w]), xv[u][w], acc[w]);
        acc[w] = live[u][w] ? prod : acc[w];
      }
    }
    bool any = false;
#pragma unroll
    for (int w = 0; w < W; ++w) any |= alive[w];
    return __ballot(any) != 0;
  };
  uint16_t pp[U][W];
  S vv[U][W];
  if constexpr (sizeof(S) < 8) {
    if (j0 < j1) load(j0, pp, vv);
    for (int j = j0; j < j1; j += U) {
      uint16_t np[U][W];
      S nv[U][W];
      const bool more = j + U < j1;
      if (more) load(j + U, np, nv);
      if (!consume(pp, vv) || !more) break;
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int w = 0; w < W; ++w) { pp[u][w] = np[u][w]; vv[u][w] = nv[u][w]; }
      }
    }
  } else {
    for (int j = j0; j < j1; j += U) {
      load(j, pp, vv);
      if (!consume(pp, vv)) break;
    }
  }
}

// LDS bytes of one wave of the staged kernel: its x tiles (XLDS), reused
// after the chunk loop for its row-end table (T ints) and, in a heavy block,
// for the partial sums it hands to wave 0 (T values).
template <int DT, int W, bool XLDS>
__host__ __device__ constexpr uint32_t staged_region_bytes(int32_t lds_tiles) {
  using A = typename Val<DT>::acc;
  const uint32_t tiles = XLDS ? uint32_t(lds_tiles) * 64u * uint32_t(sizeof(A)) : 0u;
  const uint32_t rows = 64u * W * uint32_t(sizeof(A) > 4 ? sizeof(A) : 4);
  return ((tiles > rows ? tiles : rows) + 15u) & ~15u;
}

// Single-matrix launch over a staged matrix; the block layout is that of
// argcsr_spmv_kernel (heavy groups first, split over the block's waves;
// then one group per wave).  Dynamic LDS only: kSpmvWaves regions of
// staged_region_bytes each.
template <int DT, int W, int U, bool XLDS>
__global__ __launch_bounds__(kSpmvWaves * 64) void argcsr_spmv_staged_kernel(
    const argcsr_group_info* __restrict__ groups, int32_t n_groups,
    const int32_t* __restrict__ tm, const uint16_t* __restrict__ local,
    const typename Val<DT>::storage* __restrict__ values,
    const int32_t* __restrict__ tile_ptr, const int32_t* __restrict__ tile_start,
    const int32_t* __restrict__ tile_len, int32_t lds_tiles,
    const typename Val<DT>::acc* __restrict__ x, int32_t n_cols,
    typename Val<DT>::acc* __restrict__ y,
    const int32_t* __restrict__ heavy, int32_t n_heavy, int32_t heavy_chunk) {
  using A = typename Val<DT>::acc;
  extern __shared__ __align__(16) unsigned char stage_lds[];
  const int wv = wave_uniform(int(threadIdx.x >> 6));
  const int lane = lane_id();
  const XGather<A> gx(x, n_cols);
  const uint32_t region = staged_region_bytes<DT, W, XLDS>(lds_tiles);
  unsigned char* mine = stage_lds + size_t(wv) * region;
  A* xs = reinterpret_cast<A*>(mine);
  int32_t* ends = reinterpret_cast<int32_t*>(mine);    // after the chunk loop
  const int32_t b = int32_t(blockIdx.x);
  int g;
  bool split;
  if (b < n_heavy) {
    g = heavy[b];
    split = true;
  } else {
    const uint32_t nb = gridDim.x - uint32_t(n_heavy);
    g = int(xcd_remap(uint32_t(b - n_heavy), nb)) * kSpmvWaves + wv;
    split = false;
    if (g >= n_groups) return;
  }
  const argcsr_group_info gi = groups[g];
  if (!split && gi.chunk_size > heavy_chunk) return;   // processed by a heavy block
  const int32_t tp = tile_ptr[g];
  // at most the tiles this wave's LDS region holds (all, for a staging made
  // by argcsr_stage)
  const int32_t nt = min(tile_ptr[g + 1] - tp, lds_tiles);
  int32_t tmv[W];
  load_mapping<W>(gi.first_row, gi.size, tm, tmv);
  const TileTable tt = load_tile_table(tile_start, tile_len, tp, nt);
  if constexpr (XLDS) stage_tiles<A>(x, n_cols, tt, nt, xs);
  A acc[W];
  if (!split) {
    const int32_t n_mapped = tm[gi.first_row + gi.size - 1];
    chunk_partials_staged<DT, W, U, XLDS>(gi.offset, 0, gi.chunk_size, local, values, xs, tt, gx,
                                         acc);
    wave_lds_sync();                                   // x tiles read: the region is free
    uint64_t emask[W];
    row_end_mask<W>(tmv, ends, emask);
    row_sums<DT, W>(gi.first_row, gi.size, n_mapped, emask, acc, y);
    return;
  }
  // heavy group: every wave staged the tiles in its own region and sums a
  // contiguous share of the steps; waves 1.. leave their sums in their own
  // regions and wave 0 adds them in wave order
  const int32_t c = gi.chunk_size;
  const int32_t share = (c + kSpmvWaves - 1) / kSpmvWaves;
  const int32_t j0 = min(c, wv * share), j1 = min(c, j0 + share);
  chunk_partials_staged<DT, W, U, XLDS>(gi.offset, j0, j1, local, values, xs, tt, gx, acc);
  wave_lds_sync();
  if (wv > 0) {
#pragma unroll
    for (int w = 0; w < W; ++w) xs[w * 64 + lane] = acc[w];
  }
  __syncthreads();
  if (wv == 0) {
#pragma unroll
    for (int q = 1; q < kSpmvWaves; ++q) {
      const A* part = reinterpret_cast<const A*>(stage_lds + size_t(q) * region);
#pragma unroll
      for (int w = 0; w < W; ++w) acc[w] += part[w * 64 + lane];
    }
    uint64_t emask[W];
    row_end_mask<W>(tmv, ends, emask);
    row_sums<DT, W>(gi.first_row, gi.size, tm[gi.first_row + gi.size - 1], emask, acc, y);
  }
}

}  // namespace argcsr
