// Staging of x for banded matrices: an extension of the ARG-CSR storage.
//
// Sec. 4 stages in shared memory the data a block of threads reuses.  In a
// banded matrix the rows of a group name a few runs of consecutive columns
// (for a stencil: the grid lines around the group's own), so the part of x a
// group reads is small and can be staged the same way.  Per group, the
// distinct columns its slots name are merged into windows (two neighbouring
// columns stay in one window when at most `gap` columns between them are
// absent), and every window is cut into tiles of 64 consecutive columns
// (the last one shorter).  A slot then stores, instead of its column, a
// 16-bit position in its group's staged tiles: 64*q + (column - start of
// tile q), 0xFFFF for an artificial zero.  The SpMV loads a group's tiles
// into LDS with coalesced loads and reads x from there; the index stream is
// 2 bytes per slot instead of 4.
//
//   stage_kernel<false>  per group: its tile count (written to tile_ptr[g+1])
//   stage_scan_kernel    tile_ptr as an exclusive scan, the total and the
//                        largest group's count
//   stage_kernel<true>   per group: its tiles (first column, length) and the
//                        position of every slot
//
// One wave per group.  The group's columns are marked in a bitmap in LDS
// (offset by the group's smallest column); the windows follow from the
// distances between consecutive set bits, which each lane finds over its
// own range of bitmap words with the last set bit of the lanes before it.
#include <hip/hip_runtime.h>

#include <climits>

#include "common.hpp"
#include "group.hpp"
#include "stage.hpp"

namespace argcsr {
namespace {

constexpr int kStageWords = kStageSpanBits / 32;

struct StageStatus {
  int unstageable;        // bit 0: a group spans too many columns; bit 1: too many tiles
  int mismatch;           // tile_ptr does not match the group's count
  int total;
  int max_tiles;
};

__global__ void stage_clear_kernel(StageStatus* st) { *st = StageStatus{}; }

__device__ __forceinline__ int wave_min_i32(int v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const int t = __shfl_xor(v, d, 64);
    v = t < v ? t : v;
  }
  return v;
}

// Exclusive max-scan over lanes (lanes before this one), -1 if none.
__device__ __forceinline__ int wave_excl_max(int v) {
  const int lane = lane_id();
  int incl = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(incl, d, 64);
    if (lane >= d) incl = t > incl ? t : incl;
  }
  const int prev = __shfl_up(incl, 1, 64);
  return lane == 0 ? -1 : prev;
}

template <bool FILL>
__global__ __launch_bounds__(64) void stage_kernel(
    const argcsr_group_info* __restrict__ groups, int32_t n_groups, int32_t T,
    const int32_t* __restrict__ columns, int32_t gap, int32_t* __restrict__ tile_ptr,
    int32_t n_stage_tiles, int32_t* __restrict__ tile_start, int32_t* __restrict__ tile_len,
    uint16_t* __restrict__ local, StageStatus* st) {
  __shared__ uint32_t bm[kStageWords];
  __shared__ int32_t win_start[kStageMaxTiles];   // window start (relative to the smallest column)
  __shared__ int32_t win_prev[kStageMaxTiles];    // the set bit before it (-1 for the first)
  __shared__ int32_t win_tile[kStageMaxTiles];    // first tile of the window
  const int g = int(blockIdx.x);
  if (g >= n_groups) return;
  const int lane = lane_id();
  const argcsr_group_info gi = groups[g];
  const int64_t slots = int64_t(gi.chunk_size) * T;
  const int32_t* cb = columns + gi.offset;

  // the group's smallest and largest column
  int mn = INT_MAX, mx = -1;
  for (int64_t s = lane; s < slots; s += 64) {
    const int c = cb[s];
    if (c >= 0) {
      mn = c < mn ? c : mn;
      mx = c > mx ? c : mx;
    }
  }
  mn = wave_min_i32(mn);
  mx = wave_max(mx);
  int n_tiles = 0;
  bool ok = true;
  int n_win = 0, last_all = -1;
  if (mx >= 0) {
    const int64_t span = int64_t(mx) - mn + 1;
    if (span > kStageSpanBits) {
      if (lane == 0) atomicOr(&st->unstageable, 1);
      ok = false;
    } else {
      const int nw = int((span + 31) / 32);
      for (int w = lane; w < nw; w += 64) bm[w] = 0u;
      wave_lds_sync();
      for (int64_t s = lane; s < slots; s += 64) {
        const int c = cb[s];
        if (c >= 0) atomicOr(&bm[(c - mn) >> 5], 1u << ((c - mn) & 31));
      }
      wave_lds_sync();
      // this lane's words [lo, hi)
      const int per = (nw + 63) / 64;
      const int lo = lane * per < nw ? lane * per : nw;
      const int hi = lo + per < nw ? lo + per : nw;
      int distinct = 0, last = -1;
      for (int w = lo; w < hi; ++w) {
        const uint32_t b = bm[w];
        distinct += __popc(b);
        if (b) last = 32 * w + 31 - __clz(int(b));
      }
      // a tile holds at most 64 distinct columns
      const int all_distinct = int(wave_sum_i64(distinct));
      if (all_distinct > 64 * kStageMaxTiles) {
        ok = false;
      } else {
        last_all = wave_max(last);
        int prev = wave_excl_max(last);
        // window starts in this lane's range: a set bit more than gap+1
        // columns after the previous one (or the first)
        int starts = 0;
        for (int w = lo; w < hi; ++w) {
          uint32_t b = bm[w];
          while (b) {
            const int p = 32 * w + __builtin_ctz(b);
            b &= b - 1;
            if (prev < 0 || int64_t(p) - prev - 1 > int64_t(gap)) ++starts;
            prev = p;
          }
        }
        const int incl = wave_inclusive_scan(starts);
        n_win = __shfl(incl, 63, 64);
        if (n_win > kStageMaxTiles) {
          ok = false;
        } else {
          int idx = incl - starts;
          prev = wave_excl_max(last);
          for (int w = lo; w < hi; ++w) {
            uint32_t b = bm[w];
            while (b) {
              const int p = 32 * w + __builtin_ctz(b);
              b &= b - 1;
              if (prev < 0 || int64_t(p) - prev - 1 > int64_t(gap)) {
                win_start[idx] = p;
                win_prev[idx] = prev;
                ++idx;
              }
              prev = p;
            }
          }
          wave_lds_sync();
          // tiles per window: window i spans [start_i, end_i], end_i being the
          // set bit before the next window's start (the last set bit for the
          // last window)
          int wt = 0, ws = 0, we = 0;
          if (lane < n_win) {
            ws = win_start[lane];
            we = lane + 1 < n_win ? win_prev[lane + 1] : last_all;
            wt = (we - ws + 64) / 64;
          }
          const int tincl = wave_inclusive_scan(wt);
          n_tiles = __shfl(tincl, 63, 64);
          if (n_tiles > kStageMaxTiles) {
            ok = false;
          } else if (FILL) {
            const int first_tile = tincl - wt;
            wave_lds_sync();
            if (lane < n_win) win_tile[lane] = first_tile;
            const int tp = tile_ptr[g];
            if (tile_ptr[g + 1] - tp != n_tiles || tp < 0 || tp + n_tiles > n_stage_tiles) {
              if (lane == 0) atomicOr(&st->mismatch, 1);
            } else if (lane < n_win) {
              for (int m = 0; m < wt; ++m) {
                const int t0 = ws + 64 * m;
                tile_start[tp + first_tile + m] = mn + t0;
                tile_len[tp + first_tile + m] = we - t0 + 1 < 64 ? we - t0 + 1 : 64;
              }
            }
            wave_lds_sync();
          }
        }
      }
      if (!ok && lane == 0) atomicOr(&st->unstageable, 2);
    }
  }
  if (!FILL) {
    if (lane == 0) {
      tile_ptr[g + 1] = ok ? n_tiles : 0;
      if (g == 0) tile_ptr[0] = 0;
    }
    return;
  }
  if (!ok) return;
  // every slot's position in the staged tiles
  for (int64_t s = lane; s < slots; s += 64) {
    const int c = cb[s];
    uint16_t v = 0xFFFF;
    if (c >= 0) {
      const int r = c - mn;
      // the last window starting at or before r (binary search; n_win <= 64)
      int lo_w = 0, hi_w = n_win - 1;
      while (lo_w < hi_w) {
        const int mid = (lo_w + hi_w + 1) >> 1;
        if (win_start[mid] <= r) lo_w = mid; else hi_w = mid - 1;
      }
      v = uint16_t(64 * win_tile[lo_w] + (r - win_start[lo_w]));
    }
    __builtin_nontemporal_store(v, local + gi.offset + s);
  }
}

// tile_ptr[1..G] holds per-group counts; turns tile_ptr into the exclusive
// scan (tile_ptr[0] = 0) and records the total and the largest count.
__global__ __launch_bounds__(1024) void stage_scan_kernel(int32_t* __restrict__ tile_ptr,
                                                        int32_t n_groups, StageStatus* st) {
  __shared__ int wave_tot[16];
  __shared__ int wave_max_s[16];
  const int lane = lane_id(), w = int(threadIdx.x >> 6);
  int carry = 0, biggest = 0;
  for (int32_t base = 0; base < n_groups; base += 1024) {
    const int32_t i = base + int32_t(threadIdx.x);
    const int v = i < n_groups ? tile_ptr[i + 1] : 0;
    const int incl = wave_inclusive_scan(v);
    const int m = wave_max(v);
    if (lane == 63) wave_tot[w] = incl;
    if (lane == 0) wave_max_s[w] = m;
    __syncthreads();
    int before = 0, all = 0, bm = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      if (q < w) before += wave_tot[q];
      all += wave_tot[q];
      bm = wave_max_s[q] > bm ? wave_max_s[q] : bm;
    }
    if (i < n_groups) tile_ptr[i + 1] = carry + before + incl;
    carry += all;
    biggest = bm > biggest ? bm : biggest;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    tile_ptr[0] = 0;
    st->total = carry;
    st->max_tiles = biggest;
  }
}

int check_stage_input(const argcsr_matrix* A) {
  if (!A) return fail(ARGCSR_EINVAL, "matrix is NULL");
  if (A->n_groups < 0 || A->n_slots < 0 || A->block_dim < 1)
    return fail(ARGCSR_EINVAL, "malformed matrix descriptor");
  if (A->n_slots > INT32_MAX) return fail(ARGCSR_EOVERFLOW, "n_slots exceeds INT32_MAX");
  if (A->n_groups > 0 && (!A->groups || !A->columns))
    return fail(ARGCSR_EINVAL, "staging needs the converted groups and columns");
  return ARGCSR_OK;
}

}  // namespace
}  // namespace argcsr

extern "C" int argcsr_stage_plan(const argcsr_matrix* A, int32_t gap, int32_t* tile_ptr,
                                 int32_t* n_tiles, int32_t* max_group_tiles, void* stream) {
  using namespace argcsr;
  clear_error();
  int rc = check_stage_input(A);
  if (rc) return rc;
  if (gap < 0) return fail(ARGCSR_EINVAL, "gap < 0");
  if (!tile_ptr || !n_tiles) return fail(ARGCSR_EINVAL, "NULL argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  *n_tiles = 0;
  if (max_group_tiles) *max_group_tiles = 0;
  if (A->n_groups == 0) {
    const int32_t zero = 0;
    ARGCSR_HIP(hipMemcpyAsync(tile_ptr, &zero, sizeof(zero), hipMemcpyHostToDevice, s));
    ARGCSR_HIP(hipStreamSynchronize(s));
    return ARGCSR_OK;
  }
  StreamScratch ws;
  rc = ws.alloc(sizeof(StageStatus), s);
  if (rc) return rc;
  auto* st = static_cast<StageStatus*>(ws.ptr);
  stage_clear_kernel<<<1, 1, 0, s>>>(st);
  stage_kernel<false><<<A->n_groups, 64, 0, s>>>(A->groups, A->n_groups, A->block_dim, A->columns,
                                                 gap, tile_ptr, 0, nullptr, nullptr, nullptr, st);
  stage_scan_kernel<<<1, 1024, 0, s>>>(tile_ptr, A->n_groups, st);
  ARGCSR_HIP(hipGetLastError());
  StageStatus h{};
  ARGCSR_HIP(hipMemcpyAsync(&h, st, sizeof(h), hipMemcpyDeviceToHost, s));
  ARGCSR_HIP(hipStreamSynchronize(s));
  if (h.unstageable & 1)
    return fail(ARGCSR_EUNSUPPORTED, "a group's columns span more than %d columns", kStageSpanBits);
  if (h.unstageable & 2)
    return fail(ARGCSR_EUNSUPPORTED, "a group needs more than %d tiles of x", kStageMaxTiles);
  *n_tiles = h.total;
  if (max_group_tiles) *max_group_tiles = h.max_tiles;
  return ARGCSR_OK;
}

extern "C" int argcsr_stage(argcsr_matrix* A, void* stream) {
  using namespace argcsr;
  clear_error();
  int rc = check_stage_input(A);
  if (rc) return rc;
  if (A->stage_gap < 0) return fail(ARGCSR_EINVAL, "stage_gap < 0");
  if (A->n_stage_tiles < 0 || A->stage_max_tiles < 0 || A->stage_max_tiles > kStageMaxTiles)
    return fail(ARGCSR_EINVAL, "malformed staging sizes");
  if (A->n_groups == 0) return ARGCSR_OK;
  if (!A->tile_ptr || !A->local || (A->n_stage_tiles > 0 && (!A->tile_start || !A->tile_len)))
    return fail(ARGCSR_EINVAL, "NULL staging buffer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  StreamScratch ws;
  rc = ws.alloc(sizeof(StageStatus), s);
  if (rc) return rc;
  auto* st = static_cast<StageStatus*>(ws.ptr);
  stage_clear_kernel<<<1, 1, 0, s>>>(st);
  stage_kernel<true><<<A->n_groups, 64, 0, s>>>(A->groups, A->n_groups, A->block_dim, A->columns,
                                                A->stage_gap, A->tile_ptr, A->n_stage_tiles,
                                                A->tile_start, A->tile_len, A->local, st);
  ARGCSR_HIP(hipGetLastError());
  StageStatus h{};
  ARGCSR_HIP(hipMemcpyAsync(&h, st, sizeof(h), hipMemcpyDeviceToHost, s));
  ARGCSR_HIP(hipStreamSynchronize(s));
  if (h.unstageable)
    return fail(ARGCSR_EUNSUPPORTED, "the matrix cannot be staged with gap %d", A->stage_gap);
  if (h.mismatch)
    return fail(ARGCSR_EINVAL, "tile_ptr was not made by argcsr_stage_plan with this gap");
  return ARGCSR_OK;
}
