// CSR -> ARG-CSR conversion on the GPU (Sec. 3 of the paper).
//
// Step 1 (grouping) is a sequential scan; it runs on the host (plan.cpp), or
// on the device by binary lifting (group.hip) when the caller has row_ptr on
// the device only.  The kernels here run steps 2-4, every group independently:
//   chunks_kernel   step 2: chunk size c_g = min{c >= 1 : sum_r max(1,ceil(L_r/c)) <= T}
//                   (row-grouped CSR: c_g = max(1, longest row)) and
//                   t_r = max(1, ceil(L_r/c_g)) chunks per row;
//                   step 3: inclusive per-group prefix sum of t_r -> threadsMapping
//   offsets kernels exclusive scan of c_g*T over the groups -> groupInfo.offset
//   heavy kernels   the launch schedule: ascending indices of groups whose
//                   chunk loop is long (compaction by an exclusive scan)
//   fill_kernel     step 4: every slot (j, k) of a group -- element j of chunk
//   fill_long_kernel k at offset + j*T + k -- is written exactly once: the
//                   matching CSR element if chunk k's row has one there,
//                   otherwise the artificial zero (0, -1); the CSR elements
//                   pass through LDS so that reads and writes are coalesced
//                   (fill_long_kernel takes the blocks of long rows, tile by
//                   tile, from a list the fill kernel makes); every CSR element
//                   passes through one of the two, which also check its column
//                   index against [0, n_cols).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "common.hpp"
#include "group.hpp"
#include "plan.hpp"
#include "schedule.hpp"
#include "values.hpp"

namespace argcsr {
namespace {

constexpr int kWaves = 4;             // waves per workgroup, one group per wave
constexpr int kMaxBlockDim = 1024;    // conversion accepts 1 <= T <= 1024
constexpr int kScanBlock = 256;
constexpr int kScanItems = 4;         // groups per thread in the offset scan
constexpr int kScanTile = kScanBlock * kScanItems;
constexpr int kMinStage = 256;        // CSR elements one fill wave stages in LDS
constexpr int kMaxStage = 2048;
constexpr int kMaxFillWaves = 4;
constexpr int kLongSteps = 16;        // steps per LDS tile in fill_long_kernel
constexpr int kLongGrid = 4096;       // one-wave workgroups of fill_long_kernel

struct Status {                       // device-side results read back by the host
  int bad_column;
  int long_items;                     // entries of the fill's long-row work list
  long long total_slots;
  long long total_heavy;
};

__global__ void clear_status_kernel(Status* st) { *st = Status{}; }

// dst[i] = src[i] for n 32-bit words (a device plan's tables into the
// caller's buffers)
__global__ __launch_bounds__(256) void copy_words_kernel(const int32_t* __restrict__ src,
                                                        int32_t* __restrict__ dst, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
    dst[i] = src[i];
}

void copy_words(const void* src, void* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  copy_words_kernel<<<dim3(uint32_t(blocks)), 256, 0, s>>>(static_cast<const int32_t*>(src),
                                                          static_cast<int32_t*>(dst), n);
}

// LDS of one fill wave: chunk starts and lengths, then the staged columns and
// values (the byte count keeps the next wave's region 8-byte aligned)
template <typename S>
__host__ __device__ inline size_t fill_lds_bytes(int32_t T, int32_t stage) {
  const size_t b = sizeof(int32_t) * (2 * size_t(T) + size_t(stage)) + sizeof(S) * size_t(stage);
  return (b + 7) & ~size_t(7);
}

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const int t = __shfl_xor(v, d, 64);
    v = t < v ? t : v;
  }
  return v;
}

// Step 2 + 3, one wave per group.  Row l of the group lives in lane l % 64,
// sub-row l / 64.
__global__ __launch_bounds__(kWaves * 64) void chunks_kernel(
    const int32_t* __restrict__ rp, argcsr_group_info* __restrict__ groups,
    int32_t n_groups, int32_t T, int32_t row_grouped, int32_t* __restrict__ tm) {
  const int lane = lane_id();
  const int g = blockIdx.x * kWaves + wave_uniform(int(threadIdx.x >> 6));
  if (g >= n_groups) return;
  const int32_t first = groups[g].first_row;
  const int32_t size = groups[g].size;
  const int sub_rows = (size + 63) / 64;

  int64_t my_nnz = 0;
  int my_longest = 0;
  for (int s = 0; s < sub_rows; ++s) {
    const int l = s * 64 + lane;
    if (l < size) {
      const int L = rp[first + l + 1] - rp[first + l];
      my_nnz += L;
      my_longest = L > my_longest ? L : my_longest;
    }
  }
  const int64_t total = wave_sum_i64(my_nnz);
  const int longest = wave_max(my_longest);

  auto chunks_needed = [&](uint32_t c) {
    int64_t need = 0;
    for (int s = 0; s < sub_rows; ++s) {
      const int l = s * 64 + lane;
      if (l < size) {
        const uint32_t L = uint32_t(rp[first + l + 1] - rp[first + l]);
        need += L > c ? (L - 1u) / c + 1u : 1u;
      }
    }
    return wave_sum_i64(need);
  };
  // binary search on the non-increasing chunks_needed(c) between two bounds:
  // no c below total/T fits, and c = longest (one chunk per row) always does;
  // since max(1, ceil(L/c)) <= L/c + 1, every c >= total/(T - size) fits too.
  // Row-grouped CSR, and a group of T rows, take one chunk per row.
  uint32_t lo = uint32_t((total + T - 1) / T);
  lo = lo < 1u ? 1u : lo;
  uint32_t hi = longest < 1 ? 1u : uint32_t(longest);
  if (row_grouped || size >= T) {
    lo = hi;
  } else {
    const int64_t fit = (total + (T - size) - 1) / (T - size);
    if (fit < int64_t(hi)) hi = fit < 1 ? 1u : uint32_t(fit);
  }
  while (lo < hi) {
    const uint32_t mid = lo + (hi - lo) / 2;
    if (chunks_needed(mid) <= T) hi = mid;
    else lo = mid + 1;
  }
  const uint32_t c = lo;

  int carry = 0;
  for (int s = 0; s < sub_rows; ++s) {
    const int l = s * 64 + lane;
    int t = 0;
    if (l < size) {
      const uint32_t L = uint32_t(rp[first + l + 1] - rp[first + l]);
      t = L > c ? int((L - 1u) / c + 1u) : 1;
    }
    const int incl = wave_inclusive_scan(t) + carry;
    if (l < size) tm[first + l] = incl;
    carry = __shfl(incl, 63, 64);
  }
  if (lane == 0) groups[g].chunk_size = int32_t(c);
}

// Offsets: block-local sums of c_g*T, a single-block scan of those, then the
// block-local exclusive scan plus the block's base.
__device__ int64_t block_exclusive_scan(int64_t v, int64_t* total) {
  __shared__ int64_t wave_tot[kScanBlock / 64];
  const int lane = lane_id(), w = threadIdx.x >> 6;
  int64_t incl = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int64_t t = __shfl_up(incl, d, 64);
    if (lane >= d) incl += t;
  }
  if (lane == 63) wave_tot[w] = incl;
  __syncthreads();
  int64_t before = 0, all = 0;
  for (int i = 0; i < kScanBlock / 64; ++i) {
    if (i < w) before += wave_tot[i];
    all += wave_tot[i];
  }
  __syncthreads();
  *total = all;
  return before + incl - v;
}

__global__ __launch_bounds__(kScanBlock) void offsets_reduce_kernel(
    const argcsr_group_info* __restrict__ groups, int32_t n_groups, int32_t T,
    int64_t* __restrict__ tile_sums) {
  int64_t s = 0;
  const int64_t base = int64_t(blockIdx.x) * kScanTile + threadIdx.x * kScanItems;
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n_groups) s += int64_t(groups[base + i].chunk_size) * T;
  int64_t total;
  (void)block_exclusive_scan(s, &total);
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanBlock) void tiles_scan_kernel(
    int64_t* __restrict__ tile_sums, int32_t n_tiles, long long* total_out) {
  int64_t carry = 0;
  for (int32_t base = 0; base < n_tiles; base += kScanBlock) {
    const int32_t i = base + threadIdx.x;
    const int64_t v = i < n_tiles ? tile_sums[i] : 0;
    int64_t total;
    const int64_t ex = block_exclusive_scan(v, &total);
    if (i < n_tiles) tile_sums[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) *total_out = carry;
}

__global__ __launch_bounds__(kScanBlock) void offsets_apply_kernel(
    argcsr_group_info* __restrict__ groups, int32_t n_groups, int32_t T,
    const int64_t* __restrict__ tile_base) {
  const int64_t base = int64_t(blockIdx.x) * kScanTile + threadIdx.x * kScanItems;
  int64_t s = 0;
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n_groups) s += int64_t(groups[base + i].chunk_size) * T;
  int64_t total;
  int64_t off = tile_base[blockIdx.x] + block_exclusive_scan(s, &total);
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n_groups) {
      groups[base + i].offset = int32_t(off);     // host checks the total fits int32
      off += int64_t(groups[base + i].chunk_size) * T;
    }
  }
}

// Heavy-group schedule: per-tile counts, then (after the tile scan) each
// tile writes the indices of its heavy groups in ascending order.
__global__ __launch_bounds__(kScanBlock) void heavy_count_kernel(
    const argcsr_group_info* __restrict__ groups, int32_t n_groups, int32_t heavy_chunk,
    int64_t* __restrict__ tile_sums) {
  int64_t s = 0;
  const int64_t base = int64_t(blockIdx.x) * kScanTile + threadIdx.x * kScanItems;
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n_groups) s += groups[base + i].chunk_size > heavy_chunk;
  int64_t total;
  (void)block_exclusive_scan(s, &total);
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanBlock) void heavy_scatter_kernel(
    const argcsr_group_info* __restrict__ groups, int32_t n_groups, int32_t heavy_chunk,
    const int64_t* __restrict__ tile_base, int32_t* __restrict__ heavy) {
  const int64_t base = int64_t(blockIdx.x) * kScanTile + threadIdx.x * kScanItems;
  int64_t s = 0;
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n_groups) s += groups[base + i].chunk_size > heavy_chunk;
  int64_t total;
  int64_t pos = tile_base[blockIdx.x] + block_exclusive_scan(s, &total);
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n_groups && groups[base + i].chunk_size > heavy_chunk)
      heavy[pos++] = int32_t(base + i);
}

// For every chunk k of the group: where its elements start in the CSR arrays
// and how many there are (0 for free chunks), in the wave's LDS tables.
__device__ inline void chunk_sources(const argcsr_group_info& gi, const int32_t* __restrict__ rp,
                                     const int32_t* __restrict__ tm, int32_t T, int lane,
                                     int32_t* src_start, int32_t* src_len) {
  const int32_t c = gi.chunk_size;
  for (int k = lane; k < T; k += 64) src_len[k] = 0;
  wave_lds_sync();
  for (int l = lane; l < gi.size; l += 64) {
    const int32_t r = gi.first_row + l;
    const int32_t begin = l == 0 ? 0 : tm[r - 1];
    const int32_t end = tm[r];
    const int32_t row_start = rp[r];
    const int32_t L = rp[r + 1] - row_start;
    for (int32_t k = begin; k < end; ++k) {
      const int32_t q = k - begin;                    // chunk q of row r
      const int32_t first_elem = q * c;
      src_start[k] = row_start + first_elem;
      const int32_t left = L - first_elem;
      src_len[k] = left < 0 ? 0 : (left < c ? left : c);
    }
  }
  wave_lds_sync();
}

// The CSR range [lo, lo + extent) that holds the elements of the wave's 64
// chunks (start, len per lane); extent 0 when they have none.
__device__ inline int32_t block_extent(int32_t start, int32_t len, int32_t* lo_out) {
  const int32_t lo = wave_min(len > 0 ? start : INT32_MAX);
  const int32_t hi = wave_max(len > 0 ? start + len : 0);
  *lo_out = lo;
  return hi > lo ? hi - lo : 0;
}

// Step 4, one wave per group.  For every chunk k the wave first records in
// LDS where its elements start in the CSR arrays and how many there are (0 for
// free chunks).  It then takes the chunks 64 at a time.  The elements of 64
// consecutive chunks form one contiguous CSR range (a row's chunks follow each
// other, and so do the rows), so when that range fits the wave's stage of
// `stage` elements the wave copies it into LDS with coalesced loads,
// converting the values to their storage type, and then writes the block's
// slots step by step, 64 consecutive slots per store, each lane taking its
// chunk's element from LDS.  Blocks whose range is longer than the stage are
// left to fill_long_kernel: a group whose chunks are longer than stage/64
// elements, the only kind that can have such blocks, appends one work item per
// tile of kLongSteps steps to a list.  Every staged column index is checked
// against [0, n_cols) (a negative one wraps above the limit as unsigned).
template <int DT>
__global__ __launch_bounds__(kMaxFillWaves * 64) void fill_kernel(
    const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
    const double* __restrict__ val, const argcsr_group_info* __restrict__ groups,
    int32_t n_groups, int32_t n_cols, int32_t T, const int32_t* __restrict__ tm, int32_t stage,
    Status* __restrict__ st, int32_t* __restrict__ long_list,
    int32_t* __restrict__ columns, typename Val<DT>::storage* __restrict__ values) {
  using S = typename Val<DT>::storage;
  extern __shared__ int32_t fill_lds[];   // per wave: [T] starts, [T] lengths, stage
  const int lane = lane_id();
  const int w = wave_uniform(int(threadIdx.x >> 6));
  const size_t wave_bytes = fill_lds_bytes<S>(T, stage);
  int32_t* src_start = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(fill_lds) + w * wave_bytes);
  int32_t* src_len = src_start + T;
  int32_t* stage_col = src_start + 2 * T;
  S* stage_val = reinterpret_cast<S*>(stage_col + stage);
  const int g = blockIdx.x * (blockDim.x >> 6) + w;
  if (g >= n_groups) return;
  const argcsr_group_info gi = groups[g];
  const int32_t c = gi.chunk_size;
  if (int64_t(c) * 64 > stage) {   // one work item per tile of kLongSteps steps
    const int32_t n_items = (c + kLongSteps - 1) / kLongSteps;
    int32_t base = 0;
    if (lane == 0) base = atomicAdd(&st->long_items, n_items);
    base = __shfl(base, 0, 64);
    for (int32_t t = lane; t < n_items; t += 64) {
      long_list[2 * int64_t(base + t)] = g;
      long_list[2 * int64_t(base + t) + 1] = t * kLongSteps;
    }
  }
  chunk_sources(gi, rp, tm, T, lane, src_start, src_len);
  const uint32_t limit = uint32_t(n_cols);
  bool bad = false;
  for (int32_t k0 = 0; k0 < T; k0 += 64) {
    const int32_t k = k0 + lane;
    const bool mine = k < T;
    const int32_t start = mine ? src_start[k] : 0;
    const int32_t len = mine ? src_len[k] : 0;
    int32_t lo;
    const int32_t extent = block_extent(start, len, &lo);
    const int64_t dst0 = int64_t(gi.offset) + k;
    if (extent <= stage) {
#pragma unroll 8
      for (int32_t p = lane; p < extent; p += 64) {
        const int32_t cp = col[lo + p];
        bad |= uint32_t(cp) >= limit;
        stage_col[p] = cp;
        stage_val[p] = Val<DT>::from_f64(val[lo + p]);
      }
      wave_lds_sync();
      const int32_t rel = start - lo;
      for (int32_t j = 0; j < c; ++j) {
        if (!mine) continue;
        const int64_t dst = dst0 + int64_t(j) * T;
        if (j < len) {
          columns[dst] = stage_col[rel + j];
          values[dst] = stage_val[rel + j];
        } else {
          columns[dst] = -1;
          values[dst] = S(0);
        }
      }
      wave_lds_sync();   // the next block overwrites the stage
    }
  }
  if (__ballot(bad) != 0 && lane == 0) atomicOr(&st->bad_column, 1);
}

// Step 4 for the blocks fill_kernel leaves: those whose CSR range is longer
// than the stage, from the list of (group, first step) work items (in any
// order: every slot belongs to one block and one tile).  One-wave workgroups
// stride over the list; an item moves kLongSteps steps of the group's long
// blocks through LDS: each load instruction reads kLongSteps consecutive
// elements of each of 64/kLongSteps chunks (a lane past its chunk's end reads
// an element of the block and keeps the padding value, so the loads carry no
// branch and are issued together), and each store writes one step of the 64
// chunks, 64 consecutive slots.  The column indices of the elements it moves
// are checked as in fill_kernel.
template <int DT>
__global__ __launch_bounds__(64) void fill_long_kernel(
    const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
    const double* __restrict__ val, const argcsr_group_info* __restrict__ groups,
    int32_t n_cols, int32_t T, const int32_t* __restrict__ tm, int32_t stage,
    Status* __restrict__ st,
    const int32_t* __restrict__ long_list, int32_t* __restrict__ columns,
    typename Val<DT>::storage* __restrict__ values) {
  using S = typename Val<DT>::storage;
  constexpr int kPer = 64 / kLongSteps;           // chunks per load instruction
  __shared__ int32_t tile_col[kLongSteps][65];    // [step][chunk], padded rows
  __shared__ S tile_val[kLongSteps][65];
  extern __shared__ int32_t long_tables[];        // [T] starts, [T] lengths
  int32_t* src_start = long_tables;
  int32_t* src_len = long_tables + T;
  const int lane = lane_id();
  const int jj = lane % kLongSteps, kq = lane / kLongSteps;
  const int32_t n_items = st->long_items;
  const uint32_t limit = uint32_t(n_cols);
  bool bad = false;
  for (int32_t i = blockIdx.x; i < n_items; i += gridDim.x) {
    const argcsr_group_info gi = groups[long_list[2 * int64_t(i)]];
    const int32_t j0 = long_list[2 * int64_t(i) + 1];
    const int32_t c = gi.chunk_size;
    chunk_sources(gi, rp, tm, T, lane, src_start, src_len);
    for (int32_t k0 = 0; k0 < T; k0 += 64) {
      const int32_t k = k0 + lane;
      int32_t lo;
      if (block_extent(k < T ? src_start[k] : 0, k < T ? src_len[k] : 0, &lo) <= stage) continue;
      int32_t cv[kLongSteps];
      double v[kLongSteps];
      bool ok[kLongSteps];
#pragma unroll
      for (int it = 0; it < kLongSteps; ++it) {
        const int32_t kk = k0 + it * kPer + kq;
        const int32_t kc = kk < T ? kk : T - 1;
        const int32_t j = j0 + jj;
        ok[it] = kk < T && j < src_len[kc];
        const int32_t e = ok[it] ? src_start[kc] + j : lo;
        cv[it] = col[e];
        v[it] = val[e];
        bad |= ok[it] && uint32_t(cv[it]) >= limit;
      }
#pragma unroll
      for (int it = 0; it < kLongSteps; ++it) {
        const int32_t kl = it * kPer + kq;          // chunk within the block
        tile_col[jj][kl] = ok[it] ? cv[it] : -1;
        tile_val[jj][kl] = ok[it] ? Val<DT>::from_f64(v[it]) : S(0);
      }
      wave_lds_sync();
      const int32_t steps = c - j0 < kLongSteps ? c - j0 : kLongSteps;
      if (k < T)
#pragma unroll 4
        for (int32_t u = 0; u < steps; ++u) {
          const int64_t dst = int64_t(gi.offset) + int64_t(j0 + u) * T + k;
          columns[dst] = tile_col[u][lane];
          values[dst] = tile_val[u][lane];
        }
      wave_lds_sync();   // the next block or item overwrites the tile and tables
    }
  }
  if (__ballot(bad) != 0 && lane == 0) atomicOr(&st->bad_column, 1);
}

// The stage holds the blocks of chunks up to twice the matrix's mean chunk
// size (at least 4 and at most 32 elements per chunk); small stages leave room
// for 4 waves per workgroup, which the many short groups of irregular
// matrices need to hide their latency.
template <int DT>
void launch_fill(int32_t n_groups, hipStream_t s, const int32_t* rp, const int32_t* col,
                 const double* val, Status* st, int32_t* long_list, const argcsr_matrix* out) {
  using S = typename Val<DT>::storage;
  const int64_t T = out->block_dim;
  const int64_t mean_chunk = (out->n_slots + int64_t(n_groups) * T - 1) / (int64_t(n_groups) * T);
  int32_t stage = kMinStage;
  while (stage < kMaxStage && stage < 128 * mean_chunk) stage *= 2;
  const int waves = stage <= 512 ? kMaxFillWaves : 1;
  const size_t lds = fill_lds_bytes<S>(int32_t(T), stage) * size_t(waves);
  const uint32_t blocks = uint32_t((int64_t(n_groups) + waves - 1) / waves);
  fill_kernel<DT><<<dim3(blocks), 64 * waves, lds, s>>>(
      rp, col, val, out->groups, out->n_groups, out->n_cols, out->block_dim, out->threads_mapping,
      stage, st, long_list, out->columns, static_cast<S*>(out->values));
  const int64_t long_blocks = std::min<int64_t>(n_groups, kLongGrid);
  fill_long_kernel<DT><<<dim3(uint32_t(long_blocks)), 64, sizeof(int32_t) * 2 * size_t(T), s>>>(
      rp, col, val, out->groups, out->n_cols, out->block_dim, out->threads_mapping, stage, st,
      long_list, out->columns, static_cast<S*>(out->values));
}

}  // namespace
}  // namespace argcsr

// A device plan (argcsr_plan_device_keep): steps 1-3 of one matrix kept on
// the device for argcsr_convert_planned.
// Its buffers are stream-ordered allocations on the planning stream (freed
// on it too: every conversion with the plan has waited for its own work).
struct argcsr_device_plan {
  int32_t n_rows = 0, block_dim = 0, desired_chunk_size = 0, format = 0;
  int32_t n_groups = 0, n_heavy = 0;
  int64_t n_slots = 0;
  argcsr_group_info* groups = nullptr;    // first_row, size, chunk_size (offset not yet set)
  int32_t* tm = nullptr;                  // threads mapping
  void* block = nullptr;                  // the one allocation holding both
  hipStream_t stream = nullptr;
  ~argcsr_device_plan() {
    if (block) (void)hipFreeAsync(block, stream);
  }
};

// Fixed scratch of argcsr_convert_noalloc: one copy per GPU (this process's
// code object), held until the process ends.  Host code reaches it only
// through the address hipGetSymbolAddress returns for the current device.
constexpr size_t kNoAllocScratchBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace argcsr {
namespace {

// Device scratch of one conversion: status words, the two tile-sum arrays of
// the offset and heavy scans, and the fill's long-row list.  Items of that
// list: a group makes them only when its chunk size c exceeds
// stage/64 >= kMinStage/64 = 4, and then ceil(c/16) <= c/4 of them, so all
// groups together make at most n_slots/(4T).
static_assert(kMinStage / 64 >= 4 && kLongSteps == 16, "long-list bound");
struct ConvertScratch {
  int32_t n_tiles;
  int64_t long_capacity;
  size_t bytes;
};

ConvertScratch convert_scratch(int32_t n_groups, int64_t n_slots, int32_t T) {
  ConvertScratch c;
  c.n_tiles = (n_groups + kScanTile - 1) / kScanTile;
  c.long_capacity = n_slots / (4 * int64_t(T)) + 1;
  c.bytes = sizeof(Status) + 2 * sizeof(int64_t) * size_t(c.n_tiles) +
            2 * sizeof(int32_t) * size_t(c.long_capacity);
  return c;
}

constexpr int kMaxDevices = 64;
// Step-1 groups of argcsr_convert_noalloc pass through this host buffer on
// their way to the device (copied and waited for chunk by chunk).
constexpr int32_t kGroupChunk = 1 << 16;
argcsr_group_info g_group_chunk[kGroupChunk];
std::mutex g_noalloc_mu;                    // one argcsr_convert_noalloc at a time
void* g_noalloc_ptr[kMaxDevices] = {};       // device address of `scratch`, per device

// The current device's address of `scratch` (looked up once per device,
// with that device current).  Caller holds g_noalloc_mu.
int noalloc_scratch(void** out) {
  int dev = -1;
  ARGCSR_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(ARGCSR_EUNSUPPORTED, "device %d", dev);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(ARGCSR_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_noalloc_ptr[dev] = p;
  }
  *out = g_noalloc_ptr[dev];
  return ARGCSR_OK;
}

// All four steps.  With `fixed` (argcsr_convert_noalloc) the scratch is the
// given device memory of fixed_bytes, step 1 runs on the host from
// row_ptr_host (required) and its groups reach the device through
// g_group_chunk; nothing is allocated.
int convert_impl(int32_t n_rows, int32_t n_cols, const int32_t* row_ptr_host,
                 const int32_t* row_ptr, const int32_t* col, const double* val,
                 argcsr_matrix* out, hipStream_t s, bool fixed,
                 const argcsr_device_plan* planned = nullptr,
                 const argcsr_group_info* pregrouped = nullptr) {
  if (!out) return fail(ARGCSR_EINVAL, "out is NULL");
  if (n_rows < 0 || n_cols < 0) return fail(ARGCSR_EINVAL, "negative dimension");
  if (out->n_rows != n_rows || out->n_cols != n_cols)
    return fail(ARGCSR_EINVAL, "out->n_rows/n_cols do not match the arguments");
  const int32_t T = out->block_dim;
  if (T < 1 || T > kMaxBlockDim)
    return fail(ARGCSR_EUNSUPPORTED, "block_dim %d outside [1, %d]", T, kMaxBlockDim);
  if (out->format != ARGCSR_FORMAT_ARG && out->format != ARGCSR_FORMAT_RG)
    return fail(ARGCSR_EINVAL, "unknown format %d", out->format);
  if (out->format == ARGCSR_FORMAT_ARG && out->desired_chunk_size < 1 && !out->region_desired)
    return fail(ARGCSR_EINVAL, "desired_chunk_size < 1");
  if (out->dtype < ARGCSR_F64 || out->dtype > ARGCSR_F16)
    return fail(ARGCSR_EINVAL, "unknown dtype %d", out->dtype);
  if (out->n_groups < 0 || out->n_slots < 0) return fail(ARGCSR_EINVAL, "negative size in out");
  const int32_t* regions = out->format == ARGCSR_FORMAT_ARG ? out->region_desired : nullptr;
  int rc = check_regions(n_rows, out->region_rows, regions);
  if (rc) return rc;
  void* fixed_ptr = nullptr;
  if (fixed) {
    if (!row_ptr_host)
      return fail(ARGCSR_EINVAL, "argcsr_convert_noalloc needs row_ptr_host (step 1 on the host)");
    const ConvertScratch need = convert_scratch(out->n_groups, out->n_slots, T);
    if (need.bytes > kNoAllocScratchBytes)
      return fail(ARGCSR_EINVAL,
                  "the conversion needs %zu bytes of scratch, more than the %zu bytes "
                  "argcsr_convert_noalloc holds", need.bytes, kNoAllocScratchBytes);
  }
  // step 1: on the host from row_ptr_host, or on the device (group.hip)
  std::vector<argcsr_group_info> host_groups;
  DeviceGrouping device_groups;
  int64_t nnz = 0;
  int32_t G = 0;
  bool groups_uploaded = false;
  if (planned) {
    // steps 1-3 were kept by argcsr_plan_device_keep
    if (n_rows > 0 && !row_ptr) return fail(ARGCSR_EINVAL, "row_ptr is NULL");
    G = planned->n_groups;
    if (n_rows > 0) {
      int32_t last = 0;
      ARGCSR_HIP(hipMemcpyAsync(&last, row_ptr + n_rows, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      ARGCSR_HIP(hipStreamSynchronize(s));
      nnz = last;
    }
  } else if (row_ptr_host && pregrouped) {
    // step 1 done (and row_ptr_host validated) by the caller
    nnz = n_rows > 0 ? row_ptr_host[n_rows] : 0;
    G = out->n_groups;
    if (G > 0 && !out->groups) return fail(ARGCSR_EINVAL, "NULL device buffer");
    if (G > 0)
      ARGCSR_HIP(hipMemcpyAsync(out->groups, pregrouped, sizeof(argcsr_group_info) * size_t(G),
                                hipMemcpyHostToDevice, s));
    groups_uploaded = true;
  } else if (row_ptr_host) {
    rc = check_row_ptr(n_rows, row_ptr_host);
    if (rc) return rc;
    nnz = n_rows > 0 ? row_ptr_host[n_rows] : 0;
    if (fixed) {
      if (out->n_groups > 0 && !out->groups) return fail(ARGCSR_EINVAL, "NULL device buffer");
      rc = noalloc_scratch(&fixed_ptr);
      if (rc) return rc;
      // groups go to out->groups a chunk at a time, never past out->n_groups
      int32_t filled = 0;
      auto flush = [&]() -> int {
        if (filled == 0) return ARGCSR_OK;
        ARGCSR_HIP(hipMemcpyAsync(out->groups + (G - filled), g_group_chunk,
                                  sizeof(argcsr_group_info) * size_t(filled),
                                  hipMemcpyHostToDevice, s));
        ARGCSR_HIP(hipStreamSynchronize(s));       // the buffer is reused next
        filled = 0;
        return ARGCSR_OK;
      };
      rc = for_each_group(n_rows, row_ptr_host, T, out->desired_chunk_size, out->format,
                          out->region_rows, regions, [&](int32_t first, int32_t size) -> int {
                            if (G >= out->n_groups)
                              return fail(ARGCSR_EINVAL, "out->n_groups = %d but the matrix "
                                          "has more groups", out->n_groups);
                            g_group_chunk[filled++] = argcsr_group_info{first, size, 0, 0};
                            ++G;
                            return filled == kGroupChunk ? flush() : 0;
                          });
      if (rc) return rc;
      rc = flush();
      if (rc) return rc;
      groups_uploaded = true;
    } else {
      rc = group_rows(n_rows, row_ptr_host, T, out->desired_chunk_size, out->format,
                      &host_groups, out->region_rows, regions);
      if (rc) return rc;
      G = (int32_t)host_groups.size();
    }
  } else {
    if (n_rows > 0 && !row_ptr) return fail(ARGCSR_EINVAL, "row_ptr is NULL");
    rc = device_groups.build(n_rows, row_ptr, T, out->desired_chunk_size, out->format, s,
                             out->region_rows, regions);
    if (rc) return rc;
    G = device_groups.n_groups;
    if (n_rows > 0) {
      int32_t last = 0;
      ARGCSR_HIP(hipMemcpyAsync(&last, row_ptr + n_rows, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      ARGCSR_HIP(hipStreamSynchronize(s));
      nnz = last;
    }
  }
  if (G != out->n_groups)
    return fail(ARGCSR_EINVAL, "out->n_groups = %d but the matrix has %d groups", out->n_groups, G);
  out->nnz = nnz;
  out->heavy_chunk = heavy_chunk_for(T, out->n_slots, G);
  if (G == 0) {
    out->n_heavy = 0;
    if (out->n_slots != 0) return fail(ARGCSR_EINVAL, "out->n_slots must be 0 for an empty matrix");
    return ARGCSR_OK;
  }
  if (!row_ptr || !out->groups || !out->threads_mapping || !out->columns || !out->values ||
      (nnz > 0 && (!col || !val)))
    return fail(ARGCSR_EINVAL, "NULL device buffer");

  const ConvertScratch cs = convert_scratch(G, out->n_slots, T);
  const int32_t n_tiles = cs.n_tiles;
  StreamScratch ws;
  void* base = fixed_ptr;
  if (!fixed) {
    rc = ws.alloc(cs.bytes, s);
    if (rc) return rc;
    base = ws.ptr;
  }
  Status* st = static_cast<Status*>(base);
  int64_t* tile_sums = reinterpret_cast<int64_t*>(st + 1);
  int64_t* heavy_tiles = tile_sums + n_tiles;
  // (group, first step) per tile of the fill's long blocks
  int32_t* long_list = reinterpret_cast<int32_t*>(heavy_tiles + n_tiles);
  // uses the caller's slot count; it is checked against the device total
  // before anything is written to the caller's heavy_groups buffer
  const int32_t heavy_chunk = out->heavy_chunk;

  clear_status_kernel<<<1, 1, 0, s>>>(st);
  if (planned) {
    copy_words(planned->groups, out->groups, 4 * int64_t(G), s);
    copy_words(planned->tm, out->threads_mapping, int64_t(n_rows), s);
  } else {
    if (row_ptr_host) {
      if (!groups_uploaded)
        ARGCSR_HIP(hipMemcpyAsync(out->groups, host_groups.data(),
                                  sizeof(argcsr_group_info) * size_t(G), hipMemcpyHostToDevice,
                                  s));
    } else {
      rc = device_groups.write(out->groups);
      if (rc) return rc;
    }
    const int wave_blocks = (G + kWaves - 1) / kWaves;
    chunks_kernel<<<wave_blocks, kWaves * 64, 0, s>>>(row_ptr, out->groups, G, T,
                                                     out->format == ARGCSR_FORMAT_RG ? 1 : 0,
                                                     out->threads_mapping);
  }
  ARGCSR_HIP(hipGetLastError());
  offsets_reduce_kernel<<<n_tiles, kScanBlock, 0, s>>>(out->groups, G, T, tile_sums);
  tiles_scan_kernel<<<1, kScanBlock, 0, s>>>(tile_sums, n_tiles, &st->total_slots);
  offsets_apply_kernel<<<n_tiles, kScanBlock, 0, s>>>(out->groups, G, T, tile_sums);
  heavy_count_kernel<<<n_tiles, kScanBlock, 0, s>>>(out->groups, G, heavy_chunk, heavy_tiles);
  tiles_scan_kernel<<<1, kScanBlock, 0, s>>>(heavy_tiles, n_tiles, &st->total_heavy);
  ARGCSR_HIP(hipGetLastError());

  Status host_st{};
  ARGCSR_HIP(hipMemcpyAsync(&host_st, st, sizeof(Status), hipMemcpyDeviceToHost, s));
  ARGCSR_HIP(hipStreamSynchronize(s));
  if (host_st.total_slots > INT32_MAX)
    return fail(ARGCSR_EOVERFLOW, "%lld slots exceed INT32_MAX", host_st.total_slots);
  if (host_st.total_slots != out->n_slots)
    return fail(ARGCSR_EINVAL, "out->n_slots = %lld but the matrix needs %lld",
                (long long)out->n_slots, host_st.total_slots);
  if (out->heavy_groups && host_st.total_heavy != out->n_heavy)
    return fail(ARGCSR_EINVAL, "out->n_heavy = %d but the matrix has %lld heavy groups",
                out->n_heavy, host_st.total_heavy);
  out->n_heavy = int32_t(host_st.total_heavy);
  if (out->heavy_groups && out->n_heavy > 0)
    heavy_scatter_kernel<<<n_tiles, kScanBlock, 0, s>>>(out->groups, G, heavy_chunk, heavy_tiles,
                                                        out->heavy_groups);

  switch (out->dtype) {
    case ARGCSR_F64: launch_fill<ARGCSR_F64>(G, s, row_ptr, col, val, st, long_list, out); break;
    case ARGCSR_F32: launch_fill<ARGCSR_F32>(G, s, row_ptr, col, val, st, long_list, out); break;
    case ARGCSR_BF16: launch_fill<ARGCSR_BF16>(G, s, row_ptr, col, val, st, long_list, out); break;
    default: launch_fill<ARGCSR_F16>(G, s, row_ptr, col, val, st, long_list, out); break;
  }
  ARGCSR_HIP(hipGetLastError());
  ARGCSR_HIP(hipMemcpyAsync(&host_st, st, sizeof(Status), hipMemcpyDeviceToHost, s));
  ARGCSR_HIP(hipStreamSynchronize(s));
  if (host_st.bad_column)
    return fail(ARGCSR_EINVAL, "a column index lies outside [0, %d)", n_cols);
  return ARGCSR_OK;
}

}  // namespace
}  // namespace argcsr

namespace argcsr {

int convert_pregrouped(int32_t n_rows, int32_t n_cols, const int32_t* row_ptr_host,
                       const argcsr_group_info* groups_host, const int32_t* row_ptr,
                       const int32_t* col, const double* val, argcsr_matrix* out,
                       hipStream_t s) {
  if (!row_ptr_host || (out && out->n_groups > 0 && !groups_host))
    return fail(ARGCSR_EINVAL, "a pregrouped conversion needs row_ptr_host and the groups");
  return convert_impl(n_rows, n_cols, row_ptr_host, row_ptr, col, val, out, s, false, nullptr,
                      groups_host);
}

}  // namespace argcsr

extern "C" int argcsr_convert(int32_t n_rows, int32_t n_cols, const int32_t* row_ptr_host,
                              const int32_t* row_ptr, const int32_t* col, const double* val,
                              argcsr_matrix* out, void* stream) {
  argcsr::clear_error();
  return argcsr::convert_impl(n_rows, n_cols, row_ptr_host, row_ptr, col, val, out,
                              static_cast<hipStream_t>(stream), false);
}

extern "C" int argcsr_convert_noalloc(int32_t n_rows, int32_t n_cols, const int32_t* row_ptr_host,
                                      const int32_t* row_ptr, const int32_t* col,
                                      const double* val, argcsr_matrix* out, void* stream) {
  argcsr::clear_error();
  std::lock_guard<std::mutex> lock(argcsr::g_noalloc_mu);
  return argcsr::convert_impl(n_rows, n_cols, row_ptr_host, row_ptr, col, val, out,
                              static_cast<hipStream_t>(stream), true);
}

namespace argcsr {
namespace {

// Steps 1-3 from a device row_ptr; the sizes of the result.  With `keep`,
// the group table and the threads mapping stay in device memory the plan
// owns; otherwise they live in stream-ordered scratch and are dropped.
int plan_device_impl(int32_t n_rows, const int32_t* row_ptr, int32_t block_dim,
                     int32_t desired_chunk_size, int32_t format, int32_t* n_groups,
                     int64_t* n_slots, int32_t* n_heavy, hipStream_t s, argcsr_device_plan* keep) {
  if (!n_groups || !n_slots) return fail(ARGCSR_EINVAL, "NULL output pointer");
  if (n_rows < 0) return fail(ARGCSR_EINVAL, "n_rows < 0");
  if (format != ARGCSR_FORMAT_ARG && format != ARGCSR_FORMAT_RG)
    return fail(ARGCSR_EINVAL, "unknown format %d", format);
  if (block_dim < 1 || block_dim > kMaxBlockDim ||
      (format == ARGCSR_FORMAT_ARG && desired_chunk_size < 1))
    return fail(ARGCSR_EINVAL, "block_dim must be in [1, %d] and desired_chunk_size >= 1",
                kMaxBlockDim);
  if (n_rows > 0 && !row_ptr) return fail(ARGCSR_EINVAL, "row_ptr is NULL");
  DeviceGrouping dg;
  int rc = dg.build(n_rows, row_ptr, block_dim, desired_chunk_size, format, s);
  if (rc) return rc;
  const int32_t G = dg.n_groups;
  *n_groups = G;
  *n_slots = 0;
  if (n_heavy) *n_heavy = 0;
  if (G == 0) return ARGCSR_OK;
  // steps 2-3 (into the plan's buffers or scratch): the chunk sizes give the
  // slot count and the heavy-group count exactly as argcsr_plan computes
  // them on the host
  const int32_t n_tiles = (G + kScanTile - 1) / kScanTile;
  const size_t groups_bytes = sizeof(argcsr_group_info) * size_t(G);
  const size_t tm_bytes = (sizeof(int32_t) * size_t(n_rows) + 15) / 16 * 16;
  StreamScratch ws;
  rc = ws.alloc(groups_bytes + tm_bytes + sizeof(Status) + 2 * sizeof(int64_t) * size_t(n_tiles), s);
  if (rc) return rc;
  argcsr_group_info* groups = static_cast<argcsr_group_info*>(ws.ptr);
  int32_t* tm = reinterpret_cast<int32_t*>(static_cast<char*>(ws.ptr) + groups_bytes);
  if (keep) {                    // the plan takes the scratch over at the end (groups and mapping first)
    keep->stream = s;
    keep->groups = groups;
    keep->tm = tm;
  }
  auto* st = reinterpret_cast<Status*>(static_cast<char*>(ws.ptr) + groups_bytes + tm_bytes);
  int64_t* tile_sums = reinterpret_cast<int64_t*>(st + 1);
  int64_t* heavy_tiles = tile_sums + n_tiles;
  clear_status_kernel<<<1, 1, 0, s>>>(st);
  rc = dg.write(groups);
  if (rc) return rc;
  const int wave_blocks = (G + kWaves - 1) / kWaves;
  chunks_kernel<<<wave_blocks, kWaves * 64, 0, s>>>(row_ptr, groups, G, block_dim,
                                                   format == ARGCSR_FORMAT_RG ? 1 : 0, tm);
  offsets_reduce_kernel<<<n_tiles, kScanBlock, 0, s>>>(groups, G, block_dim, tile_sums);
  tiles_scan_kernel<<<1, kScanBlock, 0, s>>>(tile_sums, n_tiles, &st->total_slots);
  ARGCSR_HIP(hipGetLastError());
  Status host_st{};
  ARGCSR_HIP(hipMemcpyAsync(&host_st, st, sizeof(Status), hipMemcpyDeviceToHost, s));
  ARGCSR_HIP(hipStreamSynchronize(s));
  const int64_t S = host_st.total_slots;
  const int32_t heavy_chunk = heavy_chunk_for(block_dim, S, G);
  heavy_count_kernel<<<n_tiles, kScanBlock, 0, s>>>(groups, G, heavy_chunk, heavy_tiles);
  tiles_scan_kernel<<<1, kScanBlock, 0, s>>>(heavy_tiles, n_tiles, &st->total_heavy);
  ARGCSR_HIP(hipGetLastError());
  ARGCSR_HIP(hipMemcpyAsync(&host_st, st, sizeof(Status), hipMemcpyDeviceToHost, s));
  ARGCSR_HIP(hipStreamSynchronize(s));
  *n_slots = S;
  if (n_heavy) *n_heavy = int32_t(host_st.total_heavy);
  if (keep) {
    keep->block = ws.ptr;        // owned by the plan now (freed with it)
    ws.ptr = nullptr;
    keep->n_groups = G;
    keep->n_slots = S;
    keep->n_heavy = int32_t(host_st.total_heavy);
  }
  if (S > INT32_MAX) return fail(ARGCSR_EOVERFLOW, "%lld slots exceed INT32_MAX", (long long)S);
  return ARGCSR_OK;
}

}  // namespace
}  // namespace argcsr

extern "C" int argcsr_plan_device(int32_t n_rows, const int32_t* row_ptr, int32_t block_dim,
                                  int32_t desired_chunk_size, int32_t format, int32_t* n_groups,
                                  int64_t* n_slots, int32_t* n_heavy, void* stream) {
  argcsr::clear_error();
  return argcsr::plan_device_impl(n_rows, row_ptr, block_dim, desired_chunk_size, format,
                                  n_groups, n_slots, n_heavy, static_cast<hipStream_t>(stream),
                                  nullptr);
}

extern "C" int argcsr_plan_device_keep(int32_t n_rows, const int32_t* row_ptr, int32_t block_dim,
                                       int32_t desired_chunk_size, int32_t format,
                                       int32_t* n_groups, int64_t* n_slots, int32_t* n_heavy,
                                       argcsr_device_plan** plan, void* stream) {
  using namespace argcsr;
  clear_error();
  if (!plan) return fail(ARGCSR_EINVAL, "plan is NULL");
  *plan = nullptr;
  auto* p = new (std::nothrow) argcsr_device_plan();
  if (!p) return fail(ARGCSR_ENOMEM, "device plan");
  p->n_rows = n_rows;
  p->block_dim = block_dim;
  p->desired_chunk_size = format == ARGCSR_FORMAT_RG ? 0 : desired_chunk_size;
  p->format = format;
  const int rc = plan_device_impl(n_rows, row_ptr, block_dim, desired_chunk_size, format,
                                  n_groups, n_slots, n_heavy, static_cast<hipStream_t>(stream), p);
  if (rc) {
    delete p;
    return rc;
  }
  *plan = p;
  return ARGCSR_OK;
}

extern "C" int argcsr_convert_planned(const argcsr_device_plan* plan, int32_t n_cols,
                                      const int32_t* row_ptr, const int32_t* col,
                                      const double* val, argcsr_matrix* out, void* stream) {
  using namespace argcsr;
  clear_error();
  if (!plan || !out) return fail(ARGCSR_EINVAL, "plan or out is NULL");
  if (out->n_rows != plan->n_rows || out->block_dim != plan->block_dim ||
      out->format != plan->format || out->n_groups != plan->n_groups ||
      out->n_slots != plan->n_slots ||
      (plan->format == ARGCSR_FORMAT_ARG && out->desired_chunk_size != plan->desired_chunk_size))
    return fail(ARGCSR_EINVAL, "out does not describe the planned matrix");
  if (out->region_desired) return fail(ARGCSR_EINVAL, "a device plan has one desired_chunk_size");
  if (out->heavy_groups && out->n_heavy != plan->n_heavy)
    return fail(ARGCSR_EINVAL, "out->n_heavy = %d but the plan has %d", out->n_heavy,
                plan->n_heavy);
  return convert_impl(plan->n_rows, n_cols, nullptr, row_ptr, col, val, out,
                      static_cast<hipStream_t>(stream), false, plan);
}

extern "C" int argcsr_device_plan_destroy(argcsr_device_plan* plan) {
  delete plan;
  return ARGCSR_OK;
}
