// Conversion step 1 (grouping, Sec. 3) on the GPU.
//
// The rule is the host's (plan.cpp): from a group's first row s the group
// takes rows while it keeps at most block_dim rows and at most
// desired*block_dim nonzeros, and always takes row s.  So the group opened
// at s ends at
//   next(s) = max(s+1, max{e <= min(n, s+block_dim) : rp[e] - rp[s] <= budget}),
// a function of s alone, and the groups are the path 0 -> next(0) ->
// next(next(0)) -> ... -> n.  A scan along that path is sequential; here it
// is replaced by binary lifting:
//   1. next_kernel      J_0[r] = next(r) for every row (a binary search on
//                       row_ptr staged in LDS), J_0[n] = n;
//   2. jump_kernel      J_{k+1}[r] = J_k[J_k[r]]: 2^(k+1) groups ahead, and in
//                       the same launch J_{k+2}[r] = J_k[J_k[J_{k+1}[r]]];
//   3. count_kernel     the number of groups, by descending the levels from 0;
//   4. starts_kernel    group i starts at p_i = J applied along the bits of i
//                       (at most K lookups per group) and ends at J_0[p_i].
// Work O(n log n), depth O(log n); the result is the host scan's, row for
// row.  The levels take (K+1)*(n+1) int32 of stream-ordered scratch,
// K = bit length of n.
#include <hip/hip_runtime.h>

#include <mutex>

#include "common.hpp"
#include "group.hpp"

namespace argcsr {
namespace {

constexpr int kGroupBlock = 256;
constexpr int kMaxGroupDim = 1024;   // block_dim limit of plan/convert

__global__ void fill_i32_kernel(int32_t* __restrict__ p, int32_t n, int32_t v) {
  for (int32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = v;
}

// J_0 and row_ptr validation (rp[0] == 0, non-decreasing).  Block b handles
// rows [b*256, b*256+256); it stages rp over those rows plus the block_dim
// rows any of their groups can reach.
__global__ __launch_bounds__(kGroupBlock) void next_kernel(
    int32_t n, const int32_t* __restrict__ rp, int32_t block_dim, int64_t budget,
    int32_t region_rows, const int32_t* __restrict__ region_desired,
    int32_t* __restrict__ j0, int32_t* __restrict__ bad) {
  __shared__ int32_t srp[kGroupBlock + kMaxGroupDim + 1];
  const int64_t base = int64_t(blockIdx.x) * kGroupBlock;
  const int64_t span = min(int64_t(n) - base, int64_t(kGroupBlock) + block_dim);  // rows base..base+span
  for (int64_t i = threadIdx.x; i <= span; i += kGroupBlock) srp[i] = rp[base + i];
  __syncthreads();
  const int64_t r = base + threadIdx.x;
  if (r > n) return;
  if (r == n) {
    j0[n] = n;
    return;
  }
  const int32_t l = int32_t(threadIdx.x);
  if (srp[l + 1] < srp[l] || (r == 0 && srp[0] != 0)) {
    bad[0] = 1;
    j0[r] = int32_t(r + 1);       // keeps every pointer moving forward
    return;
  }
  // a per-region desiredChunkSize: the region of the group's first row r
  if (region_desired) budget = int64_t(region_desired[r / region_rows]) * block_dim;
  const int64_t limit = int64_t(srp[l]) + budget;
  const int32_t hi = int32_t(min(int64_t(n) - base, int64_t(l) + block_dim));  // local index
  // largest e in [l+1, hi] with srp[e] <= limit, or l+1 if none
  int32_t lo = l + 1, top = hi;
  if (int64_t(srp[lo]) <= limit) {
    while (lo < top) {
      const int32_t mid = lo + (top - lo + 1) / 2;
      if (int64_t(srp[mid]) <= limit) lo = mid;
      else top = mid - 1;
    }
  }
  j0[r] = int32_t(base + lo);
}

// Levels k+1 and (when jk2 is given) k+2 from level k alone; every index is
// a value of J_k, which lies in [0, n].
__global__ __launch_bounds__(kGroupBlock) void jump_kernel(int32_t n, const int32_t* __restrict__ jk,
                                                           int32_t* __restrict__ jk1,
                                                           int32_t* __restrict__ jk2) {
  const int64_t r = int64_t(blockIdx.x) * kGroupBlock + threadIdx.x;
  if (r > n) return;
  const int32_t a = jk[jk[r]];
  jk1[r] = a;
  if (jk2) jk2[r] = jk[jk[a]];
}

// groups = 1 + the largest number of jumps from row 0 that stays below n
__global__ void count_kernel(int32_t n, const int32_t* __restrict__ levels, int32_t levels_n,
                             int64_t stride, int32_t* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int32_t p = 0;
  int64_t jumps = 0;
  for (int32_t k = levels_n - 1; k >= 0; --k) {
    const int32_t q = levels[int64_t(k) * stride + p];
    if (q < n) {
      p = q;
      jumps += int64_t(1) << k;
    }
  }
  out[0] = int32_t(jumps + 1);
}

__global__ __launch_bounds__(kGroupBlock) void starts_kernel(
    int32_t n_groups, const int32_t* __restrict__ levels, int32_t levels_n, int64_t stride,
    argcsr_group_info* __restrict__ groups) {
  const int64_t i = int64_t(blockIdx.x) * kGroupBlock + threadIdx.x;
  if (i >= n_groups) return;
  int32_t p = 0;
  for (int32_t k = levels_n - 1; k >= 0; --k)
    if ((i >> k) & 1) p = levels[int64_t(k) * stride + p];
  groups[i] = argcsr_group_info{p, levels[p] - p, 0, 0};
}

}  // namespace

int scratch_alloc_async(void** p, size_t bytes, hipStream_t s) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static hipMemPool_t pools[kMaxDevices] = {};
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(ARGCSR_EHIP, "no current device");
  hipMemPool_t pool = nullptr;
  {
    std::lock_guard<std::mutex> lock(mu);
    if (!pools[dev]) {
      hipMemPoolProps props{};
      props.allocType = hipMemAllocationTypePinned;
      props.location.type = hipMemLocationTypeDevice;
      props.location.id = dev;
      hipMemPool_t created = nullptr;
      if (hipMemPoolCreate(&created, &props) != hipSuccess)
        return fail(ARGCSR_ENOMEM, "memory pool of device %d could not be created", dev);
      uint64_t keep_all = UINT64_MAX;
      (void)hipMemPoolSetAttribute(created, hipMemPoolAttrReleaseThreshold, &keep_all);
      pools[dev] = created;
    }
    pool = pools[dev];
  }
  if (hipMallocFromPoolAsync(p, bytes < 256 ? 256 : bytes, pool, s) != hipSuccess) {
    *p = nullptr;
    return fail(ARGCSR_ENOMEM, "device scratch of %zu bytes could not be allocated", bytes);
  }
  return ARGCSR_OK;
}

int StreamScratch::alloc(size_t bytes, hipStream_t s) {
  stream = s;
  if (scratch_alloc_async(&ptr, bytes, s) != ARGCSR_OK) {
    ptr = nullptr;
    return fail(ARGCSR_ENOMEM, "device scratch of %zu bytes could not be allocated", bytes);
  }
  return ARGCSR_OK;
}

int DeviceGrouping::build(int32_t n, const int32_t* rp, int32_t block_dim, int32_t desired,
                          int32_t format, hipStream_t s, int32_t region_rows,
                          const int32_t* region_desired) {
  release();
  stream = s;
  n_rows = n;
  n_groups = 0;
  if (n == 0) return ARGCSR_OK;
  const bool row_grouped = format == ARGCSR_FORMAT_RG;
  if (block_dim < 1 || block_dim > kMaxGroupDim ||
      (!row_grouped && !region_desired && desired < 1) || (region_desired && region_rows < 1))
    return fail(ARGCSR_EINVAL, "block_dim must be in [1, %d] and desired_chunk_size >= 1",
                kMaxGroupDim);
  levels_n = 1;
  while ((int64_t(1) << levels_n) <= n) ++levels_n;   // 2^levels_n > n >= any jump count
  stride = int64_t(n) + 1;
  const int64_t n_regions = region_desired ? (int64_t(n) + region_rows - 1) / region_rows : 0;
  const size_t bytes = sizeof(int32_t) * (size_t(levels_n) * size_t(stride) + 2 + size_t(n_regions));
  if (scratch_alloc_async(reinterpret_cast<void**>(&levels), bytes, s) != ARGCSR_OK) {
    levels = nullptr;
    return fail(ARGCSR_ENOMEM, "grouping tables of %zu bytes could not be allocated", bytes);
  }
  int32_t* flags = levels + size_t(levels_n) * size_t(stride);   // [0] bad row_ptr, [1] count
  int32_t* d_regions = n_regions ? flags + 2 : nullptr;
  fill_i32_kernel<<<1, 64, 0, s>>>(flags, 2, 0);
  if (d_regions)
    ARGCSR_HIP(hipMemcpyAsync(d_regions, region_desired, sizeof(int32_t) * size_t(n_regions),
                              hipMemcpyHostToDevice, s));
  const int64_t blocks = (int64_t(n) + 1 + kGroupBlock - 1) / kGroupBlock;
  next_kernel<<<dim3(uint32_t(blocks)), kGroupBlock, 0, s>>>(
      n, rp, block_dim, row_grouped ? INT64_MAX / 2 : int64_t(desired) * block_dim,
      row_grouped ? 1 : region_rows, row_grouped ? nullptr : d_regions, levels, flags);
  for (int32_t k = 0; k + 1 < levels_n; k += 2)
    jump_kernel<<<dim3(uint32_t(blocks)), kGroupBlock, 0, s>>>(
        n, levels + k * stride, levels + (k + 1) * stride,
        k + 2 < levels_n ? levels + (k + 2) * stride : nullptr);
  count_kernel<<<1, 64, 0, s>>>(n, levels, levels_n, stride, flags + 1);
  ARGCSR_HIP(hipGetLastError());
  int32_t host_flags[2] = {0, 0};
  ARGCSR_HIP(hipMemcpyAsync(host_flags, flags, sizeof(host_flags), hipMemcpyDeviceToHost, s));
  ARGCSR_HIP(hipStreamSynchronize(s));
  if (host_flags[0])
    return fail(ARGCSR_EINVAL, "row_ptr does not start at 0 or decreases");
  n_groups = host_flags[1];
  return ARGCSR_OK;
}

int DeviceGrouping::write(argcsr_group_info* groups) const {
  if (n_groups == 0) return ARGCSR_OK;
  starts_kernel<<<dim3(uint32_t((n_groups + kGroupBlock - 1) / kGroupBlock)), kGroupBlock, 0,
                  stream>>>(n_groups, levels, levels_n, stride, groups);
  ARGCSR_HIP(hipGetLastError());
  return ARGCSR_OK;
}

void DeviceGrouping::release() {
  if (levels) (void)hipFreeAsync(levels, stream);
  levels = nullptr;
}

}  // namespace argcsr
