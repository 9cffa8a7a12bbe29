// Plain CSR y = A x on the same GPU: the baseline the ARG-CSR kernel is
// measured against (CSR definition, Sec. 2).  "CSR-vector": V consecutive
// lanes (V a power of two, 1..64) share a row, stride through its nonzeros
// (coalesced), and combine their partial sums with a butterfly over the V
// lanes.  V defaults to the power of two nearest above the mean row length.
//
// Binned variant (still plain CSR, no other storage): the rows are grouped
// by length once (argcsr_csr_bin_rows: bin k < 7 holds the rows of at most
// 2^k nonzeros and more than 2^(k-1), bin 7 the longer ones), and one launch
// gives each bin its own width: 2^k lanes per row, a whole 256-lane
// workgroup per row of bin 7.  A row of bin k < 7 is summed exactly as by
// the uniform kernel with V = 2^k.
#include <hip/hip_runtime.h>

#include <vector>

#include "common.hpp"
#include "group.hpp"
#include "values.hpp"

namespace argcsr {
namespace {

constexpr int kCsrBlock = 256;
constexpr int kBins = ARGCSR_CSR_BINS;      // 8: widths 1, 2, 4, ..., 64, then a workgroup

// Sum of row `row` by V consecutive lanes; lane `sub` of the row strides
// through its nonzeros, then a butterfly over the V lanes.
template <int DT, int V>
__device__ __forceinline__ typename Val<DT>::acc csr_row_sum(
    int64_t row, bool valid, int sub, const int32_t* __restrict__ rp,
    const int32_t* __restrict__ col, const typename Val<DT>::storage* __restrict__ val,
    const typename Val<DT>::acc* __restrict__ x) {
  using Vt = Val<DT>;
  using A = typename Vt::acc;
  A sum = A(0);
  if (valid) {
    const int32_t begin = rp[row], end = rp[row + 1];
    for (int32_t k = begin + sub; k < end; k += V)
      sum = __builtin_fma(Vt::load(val[k]), x[col[k]], sum);
  }
#pragma unroll
  for (int d = V / 2; d >= 1; d >>= 1) sum += __shfl_xor(sum, d, 64);
  return sum;
}

template <int DT, int V>
__global__ __launch_bounds__(kCsrBlock) void csr_vector_kernel(
    int32_t n_rows, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
    const typename Val<DT>::storage* __restrict__ val,
    const typename Val<DT>::acc* __restrict__ x, typename Val<DT>::acc* __restrict__ y) {
  constexpr int kRowsPerBlock = kCsrBlock / V;
  const int sub = threadIdx.x % V;
  const int64_t row = int64_t(xcd_remap(blockIdx.x, gridDim.x)) * kRowsPerBlock + threadIdx.x / V;
  const bool valid = row < n_rows;     // all V lanes of a row agree
  const auto sum = csr_row_sum<DT, V>(row, valid, sub, rp, col, val, x);
  if (valid && sub == 0) y[row] = sum;
}

// bin of a row of length L: the smallest k with L <= 2^k, 7 above 64
__host__ __device__ __forceinline__ int row_bin(int32_t L) {
  int k = 0;
  while (k < kBins - 1 && L > (1 << k)) ++k;
  return k;
}

struct BinLaunch {
  int32_t row_start[kBins + 1];     // bin k's rows: rows[row_start[k] .. row_start[k+1])
  int32_t block_start[kBins + 1];   // bin k's workgroups: [block_start[k], block_start[k+1])
};

template <int DT, int V>
__device__ __forceinline__ void binned_rows(const BinLaunch& bl, int k, int32_t b,
                                            const int32_t* __restrict__ rows,
                                            const int32_t* __restrict__ rp,
                                            const int32_t* __restrict__ col,
                                            const typename Val<DT>::storage* __restrict__ val,
                                            const typename Val<DT>::acc* __restrict__ x,
                                            typename Val<DT>::acc* __restrict__ y) {
  constexpr int kRowsPerBlock = kCsrBlock / V;
  const int sub = threadIdx.x % V;
  const int64_t i = int64_t(b - bl.block_start[k]) * kRowsPerBlock + threadIdx.x / V;
  const bool valid = i < bl.row_start[k + 1] - bl.row_start[k];
  const int64_t row = valid ? rows[bl.row_start[k] + i] : 0;
  const auto sum = csr_row_sum<DT, V>(row, valid, sub, rp, col, val, x);
  if (valid && sub == 0) y[row] = sum;
}

template <int DT>
__global__ __launch_bounds__(kCsrBlock) void csr_binned_kernel(
    BinLaunch bl, const int32_t* __restrict__ rows, const int32_t* __restrict__ rp,
    const int32_t* __restrict__ col, const typename Val<DT>::storage* __restrict__ val,
    const typename Val<DT>::acc* __restrict__ x, typename Val<DT>::acc* __restrict__ y) {
  using Vt = Val<DT>;
  using A = typename Vt::acc;
  const int32_t b = int32_t(blockIdx.x);
  int k = 0;
  while (k < kBins - 1 && b >= bl.block_start[k + 1]) ++k;
  switch (k) {
    case 0: binned_rows<DT, 1>(bl, k, b, rows, rp, col, val, x, y); return;
    case 1: binned_rows<DT, 2>(bl, k, b, rows, rp, col, val, x, y); return;
    case 2: binned_rows<DT, 4>(bl, k, b, rows, rp, col, val, x, y); return;
    case 3: binned_rows<DT, 8>(bl, k, b, rows, rp, col, val, x, y); return;
    case 4: binned_rows<DT, 16>(bl, k, b, rows, rp, col, val, x, y); return;
    case 5: binned_rows<DT, 32>(bl, k, b, rows, rp, col, val, x, y); return;
    case 6: binned_rows<DT, 64>(bl, k, b, rows, rp, col, val, x, y); return;
    default: break;
  }
  // bin 7: the workgroup's 256 lanes stride through one row; wave sums
  // added in wave order
  __shared__ A part[kCsrBlock / 64];
  const int64_t row = rows[bl.row_start[kBins - 1] + (b - bl.block_start[kBins - 1])];
  A sum = A(0);
  const int32_t begin = rp[row], end = rp[row + 1];
  for (int32_t k2 = begin + int32_t(threadIdx.x); k2 < end; k2 += kCsrBlock)
    sum = __builtin_fma(Vt::load(val[k2]), x[col[k2]], sum);
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) sum += __shfl_xor(sum, d, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    A t = part[0];
#pragma unroll
    for (int w = 1; w < kCsrBlock / 64; ++w) t += part[w];
    y[row] = t;
  }
}

// Binning: per workgroup of 256 rows, the count of each bin (pass 1), and
// the rows written to their bin's range in ascending order (pass 2) at the
// offsets the host computes from the counts.
__global__ __launch_bounds__(kCsrBlock) void bin_count_kernel(int32_t n_rows,
                                                            const int32_t* __restrict__ rp,
                                                            int32_t* __restrict__ counts) {
  __shared__ int32_t c[kBins];
  if (threadIdx.x < kBins) c[threadIdx.x] = 0;
  __syncthreads();
  const int64_t r = int64_t(blockIdx.x) * kCsrBlock + threadIdx.x;
  if (r < n_rows) atomicAdd(&c[row_bin(rp[r + 1] - rp[r])], 1);
  __syncthreads();
  if (threadIdx.x < kBins) counts[int64_t(blockIdx.x) * kBins + threadIdx.x] = c[threadIdx.x];
}

__global__ __launch_bounds__(kCsrBlock) void bin_scatter_kernel(int32_t n_rows,
                                                              const int32_t* __restrict__ rp,
                                                              const int32_t* __restrict__ offsets,
                                                              int32_t* __restrict__ rows) {
  __shared__ int32_t wave_counts[kCsrBlock / 64][kBins];
  const int lane = lane_id(), w = int(threadIdx.x >> 6);
  const int64_t r = int64_t(blockIdx.x) * kCsrBlock + threadIdx.x;
  const int bin = r < n_rows ? row_bin(rp[r + 1] - rp[r]) : -1;
  // rank among this wave's lanes of the same bin, and the wave's counts
  int rank = 0;
#pragma unroll
  for (int k = 0; k < kBins; ++k) {
    const uint64_t m = __ballot(bin == k);
    if (bin == k) rank = __popcll(m & ((uint64_t(1) << lane) - 1));
    if (lane == 0) wave_counts[w][k] = __popcll(m);
  }
  __syncthreads();
  if (bin >= 0) {
    int before = 0;
    for (int q = 0; q < w; ++q) before += wave_counts[q][bin];
    rows[offsets[int64_t(blockIdx.x) * kBins + bin] + before + rank] = int32_t(r);
  }
}

template <int DT, int V>
void launch(int32_t n_rows, const int32_t* rp, const int32_t* col, const void* val,
            const void* x, void* y, hipStream_t s) {
  using Vt = Val<DT>;
  constexpr int kRowsPerBlock = kCsrBlock / V;
  const int blocks = int((int64_t(n_rows) + kRowsPerBlock - 1) / kRowsPerBlock);
  csr_vector_kernel<DT, V><<<blocks, kCsrBlock, 0, s>>>(
      n_rows, rp, col, static_cast<const typename Vt::storage*>(val),
      static_cast<const typename Vt::acc*>(x), static_cast<typename Vt::acc*>(y));
}

template <int DT>
void launch_v(int V, int32_t n_rows, const int32_t* rp, const int32_t* col, const void* val,
              const void* x, void* y, hipStream_t s) {
  switch (V) {
    case 1: launch<DT, 1>(n_rows, rp, col, val, x, y, s); break;
    case 2: launch<DT, 2>(n_rows, rp, col, val, x, y, s); break;
    case 4: launch<DT, 4>(n_rows, rp, col, val, x, y, s); break;
    case 8: launch<DT, 8>(n_rows, rp, col, val, x, y, s); break;
    case 16: launch<DT, 16>(n_rows, rp, col, val, x, y, s); break;
    case 32: launch<DT, 32>(n_rows, rp, col, val, x, y, s); break;
    default: launch<DT, 64>(n_rows, rp, col, val, x, y, s); break;
  }
}

}  // namespace
}  // namespace argcsr

extern "C" int argcsr_csr_spmv(int32_t n_rows, int32_t n_cols, int64_t nnz,
                               const int32_t* row_ptr, const int32_t* col, const void* val,
                               int32_t dtype, int32_t lanes_per_row, const void* x, void* y,
                               void* stream) {
  using namespace argcsr;
  clear_error();
  if (n_rows < 0 || n_cols < 0 || nnz < 0) return fail(ARGCSR_EINVAL, "negative size");
  if (dtype < ARGCSR_F64 || dtype > ARGCSR_F16) return fail(ARGCSR_EINVAL, "unknown dtype %d", dtype);
  if (lanes_per_row != 0 &&
      (lanes_per_row < 1 || lanes_per_row > 64 || (lanes_per_row & (lanes_per_row - 1))))
    return fail(ARGCSR_EINVAL, "lanes_per_row must be 0 or a power of two in [1, 64]");
  if (n_rows == 0) return ARGCSR_OK;
  if (!row_ptr || !x || !y || (nnz > 0 && (!col || !val)))
    return fail(ARGCSR_EINVAL, "NULL device buffer");
  if (x == y) return fail(ARGCSR_EINVAL, "y must not alias x");
  int V = lanes_per_row;
  if (V == 0) {
    const double mean = double(nnz) / double(n_rows);
    V = 1;
    while (V < 64 && V < mean) V <<= 1;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  switch (dtype) {
    case ARGCSR_F64: launch_v<ARGCSR_F64>(V, n_rows, row_ptr, col, val, x, y, s); break;
    case ARGCSR_F32: launch_v<ARGCSR_F32>(V, n_rows, row_ptr, col, val, x, y, s); break;
    case ARGCSR_BF16: launch_v<ARGCSR_BF16>(V, n_rows, row_ptr, col, val, x, y, s); break;
    default: launch_v<ARGCSR_F16>(V, n_rows, row_ptr, col, val, x, y, s); break;
  }
  ARGCSR_HIP(hipGetLastError());
  return ARGCSR_OK;
}

namespace argcsr {
namespace {

template <int DT>
void launch_binned(const BinLaunch& bl, int32_t blocks, const int32_t* rows, const int32_t* rp,
                   const int32_t* col, const void* val, const void* x, void* y, hipStream_t s) {
  using Vt = Val<DT>;
  csr_binned_kernel<DT><<<blocks, kCsrBlock, 0, s>>>(
      bl, rows, rp, col, static_cast<const typename Vt::storage*>(val),
      static_cast<const typename Vt::acc*>(x), static_cast<typename Vt::acc*>(y));
}

}  // namespace
}  // namespace argcsr

extern "C" int argcsr_csr_bin_rows(int32_t n_rows, const int32_t* row_ptr, int32_t* rows,
                                   int32_t* bin_start, void* stream) {
  using namespace argcsr;
  clear_error();
  if (n_rows < 0) return fail(ARGCSR_EINVAL, "n_rows < 0");
  if (!bin_start) return fail(ARGCSR_EINVAL, "bin_start is NULL");
  for (int k = 0; k <= kBins; ++k) bin_start[k] = 0;
  if (n_rows == 0) return ARGCSR_OK;
  if (!row_ptr || !rows) return fail(ARGCSR_EINVAL, "NULL device buffer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t blocks = (int64_t(n_rows) + kCsrBlock - 1) / kCsrBlock;
  const size_t bytes = sizeof(int32_t) * size_t(blocks) * kBins;
  int32_t* d_counts = nullptr;
  int rc = scratch_alloc_async(reinterpret_cast<void**>(&d_counts), bytes, s);
  if (rc) return rc;
  bin_count_kernel<<<dim3(uint32_t(blocks)), kCsrBlock, 0, s>>>(n_rows, row_ptr, d_counts);
  std::vector<int32_t> h(size_t(blocks) * kBins);
  hipError_t e = hipMemcpyAsync(h.data(), d_counts, bytes, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    (void)hipFreeAsync(d_counts, s);
    return fail(ARGCSR_EHIP, "binning counts: %s", hipGetErrorString(e));
  }
  // offsets: bin by bin, workgroup by workgroup (rows ascend within a bin)
  int64_t total = 0;
  for (int k = 0; k < kBins; ++k) {
    bin_start[k] = int32_t(total);
    for (int64_t b = 0; b < blocks; ++b) {
      const int32_t c = h[size_t(b) * kBins + k];
      h[size_t(b) * kBins + k] = int32_t(total);
      total += c;
    }
  }
  bin_start[kBins] = int32_t(total);
  e = hipMemcpyAsync(d_counts, h.data(), bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    bin_scatter_kernel<<<dim3(uint32_t(blocks)), kCsrBlock, 0, s>>>(n_rows, row_ptr, d_counts,
                                                                   rows);
    e = hipGetLastError();
  }
  (void)hipFreeAsync(d_counts, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(ARGCSR_EHIP, "binning: %s", hipGetErrorString(e));
  return ARGCSR_OK;
}

extern "C" int argcsr_csr_spmv_binned(int32_t n_rows, int32_t n_cols, int64_t nnz,
                                      const int32_t* row_ptr, const int32_t* col, const void* val,
                                      int32_t dtype, const int32_t* rows,
                                      const int32_t* bin_start, const void* x, void* y,
                                      void* stream) {
  using namespace argcsr;
  clear_error();
  if (n_rows < 0 || n_cols < 0 || nnz < 0) return fail(ARGCSR_EINVAL, "negative size");
  if (dtype < ARGCSR_F64 || dtype > ARGCSR_F16) return fail(ARGCSR_EINVAL, "unknown dtype %d", dtype);
  if (!bin_start) return fail(ARGCSR_EINVAL, "bin_start is NULL");
  if (bin_start[0] != 0 || bin_start[kBins] != n_rows)
    return fail(ARGCSR_EINVAL, "bin_start does not cover the %d rows", n_rows);
  BinLaunch bl{};
  int64_t blocks = 0;
  for (int k = 0; k < kBins; ++k) {
    if (bin_start[k + 1] < bin_start[k]) return fail(ARGCSR_EINVAL, "bin_start decreases");
    bl.row_start[k] = bin_start[k];
    bl.block_start[k] = int32_t(blocks);
    const int64_t cnt = bin_start[k + 1] - bin_start[k];
    const int64_t per = k < kBins - 1 ? kCsrBlock / (1 << k) : 1;     // rows per workgroup
    blocks += (cnt + per - 1) / per;
  }
  bl.row_start[kBins] = bin_start[kBins];
  bl.block_start[kBins] = int32_t(blocks);
  if (n_rows == 0) return ARGCSR_OK;
  if (!row_ptr || !rows || !x || !y || (nnz > 0 && (!col || !val)))
    return fail(ARGCSR_EINVAL, "NULL device buffer");
  if (x == y) return fail(ARGCSR_EINVAL, "y must not alias x");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int32_t nb = int32_t(blocks);
  switch (dtype) {
    case ARGCSR_F64: launch_binned<ARGCSR_F64>(bl, nb, rows, row_ptr, col, val, x, y, s); break;
    case ARGCSR_F32: launch_binned<ARGCSR_F32>(bl, nb, rows, row_ptr, col, val, x, y, s); break;
    case ARGCSR_BF16: launch_binned<ARGCSR_BF16>(bl, nb, rows, row_ptr, col, val, x, y, s); break;
    default: launch_binned<ARGCSR_F16>(bl, nb, rows, row_ptr, col, val, x, y, s); break;
  }
  ARGCSR_HIP(hipGetLastError());
  return ARGCSR_OK;
}
