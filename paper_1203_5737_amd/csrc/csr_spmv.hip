// Plain CSR y = A x on the same GPU: the baseline the ARG-CSR kernel is
// measured against (CSR definition, Sec. 2).  "CSR-vector": V consecutive
// lanes (V a power of two, 1..64) share a row, stride through its nonzeros
// (coalesced), and combine their partial sums with a butterfly over the V
// lanes.  V defaults to the power of two nearest above the mean row length.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "values.hpp"

namespace argcsr {
namespace {

constexpr int kCsrBlock = 256;

template <int DT, int V>
__global__ __launch_bounds__(kCsrBlock) void csr_vector_kernel(
    int32_t n_rows, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
    const typename Val<DT>::storage* __restrict__ val,
    const typename Val<DT>::acc* __restrict__ x, typename Val<DT>::acc* __restrict__ y) {
  using Vt = Val<DT>;
  using A = typename Vt::acc;
  constexpr int kRowsPerBlock = kCsrBlock / V;
  const int sub = threadIdx.x % V;
  const int64_t row = int64_t(xcd_remap(blockIdx.x, gridDim.x)) * kRowsPerBlock + threadIdx.x / V;
  const bool valid = row < n_rows;     // all V lanes of a row agree
  A sum = A(0);
  if (valid) {
    const int32_t begin = rp[row], end = rp[row + 1];
    for (int32_t k = begin + sub; k < end; k += V)
      sum = __builtin_fma(Vt::load(val[k]), x[col[k]], sum);
  }
#pragma unroll
  for (int d = V / 2; d >= 1; d >>= 1) sum += __shfl_xor(sum, d, 64);
  if (valid && sub == 0) y[row] = sum;
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
