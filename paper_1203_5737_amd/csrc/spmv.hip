// y = A x for an ARG-CSR matrix on gfx950 (Sec. 4 of the paper: chunk
// partial sums, then per-row sums of the partial sums).
//
// Mapping to CDNA4 (a wave has 64 lanes):
//   - one wave per group; with T = 64*W chunks per group, lane i owns chunks
//     i, i+64, ..., i+64*(W-1) ("sub-blocks" w = 0..W-1).  A group's slots
//     for step j are T consecutive values/columns, so every load is a
//     contiguous, fully coalesced wave-wide access (the paper's column-major
//     chunk storage, Sec. 3);
//   - the group struct is read with scalar loads (wave-uniform); no
//     workgroup barrier is needed anywhere;
//   - the threads mapping is turned into a bitmask of row-end chunks (chunk
//     tm[l]-1 ends row l) through a small per-wave LDS table and a ballot;
//   - each chunk sums value*x[column] over its slots, stopping at the first
//     artificial zero (column -1); a wave leaves the loop once every lane
//     has hit padding (Sec. 4);
//   - row sums are a segmented inclusive scan across lanes (segments = rows,
//     delimited by the row-end mask), carried from one sub-block to the next;
//     the lane holding a row's last chunk writes y[first_row + row].
//     Summation order is fixed by the layout, so results are deterministic.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "spmv_kernels.hpp"
#include "spmv_staged.hpp"

namespace argcsr {
namespace {

template <int DT, int W, int U>
void launch(const argcsr_matrix* A, const void* x, void* y, hipStream_t s) {
  using Vt = Val<DT>;
  const bool sched = A->heavy_groups != nullptr && A->n_heavy > 0;
  const int32_t n_heavy = sched ? A->n_heavy : 0;
  const int32_t heavy_chunk = sched ? A->heavy_chunk : INT32_MAX;
  const int blocks = n_heavy + (A->n_groups + kSpmvWaves - 1) / kSpmvWaves;
  const bool serial = serial_gathers(int32_t(sizeof(typename Vt::storage)), A->block_dim,
                                     A->n_slots, A->n_groups);
  argcsr_spmv_kernel<DT, W, U><<<blocks, kSpmvWaves * 64, 0, s>>>(
      A->groups, A->n_groups, A->threads_mapping, A->columns,
      static_cast<const typename Vt::storage*>(A->values),
      static_cast<const typename Vt::acc*>(x), A->n_cols, static_cast<typename Vt::acc*>(y),
      A->heavy_groups, n_heavy, heavy_chunk, serial ? 1 : 0);
}

template <int DT, int W, int U, bool XLDS>
int launch_staged(const argcsr_matrix* A, const void* x, void* y, hipStream_t s) {
  using Vt = Val<DT>;
  const bool sched = A->heavy_groups != nullptr && A->n_heavy > 0;
  const int32_t n_heavy = sched ? A->n_heavy : 0;
  const int32_t heavy_chunk = sched ? A->heavy_chunk : INT32_MAX;
  const int blocks = n_heavy + (A->n_groups + kSpmvWaves - 1) / kSpmvWaves;
  const int32_t lds_tiles = A->stage_max_tiles > 0 ? A->stage_max_tiles : 1;
  const size_t lds = size_t(kSpmvWaves) * staged_region_bytes<DT, W, XLDS>(lds_tiles);
  auto* kern = &argcsr_spmv_staged_kernel<DT, W, U, XLDS>;
  if (lds > 64 * 1024)
    ARGCSR_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  kern<<<blocks, kSpmvWaves * 64, lds, s>>>(
      A->groups, A->n_groups, A->threads_mapping, A->local,
      static_cast<const typename Vt::storage*>(A->values), A->tile_ptr, A->tile_start,
      A->tile_len, lds_tiles,
      static_cast<const typename Vt::acc*>(x), A->n_cols, static_cast<typename Vt::acc*>(y),
      A->heavy_groups, n_heavy, heavy_chunk);
  return ARGCSR_OK;
}

// Steps per load batch of the staged kernel with x in LDS, chosen by a
// sweep on the 27-point stencil (MI355X, cold): FP64 x at W = 1 takes 16
// (124.0 us against 126.5 with 8), at W = 2 and 4 fewer steps than the plain
// kernel (139.5 us with 2 against 149.3 with 4 at W = 2; 137.5 with 1
// against 152.6 with 2 at W = 4); 4- and 2-byte values at W = 2 take 2
// (FP32 71.2 against 73.2 us, BF16 56.0 against 56.6).
template <int DT, int W>
constexpr int staged_steps() {
  if (sizeof(typename Val<DT>::acc) == 8) return W == 1 ? 16 : W == 2 ? 2 : 1;
  return W == 1 ? 8 : W == 2 ? 2 : 2;
}

template <int DT, int W, int U>
int launch_w(const argcsr_matrix* A, const void* x, void* y, hipStream_t s) {
  if (!A->local) {
    launch<DT, W, U>(A, x, y, s);
    return ARGCSR_OK;
  }
  return A->stage_lds ? launch_staged<DT, W, staged_steps<DT, W>(), true>(A, x, y, s)
                      : launch_staged<DT, W, U, false>(A, x, y, s);
}

template <int DT>
int launch_dt(const argcsr_matrix* A, const void* x, void* y, hipStream_t s) {
  switch (A->block_dim) {
    case 64: return launch_w<DT, 1, 8>(A, x, y, s);
    case 128: return launch_w<DT, 2, 4>(A, x, y, s);
    default: return launch_w<DT, 4, 2>(A, x, y, s);
  }
}

}  // namespace

int check_matrix(const argcsr_matrix* A) {
  if (!A) return fail(ARGCSR_EINVAL, "matrix is NULL");
  if (A->n_rows < 0 || A->n_cols < 0 || A->n_groups < 0 || A->n_slots < 0)
    return fail(ARGCSR_EINVAL, "negative size in matrix descriptor");
  if (A->block_dim != 64 && A->block_dim != 128 && A->block_dim != 256)
    return fail(ARGCSR_EUNSUPPORTED, "block_dim %d: the GPU kernels take 64, 128 or 256",
                A->block_dim);
  if (A->dtype < ARGCSR_F64 || A->dtype > ARGCSR_F16)
    return fail(ARGCSR_EINVAL, "unknown dtype %d", A->dtype);
  if (A->n_slots > INT32_MAX) return fail(ARGCSR_EOVERFLOW, "n_slots exceeds INT32_MAX");
  if (int64_t(A->n_cols) * (A->dtype == ARGCSR_F64 ? 8 : 4) > kMaxVectorBytes)
    return fail(ARGCSR_EUNSUPPORTED, "x of %d columns exceeds the %lld-byte gather range",
                A->n_cols, (long long)kMaxVectorBytes);
  if (A->n_groups > 0 && (!A->groups || !A->threads_mapping || !A->values ||
                          (!A->columns && !A->local)))
    return fail(ARGCSR_EINVAL, "NULL device buffer in matrix descriptor");
  if (A->local) {
    if (A->n_stage_tiles < 0 || A->stage_max_tiles < 0 || A->stage_max_tiles > kStageMaxTiles)
      return fail(ARGCSR_EINVAL, "malformed staging sizes");
    if (!A->tile_ptr || (A->n_stage_tiles > 0 && (!A->tile_start || !A->tile_len)))
      return fail(ARGCSR_EINVAL, "NULL staging buffer in matrix descriptor");
  }
  if (A->heavy_groups && (A->n_heavy < 0 || A->n_heavy > A->n_groups ||
                          A->heavy_chunk != heavy_chunk_for(A->block_dim, A->n_slots,
                                                            A->n_groups)))
    return fail(ARGCSR_EINVAL, "heavy-group schedule does not match the matrix");
  return ARGCSR_OK;
}

}  // namespace argcsr

extern "C" int argcsr_spmv(const argcsr_matrix* A, const void* x, void* y, void* stream) {
  using namespace argcsr;
  clear_error();
  int rc = check_matrix(A);
  if (rc) return rc;
  if (A->n_groups == 0) return ARGCSR_OK;
  if (!x || !y) return fail(ARGCSR_EINVAL, "x or y is NULL");
  if (x == y) return fail(ARGCSR_EINVAL, "y must not alias x");
  hipStream_t s = static_cast<hipStream_t>(stream);
  switch (A->dtype) {
    case ARGCSR_F64: rc = launch_dt<ARGCSR_F64>(A, x, y, s); break;
    case ARGCSR_F32: rc = launch_dt<ARGCSR_F32>(A, x, y, s); break;
    case ARGCSR_BF16: rc = launch_dt<ARGCSR_BF16>(A, x, y, s); break;
    default: rc = launch_dt<ARGCSR_F16>(A, x, y, s); break;
  }
  if (rc) return rc;
  ARGCSR_HIP(hipGetLastError());
  return ARGCSR_OK;
}
