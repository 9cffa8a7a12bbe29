// Many ARG-CSR matrices in one persistent launch over a global work queue.
//
// Work items are (matrix, group) pairs.  Heavy groups (a long chunk loop,
// see schedule.hpp) are taken by whole workgroups from one queue and split
// over their waves; all other groups are taken by single waves, kGrab at a
// time, from per-XCD segments of a second list in matrix and row order
// (workqueue.hpp).  Queue counters are zeroed by a one-block kernel enqueued
// before every launch (no memset, so the pair can be captured in a hipGraph).  Each group is computed by the
// same deterministic routine as argcsr_spmv, so the results do not depend on
// which wave takes which item.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "batch.hpp"
#include "common.hpp"
#include "schedule.hpp"
#include "spmv_kernels.hpp"
#include "workqueue.hpp"

namespace argcsr {
namespace {

constexpr int kGrab = 4;                 // normal items taken per queue access
constexpr int kMaxBlocksPerCu = 8;       // persistent grid: as many workgroups as fit, <= 8 per CU

template <int DT, int W, int U>
__device__ __forceinline__ void run_item(const BatchMat& m, int32_t g, int32_t* ends) {
  using Vt = Val<DT>;
  const argcsr_group_info gi = m.groups[g];
  spmv_group<DT, W, U>(gi.first_row, gi.size, gi.offset, gi.chunk_size, m.tm, m.columns,
                       static_cast<const typename Vt::storage*>(m.values),
                       XGather<typename Vt::acc>(static_cast<const typename Vt::acc*>(m.x),
                                                 m.n_cols),
                       m.serial != 0, static_cast<typename Vt::acc*>(m.y), ends);
}

template <int DT, int W, int U>
__device__ __forceinline__ void run_heavy(const BatchMat& m, int32_t g, int32_t* ends,
                                          typename Val<DT>::acc* part_mem, int wv) {
  using Vt = Val<DT>;
  using A = typename Vt::acc;
  const argcsr_group_info gi = m.groups[g];
  spmv_group_split<DT, W, U>(gi.first_row, gi.size, gi.offset, gi.chunk_size, m.tm, m.columns,
                             static_cast<const typename Vt::storage*>(m.values),
                             XGather<A>(static_cast<const A*>(m.x), m.n_cols), m.serial != 0,
                             static_cast<A*>(m.y), ends,
                             reinterpret_cast<A(*)[64 * W]>(part_mem), wv);
}

template <int DT>
__global__ __launch_bounds__(kSpmvWaves * 64) void batch_spmv_kernel(
    const BatchMat* __restrict__ mats, const int2* __restrict__ heavy, int32_t n_heavy,
    const int2* __restrict__ items, int32_t n_items, WorkQueues* q) {
  using A = typename Val<DT>::acc;
  __shared__ int32_t ends[kSpmvWaves][256];
  __shared__ A part_mem[(kSpmvWaves - 1) * 256];
  __shared__ int32_t grabbed;
  const int wv = wave_uniform(int(threadIdx.x >> 6));

  // heavy groups: the whole workgroup takes one at a time
  for (;;) {
    if (threadIdx.x == 0) grabbed = atomicAdd(&q->heavy.next, 1);
    __syncthreads();
    const int32_t h = grabbed;
    __syncthreads();                      // all waves have read `grabbed`
    if (h >= n_heavy) break;
    const int2 it = heavy[h];
    const BatchMat m = mats[it.x];
    switch (m.block_dim) {
      case 64: run_heavy<DT, 1, 8>(m, it.y, ends[0], part_mem, wv); break;
      case 128: run_heavy<DT, 2, 4>(m, it.y, ends[0], part_mem, wv); break;
      default: run_heavy<DT, 4, 2>(m, it.y, ends[0], part_mem, wv); break;
    }
    __syncthreads();                      // part_mem / ends free for the next heavy item
  }

  // all other groups: each wave takes kGrab items at a time
  QueueCursor cursor{int(blockIdx.x % kQueues), 0};
  int32_t i0, i1;
  while (cursor.take(q, n_items, kGrab, &i0, &i1)) {
    for (int32_t i = i0; i < i1; ++i) {
      const int2 it = items[i];
      const BatchMat m = mats[it.x];
      switch (m.block_dim) {
        case 64: run_item<DT, 1, 8>(m, it.y, ends[wv]); break;
        case 128: run_item<DT, 2, 4>(m, it.y, ends[wv]); break;
        default: run_item<DT, 4, 2>(m, it.y, ends[wv]); break;
      }
    }
  }
}

const void* kernel_for(int32_t dtype) {
  switch (dtype) {
    case ARGCSR_F64: return reinterpret_cast<const void*>(&batch_spmv_kernel<ARGCSR_F64>);
    case ARGCSR_F32: return reinterpret_cast<const void*>(&batch_spmv_kernel<ARGCSR_F32>);
    case ARGCSR_BF16: return reinterpret_cast<const void*>(&batch_spmv_kernel<ARGCSR_BF16>);
    default: return reinterpret_cast<const void*>(&batch_spmv_kernel<ARGCSR_F16>);
  }
}

int launch_kernels(argcsr_batch* b, hipStream_t s) {
  auto* q = static_cast<WorkQueues*>(b->queue);
  reset_work_queues_kernel<<<1, 64, 0, s>>>(q, 1);
  const dim3 grid(b->grid), block(kSpmvWaves * 64);
  switch (b->dtype) {
    case ARGCSR_F64:
      batch_spmv_kernel<ARGCSR_F64><<<grid, block, 0, s>>>(b->d_mats, b->d_heavy, b->n_heavy,
                                                            b->d_items, b->n_items, q);
      break;
    case ARGCSR_F32:
      batch_spmv_kernel<ARGCSR_F32><<<grid, block, 0, s>>>(b->d_mats, b->d_heavy, b->n_heavy,
                                                            b->d_items, b->n_items, q);
      break;
    case ARGCSR_BF16:
      batch_spmv_kernel<ARGCSR_BF16><<<grid, block, 0, s>>>(b->d_mats, b->d_heavy, b->n_heavy,
                                                             b->d_items, b->n_items, q);
      break;
    default:
      batch_spmv_kernel<ARGCSR_F16><<<grid, block, 0, s>>>(b->d_mats, b->d_heavy, b->n_heavy,
                                                            b->d_items, b->n_items, q);
      break;
  }
  ARGCSR_HIP(hipGetLastError());
  return ARGCSR_OK;
}

void free_batch(argcsr_batch* b) {
  if (!b) return;
  if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->d_mats) (void)hipFree(b->d_mats);
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_heavy) (void)hipFree(b->d_heavy);
  if (b->queue) (void)hipFree(b->queue);
  if (b->last) (void)hipEventDestroy(b->last);
  delete b;
}

}  // namespace

// Builds the work lists on the host from the converted group tables.
int build_batch(int32_t n, const argcsr_matrix* mats, const void* const* xs, void* const* ys,
                argcsr_batch* b) {
  b->n_mats = n;
  b->dtype = mats[0].dtype;
  std::vector<BatchMat> hm(n);
  std::vector<int2> items;
  std::vector<int2> heavy;
  std::vector<argcsr_group_info> g;
  for (int32_t m = 0; m < n; ++m) {
    const argcsr_matrix& A = mats[m];
    int rc = check_matrix(&A);
    if (rc) return rc;
    if (A.dtype != b->dtype)
      return fail(ARGCSR_EINVAL, "matrix %d has dtype %d, batch dtype is %d", m, A.dtype, b->dtype);
    if (A.n_groups > 0 && (!xs[m] || !ys[m]))
      return fail(ARGCSR_EINVAL, "matrix %d: x or y is NULL", m);
    if (A.n_groups > 0 && !A.columns)
      return fail(ARGCSR_EINVAL, "matrix %d: a batch reads columns (staging is not used)", m);
    hm[m] = BatchMat{A.groups, A.threads_mapping, A.columns, A.values, xs[m], ys[m],
                     A.block_dim, A.n_groups, A.n_cols,
                     serial_gathers(A.dtype == ARGCSR_F64 ? 8 : A.dtype == ARGCSR_F32 ? 4 : 2,
                                    A.block_dim, A.n_slots, A.n_groups) ? 1 : 0};
    g.resize(size_t(A.n_groups));
    if (A.n_groups > 0)
      ARGCSR_HIP(hipMemcpy(g.data(), A.groups, sizeof(argcsr_group_info) * g.size(),
                           hipMemcpyDeviceToHost));
    const int32_t hc = heavy_chunk_for(A.block_dim, A.n_slots, A.n_groups);
    for (int32_t k = 0; k < A.n_groups; ++k) {
      if (g[k].chunk_size > hc) heavy.push_back(int2{m, k});
      else items.push_back(int2{m, k});
    }
  }
  // matrix-major, row order: waves working at the same time gather from the
  // same few x vectors (sorting by length across matrices measured 13% slower)
  b->n_items = int32_t(items.size());
  b->n_heavy = int32_t(heavy.size());

  ARGCSR_HIP(hipMalloc(&b->d_mats, sizeof(BatchMat) * size_t(std::max(n, 1))));
  ARGCSR_HIP(hipMalloc(&b->d_items, sizeof(int2) * std::max<size_t>(items.size(), 1)));
  ARGCSR_HIP(hipMalloc(&b->d_heavy, sizeof(int2) * std::max<size_t>(heavy.size(), 1)));
  ARGCSR_HIP(hipMalloc(&b->queue, sizeof(WorkQueues)));
  ARGCSR_HIP(hipMemcpy(b->d_mats, hm.data(), sizeof(BatchMat) * size_t(n), hipMemcpyHostToDevice));
  if (!items.empty())
    ARGCSR_HIP(hipMemcpy(b->d_items, items.data(), sizeof(int2) * items.size(),
                         hipMemcpyHostToDevice));
  if (!heavy.empty())
    ARGCSR_HIP(hipMemcpy(b->d_heavy, heavy.data(), sizeof(int2) * heavy.size(),
                         hipMemcpyHostToDevice));
  int dev = 0, cus = 0, per_cu = 0;
  ARGCSR_HIP(hipGetDevice(&dev));
  ARGCSR_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  ARGCSR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel_for(b->dtype),
                                                          kSpmvWaves * 64, 0));
  per_cu = std::max(1, std::min(per_cu, kMaxBlocksPerCu));
  const int64_t work_blocks = int64_t(b->n_heavy) + (int64_t(b->n_items) + kGrab * kSpmvWaves - 1) /
                                                        (kGrab * kSpmvWaves);
  b->grid = int32_t(std::max<int64_t>(1, std::min<int64_t>(int64_t(cus) * per_cu, work_blocks)));
  return ARGCSR_OK;
}

}  // namespace argcsr

extern "C" int argcsr_batch_create(int32_t n_mats, const argcsr_matrix* mats,
                                   const void* const* xs, void* const* ys,
                                   argcsr_batch** out) {
  using namespace argcsr;
  clear_error();
  if (!out) return fail(ARGCSR_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_mats < 1 || !mats || !xs || !ys) return fail(ARGCSR_EINVAL, "empty or NULL batch");
  auto* b = new (std::nothrow) argcsr_batch();
  if (!b) return fail(ARGCSR_ENOMEM, "host allocation failed");
  int rc = build_batch(n_mats, mats, xs, ys, b);
  if (rc) { free_batch(b); return rc; }
  if (hipEventCreateWithFlags(&b->last, hipEventDisableTiming) != hipSuccess) {
    b->last = nullptr;
    free_batch(b);
    return fail(ARGCSR_EHIP, "hipEventCreate failed");
  }
  // capture reset + persistent kernel into a graph on a private stream
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
    free_batch(b);
    return fail(ARGCSR_EHIP, "hipStreamCreate failed");
  }
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    rc = launch_kernels(b, cs);
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cs, &graph);
    b->graph = graph;
    if (rc == ARGCSR_OK && e2 == hipSuccess)
      e = hipGraphInstantiate(&b->graph_exec, graph, nullptr, nullptr, 0);
    else
      e = e2 != hipSuccess ? e2 : hipErrorUnknown;
  }
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess || rc != ARGCSR_OK) {
    free_batch(b);
    return rc ? rc : fail(ARGCSR_EHIP, "graph capture failed: %s", hipGetErrorString(e));
  }
  *out = b;
  return ARGCSR_OK;
}

extern "C" int argcsr_batch_launch(argcsr_batch* b, void* stream) {
  using namespace argcsr;
  clear_error();
  if (!b) return fail(ARGCSR_EINVAL, "batch is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int rc = launch_kernels(b, s);
  if (rc) return rc;
  ARGCSR_HIP(hipEventRecord(b->last, s));
  b->launched = true;
  return ARGCSR_OK;
}

extern "C" int argcsr_batch_graph_launch(argcsr_batch* b, void* stream) {
  using namespace argcsr;
  clear_error();
  if (!b || !b->graph_exec) return fail(ARGCSR_EINVAL, "batch is NULL or has no graph");
  hipStream_t s = static_cast<hipStream_t>(stream);
  ARGCSR_HIP(hipGraphLaunch(b->graph_exec, s));
  ARGCSR_HIP(hipEventRecord(b->last, s));
  b->launched = true;
  return ARGCSR_OK;
}

extern "C" int argcsr_batch_info(const argcsr_batch* b, int32_t* n_items, int32_t* n_heavy,
                                 int32_t* grid) {
  using namespace argcsr;
  clear_error();
  if (!b) return fail(ARGCSR_EINVAL, "batch is NULL");
  if (n_items) *n_items = b->n_items;
  if (n_heavy) *n_heavy = b->n_heavy;
  if (grid) *grid = b->grid;
  return ARGCSR_OK;
}

extern "C" int argcsr_batch_destroy(argcsr_batch* b) {
  using namespace argcsr;
  clear_error();
  if (b) {
    // the last launch may still be in flight on a caller stream: wait for it
    // alone (launches are ordered on their streams; a caller that launches
    // on several streams at once orders them itself)
    const hipError_t e = b->launched ? hipEventSynchronize(b->last) : hipSuccess;
    free_batch(b);
    if (e != hipSuccess)
      return fail(ARGCSR_EHIP, "waiting for the batch's last launch failed: %s",
                  hipGetErrorString(e));
  }
  return ARGCSR_OK;
}
