// Autotuner for the storage format and its parameters (block_dim T,
// desired_chunk_size D; row-grouped CSR at each T).
//
// The paper finds D decisive and matrix dependent: larger D for regular
// matrices, D = 1 as the robust default, and row-grouped CSR ahead on
// finite-difference matrices (Sec. 5).  Here every (T, D) in
// {64,128,256} x {1,2,4,...,64, longest row, mean row length} and
// row-grouped CSR at each T is planned on the host (steps 1-2 give the group
// count, slot count and heavy-group count exactly), ranked by a cost model
// fitted to cold timings, and `n_finalists` of them (distinct layouts, the
// best of each block size first) are converted and timed on the device,
// cold: each timed launch follows a read-modify-write pass over a buffer
// larger than the Infinity Cache and the L2s together, so the matrix comes
// from HBM as it does in a batch of many matrices or after other work; the
// median launch time decides.  An ARG-CSR finalist is also timed with x
// staged in LDS when its groups allow it.  Choices are cached per process
// under a signature of the row-length distribution, so matrices of the same
// shape are tuned once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "plan.hpp"
#include "schedule.hpp"

namespace argcsr {
namespace {

constexpr int32_t kBlockDims[] = {64, 128, 256};
constexpr int32_t kDesired[] = {1, 2, 4, 8, 16, 32, 64};
constexpr int kTimedReps = 7;
// bytes the cache flush between timed launches reads and writes: more than
// the 256 MB Infinity Cache plus the 8 x 4 MB of L2
constexpr size_t kFlushBytes = size_t(512) << 20;

__global__ void flush_kernel(float4* __restrict__ buf, size_t n) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += size_t(gridDim.x) * blockDim.x) {
    float4 v = buf[i];
    v.x += 1.0f;
    buf[i] = v;
  }
}

// Cost model, in microseconds on MI355X, fitted to cold timings of every
// candidate on matrices of both regimes (power-law and mixed rows, whose x
// gathers miss the caches; the 27-point stencil and 2D/3D Laplacians, which
// stream; members of the 256-matrix batch from 1.5e3 to 1.9e5 rows).  A
// group costs one wave a fixed latency (group record, mapping, the first
// loads, the row sums, the store) plus a latency per step of 64 slots, four
// and a half times as long for 8-byte values; the chip keeps 256 CUs x 32
// waves of such chains in flight.  A launch takes the longest of: its bytes
// at the sustained stream rate, the summed chains over the waves in flight,
// and one group's chain (a matrix of few, long groups cannot fill the chip).
// The x gathers cost the same for every candidate of one matrix (one per
// nonzero) and are left out: the model ranks candidates, it does not predict
// the gather-bound time of a matrix with random columns.
constexpr double kStreamBytesPerUs = 5.0e6;
constexpr double kUsPerGroup = 3.0;
constexpr double kUsPerStep = 0.15;
constexpr double kStepFactorF64 = 4.5;
constexpr double kWavesInFlight = 256.0 * 32.0;
constexpr double kUsPerHeavy = 2.0e-3;

double model_us(int32_t dtype, int32_t n_rows, int32_t n_cols, int32_t G, int64_t S, int32_t H) {
  const int sv = dtype == ARGCSR_F64 ? 8 : dtype == ARGCSR_F32 ? 4 : 2;
  const int sx = dtype == ARGCSR_F64 ? 8 : 4;
  const double bytes =
      double(S) * (sv + 4) + 16.0 * G + double(n_rows) * (4 + sx) + double(n_cols) * sx;
  const double step = kUsPerStep * (dtype == ARGCSR_F64 ? kStepFactorF64 : 1.0);
  const double steps = double(S) / 64.0;
  const double chains = (kUsPerGroup * G + step * steps) / kWavesInFlight;
  const double longest = G > 0 ? kUsPerGroup + step * steps / G : 0.0;
  return std::max({bytes / kStreamBytesPerUs, chains, longest}) + kUsPerHeavy * H;
}

// Cost of a matrix as one member of a batch (argcsr_batch_create), in
// microseconds of the batch's time, fitted to whole-batch cold timings of
// the 256-matrix FP32 batch under 21 uniform (T, D) choices: the persistent
// kernel overlaps the members, so only throughput counts -- the bytes of the
// member's slots and groups at a rate that falls with the block size (a
// group's wave streams more slots per step) and a cost per group (the work
// queue hands out groups one by one).  The part that does not depend on the
// choice (x gathers, y, the row offsets) is left out.
constexpr double kMemberBytesPerUs[3] = {5.25e6, 4.9e6, 4.0e6};  // T = 64, 128, 256
constexpr double kMemberUsPerGroup = 3.5e-4;

double member_us(int32_t dtype, int32_t T, int32_t G, int64_t S) {
  const int sv = dtype == ARGCSR_F64 ? 8 : dtype == ARGCSR_F32 ? 4 : 2;
  const int t = T == 64 ? 0 : T == 128 ? 1 : 2;
  return (double(S) * (sv + 4) + 16.0 * G) / kMemberBytesPerUs[t] + kMemberUsPerGroup * G;
}

struct Candidate {
  int32_t T, D, format, G, heavy;
  int64_t S;
  double model_us;
  double measured_us;
  double staged_us;  // with x staged in LDS (gap 0); < 0 if not staged
};

std::mutex g_cache_mutex;
std::map<std::string, argcsr_tune_result> g_cache;

int value_bytes(int32_t dtype) {
  return dtype == ARGCSR_F64 ? 8 : dtype == ARGCSR_F32 ? 4 : 2;
}

// dtype, log2 of n and nnz, and the share of rows in each power-of-two
// row-length bucket (quantised to 1/32).
std::string signature(int32_t n_rows, const int32_t* rp, int32_t dtype) {
  int64_t hist[33] = {0};
  for (int32_t r = 0; r < n_rows; ++r) {
    const int64_t L = int64_t(rp[r + 1]) - rp[r];
    int b = 0;
    while (b < 32 && (int64_t(1) << b) <= L) ++b;
    hist[b]++;
  }
  const int64_t nnz = n_rows > 0 ? rp[n_rows] : 0;
  std::string key = std::to_string(dtype) + ":" +
                    std::to_string(int(std::log2(double(n_rows) + 1.0))) + ":" +
                    std::to_string(int(std::log2(double(nnz) + 1.0)));
  for (int b = 0; b < 33; ++b) {
    const int q = n_rows > 0 ? int(std::lround(32.0 * double(hist[b]) / double(n_rows))) : 0;
    key += "," + std::to_string(hist[b] > 0 ? std::max(q, 1) : 0);
  }
  return key;
}

struct DeviceBuffers {
  argcsr_matrix m{};
  void* mem[9] = {};
  ~DeviceBuffers() {
    for (void* p : mem)
      if (p) (void)hipFree(p);
  }
};

// Every candidate the tuner considers, sized by argcsr_plan (steps 1-2),
// with `cost` as its model estimate; sorted by the estimate (stable: ties
// keep the enumeration order, ARG-CSR before row-grouped CSR at each T).
template <typename Cost>
std::vector<Candidate> plan_candidates(int32_t n_rows, const int32_t* row_ptr_host, Cost cost) {
  std::vector<Candidate> cands;
  auto add = [&](int32_t T, int32_t D, int32_t format) {
    int32_t G = 0, H = 0;
    int64_t S = 0;
    if (argcsr_plan(n_rows, row_ptr_host, T, D, format, &G, &S, &H) != ARGCSR_OK) return;
    cands.push_back(Candidate{T, D, format, G, H, S, cost(T, G, S, H), -1.0, -1.0});
  };
  // besides the powers of two: the longest and the mean row length (capped
  // at 64), the values Sec. 5's rule points to for regular rows
  int64_t longest = 0;
  for (int32_t r = 0; r < n_rows; ++r)
    longest = std::max<int64_t>(longest, int64_t(row_ptr_host[r + 1]) - row_ptr_host[r]);
  const int64_t nnz = n_rows > 0 ? row_ptr_host[n_rows] : 0;
  std::vector<int32_t> desired(std::begin(kDesired), std::end(kDesired));
  for (int64_t d : {longest, n_rows > 0 ? (nnz + n_rows / 2) / n_rows : int64_t(0)})
    if (d >= 1 && d <= 64 && std::find(desired.begin(), desired.end(), int32_t(d)) == desired.end())
      desired.push_back(int32_t(d));
  for (int32_t T : kBlockDims) {
    for (int32_t D : desired) add(T, D, ARGCSR_FORMAT_ARG);
    add(T, 0, ARGCSR_FORMAT_RG);
  }
  clear_error();
  std::stable_sort(cands.begin(), cands.end(),
                   [](const Candidate& a, const Candidate& b) { return a.model_us < b.model_us; });
  return cands;
}

// Median of kTimedReps launches of A's SpMV, each after the cache flush.
int time_spmv(const argcsr_matrix* A, void* x, void* y, float4* flush, hipStream_t s,
              double* median_us) {
  hipEvent_t e0, e1;
  ARGCSR_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(ARGCSR_EHIP, "autotune: hipEventCreate failed");
  }
  int rc = argcsr_spmv(A, x, y, s);  // first launch: code and tables loaded
  std::vector<float> ms;
  for (int i = 0; i < kTimedReps && rc == ARGCSR_OK; ++i) {
    flush_kernel<<<4096, 256, 0, s>>>(flush, kFlushBytes / sizeof(float4));
    if (hipEventRecord(e0, s) != hipSuccess) rc = ARGCSR_EHIP;
    if (rc == ARGCSR_OK) rc = argcsr_spmv(A, x, y, s);
    float t = 0.f;
    if (rc == ARGCSR_OK && (hipEventRecord(e1, s) != hipSuccess ||
                            hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&t, e0, e1) != hipSuccess))
      rc = fail(ARGCSR_EHIP, "autotune: event timing failed");
    ms.push_back(t);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  std::sort(ms.begin(), ms.end());
  *median_us = 1e3 * double(ms[ms.size() / 2]);
  return ARGCSR_OK;
}

// Converts candidate c, times it, and for an ARG-CSR layout also times it
// with x staged in LDS (gap 0) when every group fits the staging limits.
int time_candidate(int32_t n_rows, int32_t n_cols, const int32_t* rp_host, const int32_t* rp,
                   const int32_t* col, const double* val, int32_t dtype, Candidate* c,
                   void* x, void* y, float4* flush, hipStream_t s) {
  DeviceBuffers b;
  argcsr_matrix& m = b.m;
  m.n_rows = n_rows;
  m.n_cols = n_cols;
  m.block_dim = c->T;
  m.desired_chunk_size = c->D;
  m.format = c->format;
  m.dtype = dtype;
  m.n_groups = c->G;
  m.n_slots = c->S;
  m.n_heavy = c->heavy;
  const size_t sizes[5] = {sizeof(argcsr_group_info) * size_t(c->G), sizeof(int32_t) * size_t(n_rows),
                           sizeof(int32_t) * size_t(c->S), size_t(value_bytes(dtype)) * size_t(c->S),
                           sizeof(int32_t) * size_t(c->heavy)};
  for (int i = 0; i < 5; ++i)
    if (sizes[i] && hipMalloc(&b.mem[i], sizes[i]) != hipSuccess)
      return fail(ARGCSR_ENOMEM, "autotune: device allocation of %zu bytes failed", sizes[i]);
  m.groups = static_cast<argcsr_group_info*>(b.mem[0]);
  m.threads_mapping = static_cast<int32_t*>(b.mem[1]);
  m.columns = static_cast<int32_t*>(b.mem[2]);
  m.values = b.mem[3];
  m.heavy_groups = static_cast<int32_t*>(b.mem[4]);
  int rc = argcsr_convert(n_rows, n_cols, rp_host, rp, col, val, &m, s);
  if (rc == ARGCSR_OK) rc = time_spmv(&m, x, y, flush, s, &c->measured_us);
  if (rc || c->format != ARGCSR_FORMAT_ARG || c->G == 0) return rc;
  if (hipMalloc(&b.mem[5], sizeof(int32_t) * (size_t(c->G) + 1)) != hipSuccess)
    return fail(ARGCSR_ENOMEM, "autotune: tile table allocation failed");
  int32_t n_tiles = 0, max_tiles = 0;
  rc = argcsr_stage_plan(&m, 0, static_cast<int32_t*>(b.mem[5]), &n_tiles, &max_tiles, s);
  if (rc == ARGCSR_EUNSUPPORTED) {  // a group beyond the staging limits: not staged
    clear_error();
    return ARGCSR_OK;
  }
  if (rc) return rc;
  if (hipMalloc(&b.mem[6], sizeof(int32_t) * std::max<size_t>(n_tiles, 1)) != hipSuccess ||
      hipMalloc(&b.mem[7], sizeof(int32_t) * std::max<size_t>(n_tiles, 1)) != hipSuccess ||
      hipMalloc(&b.mem[8], sizeof(uint16_t) * size_t(c->S)) != hipSuccess)
    return fail(ARGCSR_ENOMEM, "autotune: staging allocation failed");
  m.stage_gap = 0;
  m.n_stage_tiles = n_tiles;
  m.stage_max_tiles = max_tiles;
  m.stage_lds = 1;
  m.tile_ptr = static_cast<int32_t*>(b.mem[5]);
  m.tile_start = static_cast<int32_t*>(b.mem[6]);
  m.tile_len = static_cast<int32_t*>(b.mem[7]);
  m.local = static_cast<uint16_t*>(b.mem[8]);
  rc = argcsr_stage(&m, s);
  if (rc == ARGCSR_OK) rc = time_spmv(&m, x, y, flush, s, &c->staged_us);
  return rc;
}

}  // namespace
}  // namespace argcsr

extern "C" int argcsr_autotune(int32_t n_rows, int32_t n_cols, const int32_t* row_ptr_host,
                               const int32_t* row_ptr, const int32_t* col, const double* val,
                               int32_t dtype, int32_t n_finalists, argcsr_tune_result* out,
                               void* stream) {
  using namespace argcsr;
  clear_error();
  if (!out) return fail(ARGCSR_EINVAL, "out is NULL");
  if (dtype < ARGCSR_F64 || dtype > ARGCSR_F16) return fail(ARGCSR_EINVAL, "unknown dtype %d", dtype);
  int rc = check_row_ptr(n_rows, row_ptr_host);
  if (rc) return rc;
  const std::string key = signature(n_rows, row_ptr_host, dtype);
  {
    std::lock_guard<std::mutex> lock(g_cache_mutex);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
      *out = it->second;
      out->from_cache = 1;
      return ARGCSR_OK;
    }
  }
  const int sx = dtype == ARGCSR_F64 ? 8 : 4;
  std::vector<Candidate> cands =
      plan_candidates(n_rows, row_ptr_host, [&](int32_t, int32_t G, int64_t S, int32_t H) {
        return model_us(dtype, n_rows, n_cols, G, S, H);
      });
  int32_t n_planned = 0;
  if (cands.empty()) return fail(ARGCSR_EOVERFLOW, "no (block_dim, desired_chunk_size) fits int32");
  // finalists: candidates with a layout of their own (the same T, group
  // count, slot count and heavy count as a better-ranked one is the same
  // layout on every matrix tried: e.g. D = 27, 32, 64 and row-grouped CSR
  // on rows of 27), the best of each T first, then the next in model order
  {
    std::vector<Candidate> distinct;
    for (const Candidate& c : cands) {
      bool dup = false;
      for (const Candidate& d : distinct)
        dup |= d.T == c.T && d.G == c.G && d.S == c.S && d.heavy == c.heavy;
      if (!dup) distinct.push_back(c);
    }
    std::vector<Candidate> order;
    std::vector<bool> used(distinct.size(), false);
    for (int32_t T : kBlockDims) {
      for (size_t i = 0; i < distinct.size(); ++i)
        if (!used[i] && distinct[i].T == T) {
          used[i] = true;
          order.push_back(distinct[i]);
          break;
        }
    }
    std::stable_sort(order.begin(), order.end(),
                     [](const Candidate& a, const Candidate& b) { return a.model_us < b.model_us; });
    for (size_t i = 0; i < distinct.size(); ++i)
      if (!used[i]) order.push_back(distinct[i]);
    const int32_t planned = int32_t(cands.size());
    cands.swap(order);
    n_planned = planned;
  }
  const int n_time = std::max(0, std::min<int>(n_finalists, int(cands.size())));
  int best = 0;
  if (n_time > 0 && n_rows > 0) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    void* x = nullptr;
    void* y = nullptr;
    void* flush = nullptr;
    if (hipMalloc(&x, size_t(sx) * std::max(n_cols, 1)) != hipSuccess ||
        hipMalloc(&y, size_t(sx) * std::max(n_rows, 1)) != hipSuccess ||
        hipMalloc(&flush, kFlushBytes) != hipSuccess) {
      if (x) (void)hipFree(x);
      if (y) (void)hipFree(y);
      return fail(ARGCSR_ENOMEM, "autotune: vector or flush-buffer allocation failed");
    }
    // x = 0: timing does not depend on the values
    rc = hipMemsetAsync(x, 0, size_t(sx) * std::max(n_cols, 1), s) == hipSuccess &&
                 hipMemsetAsync(flush, 0, kFlushBytes, s) == hipSuccess
             ? ARGCSR_OK
             : ARGCSR_EHIP;
    for (int i = 0; i < n_time && rc == ARGCSR_OK; ++i)
      rc = time_candidate(n_rows, n_cols, row_ptr_host, row_ptr, col, val, dtype, &cands[i], x, y,
                          static_cast<float4*>(flush), s);
    (void)hipStreamSynchronize(s);
    (void)hipFree(x);
    (void)hipFree(y);
    (void)hipFree(flush);
    if (rc) return rc;
    auto fastest = [](const Candidate& c) {
      return c.staged_us >= 0.0 ? std::min(c.measured_us, c.staged_us) : c.measured_us;
    };
    for (int i = 1; i < n_time; ++i)
      if (fastest(cands[i]) < fastest(cands[best])) best = i;
  }
  const Candidate& c = cands[best];
  const bool staged = c.staged_us >= 0.0 && c.staged_us < c.measured_us;
  *out = argcsr_tune_result{c.T,        c.D,       c.model_us,
                            staged ? c.staged_us : c.measured_us,
                            0,          n_planned, n_time,
                            c.format,   staged ? 1 : 0};
  std::lock_guard<std::mutex> lock(g_cache_mutex);
  g_cache[key] = *out;
  return ARGCSR_OK;
}

extern "C" int argcsr_autotune_member(int32_t n_rows, const int32_t* row_ptr_host, int32_t dtype,
                                      argcsr_tune_result* out) {
  using namespace argcsr;
  clear_error();
  if (!out) return fail(ARGCSR_EINVAL, "out is NULL");
  if (dtype < ARGCSR_F64 || dtype > ARGCSR_F16) return fail(ARGCSR_EINVAL, "unknown dtype %d", dtype);
  int rc = check_row_ptr(n_rows, row_ptr_host);
  if (rc) return rc;
  const std::string key = "member:" + signature(n_rows, row_ptr_host, dtype);
  {
    std::lock_guard<std::mutex> lock(g_cache_mutex);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
      *out = it->second;
      out->from_cache = 1;
      return ARGCSR_OK;
    }
  }
  const std::vector<Candidate> cands =
      plan_candidates(n_rows, row_ptr_host, [&](int32_t T, int32_t G, int64_t S, int32_t) {
        return member_us(dtype, T, G, S);
      });
  if (cands.empty()) return fail(ARGCSR_EOVERFLOW, "no (block_dim, desired_chunk_size) fits int32");
  const Candidate& c = cands.front();
  *out = argcsr_tune_result{c.T, c.D, c.model_us, -1.0, 0, int32_t(cands.size()), 0, c.format, 0};
  std::lock_guard<std::mutex> lock(g_cache_mutex);
  g_cache[key] = *out;
  return ARGCSR_OK;
}

extern "C" int argcsr_autotune_clear_cache(void) {
  std::lock_guard<std::mutex> lock(argcsr::g_cache_mutex);
  argcsr::g_cache.clear();
  return ARGCSR_OK;
}
