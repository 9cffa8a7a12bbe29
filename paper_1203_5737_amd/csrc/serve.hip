// Serving loop: device-resident ARG-CSR matrices admitted under a memory
// budget, and continuous batching of SpMV and CG-solve requests.
//
// One scheduler thread owns all device work (one stream).  Clients submit
// requests into a queue and poll or wait on tickets.  Each scheduler step:
//   1. takes queued requests in order per matrix: ADMIT converts a matrix
//      and keeps it resident, evicting matrices no running request uses
//      (least recently used first, those no queued request names before the
//      others) if the budget is short, and waiting, with every request behind
//      it, while the matrix cannot fit until running requests end; SPMV/CG
//      requests enter free slots as slots and memory allow.  The host side
//      of an ADMIT (steps 1-2 of the conversion with the group table kept,
//      and a copy of the CSR arrays into pinned staging) is done ahead by a
//      preparation thread, and the upload and conversion kernels run on a
//      converter thread with a stream of its own; an ADMIT still preparing,
//      or waiting for the converter, is passed over together with every later
//      request of its matrix, and requests of resident matrices behind it go
//      on (an ADMIT of a resident matrix then completes only together with
//      the request of that matrix right behind it);
//   2. advances every active request by one step in a few launches for all
//      of them together: a pull of the step's descriptors from mapped pinned
//      memory, one multi-matrix ARG-CSR SpMV per precision (FP32 values for
//      SpMV requests and inner CG iterations, FP64 values for the outer
//      residual of CG), then the CG vector kernels, which also write the
//      scalars the scheduler needs into a mapped pinned mirror; requests in
//      an inner cycle then run up to cg_inner_per_step - 1 further inner
//      iterations (FP32 SpMV and vector kernels again), each skipped on the
//      device for a request whose cycle has stopped;
//   3. after one synchronisation, reads those scalars, retires finished
//      requests and copies their results to the caller's host memory.
// CG (for SPD matrices) keeps x, r, p, d and every dot product, alpha and
// beta in FP64; inner iterations use the FP32 matrix; every inner cycle ends
// with an outer refinement step r = b - A x with the FP64 matrix, and a solve
// finishes when that true residual satisfies |r| <= tol |b|.
// Requests never share reductions, so a result does not depend on which
// other requests were in flight.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "arena.hpp"
#include "hostcopy.hpp"
#include "common.hpp"
#include "mspmv.hpp"
#include "plan.hpp"
#include "schedule.hpp"
#include "serve_kernels.hpp"

namespace argcsr {
namespace {

constexpr size_t kDefaultStaging = size_t(256) << 20;   // pinned staging when the config says 0

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch()).count();
}

// The device memory budget: one allocation carved up by a RangeAllocator.
class Arena {
 public:
  int init(size_t bytes) {
    if (hipMalloc(&base_, bytes) != hipSuccess) {
      base_ = nullptr;
      return fail(ARGCSR_ENOMEM, "server arena of %zu bytes could not be allocated", bytes);
    }
    ranges_.reset(bytes);
    return ARGCSR_OK;
  }
  ~Arena() {
    if (base_) (void)hipFree(base_);
  }
  void* alloc(size_t bytes) {
    const size_t off = ranges_.alloc(bytes);
    return off == RangeAllocator::kNone ? nullptr : static_cast<char*>(base_) + off;
  }
  void release(void* p) {
    if (p) ranges_.release(size_t(static_cast<char*>(p) - static_cast<char*>(base_)));
  }
  size_t in_use() const { return ranges_.in_use(); }
  size_t capacity() const { return ranges_.capacity(); }

 private:
  void* base_ = nullptr;
  RangeAllocator ranges_;
};

// Pinned host memory for request inputs and results, carved up like the
// device arena.  Thread-safe: the scheduler allocates, the copy helper
// releases.
class PinnedArena {
 public:
  int init(size_t bytes) {
    if (bytes == 0) return ARGCSR_OK;
    if (hipHostMalloc(&base_, bytes, hipHostMallocDefault) != hipSuccess) {
      base_ = nullptr;
      return fail(ARGCSR_ENOMEM, "pinned staging of %zu bytes could not be allocated", bytes);
    }
    ranges_.reset(bytes);
    return ARGCSR_OK;
  }
  ~PinnedArena() {
    if (base_) (void)hipHostFree(base_);
  }
  void* alloc(size_t bytes) {
    std::lock_guard<std::mutex> lock(mu_);
    if (!base_) return nullptr;
    const size_t off = ranges_.alloc(bytes);
    return off == RangeAllocator::kNone ? nullptr : static_cast<char*>(base_) + off;
  }
  void release(void* p) {
    std::lock_guard<std::mutex> lock(mu_);
    if (p) ranges_.release(size_t(static_cast<char*>(p) - static_cast<char*>(base_)));
  }

 private:
  void* base_ = nullptr;
  RangeAllocator ranges_;
  std::mutex mu_;
};

struct Resident {
  int64_t id = 0;
  argcsr_matrix m64{};        // FP64 values
  float* values32 = nullptr;  // FP32 values, same layout (groups, mapping, columns shared)
  std::vector<void*> blocks;
  size_t bytes = 0;
  int64_t last_use = 0;
};

enum ReqStatus : int32_t { kPending = 1 };
// admit(): the matrix does not fit yet; memory frees up as running requests
// end, so the ADMIT stays at the head of the queue and is tried again
constexpr int kAdmitWait = 2;
// admit(): the preparation thread has not finished the ADMIT's host side
// yet; it stays at the head of the queue and is tried again
constexpr int kAdmitPending = 3;
// admit(): the matrix's memory is allocated and its conversion handed to the
// converter thread (its own stream); the ADMIT completes when that is done
constexpr int kAdmitStarted = 4;

// The host side of an ADMIT, done ahead of the scheduler by the preparation
// thread: steps 1-2 of the conversion with the group table kept, and the CSR
// arrays copied into pinned staging.  Shared by the request and the thread's
// queue.  State: kQueued -> kRunning -> kReady by the thread; the scheduler
// takes a kQueued one away (kAbandoned: the thread skips it) or waits for a
// kRunning one, so the caller's arrays are never read after its ADMIT has
// completed.
struct AdmitPrep {
  enum : int { kQueued = 0, kRunning = 1, kReady = 2, kAbandoned = 3 };
  std::atomic<int> state{kQueued};
  argcsr_request q{};
  int32_t T = 0, D = 0;
  bool found_resident = false;   // resident when the thread looked: nothing prepared
  int rc = ARGCSR_OK;            // planning error, returned by the ADMIT
  std::vector<argcsr_group_info> groups;
  int64_t n_slots = 0;
  int32_t n_heavy = 0;
  void* stage = nullptr;         // pinned row_ptr | col | val, or NULL (upload from q's arrays)
  size_t off_col = 0, off_val = 0;
};

struct Request;

// A conversion handed to the converter thread: the matrix's resident
// arrays and the CSR staging are allocated in the arena (by the scheduler,
// which owns it); the thread uploads the CSR arrays, converts, rounds the
// FP32 copy of the values and waits for its stream.
struct AdmitJob {
  Request* r = nullptr;
  std::unique_ptr<Resident> m;
  std::vector<size_t> sizes;      // arena bytes of m's blocks
  size_t resident_blocks = 0;     // m->blocks[resident_blocks..] are the CSR staging
  int32_t* d_rp = nullptr;
  int32_t* d_col = nullptr;
  double* d_val = nullptr;
  const void* src_rp = nullptr;   // pinned staging or the caller's arrays
  const void* src_col = nullptr;
  const void* src_val = nullptr;
  int64_t nnz = 0;
  const argcsr_group_info* groups = nullptr;   // prepared step 1, or NULL
  int rc = ARGCSR_OK;
};

struct Request {
  uint64_t ticket = 0;
  argcsr_request q{};
  argcsr_result res{};
  // active state
  int32_t slot = -1;
  int32_t phase = kPhaseStart;
  int32_t inner_in_cycle = 0;
  int32_t parity = 0;          // which CgScalars::rr holds |r|^2 before the next step
  double cycle_rr0 = 0.0;
  std::vector<void*> blocks;
  float* x32 = nullptr;
  float* y32 = nullptr;
  double* v64[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};  // b x r p d q64
  float* p32 = nullptr;
  float* q32 = nullptr;
  Resident* mat = nullptr;
  // ADMIT: sizes from argcsr_plan, kept while the ADMIT waits for memory
  int32_t plan_groups = -1, plan_heavy = 0;
  int64_t plan_slots = 0;
  std::shared_ptr<AdmitPrep> prep;   // host side done ahead (see AdmitPrep)
  // pinned staging of the input (set by the copy helper when filled) and of
  // the result
  void* stage = nullptr;
  std::atomic<int> staged{0};
};

// Work of the copy helper thread: fill a request's pinned input from the
// caller's buffer, or, once `done` has fired, copy its pinned result into
// the caller's buffer and publish it.
struct CopyJob {
  Request* r = nullptr;
  void* stage = nullptr;
  size_t bytes = 0;
  hipEvent_t done = nullptr;    // result copies only
};

}  // namespace
}  // namespace argcsr

struct argcsr_server {
  argcsr_server_config cfg{};
  argcsr::Arena arena;
  hipStream_t stream = nullptr;
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::deque<argcsr::Request*> incoming;                      // guarded by mu
  std::unordered_map<uint64_t, argcsr_result> results;        // guarded by mu
  std::unordered_map<int64_t, int32_t> refs;                  // matrix id -> queued/active requests (mu)
  argcsr_server_stats stats{};                                // guarded by mu
  // scheduler-thread state
  std::deque<argcsr::Request*> pending;
  std::vector<argcsr::Request*> active;
  std::vector<int32_t> free_slots;
  std::unordered_map<int64_t, std::unique_ptr<argcsr::Resident>> resident;
  // per-step device buffers
  void* d_desc = nullptr;
  size_t d_desc_bytes = 0;
  void* h_desc = nullptr;      // mapped pinned staging, pulled by the device
  const void* h_desc_dev = nullptr;   // its device address
  argcsr::CgScalars* d_scalars = nullptr;
  argcsr::CgScalars* h_scalars = nullptr;   // mapped pinned mirror written by the kernels
  argcsr::CgScalars* h_scalars_dev = nullptr;
  // pinned staging and its copy helper
  argcsr::PinnedArena pinned;
  std::thread helper;
  std::mutex hmu;
  std::condition_variable hcv;
  std::deque<argcsr::CopyJob> jobs;          // guarded by hmu
  bool helper_stop = false;                  // guarded by hmu
  std::vector<argcsr::Request*> staging;     // scheduler: waiting for their input copy
  std::vector<void*> stage_release;          // scheduler: free after the next step's sync
  // ADMIT preparation thread
  std::thread preparer;
  std::mutex pmu;
  std::condition_variable pcv;
  std::deque<std::shared_ptr<argcsr::AdmitPrep>> preps;   // guarded by pmu
  bool preparer_stop = false;                              // guarded by pmu
  std::unordered_map<int64_t, int32_t> resident_ids;       // resident matrices (mu)
  // converter thread: one conversion at a time on its own stream
  std::thread converter;
  hipStream_t conv_stream = nullptr;
  std::mutex cmu;
  std::condition_variable ccv;
  argcsr::AdmitJob* conv_todo = nullptr;                   // guarded by cmu
  bool converter_stop = false;                             // guarded by cmu
  std::unique_ptr<argcsr::AdmitJob> admitting;             // scheduler: the conversion in flight
  std::atomic<int> conv_done{0};
  // recorded on the scheduler's stream when a conversion starts; the
  // converter's stream waits for it (see start_admission)
  hipEvent_t conv_after = nullptr;
};

namespace argcsr {
namespace {

void publish(argcsr_server* s, Request* r) {
  r->res.t_done_ns = now_ns();
  std::lock_guard<std::mutex> lock(s->mu);
  s->results[r->ticket] = r->res;
  if (r->q.kind == ARGCSR_REQ_SPMV || r->q.kind == ARGCSR_REQ_CG) {
    auto it = s->refs.find(r->q.matrix_id);
    if (it != s->refs.end() && --it->second == 0) s->refs.erase(it);
    if (r->res.status == ARGCSR_OK) s->stats.completed++;
    else s->stats.failed++;
  }
  s->cv_done.notify_all();
}

bool matrix_idle(argcsr_server* s, int64_t id) {
  std::lock_guard<std::mutex> lock(s->mu);
  return s->refs.find(id) == s->refs.end();
}

// A matrix is pinned while a running request (active, or waiting for its
// input copy) uses it; queued requests do not pin.
bool pinned(const argcsr_server* s, const Resident* m) {
  for (const Request* r : s->active)
    if (r->mat == m) return true;
  for (const Request* r : s->staging)
    if (r->mat == m) return true;
  return false;
}

void evict(argcsr_server* s, Resident* m) {
  for (void* p : m->blocks) s->arena.release(p);
  std::lock_guard<std::mutex> lock(s->mu);
  s->resident_ids.erase(m->id);
  s->stats.evictions++;
  s->stats.resident_matrices--;
  s->stats.resident_bytes -= int64_t(m->bytes);
}

// Arena bytes that evicting every unpinned resident matrix (but `keep`)
// would add to the free space.
size_t evictable_bytes(const argcsr_server* s, int64_t keep) {
  size_t b = 0;
  for (const auto& kv : s->resident) {
    const Resident* m = kv.second.get();
    if (m->id != keep && !pinned(s, m)) b += m->bytes;
  }
  return b;
}

// Allocates from the arena, evicting unpinned matrices (never `keep`) until
// the request fits: first those no queued request refers to, least recently
// used first, then those that queued requests refer to (they would be
// admitted again).  Returns nullptr when every candidate is gone.
void* alloc_evicting(argcsr_server* s, size_t bytes, int64_t keep) {
  for (;;) {
    if (void* p = s->arena.alloc(bytes)) return p;
    Resident* victim = nullptr;
    bool victim_idle = false;
    for (auto& kv : s->resident) {
      Resident* m = kv.second.get();
      if (m->id == keep || pinned(s, m)) continue;
      const bool idle = matrix_idle(s, m->id);
      if (!victim || (idle && !victim_idle) ||
          (idle == victim_idle && m->last_use < victim->last_use)) {
        victim = m;
        victim_idle = idle;
      }
    }
    if (!victim) return nullptr;
    const int64_t id = victim->id;
    evict(s, victim);
    s->resident.erase(id);
  }
}

// Whether memory will free up without the scheduler's help: requests are
// running (their vectors, and the pins on their matrices, go when they end).
bool memory_will_free(const argcsr_server* s) {
  return !s->active.empty() || !s->staging.empty();
}

// Conversion parameters of an ADMIT: the server's block_dim, and its
// desired_chunk_size or else the mean row length in [1, 64].
void admit_params(const argcsr_server_config& cfg, const argcsr_request& q, int64_t nnz,
                  int32_t* T, int32_t* D) {
  *T = cfg.block_dim > 0 ? cfg.block_dim : 64;
  *D = cfg.desired_chunk_size;
  if (*D <= 0) {
    const double mean = q.n_rows > 0 ? double(nnz) / q.n_rows : 1.0;
    *D = int32_t(std::min(64.0, std::max(1.0, std::round(mean))));
  }
}

// Checks of an ADMIT's arguments that need no scan of row_ptr.
int check_admit(const argcsr_request& q) {
  if (q.n_rows < 0 || q.n_cols < 0) return fail(ARGCSR_EINVAL, "negative dimension");
  if (q.n_rows > 0 && !q.row_ptr) return fail(ARGCSR_EINVAL, "row_ptr is NULL");
  if (int64_t(q.n_cols) * 8 > kMaxVectorBytes)
    return fail(ARGCSR_EUNSUPPORTED, "x of %d columns exceeds the gather range", q.n_cols);
  return ARGCSR_OK;
}

// The preparation thread: for each ADMIT in submission order whose matrix
// is not resident, steps 1-2 on the host (group table kept) and a copy of
// the CSR arrays into pinned staging.
void preparer(argcsr_server* s) {
  for (;;) {
    std::shared_ptr<AdmitPrep> p;
    {
      std::unique_lock<std::mutex> lock(s->pmu);
      s->pcv.wait(lock, [&] { return s->preparer_stop || !s->preps.empty(); });
      if (s->preps.empty()) return;
      p = std::move(s->preps.front());
      s->preps.pop_front();
    }
    int expected = AdmitPrep::kQueued;
    if (!p->state.compare_exchange_strong(expected, AdmitPrep::kRunning)) continue;  // abandoned
    const argcsr_request& q = p->q;
    {
      std::lock_guard<std::mutex> lock(s->mu);
      p->found_resident = s->resident_ids.count(q.matrix_id) != 0;
    }
    if (!p->found_resident) {
      p->rc = check_admit(q);
      if (p->rc == ARGCSR_OK) {
        p->rc = check_row_ptr(q.n_rows, q.row_ptr);
        const int64_t nnz = p->rc == ARGCSR_OK && q.n_rows > 0 ? q.row_ptr[q.n_rows] : 0;
        if (p->rc == ARGCSR_OK && nnz > 0 && (!q.col || !q.val))
          p->rc = fail(ARGCSR_EINVAL, "NULL CSR arrays");
        if (p->rc == ARGCSR_OK) {
          // the CSR arrays go to pinned staging (row_ptr | col | val, each
          // 256-byte aligned) on copy threads while this thread groups the
          // rows (steps 1-2): the two do not depend on each other
          auto up = [](size_t b) { return (b + 255) / 256 * 256; };
          const size_t rp_b = sizeof(int32_t) * size_t(q.n_rows + 1);
          const size_t col_b = sizeof(int32_t) * size_t(nnz), val_b = sizeof(double) * size_t(nnz);
          p->off_col = up(rp_b);
          p->off_val = p->off_col + up(col_b);
          p->stage = s->pinned.alloc(p->off_val + val_b);
          std::vector<std::thread> copiers;
          if (p->stage) {
            char* st = static_cast<char*>(p->stage);
            const CopySeg segs[3] = {{st, reinterpret_cast<const char*>(q.row_ptr), rp_b},
                                     {st + p->off_col, reinterpret_cast<const char*>(q.col), nnz > 0 ? col_b : 0},
                                     {st + p->off_val, reinterpret_cast<const char*>(q.val), nnz > 0 ? val_b : 0}};
            copiers = start_copy(segs, 3);
          }
          admit_params(s->cfg, q, nnz, &p->T, &p->D);
          p->rc = plan_host_groups(q.n_rows, q.row_ptr, p->T, p->D, ARGCSR_FORMAT_ARG,
                                   &p->groups, &p->n_slots, &p->n_heavy);
          for (std::thread& t : copiers) t.join();
          if (p->rc != ARGCSR_OK && p->stage) {
            s->pinned.release(p->stage);
            p->stage = nullptr;
          }
        }
      }
    }
    p->state.store(AdmitPrep::kReady, std::memory_order_release);
    std::lock_guard<std::mutex> lock(s->mu);
    s->cv_work.notify_one();
  }
}

// Lets go of an ADMIT's preparation once the ADMIT is complete: a queued
// one is abandoned, a running one waited for (it still reads the caller's
// arrays), a ready one's staging freed.
void drop_prep(argcsr_server* s, Request* r) {
  AdmitPrep* p = r->prep.get();
  if (!p) return;
  int expected = AdmitPrep::kQueued;
  if (!p->state.compare_exchange_strong(expected, AdmitPrep::kAbandoned)) {
    while (p->state.load(std::memory_order_acquire) == AdmitPrep::kRunning)
      std::this_thread::sleep_for(std::chrono::microseconds(50));
    if (p->state.load(std::memory_order_acquire) == AdmitPrep::kReady) {
      s->pinned.release(p->stage);
      p->stage = nullptr;
    }
  }
  r->prep.reset();
}

int admit(argcsr_server* s, Request* r) {
  const argcsr_request& q = r->q;
  AdmitPrep* prep = r->prep.get();
  if (s->resident.count(q.matrix_id)) {
    // nothing to convert; a preparation still reading the caller's arrays
    // must finish first (the ADMIT completes when this returns)
    if (prep) {
      int expected = AdmitPrep::kQueued;
      if (!prep->state.compare_exchange_strong(expected, AdmitPrep::kAbandoned)) {
        if (expected == AdmitPrep::kRunning) return kAdmitPending;
        s->pinned.release(prep->stage);           // kReady: its staging is ours to free
        prep->stage = nullptr;
      }
      r->prep.reset();
    }
    s->resident[q.matrix_id]->last_use = now_ns();
    return ARGCSR_OK;
  }
  bool prepared = false;
  if (prep) {
    const int st = prep->state.load(std::memory_order_acquire);
    if (st == AdmitPrep::kQueued || st == AdmitPrep::kRunning) return kAdmitPending;
    if (st == AdmitPrep::kReady && !prep->found_resident) {
      if (prep->rc) {
        const int rc = prep->rc;
        r->prep.reset();
        return rc;
      }
      prepared = true;
    }
  }
  int rc = check_admit(q);
  if (rc) return rc;
  if (!prepared) {
    rc = check_row_ptr(q.n_rows, q.row_ptr);
    if (rc) return rc;
  }
  const int64_t nnz = q.n_rows > 0 ? q.row_ptr[q.n_rows] : 0;
  if (nnz > 0 && (!q.col || !q.val)) return fail(ARGCSR_EINVAL, "NULL CSR arrays");
  int32_t T = 0, D = 0;
  admit_params(s->cfg, q, nnz, &T, &D);
  auto m = std::make_unique<Resident>();
  m->id = q.matrix_id;
  argcsr_matrix& A = m->m64;
  A.n_rows = q.n_rows;
  A.n_cols = q.n_cols;
  A.block_dim = T;
  A.desired_chunk_size = D;
  A.dtype = ARGCSR_F64;
  if (prepared) {
    r->plan_groups = int32_t(prep->groups.size());
    r->plan_slots = prep->n_slots;
    r->plan_heavy = prep->n_heavy;
  } else if (r->plan_groups < 0) {       // planned once, also when the ADMIT has to wait
    rc = argcsr_plan(q.n_rows, q.row_ptr, T, D, ARGCSR_FORMAT_ARG, &r->plan_groups,
                     &r->plan_slots, &r->plan_heavy);
    if (rc) {
      r->plan_groups = -1;
      return rc;
    }
  }
  A.n_groups = r->plan_groups;
  A.n_slots = r->plan_slots;
  A.n_heavy = r->plan_heavy;
  // everything the conversion holds at once: the resident arrays and the
  // CSR staging (released after the conversion)
  auto rounded = [](size_t b) { return (std::max<size_t>(b, 1) + kAlign - 1) / kAlign * kAlign; };
  const size_t need = rounded(sizeof(argcsr_group_info) * size_t(A.n_groups)) +
                      rounded(sizeof(int32_t) * size_t(q.n_rows)) +
                      rounded(sizeof(int32_t) * size_t(A.n_slots)) +
                      rounded(sizeof(double) * size_t(A.n_slots)) +
                      rounded(sizeof(float) * size_t(A.n_slots)) +
                      rounded(sizeof(int32_t) * size_t(std::max(A.n_heavy, 1))) +
                      rounded(sizeof(int32_t) * size_t(q.n_rows + 1)) +
                      rounded(sizeof(int32_t) * size_t(std::max<int64_t>(nnz, 1))) +
                      rounded(sizeof(double) * size_t(std::max<int64_t>(nnz, 1)));
  if (need > s->arena.capacity())
    return fail(ARGCSR_EBUDGET, "matrix %lld needs %zu bytes; the budget is %zu",
                (long long)q.matrix_id, need, s->arena.capacity());
  // not enough room even after evicting every unpinned matrix: wait for
  // running requests to end, if any are running
  if (s->arena.capacity() - s->arena.in_use() + evictable_bytes(s, q.matrix_id) < need &&
      memory_will_free(s))
    return kAdmitWait;
  std::vector<size_t> sizes;
  auto grab = [&](size_t bytes) -> void* {
    void* p = alloc_evicting(s, bytes, q.matrix_id);
    if (p) {
      m->blocks.push_back(p);
      sizes.push_back((std::max<size_t>(bytes, 1) + kAlign - 1) / kAlign * kAlign);
    }
    return p;
  };
  auto give_back = [&]() {
    for (void* p : m->blocks) s->arena.release(p);
  };
  const size_t resident_blocks = 6;               // then the CSR staging, released after the conversion
  int32_t* d_rp = nullptr;
  int32_t* d_col = nullptr;
  double* d_val = nullptr;
  auto allocate = [&]() -> bool {
    A.groups = static_cast<argcsr_group_info*>(grab(sizeof(argcsr_group_info) * size_t(A.n_groups)));
    A.threads_mapping = static_cast<int32_t*>(grab(sizeof(int32_t) * size_t(q.n_rows)));
    A.columns = static_cast<int32_t*>(grab(sizeof(int32_t) * size_t(A.n_slots)));
    A.values = grab(sizeof(double) * size_t(A.n_slots));
    m->values32 = static_cast<float*>(grab(sizeof(float) * size_t(A.n_slots)));
    A.heavy_groups = static_cast<int32_t*>(grab(sizeof(int32_t) * size_t(std::max(A.n_heavy, 1))));
    d_rp = static_cast<int32_t*>(grab(sizeof(int32_t) * size_t(q.n_rows + 1)));
    d_col = static_cast<int32_t*>(grab(sizeof(int32_t) * size_t(std::max<int64_t>(nnz, 1))));
    d_val = static_cast<double*>(grab(sizeof(double) * size_t(std::max<int64_t>(nnz, 1))));
    if (m->blocks.size() == resident_blocks + 3) return true;
    give_back();
    m->blocks.clear();
    sizes.clear();
    return false;
  };
  if (!allocate()) {
    // the blocks already placed can split the free space (they went into the
    // holes that evictions left): with requests running, wait for them;
    // with nothing running, evict every other matrix and place the blocks
    // again on the emptied arena
    if (memory_will_free(s)) return kAdmitWait;
    for (auto it = s->resident.begin(); it != s->resident.end();) {
      if (it->first != q.matrix_id && !pinned(s, it->second.get())) {
        evict(s, it->second.get());
        it = s->resident.erase(it);
      } else {
        ++it;
      }
    }
    if (!allocate())
      return fail(ARGCSR_EBUDGET, "matrix %lld (%lld slots) does not fit the %zu-byte budget",
                  (long long)q.matrix_id, (long long)A.n_slots, s->arena.capacity());
  }
  // the conversion goes to the converter thread; the CSR arrays come from
  // the preparation's pinned staging (asynchronous DMA) or the caller's memory
  auto job = std::make_unique<AdmitJob>();
  const char* st = prepared ? static_cast<const char*>(prep->stage) : nullptr;
  job->r = r;
  job->sizes = std::move(sizes);
  job->resident_blocks = resident_blocks;
  job->d_rp = d_rp;
  job->d_col = d_col;
  job->d_val = d_val;
  job->src_rp = st ? static_cast<const void*>(st) : q.row_ptr;
  job->src_col = st ? static_cast<const void*>(st + prep->off_col) : q.col;
  job->src_val = st ? static_cast<const void*>(st + prep->off_val) : q.val;
  job->nnz = nnz;
  job->groups = prepared ? prep->groups.data() : nullptr;
  job->m = std::move(m);
  s->admitting = std::move(job);
  return kAdmitStarted;
}

// The converter thread's part of an ADMIT (on its own stream, waited for).
void convert_job(argcsr_server* s, AdmitJob* j) {
  const argcsr_request& q = j->r->q;
  argcsr_matrix& A = j->m->m64;
  hipStream_t cs = s->conv_stream;
  int rc = ARGCSR_OK;
  if (hipStreamWaitEvent(cs, s->conv_after, 0) != hipSuccess)
    rc = fail(ARGCSR_EHIP, "conversion could not be ordered after the scheduler's stream");
  if (rc == ARGCSR_OK && hipMemcpyAsync(j->d_rp, j->src_rp, sizeof(int32_t) * size_t(q.n_rows + 1),
                     hipMemcpyHostToDevice, cs) != hipSuccess ||
      (j->nnz > 0 && (hipMemcpyAsync(j->d_col, j->src_col, sizeof(int32_t) * size_t(j->nnz),
                                     hipMemcpyHostToDevice, cs) != hipSuccess ||
                      hipMemcpyAsync(j->d_val, j->src_val, sizeof(double) * size_t(j->nnz),
                                     hipMemcpyHostToDevice, cs) != hipSuccess)))
    rc = fail(ARGCSR_EHIP, "CSR upload failed");
  if (rc == ARGCSR_OK)
    rc = j->groups ? convert_pregrouped(q.n_rows, q.n_cols, q.row_ptr, j->groups, j->d_rp,
                                        j->d_col, j->d_val, &A, cs)
                   : argcsr_convert(q.n_rows, q.n_cols, q.row_ptr, j->d_rp, j->d_col, j->d_val,
                                    &A, cs);
  if (rc == ARGCSR_OK && A.n_slots > 0) {
    const int64_t blocks = std::min<int64_t>((A.n_slots + kVecBlock - 1) / kVecBlock, 8192);
    round_values_kernel<<<int(blocks), kVecBlock, 0, cs>>>(static_cast<const double*>(A.values),
                                                           j->m->values32, A.n_slots);
    if (hipGetLastError() != hipSuccess) rc = fail(ARGCSR_EHIP, "value rounding failed");
  }
  if (hipStreamSynchronize(cs) != hipSuccess && rc == ARGCSR_OK)
    rc = fail(ARGCSR_EHIP, "conversion stream failed");
  j->rc = rc;
}

void converter(argcsr_server* s) {
  (void)hipSetDevice(s->cfg.device);
  for (;;) {
    AdmitJob* j = nullptr;
    {
      std::unique_lock<std::mutex> lock(s->cmu);
      s->ccv.wait(lock, [&] { return s->converter_stop || s->conv_todo; });
      if (!s->conv_todo) return;
      j = s->conv_todo;
      s->conv_todo = nullptr;
    }
    convert_job(s, j);
    s->conv_done.store(1, std::memory_order_release);
    std::lock_guard<std::mutex> lock(s->mu);
    s->cv_work.notify_one();
  }
}

// Scheduler: the converter finished the ADMIT in flight; the CSR staging
// goes back to the arena, the matrix becomes resident (or its memory goes
// back too), and the ADMIT completes.
void finish_admission(argcsr_server* s) {
  std::unique_ptr<AdmitJob> j = std::move(s->admitting);
  s->conv_done.store(0, std::memory_order_relaxed);
  Request* r = j->r;
  Resident* m = j->m.get();
  for (size_t i = j->resident_blocks; i < m->blocks.size(); ++i) s->arena.release(m->blocks[i]);
  m->blocks.resize(j->resident_blocks);
  drop_prep(s, r);                                // its staging has been read
  if (j->rc == ARGCSR_OK) {
    argcsr_matrix& A = m->m64;
    m->bytes = 0;
    for (size_t i = 0; i < j->resident_blocks; ++i) m->bytes += j->sizes[i];
    if (A.n_heavy == 0) A.heavy_groups = nullptr;
    m->last_use = now_ns();
    {
      std::lock_guard<std::mutex> lock(s->mu);
      s->resident_ids[r->q.matrix_id] = 1;
      s->stats.admissions++;
      s->stats.resident_matrices++;
      s->stats.resident_bytes += int64_t(m->bytes);
    }
    s->resident[r->q.matrix_id] = std::move(j->m);
  } else {
    for (void* p : m->blocks) s->arena.release(p);
  }
  r->res.status = j->rc;
  r->res.iterations = j->rc == ARGCSR_OK ? 1 : 0;
  publish(s, r);
  delete r;
}

// Starts a conversion the scheduler has prepared with admit().  Arena blocks
// are freed in the order of the scheduler's stream (a finished request's
// vectors are released while the copy of its result is still queued), so
// the blocks the conversion writes may still be read there: its stream
// first waits for everything queued on the scheduler's stream so far.
void start_admission(argcsr_server* s) {
  (void)hipEventRecord(s->conv_after, s->stream);
  s->conv_done.store(0, std::memory_order_relaxed);
  std::lock_guard<std::mutex> lock(s->cmu);
  s->conv_todo = s->admitting.get();
  s->ccv.notify_one();
}

void release_request(argcsr_server* s, Request* r) {
  for (void* p : r->blocks) s->arena.release(p);
  r->blocks.clear();
  if (r->slot >= 0) s->free_slots.push_back(r->slot);
  r->slot = -1;
}

struct Span {
  void* dev;
  size_t bytes;
};

// The device vector a request's input goes to, and the one its result
// comes from (request vectors and matrix must be set).
Span input_of(const Request* r) {
  const argcsr_matrix& A = r->mat->m64;
  if (r->q.kind == ARGCSR_REQ_SPMV) return Span{r->x32, sizeof(float) * size_t(A.n_cols)};
  return Span{r->v64[0], sizeof(double) * size_t(A.n_rows)};
}

Span output_of(const Request* r) {
  const argcsr_matrix& A = r->mat->m64;
  if (r->q.kind == ARGCSR_REQ_SPMV) return Span{r->y32, sizeof(float) * size_t(A.n_rows)};
  return Span{r->v64[1], sizeof(double) * size_t(A.n_rows)};
}

// Hands a finished request's result to the caller with `status`: an
// asynchronous copy into pinned staging that the copy helper completes and
// publishes, or, without staging space, a synchronous copy and publish here.
// Frees the request's device vectors either way (in stream order, so the
// copy still reads them).
void finish(argcsr_server* s, Request* r, int status) {
  const Span out = output_of(r);
  r->res.status = status;
  void* st = s->pinned.alloc(out.bytes);
  hipEvent_t ev = nullptr;
  if (st && hipMemcpyAsync(st, out.dev, out.bytes, hipMemcpyDeviceToHost, s->stream) == hipSuccess &&
      hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess &&
      hipEventRecord(ev, s->stream) == hipSuccess) {
    release_request(s, r);
    std::lock_guard<std::mutex> lock(s->hmu);
    s->jobs.push_back(CopyJob{r, st, out.bytes, ev});
    s->hcv.notify_one();
    return;
  }
  if (ev) (void)hipEventDestroy(ev);
  if (st) {
    (void)hipStreamSynchronize(s->stream);     // the copy may have been queued
    s->pinned.release(st);
  }
  if (hipMemcpy(r->q.out, out.dev, out.bytes, hipMemcpyDeviceToHost) != hipSuccess)
    r->res.status = fail(ARGCSR_EHIP, "result copy failed");
  release_request(s, r);
  publish(s, r);
  delete r;
}

// The copy helper thread: host-side copies between callers' buffers and the
// pinned staging, so that the scheduler never waits on them.
void copy_helper(argcsr_server* s) {
  (void)hipSetDevice(s->cfg.device);
  for (;;) {
    CopyJob j;
    {
      std::unique_lock<std::mutex> lock(s->hmu);
      s->hcv.wait(lock, [&] { return s->helper_stop || !s->jobs.empty(); });
      if (s->jobs.empty()) return;
      j = s->jobs.front();
      s->jobs.pop_front();
    }
    if (j.done) {                              // a result: wait for its copy, hand it over
      if (hipEventSynchronize(j.done) != hipSuccess)
        j.r->res.status = ARGCSR_EHIP;
      else
        std::memcpy(j.r->q.out, j.stage, j.bytes);
      (void)hipEventDestroy(j.done);
      s->pinned.release(j.stage);
      publish(s, j.r);
      delete j.r;
    } else {                                   // an input: fill the staging, wake the scheduler
      std::memcpy(j.stage, j.r->q.in, j.bytes);
      j.r->staged.store(1, std::memory_order_release);
      std::lock_guard<std::mutex> lock(s->mu);
      s->cv_work.notify_one();
    }
  }
}

// Moves a queued SPMV/CG request into a slot: allocates its vectors and
// starts its input copy (staged requests become active once the copy
// helper has filled their staging).  Returns ARGCSR_EBUSY if memory is
// short right now.
int activate(argcsr_server* s, Request* r) {
  auto it = s->resident.find(r->q.matrix_id);
  if (it == s->resident.end())
    return fail(ARGCSR_ENOTFOUND, "matrix %lld is not resident (admit it first)",
                (long long)r->q.matrix_id);
  Resident* m = it->second.get();
  const argcsr_matrix& A = m->m64;
  if (!r->q.in || !r->q.out) return fail(ARGCSR_EINVAL, "request input or output is NULL");
  // the caller's buffers hold the lengths it states; they must be the matrix's
  if (r->q.n_rows != A.n_rows || r->q.n_cols != A.n_cols)
    return fail(ARGCSR_EINVAL,
                "request for matrix %lld states %d x %d, but the resident matrix is %d x %d",
                (long long)r->q.matrix_id, r->q.n_rows, r->q.n_cols, A.n_rows, A.n_cols);
  auto grab = [&](size_t bytes) -> void* {
    void* p = alloc_evicting(s, bytes, m->id);
    if (p) r->blocks.push_back(p);
    return p;
  };
  if (r->q.kind == ARGCSR_REQ_SPMV) {
    r->x32 = static_cast<float*>(grab(sizeof(float) * size_t(std::max(A.n_cols, 1))));
    r->y32 = static_cast<float*>(grab(sizeof(float) * size_t(std::max(A.n_rows, 1))));
    if (!r->x32 || !r->y32) {
      for (void* p : r->blocks) s->arena.release(p);
      r->blocks.clear();
      return ARGCSR_EBUSY;
    }
  } else {
    if (A.n_rows != A.n_cols) return fail(ARGCSR_EINVAL, "CG needs a square matrix");
    const size_t n = size_t(std::max(A.n_rows, 1));
    bool ok = true;
    for (int k = 0; k < 6; ++k) ok &= (r->v64[k] = static_cast<double*>(grab(sizeof(double) * n))) != nullptr;
    ok &= (r->p32 = static_cast<float*>(grab(sizeof(float) * n))) != nullptr;
    ok &= (r->q32 = static_cast<float*>(grab(sizeof(float) * n))) != nullptr;
    if (!ok) {
      for (void* p : r->blocks) s->arena.release(p);
      r->blocks.clear();
      return ARGCSR_EBUSY;
    }
    ARGCSR_HIP(hipMemsetAsync(r->v64[1], 0, sizeof(double) * size_t(A.n_rows), s->stream));
    r->phase = kPhaseStart;
    r->parity = 0;
  }
  r->mat = m;
  // the input: through pinned staging filled by the copy helper (the
  // scheduler uploads it once staged), or, without staging space, straight
  // from the caller's memory
  const Span in = input_of(r);
  r->stage = s->pinned.alloc(in.bytes);
  if (r->stage) {
    std::lock_guard<std::mutex> lock(s->hmu);
    s->jobs.push_back(CopyJob{r, r->stage, in.bytes, nullptr});
    s->hcv.notify_one();
  } else {
    ARGCSR_HIP(hipMemcpyAsync(in.dev, r->q.in, in.bytes, hipMemcpyHostToDevice, s->stream));
  }
  m->last_use = now_ns();
  r->slot = s->free_slots.back();
  s->free_slots.pop_back();
  r->res.t_start_ns = now_ns();
  return ARGCSR_OK;
}

void fill_matwork(MatWork& w, const argcsr_matrix& A, const void* values, const void* x, void* y,
                  int32_t& groups, int32_t& heavy) {
  w.groups = A.groups;
  w.tm = A.threads_mapping;
  w.columns = A.columns;
  w.values = values;
  w.heavy = A.heavy_groups;
  w.x = x;
  w.y = y;
  w.block_dim = A.block_dim;
  w.n_cols = A.n_cols;
  w.serial = serial_gathers(values == A.values ? 8 : 4, A.block_dim, A.n_slots, A.n_groups);
  w.heavy_chunk = A.heavy_groups ? A.heavy_chunk : INT32_MAX;
  w.group_begin = groups;
  w.heavy_begin = heavy;
  groups += A.n_groups;
  heavy += A.heavy_groups ? A.n_heavy : 0;
}

void free_desc(argcsr_server* s) {
  if (s->d_desc) (void)hipFree(s->d_desc);
  if (s->h_desc) (void)hipHostFree(s->h_desc);
  s->d_desc = nullptr;
  s->h_desc = nullptr;
  s->h_desc_dev = nullptr;
  s->d_desc_bytes = 0;
}

// Grows the descriptor buffers (device copy and mapped host block) to hold
// `bytes`; on failure the server is left with none, so the next step retries.
int ensure_desc(argcsr_server* s, size_t bytes) {
  if (bytes <= s->d_desc_bytes) return ARGCSR_OK;
  if (s->d_desc) {
    ARGCSR_HIP(hipStreamSynchronize(s->stream));
    free_desc(s);
  }
  const size_t want = std::max(bytes * 2, size_t(1) << 20);
  void *d = nullptr, *h = nullptr, *dev = nullptr;
  const bool ok =
      hipMalloc(&d, want) == hipSuccess &&
      hipHostMalloc(&h, want, hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess &&
      hipHostGetDevicePointer(&dev, h, 0) == hipSuccess;
  s->d_desc = d;
  s->h_desc = h;
  if (!ok) {
    (void)hipGetLastError();
    free_desc(s);
    return fail(ARGCSR_ENOMEM, "cannot allocate %zu bytes of request descriptors", want);
  }
  s->h_desc_dev = dev;
  s->d_desc_bytes = want;
  return ARGCSR_OK;
}

template <int DT>
void launch_mspmv(argcsr_server* s, const MatWork* d_w, int32_t n, int32_t groups, int32_t heavy) {
  const int64_t grid = int64_t(heavy) + (int64_t(groups) + kSpmvWaves - 1) / kSpmvWaves;
  const dim3 g(uint32_t(std::max<int64_t>(grid, 1))), blk(kSpmvWaves * 64);
  switch (s->cfg.block_dim > 0 ? s->cfg.block_dim : 64) {   // every resident matrix has it
    case 64: mspmv_kernel<DT, 1, 8><<<g, blk, 0, s->stream>>>(d_w, n, groups, heavy); break;
    case 128: mspmv_kernel<DT, 2, 4><<<g, blk, 0, s->stream>>>(d_w, n, groups, heavy); break;
    default: mspmv_kernel<DT, 4, 2><<<g, blk, 0, s->stream>>>(d_w, n, groups, heavy); break;
  }
}

// One step for every active request.
int step(argcsr_server* s) {
  std::vector<Request*> f32, f64, cg;
  for (Request* r : s->active) {
    if (r->q.kind == ARGCSR_REQ_SPMV) f32.push_back(r);
    else {
      cg.push_back(r);
      if (r->phase == kPhaseInner) f32.push_back(r);
      else if (r->phase == kPhaseOuter) f64.push_back(r);
    }
  }
  // Inner requests may run further iterations (passes) in this step, as many
  // as their iteration limits allow; the kernels skip a request once its
  // cycle has stopped, so later passes hold subsets of the earlier ones.
  const int passes = s->cfg.cg_inner_per_step > 0 ? s->cfg.cg_inner_per_step : 2;
  std::vector<std::vector<Request*>> extra(size_t(passes - 1));
  for (Request* r : cg) {
    if (r->phase != kPhaseInner) continue;
    const int k = std::min({passes, s->cfg.cg_max_inner - r->inner_in_cycle,
                            s->cfg.cg_max_iter - r->res.iterations});
    for (int q = 2; q <= k; ++q) extra[size_t(q - 2)].push_back(r);
  }
  auto tiles_of = [](const std::vector<Request*>& rs) {
    int32_t t = 0;
    for (Request* r : rs) t += (r->mat->m64.n_rows + kTile - 1) / kTile;
    return t;
  };
  auto align16 = [](size_t x) { return (x + 15) / 16 * 16; };
  const int32_t tiles = tiles_of(cg);
  // descriptor block: MatWork f32 | MatWork f64 | CgVec | tile table, then per
  // further pass MatWork | CgVec | tile table, then two partial arrays (every
  // pass's tiles are a subset of the first pass's)
  const size_t o_w32 = 0;
  const size_t o_f64 = o_w32 + sizeof(MatWork) * f32.size();
  const size_t o_vec = o_f64 + sizeof(MatWork) * f64.size();
  const size_t o_tile = o_vec + sizeof(CgVec) * cg.size();
  struct Pass {
    size_t o_w, o_vec, o_tile;
    int32_t tiles, groups, heavy;
  };
  std::vector<Pass> xp(extra.size());
  size_t o = align16(o_tile + sizeof(int32_t) * size_t(tiles));
  for (size_t q = 0; q < extra.size(); ++q) {
    xp[q].tiles = tiles_of(extra[q]);
    xp[q].o_w = o;
    xp[q].o_vec = o = align16(o + sizeof(MatWork) * extra[q].size());
    xp[q].o_tile = o = align16(o + sizeof(CgVec) * extra[q].size());
    o = align16(o + sizeof(int32_t) * size_t(xp[q].tiles));
  }
  const size_t o_part = o;
  const size_t o_part2 = o_part + sizeof(double) * size_t(std::max(tiles, 1));
  const size_t total = o_part2 + sizeof(double) * size_t(std::max(tiles, 1));
  int rc = ensure_desc(s, total);
  if (rc) return rc;
  char* h = static_cast<char*>(s->h_desc);
  char* d = static_cast<char*>(s->d_desc);
  int32_t g32 = 0, h32 = 0, g64 = 0, h64 = 0;
  for (size_t i = 0; i < f32.size(); ++i) {
    Request* r = f32[i];
    const argcsr_matrix& A = r->mat->m64;
    MatWork& w = reinterpret_cast<MatWork*>(h + o_w32)[i];
    if (r->q.kind == ARGCSR_REQ_SPMV) fill_matwork(w, A, r->mat->values32, r->x32, r->y32, g32, h32);
    else fill_matwork(w, A, r->mat->values32, r->p32, r->q32, g32, h32);
  }
  for (size_t i = 0; i < f64.size(); ++i) {
    Request* r = f64[i];
    MatWork& w = reinterpret_cast<MatWork*>(h + o_f64)[i];
    fill_matwork(w, r->mat->m64, r->mat->m64.values, r->v64[1], r->v64[5], g64, h64);
  }
  int32_t t = 0;
  int32_t* tile_req = reinterpret_cast<int32_t*>(h + o_tile);
  for (size_t i = 0; i < cg.size(); ++i) {
    Request* r = cg[i];
    CgVec& v = reinterpret_cast<CgVec*>(h + o_vec)[i];
    v = CgVec{r->v64[0], r->v64[1], r->v64[2], r->v64[3], r->v64[4], r->v64[5],
              r->p32, r->q32, r->mat->m64.n_rows, r->phase, t, r->slot, r->parity, 1,
              s->cfg.cg_inner_tol * s->cfg.cg_inner_tol * r->cycle_rr0};
    const int32_t nt = (r->mat->m64.n_rows + kTile - 1) / kTile;
    for (int32_t k = 0; k < nt; ++k) tile_req[t + k] = int32_t(i);
    t += nt;
  }
  for (size_t q = 0; q < extra.size(); ++q) {
    const int32_t pass = int32_t(q) + 2;
    int32_t tq = 0;
    xp[q].groups = xp[q].heavy = 0;
    int32_t* tq_req = reinterpret_cast<int32_t*>(h + xp[q].o_tile);
    for (size_t i = 0; i < extra[q].size(); ++i) {
      Request* r = extra[q][i];
      MatWork& w = reinterpret_cast<MatWork*>(h + xp[q].o_w)[i];
      fill_matwork(w, r->mat->m64, r->mat->values32, r->p32, r->q32, xp[q].groups, xp[q].heavy);
      CgVec& v = reinterpret_cast<CgVec*>(h + xp[q].o_vec)[i];
      v = CgVec{r->v64[0], r->v64[1], r->v64[2], r->v64[3], r->v64[4], r->v64[5],
                r->p32, r->q32, r->mat->m64.n_rows, kPhaseInner, tq, r->slot,
                r->parity ^ ((pass - 1) & 1), pass,
                s->cfg.cg_inner_tol * s->cfg.cg_inner_tol * r->cycle_rr0};
      const int32_t nt = (r->mat->m64.n_rows + kTile - 1) / kTile;
      for (int32_t k = 0; k < nt; ++k) tq_req[tq + k] = int32_t(i);
      tq += nt;
    }
  }
  {
    const int64_t n16 = int64_t(o_part / 16);          // o_part is a multiple of 16
    const int64_t blocks = std::min<int64_t>((n16 + kVecBlock - 1) / kVecBlock, 64);
    desc_pull_kernel<<<dim3(uint32_t(std::max<int64_t>(blocks, 1))), kVecBlock, 0, s->stream>>>(
        static_cast<const int4*>(s->h_desc_dev), reinterpret_cast<int4*>(d), n16);
  }
  const MatWork* d_w32 = reinterpret_cast<const MatWork*>(d + o_w32);
  const MatWork* d_w64 = reinterpret_cast<const MatWork*>(d + o_f64);
  const CgVec* d_vec = reinterpret_cast<const CgVec*>(d + o_vec);
  const int32_t* d_tiles = reinterpret_cast<const int32_t*>(d + o_tile);
  double* d_pq = reinterpret_cast<double*>(d + o_part);
  double* d_rr = reinterpret_cast<double*>(d + o_part2);
  const int ncg = int(cg.size());
  if (!f64.empty()) cg_pre_kernel<<<tiles, kVecBlock, 0, s->stream>>>(d_vec, d_tiles);
  if (!f32.empty()) launch_mspmv<ARGCSR_F32>(s, d_w32, int32_t(f32.size()), g32, h32);
  if (!f64.empty()) launch_mspmv<ARGCSR_F64>(s, d_w64, int32_t(f64.size()), g64, h64);
  if (ncg > 0) {
    cg_dot_kernel<<<tiles, kVecBlock, 0, s->stream>>>(d_vec, d_tiles, s->d_scalars, d_pq);
    cg_update_kernel<<<tiles, kVecBlock, 0, s->stream>>>(d_vec, d_tiles, s->d_scalars,
                                                         s->h_scalars_dev, d_pq, d_rr);
    cg_direction_kernel<<<tiles, kVecBlock, 0, s->stream>>>(d_vec, d_tiles, s->d_scalars,
                                                            s->h_scalars_dev, d_rr);
  }
  for (size_t q = 0; q < extra.size() && !extra[q].empty(); ++q) {
    const auto* dw = reinterpret_cast<const MatWork*>(d + xp[q].o_w);
    const auto* dv = reinterpret_cast<const CgVec*>(d + xp[q].o_vec);
    const auto* dt = reinterpret_cast<const int32_t*>(d + xp[q].o_tile);
    const int32_t tq = xp[q].tiles;
    launch_mspmv<ARGCSR_F32>(s, dw, int32_t(extra[q].size()), xp[q].groups, xp[q].heavy);
    cg_dot_kernel<<<tq, kVecBlock, 0, s->stream>>>(dv, dt, s->d_scalars, d_pq);
    cg_update_kernel<<<tq, kVecBlock, 0, s->stream>>>(dv, dt, s->d_scalars, s->h_scalars_dev,
                                                      d_pq, d_rr);
    cg_direction_kernel<<<tq, kVecBlock, 0, s->stream>>>(dv, dt, s->d_scalars, s->h_scalars_dev,
                                                         d_rr);
  }
  ARGCSR_HIP(hipGetLastError());
  ARGCSR_HIP(hipStreamSynchronize(s->stream));
  for (void* p : s->stage_release) s->pinned.release(p);   // their uploads have run
  s->stage_release.clear();

  // retire / advance
  std::vector<Request*> keep;
  for (Request* r : s->active) {
    bool done = false;
    int status = ARGCSR_OK;
    if (r->q.kind == ARGCSR_REQ_SPMV) {
      done = true;
    } else {
      const CgScalars& sc = s->h_scalars[r->slot];
      // inner: the step ran passes 1..n, pass j with parity parity ^ ((j-1)&1)
      // writing rr[1 - that]; the other phases ran one pass
      const int n = r->phase == kPhaseInner ? std::max(1, std::min(sc.passes, passes)) : 1;
      const double rr = sc.rr[1 - (r->parity ^ ((n - 1) & 1))];
      r->parity ^= n & 1;
      if (r->phase == kPhaseInner) {
        r->res.iterations += n;
        r->inner_in_cycle += n;
        const bool cycle_done = sc.pq <= 0.0 ||
                                rr <= s->cfg.cg_inner_tol * s->cfg.cg_inner_tol * r->cycle_rr0 ||
                                r->inner_in_cycle >= s->cfg.cg_max_inner ||
                                r->res.iterations >= s->cfg.cg_max_iter;
        if (cycle_done) r->phase = kPhaseOuter;
      } else {
        if (r->phase == kPhaseOuter) r->res.refinements++;
        r->res.relres = sc.bnorm2 > 0.0 ? std::sqrt(rr / sc.bnorm2) : 0.0;
        if (r->res.relres <= s->cfg.cg_tol || r->res.iterations >= s->cfg.cg_max_iter) {
          status = r->res.relres <= s->cfg.cg_tol ? ARGCSR_OK : ARGCSR_ENOCONV;
          done = true;
        } else {
          r->phase = kPhaseInner;
          r->inner_in_cycle = 0;
          r->cycle_rr0 = rr;
        }
      }
    }
    if (done) finish(s, r, status);
    else keep.push_back(r);
  }
  s->active.swap(keep);
  std::lock_guard<std::mutex> lock(s->mu);
  s->stats.steps++;
  return ARGCSR_OK;
}

void scheduler(argcsr_server* s) {
  (void)hipSetDevice(s->cfg.device);
  for (;;) {
    {
      auto staged_ready = [&] {
        for (Request* r : s->staging)
          if (r->staged.load(std::memory_order_acquire)) return true;
        return false;
      };
      std::unique_lock<std::mutex> lock(s->mu);
      if (s->active.empty() && s->pending.empty() && s->incoming.empty() && !s->stop &&
          !staged_ready())
        s->cv_work.wait_for(lock, std::chrono::milliseconds(2));
      if (s->stop && s->incoming.empty()) break;
      while (!s->incoming.empty()) {
        s->pending.push_back(s->incoming.front());
        s->incoming.pop_front();
      }
    }
    // the conversion in flight, if it has finished
    if (s->admitting && s->conv_done.load(std::memory_order_acquire)) finish_admission(s);
    // admissions and new requests, in submission order per matrix.  An
    // ADMIT whose preparation is still running, or that must convert while
    // a conversion runs (on the converter's stream) or behind such an ADMIT,
    // is passed over, and so is every later request of its matrix (or of the
    // matrix being converted): they keep their order and are taken up on a
    // later scan.  Requests of other, resident matrices go on meanwhile.  An
    // ADMIT waiting for memory, a full set of request slots, a request that
    // must wait for memory, and an EVICT behind anything passed over stop
    // the scan: everything behind waits (in order).
    bool admit_waiting = false;
    bool passed = false;                 // a request was passed over in this scan
    std::vector<int64_t> held;           // matrices with a passed-over request
    auto is_held = [&](int64_t id) { return std::find(held.begin(), held.end(), id) != held.end(); };
    // Starts the SPMV/CG request at pending[k] (a slot is free): false if it
    // must wait for memory (it stays queued), true once it has left the
    // queue, started or failed.
    auto start = [&](size_t k) -> bool {
      Request* q = s->pending[k];
      const int rc = activate(s, q);
      if (rc == ARGCSR_EBUSY) {
        if (memory_will_free(s) || s->admitting != nullptr) return false;   // memory frees up
        q->res.status = fail(ARGCSR_EBUDGET, "request does not fit the budget");
      } else if (rc != ARGCSR_OK) {
        q->res.status = rc;
      }
      s->pending.erase(s->pending.begin() + std::ptrdiff_t(k));
      if (rc == ARGCSR_OK) {
        if (q->stage) s->staging.push_back(q);   // starts once its input is staged
        else s->active.push_back(q);
      } else {
        release_request(s, q);
        publish(s, q);
        delete q;
      }
      return true;
    };
    for (size_t i = 0; i < s->pending.size();) {
      Request* r = s->pending[i];
      const int64_t converting = s->admitting ? s->admitting->r->q.matrix_id : -1;
      const bool busy = s->admitting != nullptr;
      const int64_t id = r->q.matrix_id;
      auto pass_over = [&]() {
        if (!is_held(id)) held.push_back(id);
        passed = true;
        ++i;
      };
      if (r->q.kind != ARGCSR_REQ_EVICT && (id == converting || is_held(id))) {
        pass_over();                                   // behind an earlier request of its matrix
        continue;
      }
      if (r->q.kind == ARGCSR_REQ_ADMIT) {
        const bool was_resident = s->resident.count(id) != 0;
        if (!was_resident && (busy || passed)) {       // conversions start in submission order
          pass_over();
          continue;
        }
        if (was_resident && passed) {
          // Behind a passed-over ADMIT, which may evict when it runs: an
          // ADMIT of a resident matrix completes only together with the
          // request of that matrix right behind it, so that the matrix stays
          // resident until the request starts (the submission-order promise).
          const bool pair = i + 1 < s->pending.size() &&
                            s->pending[i + 1]->q.kind != ARGCSR_REQ_ADMIT &&
                            s->pending[i + 1]->q.kind != ARGCSR_REQ_EVICT &&
                            s->pending[i + 1]->q.matrix_id == id;
          if (!pair) {
            pass_over();
            continue;
          }
          if (s->free_slots.empty()) break;
          if (r->res.t_start_ns == 0) r->res.t_start_ns = now_ns();
          if (admit(s, r) == kAdmitPending) {          // its preparation still reads the arrays
            admit_waiting = true;
            pass_over();
            continue;
          }
          // resident: admit() only marked the use (it does so again when retried)
          if (!start(i + 1)) break;                    // the request waits for memory, and so does the ADMIT
          s->pending.erase(s->pending.begin() + std::ptrdiff_t(i));
          drop_prep(s, r);
          r->res.status = ARGCSR_OK;
          r->res.iterations = 0;
          publish(s, r);
          delete r;
          continue;
        }
        if (r->res.t_start_ns == 0) r->res.t_start_ns = now_ns();
        const int rc = admit(s, r);
        if (rc == kAdmitPending) {                     // preparation still running
          admit_waiting = true;
          pass_over();
          continue;
        }
        if (rc == kAdmitWait) {                        // waits for memory: everything behind waits
          admit_waiting = true;
          break;
        }
        s->pending.erase(s->pending.begin() + std::ptrdiff_t(i));
        if (rc == kAdmitStarted) {                        // completes in finish_admission
          start_admission(s);
          continue;
        }
        drop_prep(s, r);
        r->res.status = rc;
        r->res.iterations = (r->res.status == ARGCSR_OK && !was_resident) ? 1 : 0;
        publish(s, r);
        delete r;
        continue;
      }
      if (r->q.kind == ARGCSR_REQ_EVICT) {
        if (busy || passed) break;
        s->pending.erase(s->pending.begin() + std::ptrdiff_t(i));
        auto it = s->resident.find(r->q.matrix_id);
        const bool used = it != s->resident.end() && pinned(s, it->second.get());
        if (it == s->resident.end()) r->res.status = ARGCSR_ENOTFOUND;
        else if (used || !matrix_idle(s, r->q.matrix_id)) r->res.status = ARGCSR_EBUSY;
        else {
          evict(s, it->second.get());
          s->resident.erase(it);
          r->res.status = ARGCSR_OK;
        }
        publish(s, r);
        delete r;
        continue;
      }
      if (s->free_slots.empty()) break;           // wait for a slot
      if (!start(i)) break;                       // memory frees up as requests finish
    }
    // staged inputs: upload (in stream order before the next step) and start
    for (size_t i = 0; i < s->staging.size();) {
      Request* r = s->staging[i];
      if (!r->staged.load(std::memory_order_acquire)) {
        ++i;
        continue;
      }
      const Span in = input_of(r);
      if (hipMemcpyAsync(in.dev, r->stage, in.bytes, hipMemcpyHostToDevice, s->stream) !=
          hipSuccess) {
        (void)hipStreamSynchronize(s->stream);
        s->pinned.release(r->stage);
        r->stage = nullptr;
        r->res.status = fail(ARGCSR_EHIP, "input upload failed");
        release_request(s, r);
        publish(s, r);
        delete r;
      } else {
        s->stage_release.push_back(r->stage);
        r->stage = nullptr;
        s->active.push_back(r);
      }
      s->staging[i] = s->staging.back();
      s->staging.pop_back();
    }
    if ((admit_waiting || s->admitting) && s->active.empty()) {
      // only input copies are in flight: give the copy helper a moment
      std::unique_lock<std::mutex> lock(s->mu);
      s->cv_work.wait_for(lock, std::chrono::microseconds(200));
    }
    if (!s->active.empty()) {
      const int rc = step(s);
      if (rc != ARGCSR_OK) {       // device or allocation error: fail everything in flight
        for (Request* r : s->active) {
          r->res.status = rc;
          release_request(s, r);
          publish(s, r);
          delete r;
        }
        s->active.clear();
      }
    }
  }
  // shut down: the conversion in flight finishes first (it writes into the
  // arena), then what is left fails
  while (s->admitting && !s->conv_done.load(std::memory_order_acquire))
    std::this_thread::sleep_for(std::chrono::microseconds(100));
  if (s->admitting) finish_admission(s);
  for (Request* r : s->active) {
    r->res.status = ARGCSR_ENOTFOUND;
    release_request(s, r);
    publish(s, r);
    delete r;
  }
  for (Request* r : s->pending) {
    drop_prep(s, r);                          // before the caller may free the arrays
    r->res.status = ARGCSR_ENOTFOUND;
    publish(s, r);
    delete r;
  }
  s->active.clear();
  s->pending.clear();
}

}  // namespace
}  // namespace argcsr

extern "C" int argcsr_server_create(const argcsr_server_config* cfg, argcsr_server** out) {
  using namespace argcsr;
  clear_error();
  if (!cfg || !out) return fail(ARGCSR_EINVAL, "NULL argument");
  *out = nullptr;
  if (cfg->budget_bytes <= 0 || cfg->max_active < 1 || cfg->max_active > kMaxLaunchMats ||
      !(cfg->cg_tol > 0) || !(cfg->cg_inner_tol > 0) || cfg->cg_max_inner < 1 ||
      cfg->cg_max_iter < 1 || (cfg->block_dim != 0 && cfg->block_dim != 64 &&
                               cfg->block_dim != 128 && cfg->block_dim != 256) ||
      cfg->cg_inner_per_step < 0 || cfg->cg_inner_per_step > kMaxInnerPerStep)
    return fail(ARGCSR_EINVAL, "invalid server configuration");
  auto* s = new (std::nothrow) argcsr_server();
  if (!s) return fail(ARGCSR_ENOMEM, "host allocation failed");
  s->cfg = *cfg;
  int rc = ARGCSR_OK;
  if (hipSetDevice(cfg->device) != hipSuccess) rc = fail(ARGCSR_EHIP, "hipSetDevice failed");
  if (!rc) rc = s->arena.init(size_t(cfg->budget_bytes));
  if (!rc && cfg->staging_bytes >= 0)
    rc = s->pinned.init(cfg->staging_bytes > 0 ? size_t(cfg->staging_bytes) : kDefaultStaging);
  // both streams at the default priority
  if (!rc && (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess ||
              hipStreamCreateWithFlags(&s->conv_stream, hipStreamNonBlocking) != hipSuccess ||
              hipEventCreateWithFlags(&s->conv_after, hipEventDisableTiming) != hipSuccess))
    rc = fail(ARGCSR_EHIP, "hipStreamCreate failed");
  if (!rc && (hipMalloc(&s->d_scalars, sizeof(CgScalars) * size_t(cfg->max_active)) != hipSuccess ||
              hipHostMalloc(&s->h_scalars, sizeof(CgScalars) * size_t(cfg->max_active),
                            hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
              hipHostGetDevicePointer(reinterpret_cast<void**>(&s->h_scalars_dev), s->h_scalars,
                                      0) != hipSuccess))
    rc = fail(ARGCSR_ENOMEM, "server buffers could not be allocated");
  if (rc) {
    if (s->stream) (void)hipStreamDestroy(s->stream);
    if (s->conv_stream) (void)hipStreamDestroy(s->conv_stream);
    if (s->conv_after) (void)hipEventDestroy(s->conv_after);
    if (s->d_scalars) (void)hipFree(s->d_scalars);
    if (s->h_scalars) (void)hipHostFree(s->h_scalars);
    delete s;
    return rc;
  }
  for (int32_t k = cfg->max_active - 1; k >= 0; --k) s->free_slots.push_back(k);
  s->helper = std::thread(copy_helper, s);
  s->preparer = std::thread(preparer, s);
  s->converter = std::thread(converter, s);
  s->worker = std::thread(scheduler, s);
  *out = s;
  return ARGCSR_OK;
}

extern "C" int argcsr_server_submit(argcsr_server* s, const argcsr_request* q, uint64_t* ticket) {
  using namespace argcsr;
  clear_error();
  if (!s || !q || !ticket) return fail(ARGCSR_EINVAL, "NULL argument");
  if (q->kind < ARGCSR_REQ_ADMIT || q->kind > ARGCSR_REQ_EVICT)
    return fail(ARGCSR_EINVAL, "unknown request kind %d", q->kind);
  auto* r = new (std::nothrow) Request();
  if (!r) return fail(ARGCSR_ENOMEM, "host allocation failed");
  r->q = *q;
  r->res.status = kPending;
  r->res.t_submit_ns = now_ns();
  std::lock_guard<std::mutex> lock(s->mu);
  if (s->stop) {
    delete r;
    return fail(ARGCSR_EINVAL, "server is shutting down");
  }
  r->ticket = s->next_ticket++;
  s->results[r->ticket] = r->res;
  if (q->kind == ARGCSR_REQ_SPMV || q->kind == ARGCSR_REQ_CG) {
    s->refs[q->matrix_id]++;
    s->stats.submitted++;
  }
  if (q->kind == ARGCSR_REQ_ADMIT) {
    auto p = std::make_shared<AdmitPrep>();
    p->q = *q;
    r->prep = p;
    std::lock_guard<std::mutex> plock(s->pmu);
    s->preps.push_back(std::move(p));
    s->pcv.notify_one();
  }
  s->incoming.push_back(r);
  *ticket = r->ticket;
  s->cv_work.notify_one();
  return ARGCSR_OK;
}

extern "C" int argcsr_server_poll(argcsr_server* s, uint64_t ticket, argcsr_result* res) {
  using namespace argcsr;
  clear_error();
  if (!s || !res) return fail(ARGCSR_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lock(s->mu);
  auto it = s->results.find(ticket);
  if (it == s->results.end()) return fail(ARGCSR_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  *res = it->second;
  return ARGCSR_OK;
}

extern "C" int argcsr_server_wait(argcsr_server* s, uint64_t ticket, int64_t timeout_ns,
                                  argcsr_result* res) {
  using namespace argcsr;
  clear_error();
  if (!s || !res) return fail(ARGCSR_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lock(s->mu);
  const auto deadline = std::chrono::steady_clock::now() + std::chrono::nanoseconds(timeout_ns);
  for (;;) {
    auto it = s->results.find(ticket);
    if (it == s->results.end()) return fail(ARGCSR_ENOTFOUND, "unknown ticket");
    if (it->second.status != kPending) {
      *res = it->second;
      return ARGCSR_OK;
    }
    if (s->cv_done.wait_until(lock, deadline) == std::cv_status::timeout) {
      *res = s->results[ticket];
      return res->status == kPending ? fail(ARGCSR_EBUSY, "timed out") : ARGCSR_OK;
    }
  }
}

extern "C" int argcsr_server_release(argcsr_server* s, uint64_t ticket) {
  using namespace argcsr;
  clear_error();
  if (!s) return fail(ARGCSR_EINVAL, "NULL server");
  std::lock_guard<std::mutex> lock(s->mu);
  auto it = s->results.find(ticket);
  if (it == s->results.end()) return fail(ARGCSR_ENOTFOUND, "unknown ticket");
  if (it->second.status == kPending) return fail(ARGCSR_EBUSY, "request still in flight");
  s->results.erase(it);
  return ARGCSR_OK;
}

extern "C" int argcsr_server_get_stats(argcsr_server* s, argcsr_server_stats* out) {
  using namespace argcsr;
  clear_error();
  if (!s || !out) return fail(ARGCSR_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lock(s->mu);
  *out = s->stats;
  out->arena_bytes = int64_t(s->arena.capacity());
  return ARGCSR_OK;
}

extern "C" int argcsr_server_destroy(argcsr_server* s) {
  using namespace argcsr;
  clear_error();
  if (!s) return ARGCSR_OK;
  {
    std::lock_guard<std::mutex> lock(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  {
    std::lock_guard<std::mutex> lock(s->hmu);   // the helper drains its queue, then exits
    s->helper_stop = true;
    s->hcv.notify_all();
  }
  if (s->helper.joinable()) s->helper.join();
  {
    std::lock_guard<std::mutex> lock(s->pmu);    // the preparer drains its queue, then exits
    s->preparer_stop = true;
    s->pcv.notify_all();
  }
  if (s->preparer.joinable()) s->preparer.join();
  {
    std::lock_guard<std::mutex> lock(s->cmu);    // the scheduler waited for its last conversion
    s->converter_stop = true;
    s->ccv.notify_all();
  }
  if (s->converter.joinable()) s->converter.join();
  for (auto& p : s->preps) s->pinned.release(p->stage);
  s->preps.clear();
  for (Request* r : s->staging) {               // never started
    s->pinned.release(r->stage);
    r->res.status = ARGCSR_ENOTFOUND;
    release_request(s, r);
    publish(s, r);
    delete r;
  }
  s->staging.clear();
  (void)hipStreamSynchronize(s->stream);
  (void)hipStreamDestroy(s->stream);
  if (s->conv_stream) (void)hipStreamDestroy(s->conv_stream);
  if (s->conv_after) (void)hipEventDestroy(s->conv_after);
  free_desc(s);
  (void)hipFree(s->d_scalars);
  (void)hipHostFree(s->h_scalars);
  delete s;
  return ARGCSR_OK;
}
