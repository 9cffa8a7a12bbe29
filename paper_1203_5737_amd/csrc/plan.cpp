// Host conversion steps used before any kernel runs: grouping (step 1, a
// sequential scan over the rows) and the slot count of the result.
#include "plan.hpp"

#include <algorithm>
#include <thread>

#include "common.hpp"
#include "schedule.hpp"

namespace argcsr {

namespace {
constexpr int32_t kMaxGroupRows = 1024;   // plan/convert accept block_dim <= 1024
}  // namespace

int check_row_ptr(int32_t n_rows, const int32_t* rp) {
  if (n_rows < 0) return fail(ARGCSR_EINVAL, "n_rows < 0");
  if (n_rows > 0 && rp == nullptr) return fail(ARGCSR_EINVAL, "row_ptr is NULL");
  if (rp == nullptr) return ARGCSR_OK;
  if (rp[0] != 0) return fail(ARGCSR_EINVAL, "row_ptr[0] = %d, expected 0", rp[0]);
  for (int32_t r = 0; r < n_rows; ++r)
    if (rp[r + 1] < rp[r])
      return fail(ARGCSR_EINVAL, "row_ptr decreases at row %d", r);
  return ARGCSR_OK;
}

int check_regions(int32_t n_rows, int32_t region_rows, const int32_t* region_desired) {
  if (!region_desired) return ARGCSR_OK;
  if (region_rows < 1) return fail(ARGCSR_EINVAL, "region_rows must be >= 1");
  for (int64_t w = 0; w * region_rows < n_rows; ++w)
    if (region_desired[w] < 1)
      return fail(ARGCSR_EINVAL, "region_desired[%lld] = %d < 1", (long long)w, region_desired[w]);
  return ARGCSR_OK;
}

int group_rows(int32_t n_rows, const int32_t* rp, int32_t block_dim,
               int32_t desired, int32_t format, std::vector<argcsr_group_info>* groups,
               int32_t region_rows, const int32_t* region_desired) {
  groups->clear();
  return for_each_group(n_rows, rp, block_dim, desired, format, region_rows, region_desired,
                        [groups](int32_t first, int32_t size) {
                          groups->push_back(argcsr_group_info{first, size, 0, 0});
                          return 0;
                        });
}

int32_t longest_row(const int32_t* rp, int32_t first, int32_t size) {
  int32_t longest = 1;
  for (int32_t l = 0; l < size; ++l) longest = std::max(longest, rp[first + l + 1] - rp[first + l]);
  return longest;
}

int32_t min_chunk_size(const int32_t* rp, int32_t first, int32_t size,
                       int32_t block_dim) {
  const uint32_t T = uint32_t(block_dim);
  uint32_t longest = 0;
  for (int32_t l = 0; l < size; ++l)
    longest = std::max(longest, uint32_t(rp[first + l + 1] - rp[first + l]));
  if (size == 1) return int32_t(longest > T ? (longest - 1) / T + 1 : 1);   // one row: ceil(L/T)
  const uint64_t total = uint64_t(rp[first + size]) - uint64_t(rp[first]);
  // chunks_needed is non-increasing in c; at c = longest every row needs one
  // chunk (size <= block_dim), no c below total/block_dim can fit, and since
  // max(1, ceil(L/c)) <= L/c + 1 every c >= total/(block_dim - size) fits.
  // A group of block_dim rows has one chunk per row.
  uint32_t lo = uint32_t(std::max<uint64_t>(1, (total + T - 1) / T));
  uint32_t hi = std::max<uint32_t>(1, longest);
  if (uint32_t(size) >= T) return int32_t(hi);
  hi = uint32_t(std::min<uint64_t>(hi, std::max<uint64_t>(1, (total + (T - size) - 1) / (T - size))));
  if (lo >= hi) return int32_t(hi);
  // for c >= lo only rows longer than lo can need more than one chunk
  uint32_t longer[kMaxGroupRows];
  int32_t n_longer = 0;
  for (int32_t l = 0; l < size; ++l) {
    const uint32_t L = uint32_t(rp[first + l + 1] - rp[first + l]);
    if (L > lo) longer[n_longer++] = L;
  }
  auto chunks_needed = [&](uint32_t c) {
    uint64_t need = uint64_t(size - n_longer);
    for (int32_t k = 0; k < n_longer; ++k)
      need += longer[k] > c ? (longer[k] - 1) / c + 1 : 1;
    return need;
  };
  // the answer is usually the lower bound or just above it
  for (int k = 0; k < 2 && lo < hi; ++k, ++lo)
    if (chunks_needed(lo) <= T) return int32_t(lo);
  while (lo < hi) {
    const uint32_t mid = lo + (hi - lo) / 2;
    if (chunks_needed(mid) <= T) hi = mid;
    else lo = mid + 1;
  }
  return int32_t(lo);
}

}  // namespace argcsr

namespace argcsr {
namespace {

int plan_impl(int32_t n_rows, const int32_t* row_ptr_host, int32_t block_dim,
              int32_t desired_chunk_size, int32_t format, int32_t region_rows,
              const int32_t* region_desired, int32_t* n_groups, int64_t* n_slots,
              int32_t* n_heavy, std::vector<argcsr_group_info>* keep = nullptr) {
  if (!n_groups || !n_slots) return fail(ARGCSR_EINVAL, "NULL output pointer");
  if (format != ARGCSR_FORMAT_ARG && format != ARGCSR_FORMAT_RG)
    return fail(ARGCSR_EINVAL, "unknown format %d", format);
  const bool row_grouped = format == ARGCSR_FORMAT_RG;
  if (block_dim < 1 || block_dim > kMaxGroupRows || (!row_grouped && desired_chunk_size < 1))
    return fail(ARGCSR_EINVAL, "block_dim must be in [1, %d] and desired_chunk_size >= 1",
                kMaxGroupRows);
  int rc = check_row_ptr(n_rows, row_ptr_host);
  if (rc) return rc;
  rc = check_regions(n_rows, region_rows, region_desired);
  if (rc) return rc;
  std::vector<argcsr_group_info> own;
  std::vector<argcsr_group_info>& groups = keep ? *keep : own;
  rc = group_rows(n_rows, row_ptr_host, block_dim, desired_chunk_size, format, &groups,
                  region_rows, region_desired);
  if (rc) return rc;
  // step 2 is independent per group: split large matrices over host threads
  std::vector<int32_t> chunk(groups.size());
  const size_t G = groups.size();
  const unsigned hw = std::max(1u, std::min(8u, std::thread::hardware_concurrency()));
  const unsigned n_threads = G >= 16384 ? hw : 1;
  auto work = [&](unsigned t) {
    for (size_t g = t * G / n_threads; g < (t + 1) * G / n_threads; ++g)
      chunk[g] = row_grouped ? longest_row(row_ptr_host, groups[g].first_row, groups[g].size)
                             : min_chunk_size(row_ptr_host, groups[g].first_row, groups[g].size,
                                              block_dim);
  };
  std::vector<std::thread> pool;
  for (unsigned t = 1; t < n_threads; ++t) pool.emplace_back(work, t);
  work(0);
  for (auto& th : pool) th.join();
  int64_t slots = 0;
  for (size_t g = 0; g < G; ++g) slots += int64_t(chunk[g]) * block_dim;
  if (keep)
    for (size_t g = 0; g < G; ++g) groups[g].chunk_size = chunk[g];
  const int32_t heavy_chunk = heavy_chunk_for(block_dim, slots, (int32_t)groups.size());
  int32_t heavy = 0;
  for (int32_t c : chunk) heavy += c > heavy_chunk;
  *n_groups = (int32_t)groups.size();
  *n_slots = slots;
  if (n_heavy) *n_heavy = heavy;
  if (slots > INT32_MAX)
    return fail(ARGCSR_EOVERFLOW, "%lld slots exceed INT32_MAX", (long long)slots);
  return ARGCSR_OK;
}

}  // namespace

int plan_host_groups(int32_t n_rows, const int32_t* rp, int32_t block_dim, int32_t desired,
                     int32_t format, std::vector<argcsr_group_info>* groups, int64_t* n_slots,
                     int32_t* n_heavy) {
  int32_t G = 0;
  return plan_impl(n_rows, rp, block_dim, desired, format, 0, nullptr, &G, n_slots, n_heavy,
                   groups);
}

}  // namespace argcsr

extern "C" int argcsr_plan(int32_t n_rows, const int32_t* row_ptr_host,
                           int32_t block_dim, int32_t desired_chunk_size, int32_t format,
                           int32_t* n_groups, int64_t* n_slots, int32_t* n_heavy) {
  argcsr::clear_error();
  return argcsr::plan_impl(n_rows, row_ptr_host, block_dim, desired_chunk_size, format, 0,
                           nullptr, n_groups, n_slots, n_heavy);
}

extern "C" int argcsr_plan_regions(int32_t n_rows, const int32_t* row_ptr_host,
                                   int32_t block_dim, int32_t region_rows,
                                   const int32_t* region_desired, int32_t* n_groups,
                                   int64_t* n_slots, int32_t* n_heavy) {
  using namespace argcsr;
  clear_error();
  if (!region_desired) return fail(ARGCSR_EINVAL, "region_desired is NULL");
  return plan_impl(n_rows, row_ptr_host, block_dim, 1, ARGCSR_FORMAT_ARG, region_rows,
                   region_desired, n_groups, n_slots, n_heavy);
}

// The Sec. 5 rule applied per region: a region whose rows are regular (its
// longest row at most twice its mean length) gets desiredChunkSize = its
// longest row, capped at max_desired, so that its groups take block_dim rows
// with one chunk each; any other region gets 1, the robust setting.
extern "C" int argcsr_choose_region_desired(int32_t n_rows, const int32_t* row_ptr_host,
                                            int32_t region_rows, int32_t max_desired,
                                            int32_t* region_desired) {
  using namespace argcsr;
  clear_error();
  if (region_rows < 1 || max_desired < 1 || (n_rows > 0 && !region_desired))
    return fail(ARGCSR_EINVAL, "region_rows and max_desired must be >= 1");
  int rc = check_row_ptr(n_rows, row_ptr_host);
  if (rc) return rc;
  for (int64_t first = 0; first < n_rows; first += region_rows) {
    const int64_t end = std::min<int64_t>(n_rows, first + region_rows);
    int64_t longest = 0;
    for (int64_t r = first; r < end; ++r)
      longest = std::max<int64_t>(longest, int64_t(row_ptr_host[r + 1]) - row_ptr_host[r]);
    const int64_t nnz = int64_t(row_ptr_host[end]) - row_ptr_host[first];
    const bool regular = longest > 0 && longest * (end - first) <= 2 * nnz;
    region_desired[first / region_rows] =
        regular ? int32_t(std::min<int64_t>(longest, max_desired)) : 1;
  }
  return ARGCSR_OK;
}
