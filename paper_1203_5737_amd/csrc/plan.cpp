// Host conversion steps used before any kernel runs: grouping (step 1, a
// sequential scan over the rows) and the slot count of the result.
#include "plan.hpp"

#include <algorithm>

#include "common.hpp"
#include "schedule.hpp"

namespace argcsr {

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

int group_rows(int32_t n_rows, const int32_t* rp, int32_t block_dim,
               int32_t desired, std::vector<argcsr_group_info>* groups) {
  groups->clear();
  const int64_t budget = int64_t(desired) * int64_t(block_dim);
  int32_t start = 0;
  while (start < n_rows) {
    // extend the group from `start` as far as both limits allow (at least one row)
    int32_t end = start + 1;
    const int32_t row_cap = (int32_t)std::min<int64_t>(n_rows, int64_t(start) + block_dim);
    const int64_t base = rp[start];
    while (end < row_cap && int64_t(rp[end + 1]) - base <= budget) ++end;
    groups->push_back(argcsr_group_info{start, end - start, 0, 0});
    start = end;
  }
  return ARGCSR_OK;
}

int32_t min_chunk_size(const int32_t* rp, int32_t first, int32_t size,
                       int32_t block_dim) {
  int64_t longest = 0;
  for (int32_t l = 0; l < size; ++l)
    longest = std::max<int64_t>(longest, int64_t(rp[first + l + 1]) - rp[first + l]);
  const int64_t total = int64_t(rp[first + size]) - rp[first];
  auto chunks_needed = [&](int64_t c) {
    int64_t need = 0;
    for (int32_t l = 0; l < size; ++l) {
      const int64_t L = int64_t(rp[first + l + 1]) - rp[first + l];
      need += L > c ? (L + c - 1) / c : 1;
    }
    return need;
  };
  // chunks_needed is non-increasing in c; at c = longest every row needs one
  // chunk (size <= block_dim), and no c below total/block_dim can fit.
  int64_t lo = std::max<int64_t>(1, (total + block_dim - 1) / block_dim);
  int64_t hi = std::max<int64_t>(1, longest);
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (chunks_needed(mid) <= block_dim) hi = mid;
    else lo = mid + 1;
  }
  return (int32_t)lo;
}

}  // namespace argcsr

extern "C" int argcsr_plan(int32_t n_rows, const int32_t* row_ptr_host,
                           int32_t block_dim, int32_t desired_chunk_size,
                           int32_t* n_groups, int64_t* n_slots, int32_t* n_heavy) {
  using namespace argcsr;
  clear_error();
  if (!n_groups || !n_slots) return fail(ARGCSR_EINVAL, "NULL output pointer");
  if (block_dim < 1 || desired_chunk_size < 1)
    return fail(ARGCSR_EINVAL, "block_dim and desired_chunk_size must be >= 1");
  int rc = check_row_ptr(n_rows, row_ptr_host);
  if (rc) return rc;
  std::vector<argcsr_group_info> groups;
  rc = group_rows(n_rows, row_ptr_host, block_dim, desired_chunk_size, &groups);
  if (rc) return rc;
  std::vector<int32_t> chunk(groups.size());
  int64_t slots = 0;
  for (size_t g = 0; g < groups.size(); ++g) {
    chunk[g] = min_chunk_size(row_ptr_host, groups[g].first_row, groups[g].size, block_dim);
    slots += int64_t(chunk[g]) * block_dim;
  }
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
