// Host side of the conversion: validation of CSR row offsets, step 1
// (grouping) and the chunk-size rule of step 2 used for sizing.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "argcsr.h"

namespace argcsr {

// rp[0] == 0 and non-decreasing.  Returns ARGCSR_OK or ARGCSR_EINVAL.
int check_row_ptr(int32_t n_rows, const int32_t* rp);

// Step 1 of the conversion (Sec. 3): consecutive rows form a group while the
// group holds at most block_dim rows and at most desired*block_dim nonzeros;
// a row that would break either limit opens the next group.  Fills
// first_row/size of every group (offset and chunk_size left 0).
// Row-grouped CSR (format ARGCSR_FORMAT_RG): groups of block_dim rows.
// With region_desired (host, ceil(n_rows / region_rows) entries >= 1) the
// group that opens at row s takes region_desired[s / region_rows] instead
// of `desired`.
int group_rows(int32_t n_rows, const int32_t* rp, int32_t block_dim,
               int32_t desired, int32_t format, std::vector<argcsr_group_info>* groups,
               int32_t region_rows = 0, const int32_t* region_desired = nullptr);

// The scan of group_rows, handing each group to emit(first_row, size) in
// row order; a nonzero return from emit stops the scan and is returned.
template <class Emit>
int for_each_group(int32_t n_rows, const int32_t* rp, int32_t block_dim, int32_t desired,
                   int32_t format, int32_t region_rows, const int32_t* region_desired,
                   Emit&& emit) {
  const bool rg = format == ARGCSR_FORMAT_RG;
  int32_t start = 0;
  while (start < n_rows) {
    // extend the group from `start` as far as both limits allow (at least one row)
    const int32_t d = region_desired ? region_desired[start / region_rows] : desired;
    const int64_t budget = rg ? INT64_MAX / 2 : int64_t(d) * int64_t(block_dim);
    int32_t end = start + 1;
    const int64_t cap = int64_t(start) + block_dim;
    const int32_t row_cap = cap < n_rows ? int32_t(cap) : n_rows;
    const int64_t base = rp[start];
    while (end < row_cap && int64_t(rp[end + 1]) - base <= budget) ++end;
    const int rc = emit(start, end - start);
    if (rc) return rc;
    start = end;
  }
  return 0;
}

// Steps 1-2 on the host, keeping the group table: first_row, size and
// chunk_size of every group (offset left 0), with the slot and heavy-group
// counts argcsr_plan reports.  Validates row_ptr.
int plan_host_groups(int32_t n_rows, const int32_t* rp, int32_t block_dim, int32_t desired,
                     int32_t format, std::vector<argcsr_group_info>* groups, int64_t* n_slots,
                     int32_t* n_heavy);

// argcsr_convert with step 1 already done on the host: groups_host holds
// out->n_groups groups (first_row, size) in row order as group_rows or
// plan_host_groups make them for out's parameters, from a row_ptr_host that
// has been validated (it is not scanned again).  Synchronous, as
// argcsr_convert.  (convert.hip)
int convert_pregrouped(int32_t n_rows, int32_t n_cols, const int32_t* row_ptr_host,
                       const argcsr_group_info* groups_host, const int32_t* row_ptr,
                       const int32_t* col, const double* val, argcsr_matrix* out,
                       hipStream_t s);

// Checks a region table: region_rows >= 1 and every entry >= 1.
int check_regions(int32_t n_rows, int32_t region_rows, const int32_t* region_desired);

// Step 2 sizing: the smallest chunk size c >= 1 for which the rows of the
// group need at most block_dim chunks, sum max(1, ceil(L_r / c)).
int32_t min_chunk_size(const int32_t* rp, int32_t first, int32_t size,
                       int32_t block_dim);

// Row-grouped CSR: one chunk per row, chunk size max(1, longest row).
int32_t longest_row(const int32_t* rp, int32_t first, int32_t size);

}  // namespace argcsr
