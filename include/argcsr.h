/*
 * argcsr.h -- C ABI of libargcsr, Adaptive Row-grouped CSR (ARG-CSR) sparse
 * matrix-vector multiplication for AMD Instinct MI355X (gfx950).
 *
 * Method: M. Heller, T. Oberhuber, "Adaptive Row-grouped CSR format for
 * storing of sparse matrices on GPU" (arXiv:1203.5737).
 *
 * Conventions (all entry points):
 *   - Every function returns int status: ARGCSR_OK (0) or a negative code.
 *     argcsr_last_error() returns a message for the calling thread's last
 *     failure.  No C++ exception crosses this interface.
 *   - "device" pointers are HIP device memory owned by the caller; the
 *     library never frees them.  "host" pointers are ordinary host memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Kernels are enqueued on it; calls documented as synchronous wait for
 *     their own work before returning.  A kernel fault surfaces as
 *     ARGCSR_EHIP at the next call that synchronises.
 *   - Indices are int32 (the group structure of Listing 1 uses int); a slot
 *     count above INT32_MAX is ARGCSR_EOVERFLOW.
 */
#ifndef ARGCSR_H
#define ARGCSR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define ARGCSR_OK          0
#define ARGCSR_EINVAL     (-1)  /* malformed argument or matrix            */
#define ARGCSR_EOVERFLOW  (-2)  /* slot count or offset exceeds int32      */
#define ARGCSR_ENOMEM     (-3)  /* device or host allocation failed        */
#define ARGCSR_EHIP       (-4)  /* a HIP runtime call failed               */
#define ARGCSR_EBUDGET    (-5)  /* request exceeds the device memory budget */
#define ARGCSR_EBUSY      (-6)  /* no free slot; retry later               */
#define ARGCSR_ENOTFOUND  (-7)  /* unknown handle, id or ticket            */
#define ARGCSR_EUNSUPPORTED (-8) /* valid, but not supported on the GPU    */
#define ARGCSR_ENOCONV    (-9)  /* CG stopped at its iteration limit       */
#define ARGCSR_PENDING     1    /* request status: not finished yet        */

/* ---- value storage types ------------------------------------------------ */
/* FP64 stores FP64 values and takes FP64 x, y.  The reduced types store
 * values rounded to nearest-even from FP64 and take FP32 x, y with FP32
 * accumulation. */
typedef enum {
  ARGCSR_F64 = 0,
  ARGCSR_F32 = 1,
  ARGCSR_BF16 = 2,
  ARGCSR_F16 = 3
} argcsr_dtype;

/* Storage formats, both held in the arrays of argcsr_matrix and computed by
 * the same SpMV kernels:
 *   ARGCSR_FORMAT_ARG  Adaptive Row-grouped CSR (Sec. 3): groups bounded by
 *                      block_dim rows and desired_chunk_size*block_dim
 *                      nonzeros, long rows spread over free chunks.
 *   ARGCSR_FORMAT_RG   Row-grouped CSR, the Sliced-ELLPACK-style storage the
 *                      paper starts from and compares with (Sec. 3, Sec. 5):
 *                      groups of block_dim consecutive rows, one chunk per
 *                      row, chunk size = the group's longest row (at least
 *                      1); desired_chunk_size plays no part.  The paper
 *                      finds it faster than ARG-CSR on finite-difference
 *                      matrices (Sec. 5). */
typedef enum {
  ARGCSR_FORMAT_ARG = 0,
  ARGCSR_FORMAT_RG = 1
} argcsr_format;

/* One group of consecutive rows (Sec. 3, Listing 1): rows
 * first_row .. first_row+size-1; its chunk_size*block_dim slots start at
 * `offset` in values/columns, element j of chunk k at offset + j*block_dim + k. */
typedef struct {
  int32_t first_row;
  int32_t size;
  int32_t offset;
  int32_t chunk_size;
} argcsr_group_info;

/* A converted matrix.  All arrays are caller-owned device memory:
 *   groups[n_groups]            group table (Listing 1)
 *   threads_mapping[n_rows]     per group, inclusive prefix sum of the number
 *                               of chunks of each row (Sec. 3, Listing 2)
 *   columns[n_slots]            column index, -1 marks an artificial zero
 *   values[n_slots]             value, element type given by dtype
 *   heavy_groups[n_heavy]       launch schedule (not part of the paper's
 *                               format): ascending indices of the groups whose
 *                               chunk_size exceeds heavy_chunk, i.e. whose
 *                               chunk loop is long enough to be split over all
 *                               waves of a workgroup and started first.  May
 *                               be NULL (then every group is processed by one
 *                               wave, in order).
 * block_dim (chunks per group, the paper's blockDim.x) must be 64, 128 or
 * 256 on the GPU; desired_chunk_size (the paper's desiredChunkSize) >= 1. */
typedef struct {
  int32_t n_rows;
  int32_t n_cols;
  int32_t block_dim;
  int32_t desired_chunk_size;
  int32_t dtype;               /* argcsr_dtype */
  int32_t n_groups;
  int64_t nnz;
  int64_t n_slots;
  argcsr_group_info* groups;
  int32_t* threads_mapping;
  int32_t* columns;
  void* values;
  int32_t n_heavy;             /* set by argcsr_plan / argcsr_convert */
  int32_t heavy_chunk;         /* set by argcsr_convert */
  int32_t* heavy_groups;
  int32_t format;              /* argcsr_format (0 = ARG-CSR) */
  /* conversion input, ARG-CSR only: a desiredChunkSize per region of
   * region_rows consecutive rows (host int32[ceil(n_rows/region_rows)],
   * each >= 1), the region of a group's first row setting the group's
   * nonzero limit; NULL = desired_chunk_size for every row.  Read by
   * argcsr_convert only. */
  int32_t region_rows;
  const int32_t* region_desired;
  /* Staging of x (optional; an extension of the format for banded
   * matrices, made by argcsr_stage_plan + argcsr_stage).  With local != NULL
   * argcsr_spmv reads each slot's 16-bit position in its group's staged
   * tiles of x instead of its column (columns may then be NULL for
   * argcsr_spmv; batches and the server use columns and ignore staging):
   *   tile_ptr[n_groups+1]        first tile of each group (exclusive scan)
   *   tile_start[n_stage_tiles]   first column of each tile
   *   tile_len[n_stage_tiles]     columns in each tile, 1..64
   *   local[n_slots]              64*q + (column - tile_start[tile_ptr[g]+q])
   *                               for the group's q-th tile, 0xFFFF for an
   *                               artificial zero
   * stage_gap is the window gap the tiles were made with, stage_max_tiles
   * the largest group's tile count (it sizes the SpMV's LDS), stage_lds
   * selects how the SpMV reads x: 1 = the group's tiles are loaded into LDS
   * first, 0 = x is gathered from memory at tile_start + position. */
  int32_t stage_gap;
  int32_t n_stage_tiles;
  int32_t stage_max_tiles;
  int32_t stage_lds;
  int32_t* tile_ptr;
  int32_t* tile_start;
  int32_t* tile_len;
  uint16_t* local;
} argcsr_matrix;

/* Message describing the calling thread's most recent failure ("" if none). */
const char* argcsr_last_error(void);

/* Library version, e.g. 100 for 0.1.0. */
int argcsr_version(void);

/*
 * argcsr_plan -- sizes of the ARG-CSR form of a CSR matrix (host only).
 * Conversion steps 1 and 2 of Sec. 3: rows are grouped in order, a row
 * joining the open group only while the group keeps at most
 * desired_chunk_size*block_dim nonzeros and at most block_dim rows (a longer
 * single row forms its own group); each group's chunk size is the smallest
 * c >= 1 with sum over its rows of max(1, ceil(L_r / c)) <= block_dim.
 *   n_rows            >= 0
 *   row_ptr_host      host int32[n_rows+1], CSR row offsets (Sec. 2)
 *   block_dim         1..1024 (the SpMV entry points accept 64, 128, 256)
 *   desired_chunk_size >= 1 (ignored for ARGCSR_FORMAT_RG)
 *   format            argcsr_format
 *   n_groups, n_slots out: group count and slot count (sum c_g*block_dim)
 *   n_heavy           out (may be NULL): length of the heavy_groups schedule
 * Errors: EINVAL (bad sizes, row_ptr not starting at 0 or decreasing),
 * EOVERFLOW (slot count > INT32_MAX).  Allocates only host memory.
 */
int argcsr_plan(int32_t n_rows, const int32_t* row_ptr_host, int32_t block_dim,
                int32_t desired_chunk_size, int32_t format, int32_t* n_groups,
                int64_t* n_slots, int32_t* n_heavy);

/*
 * argcsr_plan_regions -- argcsr_plan for ARG-CSR with a desiredChunkSize per
 * region of rows: rows [w*region_rows, (w+1)*region_rows) use
 * region_desired[w]; the group that opens at row s takes the value of the
 * region holding s for its nonzero limit (the Sec. 5 rule -- the more
 * regular the rows, the larger desiredChunkSize -- applied locally).
 *   region_rows     >= 1
 *   region_desired  host int32[ceil(n_rows / region_rows)], each >= 1
 *   other arguments as for argcsr_plan
 * Errors: as argcsr_plan; EINVAL for a bad region table.
 */
int argcsr_plan_regions(int32_t n_rows, const int32_t* row_ptr_host, int32_t block_dim,
                        int32_t region_rows, const int32_t* region_desired,
                        int32_t* n_groups, int64_t* n_slots, int32_t* n_heavy);

/*
 * argcsr_choose_region_desired -- fills region_desired (host
 * int32[ceil(n_rows / region_rows)]) by the Sec. 5 rule applied per region:
 * a region whose rows are regular (longest row <= 2 x its mean row length)
 * gets its longest row length, capped at max_desired, so that its groups
 * take block_dim rows of one chunk each; every other region gets 1.
 * Host only.  Errors: EINVAL.
 */
int argcsr_choose_region_desired(int32_t n_rows, const int32_t* row_ptr_host,
                                 int32_t region_rows, int32_t max_desired,
                                 int32_t* region_desired);

/*
 * argcsr_plan_device -- the sizes argcsr_plan computes (same grouping rule,
 * same results), from a row_ptr that lives only in device memory: steps 1-2
 * of Sec. 3 run as HIP kernels on `stream` (step 1 by binary lifting over
 * the next-group-start function of the rows; see argcsr_convert).
 *   row_ptr  device int32[n_rows+1]
 *   other arguments as for argcsr_plan (n_heavy may be NULL)
 * Synchronous (reads the counts back).  Uses stream-ordered device scratch
 * of about 4*(log2(n_rows)+2)*n_rows bytes.  Errors: EINVAL (bad sizes,
 * row_ptr not starting at 0 or decreasing), EOVERFLOW, ENOMEM, EHIP.
 */
int argcsr_plan_device(int32_t n_rows, const int32_t* row_ptr, int32_t block_dim,
                       int32_t desired_chunk_size, int32_t format, int32_t* n_groups,
                       int64_t* n_slots, int32_t* n_heavy, void* stream);

/* A device plan: steps 1-3 of Sec. 3 (groups with their chunk sizes, the
 * threads mapping) of one matrix, kept in device memory the library owns,
 * so that a caller with row_ptr on the device only sizes and converts the
 * matrix without grouping its rows twice. */
typedef struct argcsr_device_plan argcsr_device_plan;

/*
 * argcsr_plan_device_keep -- argcsr_plan_device that keeps its steps 1-3 in
 * *plan for argcsr_convert_planned (free it with argcsr_device_plan_destroy).
 * The plan holds 16 bytes per group and 4 per row of device memory.
 *   arguments as for argcsr_plan_device; plan out (NULL on error)
 * Synchronous.  Errors: as argcsr_plan_device.
 */
int argcsr_plan_device_keep(int32_t n_rows, const int32_t* row_ptr, int32_t block_dim,
                            int32_t desired_chunk_size, int32_t format, int32_t* n_groups,
                            int64_t* n_slots, int32_t* n_heavy, argcsr_device_plan** plan,
                            void* stream);

/*
 * argcsr_convert_planned -- argcsr_convert of the planned matrix: copies the
 * plan's groups and threads mapping into out's buffers and runs step 4
 * (offsets, launch schedule, fill) only.  The result equals argcsr_convert's
 * byte for byte.
 *   plan     from argcsr_plan_device_keep on the same row_ptr
 *   out      as for argcsr_convert; n_rows, block_dim, desired_chunk_size,
 *            format, n_groups and n_slots must be the plan's (EINVAL
 *            otherwise); no region table
 *   row_ptr, col, val, stream as for argcsr_convert (row_ptr_host is not used)
 * Synchronous.  Errors: as argcsr_convert.
 */
int argcsr_convert_planned(const argcsr_device_plan* plan, int32_t n_cols, const int32_t* row_ptr,
                           const int32_t* col, const double* val, argcsr_matrix* out,
                           void* stream);

/* Frees a device plan (NULL is a no-op), in the order of the stream it was
 * planned on.  No conversion may be running with it. */
int argcsr_device_plan_destroy(argcsr_device_plan* plan);

/*
 * argcsr_convert -- CSR -> ARG-CSR on the GPU (Sec. 3, all four steps).
 * Steps 2-4 (chunk size, threads mapping, offsets, fill) run as HIP kernels
 * on `stream`.  Step 1 (grouping) runs on the host from row_ptr_host when it
 * is given, and otherwise on the device from row_ptr alone: with
 * next(s) = the end of the group that opens at row s (a binary search on
 * row_ptr), the groups are the path 0 -> next(0) -> ... -> n_rows, found by
 * binary lifting (jump tables next^(2^k), then each group's start from the
 * bits of its index).  Either way the result equals, byte for byte, the
 * sequential conversion the paper describes.
 *   row_ptr_host  host int32[n_rows+1] (same content as row_ptr), or NULL
 *   row_ptr       device int32[n_rows+1]
 *   col           device int32[nnz], 0 <= col < n_cols
 *   val           device double[nnz]
 *   out           in: n_rows, n_cols, block_dim, desired_chunk_size, format,
 *                     region_rows and region_desired, dtype,
 *                     n_groups, n_slots and n_heavy as returned by
 *                     argcsr_plan (or argcsr_plan_device), and the device
 *                     buffers of those sizes
 *                     (heavy_groups may be NULL);
 *                 out: nnz, heavy_chunk, and the buffers filled.
 * Reduced dtypes round each value to nearest-even directly from FP64.
 * Synchronous: waits for its kernels (it reads back a validation flag).
 * Errors: EINVAL (malformed CSR incl. a column outside [0, n_cols), sizes
 * not matching argcsr_plan), EUNSUPPORTED (block_dim), EOVERFLOW, EHIP.
 * Column indices are checked while the fill moves them, so after an EINVAL
 * for a column the contents of out's buffers are unspecified.
 */
int argcsr_convert(int32_t n_rows, int32_t n_cols, const int32_t* row_ptr_host,
                   const int32_t* row_ptr, const int32_t* col, const double* val,
                   argcsr_matrix* out, void* stream);

/*
 * argcsr_convert_noalloc -- argcsr_convert for callers that cannot allocate
 * device memory (tight serving loops, harnesses that forbid hipMalloc): it
 * calls no hipMalloc, hipFree or other allocating routine.  Like
 * argcsr_convert it waits for its stream (it reads back the validation
 * flag), so it cannot itself be recorded into a HIP graph.  Its scratch (status words, scan partials and the
 * fill's long-row list) is a fixed 16 MiB array in device memory, one copy
 * per GPU, held by the library until the process ends; the caller still
 * passes every input and output, as for argcsr_convert, and the result is
 * byte for byte the same.
 *   arguments as for argcsr_convert, except that row_ptr_host is required
 *   (step 1 runs on the host; device grouping needs scratch proportional to
 *   n_rows*log2(n_rows))
 * A matrix whose scratch would exceed 16 MiB -- 24 + 16*ceil(n_groups/1024)
 * + 8*(n_slots/(4*block_dim) + 1) bytes, i.e. n_slots above about
 * 8*10^6*block_dim -- is rejected with EINVAL before anything is written.
 * The scratch keeps the last call's contents; each call clears what must
 * start at zero.  Calls are serialised by a process-wide lock and are
 * synchronous, so calls from several host threads never overlap on a GPU.
 * `stream` must belong to the current device.
 * Errors: as argcsr_convert.
 */
int argcsr_convert_noalloc(int32_t n_rows, int32_t n_cols, const int32_t* row_ptr_host,
                           const int32_t* row_ptr, const int32_t* col, const double* val,
                           argcsr_matrix* out, void* stream);

/*
 * argcsr_spmv -- y = A x for a converted matrix (Sec. 4, Listing 2
 * semantics: each chunk sums value*x[column] up to its first -1, each row
 * sums its chunks; y is overwritten, empty rows give 0).
 *   A   converted matrix (device buffers as filled by argcsr_convert)
 *   x   device FP64[n_cols] for ARGCSR_F64, FP32[n_cols] otherwise
 *   y   device FP64[n_rows] / FP32[n_rows]; must not alias x
 * x is gathered with 32-bit byte offsets: n_cols * sizeof(x element) must
 * not exceed 0xFFFFFFF0 (EUNSUPPORTED otherwise).
 * Asynchronous on `stream`.  Errors: EINVAL, EUNSUPPORTED, EHIP (launch).
 */
int argcsr_spmv(const argcsr_matrix* A, const void* x, void* y, void* stream);

/*
 * argcsr_csr_spmv -- plain CSR y = A x baseline on the same GPU (Sec. 2
 * definition): lanes_per_row consecutive lanes share a row and stride through
 * it, then combine their partial sums.
 *   row_ptr        device int32[n_rows+1]; col device int32[nnz] (valid
 *                  indices in [0, n_cols) are the caller's responsibility)
 *   val            device values of `dtype` (FP64, FP32, BF16 or FP16 bits)
 *   lanes_per_row  power of two in [1, 64], or 0: the power of two at or
 *                  above the mean row length (capped at 64)
 *   x, y           as for argcsr_spmv
 * Asynchronous on `stream`.  Errors: EINVAL, EHIP.
 */
int argcsr_csr_spmv(int32_t n_rows, int32_t n_cols, int64_t nnz,
                    const int32_t* row_ptr, const int32_t* col, const void* val,
                    int32_t dtype, int32_t lanes_per_row, const void* x, void* y,
                    void* stream);

/* Plain CSR with rows binned by length (still the Sec. 2 definition and
 * the CSR arrays alone, plus a row list): bin k = 0..6 holds the rows with
 * 2^(k-1) < L <= 2^k nonzeros (bin 0: L <= 1), bin 7 the rows longer than
 * 64; argcsr_csr_spmv_binned gives bin k < 7 2^k lanes per row (each such
 * row summed exactly as argcsr_csr_spmv with lanes_per_row = 2^k) and each
 * row of bin 7 a workgroup of 256 lanes, all in one launch. */
#define ARGCSR_CSR_BINS 8

/*
 * argcsr_csr_bin_rows -- the binning.
 *   row_ptr    device int32[n_rows+1] (non-decreasing; not checked)
 *   rows       device int32[n_rows], out: row indices bin by bin, ascending
 *              within a bin
 *   bin_start  host int32[ARGCSR_CSR_BINS+1], out: bin k's rows are
 *              rows[bin_start[k] .. bin_start[k+1])
 * Synchronous; uses stream-ordered scratch of 32 bytes per 256 rows.
 * Errors: EINVAL, EHIP.
 */
int argcsr_csr_bin_rows(int32_t n_rows, const int32_t* row_ptr, int32_t* rows,
                        int32_t* bin_start, void* stream);

/*
 * argcsr_csr_spmv_binned -- y = A x over the binned rows.
 *   rows, bin_start  as made by argcsr_csr_bin_rows for this row_ptr (rows
 *                    is trusted: every entry must be a row index, as the
 *                    column indices must be valid for argcsr_csr_spmv)
 *   other arguments as for argcsr_csr_spmv
 * Asynchronous on `stream`.  Errors: EINVAL, EHIP.
 */
int argcsr_csr_spmv_binned(int32_t n_rows, int32_t n_cols, int64_t nnz,
                           const int32_t* row_ptr, const int32_t* col, const void* val,
                           int32_t dtype, const int32_t* rows, const int32_t* bin_start,
                           const void* x, void* y, void* stream);

/* ---- staging of x for banded matrices --------------------------------- */

/*
 * Sec. 4 has each block stage in shared memory the data its threads reuse.
 * In a banded matrix (a stencil, a finite-difference operator) the rows of a
 * group name a few runs of consecutive columns, so the part of x a group
 * reads is small and can be staged the same way.  Per group, the distinct
 * columns its slots name are merged into windows (neighbouring columns stay
 * in one window when at most `gap` columns between them are absent) and
 * every window is cut into tiles of 64 consecutive columns (the last one
 * shorter); each slot then holds a 16-bit position in the group's tiles.
 * A group may need at most 64 tiles and its columns may span at most 2^18
 * columns (the staging marks them in a bitmap in LDS); a matrix with a
 * group beyond either limit is not staged (ARGCSR_EUNSUPPORTED).
 */

/*
 * argcsr_stage_plan -- the tile count of every group of a converted matrix.
 *   A          converted matrix (groups and columns on the device)
 *   gap        >= 0, absent columns bridged inside one window
 *   tile_ptr   device int32[n_groups+1], out: first tile of each group
 *   n_tiles    out: total tiles; max_group_tiles out (may be NULL): the
 *              largest group's count
 * Synchronous.  Errors: EINVAL, EUNSUPPORTED (a group beyond the limits),
 * ENOMEM, EHIP.
 */
int argcsr_stage_plan(const argcsr_matrix* A, int32_t gap, int32_t* tile_ptr,
                      int32_t* n_tiles, int32_t* max_group_tiles, void* stream);

/*
 * argcsr_stage -- fills tile_start, tile_len and local of A (device buffers
 * of n_stage_tiles, n_stage_tiles and n_slots entries) from A's groups and
 * columns, with A->stage_gap and the tile_ptr that argcsr_stage_plan made
 * for that gap.  Synchronous.  Errors: EINVAL (tile_ptr not from the plan of
 * this gap, NULL buffers), EUNSUPPORTED, ENOMEM, EHIP.
 */
int argcsr_stage(argcsr_matrix* A, void* stream);

/* ---- many matrices in one launch -------------------------------------- */

/* Opaque batch: device-side descriptors of several converted matrices and a
 * work list of their row groups, library-owned (free with
 * argcsr_batch_destroy). */
typedef struct argcsr_batch argcsr_batch;

/*
 * argcsr_batch_create -- prepares y_m = A_m x_m for m = 0..n_mats-1 as ONE
 * persistent kernel over a global queue of (matrix, group) work items
 * (groups with long chunk loops go to whole workgroups first, the others to
 * single waves in matrix and row order), and captures [queue reset, kernel] in a
 * hipGraph.  The same per-group computation as argcsr_spmv is used, so each
 * y_m is bitwise identical to argcsr_spmv on A_m alone.
 *   mats   host array of n_mats converted matrices, all of one dtype; block
 *          dims may differ (64, 128, 256)
 *   xs, ys host arrays of n_mats device pointers (x_m, y_m as for
 *          argcsr_spmv); the pointers are baked into the graph: later runs
 *          read the same x buffers and write the same y buffers
 * Synchronous (copies the group tables to the host to build the work list).
 * Errors: EINVAL (mixed dtypes, NULL pointers), EUNSUPPORTED, EHIP, ENOMEM.
 */
int argcsr_batch_create(int32_t n_mats, const argcsr_matrix* mats, const void* const* xs,
                        void* const* ys, argcsr_batch** out);

/* Runs the batch on `stream` by replaying its hipGraph (asynchronous). */
int argcsr_batch_graph_launch(argcsr_batch* b, void* stream);

/* Runs the batch on `stream` with ordinary kernel launches (asynchronous). */
int argcsr_batch_launch(argcsr_batch* b, void* stream);

/* Work-list sizes and persistent grid of a batch (any pointer may be NULL). */
int argcsr_batch_info(const argcsr_batch* b, int32_t* n_items, int32_t* n_heavy, int32_t* grid);

/* Waits for the batch's most recent launch (an event recorded on the stream
 * of that launch; not a device-wide synchronisation), then frees the batch
 * (NULL is a no-op).  A caller that launched the same batch on several
 * streams concurrently orders those streams itself before destroying it.
 * Errors: EHIP if the wait fails (the batch is freed either way). */
int argcsr_batch_destroy(argcsr_batch* b);

/* ---- parameter choice --------------------------------------------------- */

typedef struct {
  int32_t block_dim;           /* chosen T */
  int32_t desired_chunk_size;  /* chosen D (0 for ARGCSR_FORMAT_RG) */
  double model_us;             /* cost-model estimate of one SpMV */
  double measured_us;          /* median of timed SpMVs, each after a cache flush
                                  (cold, as in a batch); < 0 if not timed */
  int32_t from_cache;          /* 1 if the choice came from the process cache */
  int32_t n_candidates;        /* candidates planned */
  int32_t n_timed;             /* candidates converted and timed */
  int32_t format;              /* chosen argcsr_format */
  int32_t staged;              /* 1: faster with x staged in LDS (argcsr_stage_plan
                                  and argcsr_stage with gap 0, stage_lds = 1) */
} argcsr_tune_result;

/*
 * argcsr_autotune -- picks the storage format and its parameters for a
 * matrix.  The paper makes desiredChunkSize the key, matrix-dependent
 * parameter, block size 128 its best on its GPU, and advises trying more
 * than one format, row-grouped CSR winning on finite-difference matrices
 * (Sec. 5).  Every ARG-CSR pair in {64,128,256} x {1,2,4,8,16,32,64, the
 * longest and the mean row length when at most 64} and row-grouped CSR at
 * {64,128,256} (24 to 30 candidates) is sized with argcsr_plan and ranked
 * by a cost model fitted to cold timings on matrices of both regimes (the
 * longest of: padded bytes at the stream rate, the groups' latency chains
 * over the waves the chip keeps in flight, one group's chain), and
 * n_finalists of them are converted and timed on `stream` -- candidates
 * whose layout repeats a better-ranked one's are skipped, and the best of
 * each block size comes first -- each launch after a 512 MiB
 * read-modify-write that evicts the caches (the median of 7 decides).  An
 * ARG-CSR finalist whose groups fit the staging limits is timed again with
 * x staged in LDS, and `staged` reports whether that was faster.
 * The choice is cached for the process under a signature of the row-length
 * distribution.
 *   arguments as for argcsr_convert; dtype is the value storage type
 *   n_finalists  candidates to time (0: model only)
 * Synchronous; allocates and frees temporary device memory.
 * Errors: EINVAL, ENOMEM, EHIP, EOVERFLOW.
 */
int argcsr_autotune(int32_t n_rows, int32_t n_cols, const int32_t* row_ptr_host,
                    const int32_t* row_ptr, const int32_t* col, const double* val, int32_t dtype,
                    int32_t n_finalists, argcsr_tune_result* out, void* stream);

/*
 * argcsr_autotune_member -- the (T, D, format) for a matrix that will run as
 * one member of a batch (argcsr_batch_create), where the persistent kernel
 * overlaps the members and a member's cost is its share of the batch's
 * throughput rather than the time of its own launch.  The same candidates as
 * argcsr_autotune are ranked, without timing, by a model fitted to
 * whole-batch timings: the bytes of the member's slots and groups at a rate
 * that depends on the block size, plus a cost per group.  Host only (no
 * device memory or stream); model_us is the member's estimated share of the
 * batch time, measured_us is -1.  Cached like argcsr_autotune (separately).
 * Errors: EINVAL, EOVERFLOW.
 */
int argcsr_autotune_member(int32_t n_rows, const int32_t* row_ptr_host, int32_t dtype,
                           argcsr_tune_result* out);

/* Forgets all cached autotune choices. */
int argcsr_autotune_clear_cache(void);

/* ---- measurement probes ------------------------------------------------ */

/* Not part of the SpMV path: two kernels that measure the ceilings an SpMV
 * on this GPU is held against (the HBM roofline of an SpMV is its bytes over
 * the achievable bandwidth; its random x gathers have a rate of their own).
 * Each wave folds what it read into one value and writes it to
 * sink[wave], so `sink` is device double[ARGCSR_PROBE_SINK] (caller-owned;
 * its contents are meaningless).  Asynchronous on `stream`. */
#define ARGCSR_PROBE_SINK 16384

/* Reads bytes/16 16-byte words of the device buffer `buf` (16-byte aligned)
 * once, with non-temporal loads, each wave a contiguous kilobyte per load.
 * Errors: EINVAL, EHIP. */
int argcsr_probe_read(const void* buf, int64_t bytes, double* sink, void* stream);

/* Reads the device index stream idx[n] in tiles of 512 consecutive entries
 * per wave and gathers x[idx[i]] for every idx[i] >= 0 (all of a tile's
 * gathers in flight at once), x being device FP64 (x_bytes 8) or FP32
 * (x_bytes 4) of n_x elements; indices must lie in [-1, n_x).  Run on the
 * column array of a converted matrix, it isolates the cost of the SpMV's x
 * gathers.  Errors: EINVAL, EUNSUPPORTED (x above the 32-bit gather range),
 * EHIP. */
int argcsr_probe_gather(const int32_t* idx, int64_t n, const void* x, int32_t n_x,
                        int32_t x_bytes, double* sink, void* stream);

/* ---- serving ----------------------------------------------------------- */

/* A request server: converted matrices stay resident on one GPU inside a
 * device arena of budget_bytes; SpMV and CG-solve requests are batched
 * continuously (every scheduler step advances all active requests; new ones
 * join as slots and memory free up).  Library-owned; one scheduler thread per
 * server.  Results of a request do not depend on the other requests in
 * flight (no shared reductions). */
typedef struct argcsr_server argcsr_server;

typedef struct {
  int64_t budget_bytes;        /* device arena: resident matrices + request vectors */
  int32_t max_active;          /* requests advanced together, 1..512 */
  int32_t device;              /* HIP device ordinal */
  int32_t block_dim;           /* conversion T: 0 (= 64), 64, 128 or 256 */
  int32_t desired_chunk_size;  /* conversion D: 0 = mean row length in [1, 64] */
  double cg_tol;               /* CG stops when |b - A x| <= cg_tol |b| (FP64 A) */
  double cg_inner_tol;         /* residual reduction of one FP32-matrix inner cycle */
  int32_t cg_max_inner;        /* inner iterations per refinement cycle */
  int32_t cg_max_iter;         /* inner iterations per solve; then ARGCSR_ENOCONV */
  int64_t staging_bytes;       /* pinned host staging for request inputs and results,
                                  filled and drained by a copy thread so the scheduler
                                  never waits on host copies: 0 = 256 MiB, < 0 = none
                                  (then copies go straight to/from the caller's memory) */
  int32_t cg_inner_per_step;   /* inner CG iterations one scheduler step may run for a
                                  request, 0 (= 2) or 1..8; results do not depend on it */
} argcsr_server_config;

typedef enum {
  ARGCSR_REQ_ADMIT = 0,  /* make matrix_id resident from host CSR (n_rows, n_cols,
                            row_ptr, col, val); a no-op if it already is */
  ARGCSR_REQ_SPMV = 1,   /* out[n_rows] (float) = A in[n_cols] (float), FP32 values */
  ARGCSR_REQ_CG = 2,     /* out[n] (double) = x with A x = in (double b[n]), A SPD,
                            n = n_rows = n_cols */
  ARGCSR_REQ_EVICT = 3   /* drop matrix_id (EBUSY while running or queued
                            requests use it) */
} argcsr_request_kind;

typedef struct {
  int32_t kind;                /* argcsr_request_kind */
  int32_t n_rows, n_cols;      /* ADMIT: the matrix's size.  SPMV / CG: the
                                  lengths of out (n_rows) and in (n_cols) the
                                  caller provides; a request whose lengths are
                                  not the resident matrix's fails with EINVAL
                                  before any of its buffers is touched */
  int64_t matrix_id;
  const int32_t* row_ptr;      /* ADMIT, host, valid until the request completes */
  const int32_t* col;
  const double* val;
  const void* in;              /* SPMV / CG input, host, valid until completion */
  void* out;                   /* SPMV / CG output, host */
} argcsr_request;

typedef struct {
  int32_t status;              /* ARGCSR_PENDING, ARGCSR_OK or an error code */
  int32_t iterations;          /* CG: inner iterations (FP32 matrix); ADMIT: 1 if the
                                  matrix was converted now, 0 if already resident */
  int32_t refinements;         /* CG: outer residual evaluations (FP64 matrix) */
  int32_t reserved;
  double relres;               /* CG: final |b - A x| / |b| with the FP64 matrix */
  int64_t t_submit_ns, t_start_ns, t_done_ns;   /* steady clock */
} argcsr_result;

typedef struct {
  int64_t submitted, completed, failed;   /* SPMV + CG requests */
  int64_t admissions, evictions, steps;
  int64_t resident_matrices, resident_bytes, arena_bytes;
} argcsr_server_stats;

/* Creates a server and starts its scheduler thread.  Allocates the arena
 * (budget_bytes of device memory) up front.  Errors: EINVAL, ENOMEM, EHIP. */
int argcsr_server_create(const argcsr_server_config* cfg, argcsr_server** out);

/* Queues a request (thread-safe, non-blocking) and returns its ticket.
 * Requests are taken in submission order per matrix.  An ADMIT whose host
 * preparation is still running, an ADMIT that must convert while another
 * conversion runs (conversions run one at a time, on a stream of their own,
 * in submission order), and every later request of the same matrix wait,
 * while the requests behind them that name other, resident matrices start:
 * an ADMIT of a resident matrix then completes together with the SPMV/CG
 * request of that matrix submitted right behind it (or waits with it), so
 * the matrix stays resident until that request starts.  An EVICT waits for
 * every earlier request.  A matrix that a running request
 * uses is never evicted; queued requests do not pin their matrices (an ADMIT
 * evicts matrices no queued request names first).  An ADMIT that finds the
 * budget full even after evicting every matrix no running request uses
 * waits, and every request behind it with it, until running requests end
 * and free memory; it fails with EBUDGET only if the matrix can never fit
 * (it needs more than the whole budget, or nothing is running).  An
 * SPMV/CG request for a matrix that is not resident when it is started
 * fails with ENOTFOUND: submit the ADMIT (a no-op for a resident matrix)
 * right before the request that needs it; in-order processing then keeps
 * the matrix resident until the request starts. */
int argcsr_server_submit(argcsr_server* s, const argcsr_request* r, uint64_t* ticket);

/* Current result of a ticket (status ARGCSR_PENDING while in flight). */
int argcsr_server_poll(argcsr_server* s, uint64_t ticket, argcsr_result* res);

/* Blocks until the ticket finishes or timeout_ns passes (EBUSY). */
int argcsr_server_wait(argcsr_server* s, uint64_t ticket, int64_t timeout_ns, argcsr_result* res);

/* Forgets a finished ticket's result. */
int argcsr_server_release(argcsr_server* s, uint64_t ticket);

int argcsr_server_get_stats(argcsr_server* s, argcsr_server_stats* out);

/* Stops the scheduler (requests still queued fail with ENOTFOUND) and frees
 * the server. */
int argcsr_server_destroy(argcsr_server* s);

#ifdef __cplusplus
}
#endif
#endif /* ARGCSR_H */
