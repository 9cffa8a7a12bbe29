/*
 * oracle.h -- plain, slow, obviously-correct CPU reference for ARG-CSR SpMV.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path
 * (the HIP library under paper_1203_5737_amd/) never links, loads or calls it,
 * and this file shares no code with that library.
 *
 * Everything is computed in FP64 (the paper's precision, Sec. 5) with
 * sequential loops in the order the paper describes, compiled without
 * floating-point contraction (no FMA).
 *
 * Source: M. Heller, T. Oberhuber, "Adaptive Row-grouped CSR format for
 * storing of sparse matrices on GPU" (arXiv:1203.5737).
 *   - CSR storage: Sec. 2 (Fig. 1).
 *   - ARG-CSR layout, chunks, group structure: Sec. 3, Listing 1, Fig. 3.
 *   - Conversion CSR -> ARG-CSR (four steps): Sec. 3, the paragraph after
 *     Listing 1.
 *   - SpMV semantics, padding marker -1, threads mapping use: Sec. 4,
 *     Listing 2 and the paragraph after it.
 *
 * Readings of points the paper leaves open (the contract for the GPU path):
 *   R1  a row joins the open group only if the group's nonzero count stays
 *       <= desiredChunkSize*blockDim and its row count <= blockDim; a row
 *       longer than desiredChunkSize*blockDim forms a group of its own.
 *   R2  rows get t_r = max(1, ceil(L_r / c_g)) chunks, c_g being the final
 *       maximum chunk filling of the greedy distribution; left-over chunks
 *       stay free (this reproduces the Fig. 3 example: 4 chunks, 1 free).
 *   R3  threadsMapping holds the INCLUSIVE per-group prefix sum of t_r (the
 *       kernel of Listing 2 reads begin = tm[l-1], end = tm[l]).
 *   R4  chunk q of a row holds its elements [q*c, min((q+1)*c, L)).
 *   R5  every slot not holding an element (also in free chunks) is the
 *       artificial zero (value 0, column -1).
 *   R6  a group whose rows are all empty has chunkSize 1.
 *   R7  reduced-precision storage rounds the FP64 value to nearest, ties to
 *       even, directly from FP64.
 *   R8  all indices are int32; a slot count above INT32_MAX is an error.
 *   R10 a desiredChunkSize per region of consecutive rows (the Sec. 5 rule
 *       -- the more regular the rows, the larger desiredChunkSize -- applied
 *       locally): the group that opens at row s uses the value of the region
 *       holding s for its nonzero limit.
 *   R11 Staging of x (an extension; Sec. 4 stages the data each group
 *       reuses in shared memory, not x): the columns a group's slots name
 *       are merged into windows (holes of at most `gap` absent columns
 *       bridged) and cut into tiles of 64 columns; slots then hold 16-bit
 *       positions in the group's staged tiles (0xFFFF = artificial zero).
 *   R9  Row-grouped CSR (the Sliced-ELLPACK-style storage Sec. 3 builds on,
 *       compared against in Sec. 5): slices of blockDim consecutive rows,
 *       one chunk per row, chunk size = the slice's longest row, but at
 *       least 1 (as R6); stored in the same arrays as ARG-CSR, with
 *       threadsMapping[row] = its position in the slice + 1.
 */
#ifndef ARGCSR_ORACLE_H
#define ARGCSR_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Value storage types of the converted matrix. */
enum { ORA_F64 = 0, ORA_F32 = 1, ORA_BF16 = 2, ORA_F16 = 3 };

/* Return codes. */
enum { ORA_OK = 0, ORA_EINVAL = -1, ORA_EOVERFLOW = -2, ORA_ENOMEM = -3 };

/* CSR SpMV by definition (Sec. 2):
 * y_i = sum_{k=rp[i]}^{rp[i+1]-1} val[k] * x[col[k]], left to right, FP64.
 * n_threads > 1 splits the ROWS over OpenMP threads; each row's sum keeps
 * the same order, so y is identical. */
void ora_csr_spmv(int32_t n_rows, const int32_t* rp, const int32_t* col,
                  const double* val, const double* x, double* y,
                  int32_t n_threads);

/* CSR validity: rp[0]=0, rp non-decreasing, rp[n]=nnz, 0<=col<n_cols.
 * Returns ORA_OK or ORA_EINVAL. */
int ora_csr_check(int32_t n_rows, int32_t n_cols, int64_t nnz,
                  const int32_t* rp, const int32_t* col);

/* Conversion step 1 (grouping).  Writes first_row[g], size[g] for every
 * group (capacity n_rows) and returns the group count in *n_groups. */
int ora_group_rows(int32_t n_rows, const int32_t* rp, int32_t block_dim,
                   int32_t desired_chunk_size, int32_t* first_row,
                   int32_t* size, int32_t* n_groups);

/* Step 1 with desired[w] for rows [w*region_rows, (w+1)*region_rows)
 * (reading R10); desired has ceil(n_rows / region_rows) entries, all >= 1. */
int ora_group_rows_regions(int32_t n_rows, const int32_t* rp, int32_t block_dim,
                           int32_t region_rows, const int32_t* desired,
                           int32_t* first_row, int32_t* size, int32_t* n_groups);

/* Conversion step 2 for one group of `size` rows with lengths L[0..size):
 * the paper's greedy thread distribution.  Returns the chunk size c_g and
 * writes t[l] = max(1, ceil(L[l]/c_g)) (reading R2).  block_dim >= size. */
int32_t ora_chunk_size(int32_t size, const int64_t* L, int32_t block_dim,
                       int32_t* t);

/* Sizes of the converted matrix: group count and slot count S. */
int ora_argcsr_sizes(int32_t n_rows, const int32_t* rp, int32_t block_dim,
                     int32_t desired_chunk_size, int32_t* n_groups,
                     int64_t* n_slots);

/* ora_argcsr_sizes / ora_argcsr_convert with a desiredChunkSize per region
 * of rows (reading R10). */
int ora_argcsr_sizes_regions(int32_t n_rows, const int32_t* rp, int32_t block_dim,
                             int32_t region_rows, const int32_t* desired,
                             int32_t* n_groups, int64_t* n_slots);
int ora_argcsr_convert_regions(int32_t n_rows, const int32_t* rp, const int32_t* col,
                               const double* val, int32_t block_dim, int32_t region_rows,
                               const int32_t* desired, int32_t dtype, int32_t* groups,
                               int32_t* tm, int32_t* columns, void* values);

/* Full conversion CSR -> ARG-CSR (steps 1-4).  Output buffers are sized by
 * ora_argcsr_sizes: groups[4*G] = {firstRow,size,offset,chunkSize} per group
 * (Listing 1), tm[n_rows], columns[S], values[S] elements of `dtype`
 * (8, 4, 2, 2 bytes; bf16/f16 stored as raw uint16 bits). */
int ora_argcsr_convert(int32_t n_rows, const int32_t* rp, const int32_t* col,
                       const double* val, int32_t block_dim,
                       int32_t desired_chunk_size, int32_t dtype,
                       int32_t* groups, int32_t* tm, int32_t* columns,
                       void* values);

/* Row-grouped CSR (reading R9) in the same arrays: sizes, and the full
 * conversion with the buffer conventions of ora_argcsr_convert. */
int ora_rgcsr_sizes(int32_t n_rows, const int32_t* rp, int32_t block_dim,
                    int32_t* n_groups, int64_t* n_slots);
int ora_rgcsr_convert(int32_t n_rows, const int32_t* rp, const int32_t* col,
                      const double* val, int32_t block_dim, int32_t dtype,
                      int32_t* groups, int32_t* tm, int32_t* columns,
                      void* values);

/* Staging of x for banded matrices (reading R11): per group, the distinct
 * columns of its slots merged into windows (at most `gap` absent columns
 * between neighbours inside a window), each window cut into tiles of 64
 * columns; local[slot] = 64*q + (c - tile_start) for the group's q-th tile
 * holding column c, 0xFFFF for an artificial zero.  tile_ptr has
 * n_groups+1 entries.  Returns the tile count, ORA_EINVAL if a group needs
 * more than max_tiles (<= 1023) tiles, ORA_EOVERFLOW if tile_cap is too
 * small; with tile_start == NULL only tile_ptr is filled (sizing). */
int64_t ora_stage(int32_t n_groups, const int32_t* groups, const int32_t* columns,
                  int32_t block_dim, int32_t gap, int32_t max_tiles, int32_t* tile_ptr,
                  int32_t* tile_start, int32_t* tile_len, int64_t tile_cap,
                  uint16_t* local);

/* Column index of every slot from its local index (-1 for 0xFFFF). */
void ora_unstage(int32_t n_groups, const int32_t* groups, int32_t block_dim,
                 const int32_t* tile_ptr, const int32_t* tile_start,
                 const uint16_t* local, int32_t* columns_out);

/* SpMV read from the ARG-CSR storage by the format's definition (Sec. 3,
 * Sec. 4), FP64: each row's elements are found through the threads mapping
 * (its chunks) and the chunk layout (slots offset + j*blockDim + k up to the
 * first column -1), and summed left to right in the row's element order.
 * With a correct layout this is bitwise the CSR definition.  values are FP64. */
void ora_argcsr_spmv(int32_t n_groups, const int32_t* groups, const int32_t* tm,
                     const int32_t* columns, const double* values,
                     int32_t block_dim, const double* x, double* y);

/* Inverse ARG-CSR -> CSR (values FP64).  rp_out[n_rows+1], col_out and
 * val_out of capacity nnz.  Returns the emitted nonzero count, or <0. */
int64_t ora_argcsr_to_csr(int32_t n_rows, int32_t n_groups,
                          const int32_t* groups, const int32_t* tm,
                          const int32_t* columns, const double* values,
                          int32_t block_dim, int32_t* rp_out,
                          int32_t* col_out, double* val_out);

/* Round-to-nearest-even of an FP64 value into bfloat16 / binary16 bits,
 * computed from the definition (scaling by the format's quantum). */
uint16_t ora_round_bf16(double v);
uint16_t ora_round_f16(double v);
/* Exact value of bfloat16 / binary16 bits as FP64. */
double ora_bf16_value(uint16_t b);
double ora_f16_value(uint16_t h);

/* Element-wise: FP64 -> storage representation of `dtype` (as stored by
 * ora_argcsr_convert), and storage -> exact FP64 value. */
void ora_round_array(int64_t n, const double* v, int32_t dtype, void* out);
void ora_decode_array(int64_t n, const void* stored, int32_t dtype, double* out);

/* Textbook conjugate gradients in FP64 from x0 = 0 on a CSR matrix;
 * stops when the TRUE residual ||b - A x||_2 <= tol * ||b||_2 or after
 * max_iter iterations.  Returns the iteration count; *relres receives the
 * final true relative residual. */
int32_t ora_cg(int32_t n, const int32_t* rp, const int32_t* col,
               const double* val, const double* b, double* x, double tol,
               int32_t max_iter, double* relres);

#ifdef __cplusplus
}
#endif
#endif
