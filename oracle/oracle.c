/*
 * oracle.c -- plain CPU reference for ARG-CSR SpMV and its conversion.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Written from the paper's
 * description; every function names the passage it follows.  Compile with
 * floating-point contraction off so that every multiply and add rounds
 * separately.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* CSR (Sec. 2, Fig. 1): values row by row, their columns, row offsets.       */
/* ------------------------------------------------------------------------ */

static double csr_row_dot(const int32_t* rp, const int32_t* col,
                          const double* val, const double* x, int32_t i)
{
    double sum = 0.0;
    for (int64_t k = rp[i]; k < rp[i + 1]; k++)
        sum = sum + val[k] * x[col[k]];
    return sum;
}

void ora_csr_spmv(int32_t n_rows, const int32_t* rp, const int32_t* col,
                  const double* val, const double* x, double* y,
                  int32_t n_threads)
{
#ifdef _OPENMP
    if (n_threads > 1) {
#pragma omp parallel for schedule(static) num_threads(n_threads)
        for (int32_t i = 0; i < n_rows; i++)
            y[i] = csr_row_dot(rp, col, val, x, i);
        return;
    }
#else
    (void)n_threads;
#endif
    for (int32_t i = 0; i < n_rows; i++)
        y[i] = csr_row_dot(rp, col, val, x, i);
}

int ora_csr_check(int32_t n_rows, int32_t n_cols, int64_t nnz,
                  const int32_t* rp, const int32_t* col)
{
    if (n_rows < 0 || n_cols < 0 || nnz < 0) return ORA_EINVAL;
    if (rp[0] != 0 || (int64_t)rp[n_rows] != nnz) return ORA_EINVAL;
    for (int32_t i = 0; i < n_rows; i++)
        if (rp[i + 1] < rp[i]) return ORA_EINVAL;
    /* Column -1 marks artificial zeros in ARG-CSR (Sec. 4), so a negative
     * column can never be a real entry. */
    for (int64_t k = 0; k < nnz; k++)
        if (col[k] < 0 || col[k] >= n_cols) return ORA_EINVAL;
    return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* Conversion, step 1 (Sec. 3): read rows in order, counting nonzeros of the  */
/* open group; close it when it would exceed desiredChunkSize*blockDim        */
/* nonzeros or blockDim rows (reading R1: the row that would overflow opens   */
/* the next group).                                                           */
/* ------------------------------------------------------------------------ */

/* Step 1 with a desiredChunkSize per region of region_rows consecutive rows
 * (reading R10): the group that opens at row s may hold at most
 * desired[s / region_rows] * blockDim nonzeros.  One region covering every
 * row is the paper's rule with a single desiredChunkSize. */
static int group_rows_regions(int32_t n_rows, const int32_t* rp, int32_t block_dim,
                              int32_t region_rows, const int32_t* desired,
                              int32_t* first_row, int32_t* size, int32_t* n_groups)
{
    if (n_rows < 0 || block_dim < 1 || region_rows < 1) return ORA_EINVAL;
    for (int64_t w = 0; w * region_rows < n_rows; w++)
        if (desired[w] < 1) return ORA_EINVAL;
    int64_t limit = 0;
    int32_t g = 0;
    int32_t open_first = 0, open_size = 0;
    int64_t open_count = 0;
    for (int32_t r = 0; r < n_rows; r++) {
        const int64_t L = (int64_t)rp[r + 1] - (int64_t)rp[r];
        if (open_size > 0 &&
            (open_size + 1 > block_dim || open_count + L > limit)) {
            first_row[g] = open_first;
            size[g] = open_size;
            g++;
            open_first = r;
            open_size = 0;
            open_count = 0;
        }
        if (open_size == 0)                  /* row r opens a group */
            limit = (int64_t)desired[r / region_rows] * (int64_t)block_dim;
        open_size += 1;
        open_count += L;
    }
    if (open_size > 0) {
        first_row[g] = open_first;
        size[g] = open_size;
        g++;
    }
    *n_groups = g;
    return ORA_OK;
}

int ora_group_rows(int32_t n_rows, const int32_t* rp, int32_t block_dim,
                   int32_t desired_chunk_size, int32_t* first_row,
                   int32_t* size, int32_t* n_groups)
{
    return group_rows_regions(n_rows, rp, block_dim, INT32_MAX, &desired_chunk_size,
                              first_row, size, n_groups);
}

int ora_group_rows_regions(int32_t n_rows, const int32_t* rp, int32_t block_dim,
                           int32_t region_rows, const int32_t* desired,
                           int32_t* first_row, int32_t* size, int32_t* n_groups)
{
    return group_rows_regions(n_rows, rp, block_dim, region_rows, desired, first_row,
                              size, n_groups);
}

/* ------------------------------------------------------------------------ */
/* Conversion, step 2 (Sec. 3; example of Fig. 3): map one thread to every   */
/* row, then hand each remaining thread to the row whose chunk filling        */
/* ceil(L / threads) is greatest.  The chunk size is the final greatest       */
/* filling (at least 1, reading R6); each row then keeps                      */
/* max(1, ceil(L / chunkSize)) chunks (reading R2).                           */
/* ------------------------------------------------------------------------ */

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

int32_t ora_chunk_size(int32_t size, const int64_t* L, int32_t block_dim,
                       int32_t* t)
{
    for (int32_t l = 0; l < size; l++) t[l] = 1;
    for (int32_t left = block_dim - size; left > 0; left--) {
        int32_t best = 0;
        int64_t best_fill = -1;
        for (int32_t l = 0; l < size; l++) {
            const int64_t fill = ceil_div(L[l], t[l]);
            if (fill > best_fill) { best_fill = fill; best = l; }
        }
        t[best] += 1;
    }
    int64_t chunk = 1;
    for (int32_t l = 0; l < size; l++) {
        const int64_t fill = ceil_div(L[l], t[l]);
        if (fill > chunk) chunk = fill;
    }
    for (int32_t l = 0; l < size; l++) {
        const int64_t need = ceil_div(L[l], chunk);
        t[l] = (int32_t)(need > 1 ? need : 1);
    }
    return (int32_t)chunk;
}

int ora_argcsr_sizes(int32_t n_rows, const int32_t* rp, int32_t block_dim,
                     int32_t desired_chunk_size, int32_t* n_groups,
                     int64_t* n_slots)
{
    return ora_argcsr_sizes_regions(n_rows, rp, block_dim, INT32_MAX, &desired_chunk_size,
                                    n_groups, n_slots);
}

int ora_argcsr_sizes_regions(int32_t n_rows, const int32_t* rp, int32_t block_dim,
                             int32_t region_rows, const int32_t* desired,
                             int32_t* n_groups, int64_t* n_slots)
{
    int32_t* first = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_rows + 1));
    int32_t* size = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_rows + 1));
    int64_t* L = (int64_t*)malloc(sizeof(int64_t) * (size_t)(block_dim + 1));
    int32_t* t = (int32_t*)malloc(sizeof(int32_t) * (size_t)(block_dim + 1));
    int rc = group_rows_regions(n_rows, rp, block_dim, region_rows, desired, first,
                                size, n_groups);
    int64_t S = 0;
    for (int32_t g = 0; rc == ORA_OK && g < *n_groups; g++) {
        for (int32_t l = 0; l < size[g]; l++)
            L[l] = (int64_t)rp[first[g] + l + 1] - rp[first[g] + l];
        const int32_t c = ora_chunk_size(size[g], L, block_dim, t);
        S += (int64_t)c * block_dim;
    }
    if (rc == ORA_OK && S > INT32_MAX) rc = ORA_EOVERFLOW;
    *n_slots = S;
    free(first); free(size); free(L); free(t);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Reduced-precision storage (reading R7): round to nearest, ties to even,   */
/* written from the definition.  A positive value a is a multiple of the     */
/* target's quantum q (the spacing of representable numbers in a's binade,    */
/* or the subnormal spacing below the normal range); a/q is rounded to an     */
/* integer with ties going to the even integer.                               */
/* ------------------------------------------------------------------------ */

static uint16_t round_small_float(double v, int exp_bits, int man_bits)
{
    const int bias = (1 << (exp_bits - 1)) - 1;
    const uint16_t sign = signbit(v) ? (uint16_t)(1u << (exp_bits + man_bits)) : 0;
    const uint16_t inf_bits = (uint16_t)(((1u << exp_bits) - 1u) << man_bits);
    if (isnan(v)) return (uint16_t)(sign | inf_bits | (1u << (man_bits - 1)));
    const double a = fabs(v);
    if (isinf(a)) return (uint16_t)(sign | inf_bits);
    if (a == 0.0) return sign;
    int e2;
    (void)frexp(a, &e2);              /* a = m * 2^e2, m in [0.5, 1)   */
    int ue = e2 - 1;                  /* a in [2^ue, 2^(ue+1))          */
    const int emin = 1 - bias;        /* smallest normal exponent       */
    const int qexp = (ue < emin ? emin : ue) - man_bits;
    const double n = ldexp(a, -qexp); /* exact: scaling by 2^-qexp      */
    double k = floor(n);
    const double frac = n - k;        /* exact                          */
    if (frac > 0.5 || (frac == 0.5 && fmod(k, 2.0) != 0.0)) k += 1.0;
    uint32_t bits;
    if (ue < emin) {
        bits = (uint32_t)k;           /* subnormal (k = 2^man -> min normal) */
    } else {
        bits = ((uint32_t)(ue + bias) << man_bits) +
               ((uint32_t)k - (1u << man_bits));
    }
    if (bits >= inf_bits) bits = inf_bits;   /* overflow to infinity */
    return (uint16_t)(sign | bits);
}

uint16_t ora_round_bf16(double v) { return round_small_float(v, 8, 7); }
uint16_t ora_round_f16(double v) { return round_small_float(v, 5, 10); }

static double small_float_value(uint16_t b, int exp_bits, int man_bits)
{
    const int bias = (1 << (exp_bits - 1)) - 1;
    const int s = (b >> (exp_bits + man_bits)) & 1;
    const int e = (b >> man_bits) & ((1 << exp_bits) - 1);
    const int m = b & ((1 << man_bits) - 1);
    double v;
    if (e == (1 << exp_bits) - 1) v = m ? NAN : INFINITY;
    else if (e == 0) v = ldexp((double)m, 1 - bias - man_bits);
    else v = ldexp((double)(m + (1 << man_bits)), e - bias - man_bits);
    return s ? -v : v;
}

double ora_bf16_value(uint16_t b) { return small_float_value(b, 8, 7); }
double ora_f16_value(uint16_t h) { return small_float_value(h, 5, 10); }

void ora_round_array(int64_t n, const double* v, int32_t dtype, void* out)
{
    for (int64_t i = 0; i < n; i++) {
        switch (dtype) {
        case ORA_F64: ((double*)out)[i] = v[i]; break;
        case ORA_F32: ((float*)out)[i] = (float)v[i]; break;
        case ORA_BF16: ((uint16_t*)out)[i] = ora_round_bf16(v[i]); break;
        default: ((uint16_t*)out)[i] = ora_round_f16(v[i]); break;
        }
    }
}

void ora_decode_array(int64_t n, const void* stored, int32_t dtype, double* out)
{
    for (int64_t i = 0; i < n; i++) {
        switch (dtype) {
        case ORA_F64: out[i] = ((const double*)stored)[i]; break;
        case ORA_F32: out[i] = (double)((const float*)stored)[i]; break;
        case ORA_BF16: out[i] = ora_bf16_value(((const uint16_t*)stored)[i]); break;
        default: out[i] = ora_f16_value(((const uint16_t*)stored)[i]); break;
        }
    }
}

static void store_value(void* values, int32_t dtype, int64_t slot, double v)
{
    switch (dtype) {
    case ORA_F64: ((double*)values)[slot] = v; break;
    case ORA_F32: ((float*)values)[slot] = (float)v; break;
    case ORA_BF16: ((uint16_t*)values)[slot] = ora_round_bf16(v); break;
    default: ((uint16_t*)values)[slot] = ora_round_f16(v); break;
    }
}

/* ------------------------------------------------------------------------ */
/* Full conversion (Sec. 3).                                                  */
/*   step 1: groups (ora_group_rows);                                         */
/*   step 2: chunk size per group and chunks per row (ora_chunk_size);        */
/*   step 3: per-group prefix sum of chunks per row -> threadsMapping         */
/*           (reading R3: inclusive);                                         */
/*   step 4: each group owns chunkSize*blockDim slots from `offset`; chunks   */
/*           are stored like the rows of a column-major ELLPACK slice, i.e.   */
/*           element j of chunk k sits at offset + j*blockDim + k (Sec. 3,    */
/*           Listing 1 text); copy the CSR data chunk by chunk (reading R4),  */
/*           every other slot is the artificial zero (0, -1) (reading R5).    */
/* ------------------------------------------------------------------------ */

int ora_argcsr_convert(int32_t n_rows, const int32_t* rp, const int32_t* col,
                       const double* val, int32_t block_dim,
                       int32_t desired_chunk_size, int32_t dtype,
                       int32_t* groups, int32_t* tm, int32_t* columns,
                       void* values)
{
    return ora_argcsr_convert_regions(n_rows, rp, col, val, block_dim, INT32_MAX,
                                      &desired_chunk_size, dtype, groups, tm, columns,
                                      values);
}

int ora_argcsr_convert_regions(int32_t n_rows, const int32_t* rp, const int32_t* col,
                               const double* val, int32_t block_dim, int32_t region_rows,
                               const int32_t* desired, int32_t dtype, int32_t* groups,
                               int32_t* tm, int32_t* columns, void* values)
{
    if (dtype < ORA_F64 || dtype > ORA_F16) return ORA_EINVAL;
    int32_t* first = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_rows + 1));
    int32_t* size = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_rows + 1));
    int64_t* L = (int64_t*)malloc(sizeof(int64_t) * (size_t)(block_dim + 1));
    int32_t* t = (int32_t*)malloc(sizeof(int32_t) * (size_t)(block_dim + 1));
    int32_t G = 0;
    int rc = group_rows_regions(n_rows, rp, block_dim, region_rows, desired, first,
                                size, &G);
    int64_t offset = 0;
    for (int32_t g = 0; rc == ORA_OK && g < G; g++) {
        /* step 2 */
        for (int32_t l = 0; l < size[g]; l++)
            L[l] = (int64_t)rp[first[g] + l + 1] - rp[first[g] + l];
        const int32_t c = ora_chunk_size(size[g], L, block_dim, t);
        if (offset + (int64_t)c * block_dim > INT32_MAX) { rc = ORA_EOVERFLOW; break; }
        groups[4 * g + 0] = first[g];
        groups[4 * g + 1] = size[g];
        groups[4 * g + 2] = (int32_t)offset;
        groups[4 * g + 3] = c;
        /* step 3 */
        int32_t running = 0;
        for (int32_t l = 0; l < size[g]; l++) {
            running += t[l];
            tm[first[g] + l] = running;
        }
        /* step 4: artificial zeros first, then the chunks of every row */
        for (int64_t s = 0; s < (int64_t)c * block_dim; s++) {
            columns[offset + s] = -1;
            store_value(values, dtype, offset + s, 0.0);
        }
        for (int32_t l = 0; l < size[g]; l++) {
            const int32_t r = first[g] + l;
            const int32_t first_chunk = (l == 0) ? 0 : tm[r - 1];
            for (int32_t q = 0; q < t[l]; q++) {          /* chunk q of row r */
                for (int32_t j = 0; j < c; j++) {          /* its j-th element */
                    const int64_t e = (int64_t)q * c + j;
                    if (e >= L[l]) break;
                    const int64_t slot = offset + (int64_t)j * block_dim +
                                         first_chunk + q;
                    columns[slot] = col[rp[r] + e];
                    store_value(values, dtype, slot, val[rp[r] + e]);
                }
            }
        }
        offset += (int64_t)c * block_dim;
    }
    free(first); free(size); free(L); free(t);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Row-grouped CSR (reading R9): slice g holds rows g*T .. g*T+T-1; its      */
/* width w is its longest row (at least 1); element e of the row in slice    */
/* position l is stored at offset + e*T + l, everything else is padding.     */
/* ------------------------------------------------------------------------ */

int ora_rgcsr_sizes(int32_t n_rows, const int32_t* rp, int32_t block_dim,
                    int32_t* n_groups, int64_t* n_slots)
{
    if (n_rows < 0 || block_dim < 1) return ORA_EINVAL;
    int64_t S = 0;
    int32_t G = 0;
    for (int64_t first = 0; first < n_rows; first += block_dim, G++) {
        int64_t w = 1;
        for (int64_t r = first; r < n_rows && r < first + block_dim; r++)
            if ((int64_t)rp[r + 1] - rp[r] > w) w = (int64_t)rp[r + 1] - rp[r];
        S += w * block_dim;
    }
    *n_groups = G;
    *n_slots = S;
    return S > INT32_MAX ? ORA_EOVERFLOW : ORA_OK;
}

int ora_rgcsr_convert(int32_t n_rows, const int32_t* rp, const int32_t* col,
                      const double* val, int32_t block_dim, int32_t dtype,
                      int32_t* groups, int32_t* tm, int32_t* columns,
                      void* values)
{
    if (dtype < ORA_F64 || dtype > ORA_F16 || block_dim < 1) return ORA_EINVAL;
    int64_t offset = 0;
    int32_t g = 0;
    for (int64_t first = 0; first < n_rows; first += block_dim, g++) {
        const int64_t rows = (n_rows - first < block_dim) ? n_rows - first : block_dim;
        int64_t w = 1;
        for (int64_t l = 0; l < rows; l++)
            if ((int64_t)rp[first + l + 1] - rp[first + l] > w)
                w = (int64_t)rp[first + l + 1] - rp[first + l];
        if (offset + w * block_dim > INT32_MAX) return ORA_EOVERFLOW;
        groups[4 * g + 0] = (int32_t)first;
        groups[4 * g + 1] = (int32_t)rows;
        groups[4 * g + 2] = (int32_t)offset;
        groups[4 * g + 3] = (int32_t)w;
        for (int64_t s = 0; s < w * block_dim; s++) {
            columns[offset + s] = -1;
            store_value(values, dtype, offset + s, 0.0);
        }
        for (int64_t l = 0; l < rows; l++) {
            const int64_t r = first + l;
            tm[r] = (int32_t)(l + 1);
            for (int64_t e = 0; e < (int64_t)rp[r + 1] - rp[r]; e++) {
                columns[offset + e * block_dim + l] = col[rp[r] + e];
                store_value(values, dtype, offset + e * block_dim + l, val[rp[r] + e]);
            }
        }
        offset += w * block_dim;
    }
    return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* SpMV read from the ARG-CSR storage by the format's definition (Sec. 3,    */
/* Sec. 4): the rows of group g are firstRow .. firstRow+size-1; row r owns  */
/* the consecutive chunks b_r .. tm[r]-1 of its group (b_r = tm[r-1] inside  */
/* the group, 0 for its first row); the elements of a chunk k are the slots  */
/* offset + j*blockDim + k, j = 0, 1, ..., up to the first artificial zero   */
/* (column -1) or chunkSize slots; a row's elements are its chunks' elements */
/* in chunk order.  y_r is the sum of value*x[column] over those elements,   */
/* added left to right (the element order of the row, as in the CSR         */
/* definition), and overwrites y_r; a row without elements gets 0.          */
/* ------------------------------------------------------------------------ */

void ora_argcsr_spmv(int32_t n_groups, const int32_t* groups, const int32_t* tm,
                     const int32_t* columns, const double* values,
                     int32_t block_dim, const double* x, double* y)
{
    for (int32_t g = 0; g < n_groups; g++) {
        const int32_t first = groups[4 * g + 0], size = groups[4 * g + 1];
        const int32_t offset = groups[4 * g + 2], chunk = groups[4 * g + 3];
        for (int32_t r = first; r < first + size; r++) {
            const int32_t b = (r == first) ? 0 : tm[r - 1];
            double sum = 0.0;
            for (int32_t k = b; k < tm[r]; k++) {
                for (int32_t j = 0; j < chunk; j++) {
                    const int64_t s = (int64_t)offset + (int64_t)j * block_dim + k;
                    if (columns[s] == -1) break;
                    sum = sum + values[s] * x[columns[s]];
                }
            }
            y[r] = sum;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Staging of x for banded matrices (a storage extension, reading R11): the   */
/* paper's kernel fetches the data each group reuses into fast shared memory  */
/* (Sec. 4); here the part of x a group reads is listed so that it can be     */
/* staged the same way.  For group g: u_0 < u_1 < ... are the distinct       */
/* column indices its slots hold (artificial zeros excluded).  A window is a  */
/* maximal run of them in which two neighbours have at most `gap` absent      */
/* columns between them (u_{i+1} - u_i - 1 <= gap); window [s, e] covers      */
/* every column s..e.  Each window is cut into tiles of 64 consecutive        */
/* columns from its start (the last tile may be shorter).  The tiles of g,    */
/* in column order, are tile_start/tile_len[tile_ptr[g] .. tile_ptr[g+1]).    */
/* A slot holding column c gets the local index 64*q + (c - tile_start) for  */
/* the q-th tile of its group that contains c; an artificial zero gets        */
/* 0xFFFF.  Returns the number of tiles, or ORA_EINVAL when a group needs     */
/* more than max_tiles (<= 1023) tiles, or ORA_EOVERFLOW when tile_cap is     */
/* too small.  With tile_start == NULL only tile_ptr is filled.               */
/* ------------------------------------------------------------------------ */

static int cmp_i32(const void* a, const void* b)
{
    const int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

int64_t ora_stage(int32_t n_groups, const int32_t* groups, const int32_t* columns,
                  int32_t block_dim, int32_t gap, int32_t max_tiles, int32_t* tile_ptr,
                  int32_t* tile_start, int32_t* tile_len, int64_t tile_cap,
                  uint16_t* local)
{
    if (gap < 0 || max_tiles < 1 || max_tiles > 1023 || block_dim < 1) return ORA_EINVAL;
    int64_t total = 0;
    int64_t biggest = 1;
    for (int32_t g = 0; g < n_groups; g++) {
        const int64_t slots = (int64_t)groups[4 * g + 3] * block_dim;
        if (slots > biggest) biggest = slots;
    }
    int32_t* u = (int32_t*)malloc(sizeof(int32_t) * (size_t)biggest);
    int32_t* ts = (int32_t*)malloc(sizeof(int32_t) * (size_t)(max_tiles + 1));
    int32_t* tl = (int32_t*)malloc(sizeof(int32_t) * (size_t)(max_tiles + 1));
    if (!u || !ts || !tl) { free(u); free(ts); free(tl); return ORA_ENOMEM; }
    tile_ptr[0] = 0;
    int64_t rc = 0;
    for (int32_t g = 0; g < n_groups && rc == 0; g++) {
        const int64_t offset = groups[4 * g + 2];
        const int64_t slots = (int64_t)groups[4 * g + 3] * block_dim;
        /* the distinct columns of the group, ascending */
        int64_t m = 0;
        for (int64_t s = 0; s < slots; s++)
            if (columns[offset + s] != -1) u[m++] = columns[offset + s];
        qsort(u, (size_t)m, sizeof(int32_t), cmp_i32);
        int64_t distinct = 0;
        for (int64_t i = 0; i < m; i++)
            if (distinct == 0 || u[i] != u[distinct - 1]) u[distinct++] = u[i];
        /* windows, then tiles of 64 columns */
        int32_t nt = 0;
        int64_t i = 0;
        while (i < distinct && rc == 0) {
            const int64_t start = u[i];
            int64_t last = u[i];
            while (i + 1 < distinct && (int64_t)u[i + 1] - last - 1 <= gap) last = u[++i];
            i++;
            for (int64_t t = start; t <= last; t += 64) {
                if (nt == max_tiles) { rc = ORA_EINVAL; break; }
                ts[nt] = (int32_t)t;
                tl[nt] = (int32_t)(last - t + 1 < 64 ? last - t + 1 : 64);
                nt++;
            }
        }
        if (rc) break;
        if (tile_start) {
            if (total + nt > tile_cap) { rc = ORA_EOVERFLOW; break; }
            for (int32_t q = 0; q < nt; q++) {
                tile_start[total + q] = ts[q];
                tile_len[total + q] = tl[q];
            }
            /* local index of every slot: the tile holding its column */
            for (int64_t s = 0; s < slots; s++) {
                const int32_t c = columns[offset + s];
                uint16_t v = 0xFFFF;
                if (c != -1) {
                    for (int32_t q = 0; q < nt; q++)
                        if (c >= ts[q] && c < ts[q] + tl[q]) { v = (uint16_t)(64 * q + (c - ts[q])); break; }
                }
                local[offset + s] = v;
            }
        }
        total += nt;
        tile_ptr[g + 1] = (int32_t)total;
    }
    free(u); free(ts); free(tl);
    return rc ? rc : total;
}

/* The inverse of the local indices: the column index each slot names,      */
/* tile_start[tile_ptr[g] + local/64] + local%64, -1 for 0xFFFF.             */
void ora_unstage(int32_t n_groups, const int32_t* groups, int32_t block_dim,
                 const int32_t* tile_ptr, const int32_t* tile_start,
                 const uint16_t* local, int32_t* columns_out)
{
    for (int32_t g = 0; g < n_groups; g++) {
        const int64_t offset = groups[4 * g + 2];
        const int64_t slots = (int64_t)groups[4 * g + 3] * block_dim;
        for (int64_t s = 0; s < slots; s++) {
            const uint16_t v = local[offset + s];
            columns_out[offset + s] = v == 0xFFFF ? -1
                : tile_start[tile_ptr[g] + v / 64] + v % 64;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Inverse conversion: walk each row's chunks in order, emitting elements     */
/* until the artificial-zero marker.                                          */
/* ------------------------------------------------------------------------ */

int64_t ora_argcsr_to_csr(int32_t n_rows, int32_t n_groups,
                          const int32_t* groups, const int32_t* tm,
                          const int32_t* columns, const double* values,
                          int32_t block_dim, int32_t* rp_out,
                          int32_t* col_out, double* val_out)
{
    int64_t nnz = 0;
    int32_t row = 0;
    rp_out[0] = 0;
    for (int32_t g = 0; g < n_groups; g++) {
        const int32_t first = groups[4 * g + 0], size = groups[4 * g + 1];
        const int32_t offset = groups[4 * g + 2], chunk = groups[4 * g + 3];
        if (first != row) return -1;
        for (int32_t l = 0; l < size; l++) {
            const int32_t begin = (l == 0) ? 0 : tm[first + l - 1];
            const int32_t end = tm[first + l];
            for (int32_t k = begin; k < end; k++) {
                for (int32_t j = 0; j < chunk; j++) {
                    const int64_t s = (int64_t)offset + (int64_t)j * block_dim + k;
                    if (columns[s] == -1) break;
                    col_out[nnz] = columns[s];
                    val_out[nnz] = values[s];
                    nnz++;
                }
            }
            row++;
            if (nnz > INT32_MAX) return -2;
            rp_out[row] = (int32_t)nnz;
        }
    }
    if (row != n_rows) return -1;
    return nnz;
}

/* ------------------------------------------------------------------------ */
/* Textbook conjugate gradients (Hestenes-Stiefel), FP64, x0 = 0.  The        */
/* recursive residual drives the iteration; convergence is accepted only on   */
/* the true residual b - A x (recomputed by the CSR definition above).        */
/* ------------------------------------------------------------------------ */

static double dot(int32_t n, const double* a, const double* b)
{
    double s = 0.0;
    for (int32_t i = 0; i < n; i++) s = s + a[i] * b[i];
    return s;
}

static double true_relres(int32_t n, const int32_t* rp, const int32_t* col,
                          const double* val, const double* b, const double* x,
                          double* work, double bnorm)
{
    ora_csr_spmv(n, rp, col, val, x, work, 1);
    for (int32_t i = 0; i < n; i++) work[i] = b[i] - work[i];
    return sqrt(dot(n, work, work)) / bnorm;
}

int32_t ora_cg(int32_t n, const int32_t* rp, const int32_t* col,
               const double* val, const double* b, double* x, double tol,
               int32_t max_iter, double* relres)
{
    double* r = (double*)malloc(sizeof(double) * (size_t)(n + 1));
    double* p = (double*)malloc(sizeof(double) * (size_t)(n + 1));
    double* Ap = (double*)malloc(sizeof(double) * (size_t)(n + 1));
    const double bnorm = sqrt(dot(n, b, b));
    int32_t it = 0;
    for (int32_t i = 0; i < n; i++) { x[i] = 0.0; r[i] = b[i]; p[i] = b[i]; }
    if (bnorm == 0.0) {
        *relres = 0.0;
        free(r); free(p); free(Ap);
        return 0;
    }
    double rr = dot(n, r, r);
    double rel = 1.0;
    while (it < max_iter) {
        ora_csr_spmv(n, rp, col, val, p, Ap, 1);
        const double alpha = rr / dot(n, p, Ap);
        for (int32_t i = 0; i < n; i++) {
            x[i] = x[i] + alpha * p[i];
            r[i] = r[i] - alpha * Ap[i];
        }
        it++;
        double rr_new = dot(n, r, r);
        if (sqrt(rr_new) <= tol * bnorm) {
            rel = true_relres(n, rp, col, val, b, x, Ap, bnorm);
            if (rel <= tol) break;
            /* recursive residual drifted: restart from the true residual */
            ora_csr_spmv(n, rp, col, val, x, Ap, 1);
            for (int32_t i = 0; i < n; i++) { r[i] = b[i] - Ap[i]; p[i] = r[i]; }
            rr = dot(n, r, r);
            continue;
        }
        const double beta = rr_new / rr;
        for (int32_t i = 0; i < n; i++) p[i] = r[i] + beta * p[i];
        rr = rr_new;
    }
    *relres = true_relres(n, rp, col, val, b, x, Ap, bnorm);
    free(r); free(p); free(Ap);
    return it;
}
