/*
 * CPU oracle for column-wise sparse matrix product C = A x B on CSC matrices.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may call into this library. The GPU library
 * shares no code, header or table with it.
 *
 * Everything here is the plain definition, written for a reader to check
 * against the paper by eye:
 *   - CSC storage as in Section 2.1 (values, row indices, column pointers with
 *     colptr[0] = 0 and colptr[n] = nnz; order inside a column is free).
 *   - the Gustavson column method of Section 2.1: column j of C is the sum over
 *     the stored B(k,j) of B(k,j) times column k of A;
 *   - computed as the sequential sparse accumulator (SPA) of Algorithm 1: a
 *     dense value array, a touched flag and a list of touched rows per column.
 *
 * Arithmetic: every product A(i,k)*B(k,j) is rounded on its own and added to
 * the running value of row i in the order the B entries of column j are
 * stored, starting from 0.0 (Algorithm 1 initialises the accumulator with
 * zeros and adds). No fused multiply-add: the library is compiled with
 * -ffp-contract=off.
 *
 * Output: rows of every C column in ascending order; a row touched by any
 * product is a stored entry even if its value cancels to zero.
 */
#ifndef SPGEMM_ORACLE_H
#define SPGEMM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes of the oracle (independent of the GPU library's codes) */
#define ORACLE_OK 0
#define ORACLE_EBADCSC 1   /* colptr not starting at 0 / decreasing / rows out of range / duplicates */
#define ORACLE_ESHAPE 2    /* A.ncols != B.nrows */
#define ORACLE_ENOMEM 3
#define ORACLE_EOVERFLOW 4 /* nnz(C) or a product count exceeds int32 */

/* Check a CSC matrix: colptr[0] == 0, non-decreasing, colptr[n] == nnz,
 * 0 <= rowidx < nrows, no row repeated inside a column. */
int oracle_check_csc(int32_t nrows, int32_t ncols, const int32_t *colptr,
                     const int32_t *rowidx);

/* Op_j of Section 3.1: number of products for column j of C, the sum of
 * nnz(A(:,k)) over the stored B(k,j). */
int oracle_opcount(int32_t a_ncols, const int32_t *a_colptr,
                   int32_t b_ncols, const int32_t *b_colptr, const int32_t *b_rowidx,
                   int64_t *op /* [b_ncols] */);

/* Structure of C: nnz of every column (size of the union of the row sets of
 * the A columns selected by B(:,j)), written as the column pointer array. */
int oracle_symbolic(int32_t a_nrows, int32_t a_ncols, const int32_t *a_colptr,
                    const int32_t *a_rowidx,
                    int32_t b_nrows, int32_t b_ncols, const int32_t *b_colptr,
                    const int32_t *b_rowidx,
                    int32_t *c_colptr /* [b_ncols + 1] */);

/* Full product, double precision, Algorithm 1 order. c_rowidx / c_val must
 * hold c_colptr[b_ncols] entries (from oracle_symbolic). */
int oracle_spgemm_f64(int32_t a_nrows, int32_t a_ncols, const int32_t *a_colptr,
                      const int32_t *a_rowidx, const double *a_val,
                      int32_t b_nrows, int32_t b_ncols, const int32_t *b_colptr,
                      const int32_t *b_rowidx, const double *b_val,
                      const int32_t *c_colptr, int32_t *c_rowidx, double *c_val);

/* The same loops carried out in single precision (products and sums rounded
 * to float). A twin of the double oracle for float inputs. */
int oracle_spgemm_f32(int32_t a_nrows, int32_t a_ncols, const int32_t *a_colptr,
                      const int32_t *a_rowidx, const float *a_val,
                      int32_t b_nrows, int32_t b_ncols, const int32_t *b_colptr,
                      const int32_t *b_rowidx, const float *b_val,
                      const int32_t *c_colptr, int32_t *c_rowidx, float *c_val);

/* Per-entry magnitude sum s_ij = sum_k |A(i,k) B(k,j)| on the pattern of C,
 * used for error bounds of entries that cancel. */
int oracle_absprod_f64(int32_t a_nrows, int32_t a_ncols, const int32_t *a_colptr,
                       const int32_t *a_rowidx, const double *a_val,
                       int32_t b_nrows, int32_t b_ncols, const int32_t *b_colptr,
                       const int32_t *b_rowidx, const double *b_val,
                       const int32_t *c_colptr, const int32_t *c_rowidx,
                       double *c_abs, int32_t *c_terms);

/* Gradients of L = <G, C> with respect to the stored values of A and B, with
 * the sparsity patterns fixed:
 *   dA(i,k) = sum over stored B(k,j), j ascending, of G(i,j) * B(k,j)
 *   dB(k,j) = sum over stored A(i,k), in A's storage order, of A(i,k) * G(i,j)
 * where G(i,j) is the value G holds at C's stored position (i,j). */
int oracle_backward_f64(int32_t a_nrows, int32_t a_ncols, const int32_t *a_colptr,
                        const int32_t *a_rowidx, const double *a_val,
                        int32_t b_nrows, int32_t b_ncols, const int32_t *b_colptr,
                        const int32_t *b_rowidx, const double *b_val,
                        const int32_t *c_colptr, const int32_t *c_rowidx,
                        const double *g_val, double *da_val, double *db_val);

int oracle_backward_f32(int32_t a_nrows, int32_t a_ncols, const int32_t *a_colptr,
                        const int32_t *a_rowidx, const float *a_val,
                        int32_t b_nrows, int32_t b_ncols, const int32_t *b_colptr,
                        const int32_t *b_rowidx, const float *b_val,
                        const int32_t *c_colptr, const int32_t *c_rowidx,
                        const float *g_val, float *da_val, float *db_val);

/* Section 3.1 planning steps, written out for the pins of Figure 2.
 * oracle_sort_columns: permutation of column indices by decreasing Op
 * (ties by ascending column index). oracle_blocking: block boundaries of the
 * Blocking Algorithm over Op values already in that order; returns the number
 * of blocks and writes their first indices (block b covers
 * [starts[b], starts[b+1]) with starts[nblocks] = n). */
int oracle_sort_columns(int32_t n, const int64_t *op, int32_t *perm);
int oracle_blocking(int32_t n, const int64_t *op_sorted, int32_t bmin, int32_t bmax,
                    int32_t *starts /* [n + 1] */, int32_t *nblocks);

/* Section 3.2: hash table size H = 2^k with 2^(k-1) <= maxop < 2^k. */
int64_t oracle_hash_size(int64_t maxop);

/* The FP64 product of oracle_symbolic + oracle_spgemm_f64 with the columns
 * spread over `nthreads` OpenMP threads (0: the runtime's default). Each
 * column is still computed by one thread in Algorithm 1's order, with that
 * thread's own SPA arrays, so the result equals the single-threaded one bit
 * for bit. c_colptr [b_ncols + 1] is filled; c_rowidx / c_val must hold
 * *nnz_cap entries, else ORACLE_EOVERFLOW with *nnz_cap set to nnz(C).
 * *threads_used receives the thread count of the parallel region. */
int oracle_spgemm_f64_parallel(int32_t a_nrows, int32_t a_ncols, const int32_t *a_colptr,
                               const int32_t *a_rowidx, const double *a_val,
                               int32_t b_nrows, int32_t b_ncols, const int32_t *b_colptr,
                               const int32_t *b_rowidx, const double *b_val,
                               int32_t *c_colptr, int64_t *nnz_cap, int32_t *c_rowidx,
                               double *c_val, int32_t nthreads, int32_t *threads_used);

#ifdef __cplusplus
}
#endif
#endif
