/*
 * CPU oracle for C = A x B on CSC matrices -- TEST INFRASTRUCTURE ONLY.
 *
 * Written from the paper's definitions (Section 2.1 CSC storage and the
 * Gustavson column method, Algorithm 1 sequential SPA, Section 3.1 operation
 * count and blocking, Section 3.2 hash-size rule). Plain, single-threaded,
 * obviously correct; no blocking, fusion or reordering beyond what those
 * definitions state. Compiled with -ffp-contract=off so that every product and
 * every sum is rounded on its own.
 *
 * Pins (see tests/test_oracle_*.py): the Figure 1 worked example, dense
 * brute-force products on tiny inputs, structural invariants (boolean
 * product, identity and permutation factors, transposition), the closed form
 * of the squared 2-D Laplacian, Op_j = Z^2 for constant-Z inputs (Section
 * 5.2), the Figure 2 block costs, and central finite differences for the
 * gradients.
 */
#include "oracle.h"

#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_check_csc(int32_t nrows, int32_t ncols, const int32_t *colptr,
                     const int32_t *rowidx) {
    if (nrows < 0 || ncols < 0 || colptr == NULL) return ORACLE_EBADCSC;
    if (colptr[0] != 0) return ORACLE_EBADCSC;
    for (int32_t j = 0; j < ncols; ++j)
        if (colptr[j + 1] < colptr[j]) return ORACLE_EBADCSC;
    int32_t nnz = colptr[ncols];
    if (nnz > 0 && rowidx == NULL) return ORACLE_EBADCSC;
    for (int32_t p = 0; p < nnz; ++p)
        if (rowidx[p] < 0 || rowidx[p] >= nrows) return ORACLE_EBADCSC;
    /* duplicates: mark rows of each column in a dense stamp array */
    int32_t *stamp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nrows > 0 ? nrows : 1));
    if (!stamp) return ORACLE_ENOMEM;
    for (int32_t i = 0; i < nrows; ++i) stamp[i] = -1;
    int rc = ORACLE_OK;
    for (int32_t j = 0; j < ncols && rc == ORACLE_OK; ++j)
        for (int32_t p = colptr[j]; p < colptr[j + 1]; ++p) {
            if (stamp[rowidx[p]] == j) { rc = ORACLE_EBADCSC; break; }
            stamp[rowidx[p]] = j;
        }
    free(stamp);
    return rc;
}

int oracle_opcount(int32_t a_ncols, const int32_t *a_colptr,
                   int32_t b_ncols, const int32_t *b_colptr, const int32_t *b_rowidx,
                   int64_t *op) {
    for (int32_t j = 0; j < b_ncols; ++j) {
        int64_t s = 0;
        for (int32_t p = b_colptr[j]; p < b_colptr[j + 1]; ++p) {
            int32_t k = b_rowidx[p];
            if (k < 0 || k >= a_ncols) return ORACLE_EBADCSC;
            s += (int64_t)(a_colptr[k + 1] - a_colptr[k]); /* Z^A_k */
        }
        op[j] = s;
    }
    return ORACLE_OK;
}

static int check_pair(int32_t a_nrows, int32_t a_ncols, const int32_t *a_colptr,
                      const int32_t *a_rowidx, int32_t b_nrows, int32_t b_ncols,
                      const int32_t *b_colptr, const int32_t *b_rowidx) {
    if (a_ncols != b_nrows) return ORACLE_ESHAPE;
    int rc = oracle_check_csc(a_nrows, a_ncols, a_colptr, a_rowidx);
    if (rc) return rc;
    return oracle_check_csc(b_nrows, b_ncols, b_colptr, b_rowidx);
}

static int cmp_i32(const void *x, const void *y) {
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}

int oracle_symbolic(int32_t a_nrows, int32_t a_ncols, const int32_t *a_colptr,
                    const int32_t *a_rowidx,
                    int32_t b_nrows, int32_t b_ncols, const int32_t *b_colptr,
                    const int32_t *b_rowidx, int32_t *c_colptr) {
    int rc = check_pair(a_nrows, a_ncols, a_colptr, a_rowidx, b_nrows, b_ncols,
                        b_colptr, b_rowidx);
    if (rc) return rc;
    /* SPA_flags of Algorithm 1, cleared after each column through the list
     * of touched rows */
    unsigned char *flag = (unsigned char *)calloc((size_t)(a_nrows > 0 ? a_nrows : 1), 1);
    int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (size_t)(a_nrows > 0 ? a_nrows : 1));
    if (!flag || !touched) { free(flag); free(touched); return ORACLE_ENOMEM; }
    int64_t total = 0;
    c_colptr[0] = 0;
    for (int32_t j = 0; j < b_ncols; ++j) {
        int32_t counter = 0;
        for (int32_t p = b_colptr[j]; p < b_colptr[j + 1]; ++p) {
            int32_t k = b_rowidx[p];
            for (int32_t q = a_colptr[k]; q < a_colptr[k + 1]; ++q) {
                int32_t i = a_rowidx[q];
                if (!flag[i]) { flag[i] = 1; touched[counter++] = i; }
            }
        }
        for (int32_t r = 0; r < counter; ++r) flag[touched[r]] = 0;
        total += counter;
        if (total > 2147483647LL) { free(flag); free(touched); return ORACLE_EOVERFLOW; }
        c_colptr[j + 1] = (int32_t)total;
    }
    free(flag);
    free(touched);
    return ORACLE_OK;
}

/* Algorithm 1 for one value type. The body is spelled out twice (double and
 * float) rather than generated, so each can be read on its own. */
int oracle_spgemm_f64(int32_t a_nrows, int32_t a_ncols, const int32_t *a_colptr,
                      const int32_t *a_rowidx, const double *a_val,
                      int32_t b_nrows, int32_t b_ncols, const int32_t *b_colptr,
                      const int32_t *b_rowidx, const double *b_val,
                      const int32_t *c_colptr, int32_t *c_rowidx, double *c_val) {
    int rc = check_pair(a_nrows, a_ncols, a_colptr, a_rowidx, b_nrows, b_ncols,
                        b_colptr, b_rowidx);
    if (rc) return rc;
    size_t m = (size_t)(a_nrows > 0 ? a_nrows : 1);
    double *spa_values = (double *)calloc(m, sizeof(double));   /* zeros */
    unsigned char *spa_flags = (unsigned char *)calloc(m, 1);  /* zeros */
    int32_t *spa_indices = (int32_t *)malloc(m * sizeof(int32_t));
    if (!spa_values || !spa_flags || !spa_indices) {
        free(spa_values); free(spa_flags); free(spa_indices);
        return ORACLE_ENOMEM;
    }
    for (int32_t j = 0; j < b_ncols; ++j) {
        int32_t counter = 0;
        for (int32_t p = b_colptr[j]; p < b_colptr[j + 1]; ++p) {      /* B(k,j) */
            int32_t k = b_rowidx[p];
            double bkj = b_val[p];
            for (int32_t q = a_colptr[k]; q < a_colptr[k + 1]; ++q) {  /* A(i,k) */
                int32_t i = a_rowidx[q];
                double tmp_val = a_val[q] * bkj;
                spa_values[i] = spa_values[i] + tmp_val;
                if (spa_flags[i] == 0) {
                    spa_flags[i] = 1;
                    spa_indices[counter++] = i;
                }
            }
        }
        if (counter != c_colptr[j + 1] - c_colptr[j]) {
            free(spa_values); free(spa_flags); free(spa_indices);
            return ORACLE_EBADCSC;
        }
        /* rows of the output column in ascending order */
        qsort(spa_indices, (size_t)counter, sizeof(int32_t), cmp_i32);
        for (int32_t r = 0; r < counter; ++r) {
            int32_t i = spa_indices[r];
            c_rowidx[c_colptr[j] + r] = i;
            c_val[c_colptr[j] + r] = spa_values[i];
            spa_values[i] = 0.0;
            spa_flags[i] = 0;
        }
    }
    free(spa_values); free(spa_flags); free(spa_indices);
    return ORACLE_OK;
}

int oracle_spgemm_f32(int32_t a_nrows, int32_t a_ncols, const int32_t *a_colptr,
                      const int32_t *a_rowidx, const float *a_val,
                      int32_t b_nrows, int32_t b_ncols, const int32_t *b_colptr,
                      const int32_t *b_rowidx, const float *b_val,
                      const int32_t *c_colptr, int32_t *c_rowidx, float *c_val) {
    int rc = check_pair(a_nrows, a_ncols, a_colptr, a_rowidx, b_nrows, b_ncols,
                        b_colptr, b_rowidx);
    if (rc) return rc;
    size_t m = (size_t)(a_nrows > 0 ? a_nrows : 1);
    float *spa_values = (float *)calloc(m, sizeof(float));
    unsigned char *spa_flags = (unsigned char *)calloc(m, 1);
    int32_t *spa_indices = (int32_t *)malloc(m * sizeof(int32_t));
    if (!spa_values || !spa_flags || !spa_indices) {
        free(spa_values); free(spa_flags); free(spa_indices);
        return ORACLE_ENOMEM;
    }
    for (int32_t j = 0; j < b_ncols; ++j) {
        int32_t counter = 0;
        for (int32_t p = b_colptr[j]; p < b_colptr[j + 1]; ++p) {
            int32_t k = b_rowidx[p];
            float bkj = b_val[p];
            for (int32_t q = a_colptr[k]; q < a_colptr[k + 1]; ++q) {
                int32_t i = a_rowidx[q];
                float tmp_val = a_val[q] * bkj;
                spa_values[i] = spa_values[i] + tmp_val;
                if (spa_flags[i] == 0) {
                    spa_flags[i] = 1;
                    spa_indices[counter++] = i;
                }
            }
        }
        if (counter != c_colptr[j + 1] - c_colptr[j]) {
            free(spa_values); free(spa_flags); free(spa_indices);
            return ORACLE_EBADCSC;
        }
        qsort(spa_indices, (size_t)counter, sizeof(int32_t), cmp_i32);
        for (int32_t r = 0; r < counter; ++r) {
            int32_t i = spa_indices[r];
            c_rowidx[c_colptr[j] + r] = i;
            c_val[c_colptr[j] + r] = spa_values[i];
            spa_values[i] = 0.0f;
            spa_flags[i] = 0;
        }
    }
    free(spa_values); free(spa_flags); free(spa_indices);
    return ORACLE_OK;
}

int oracle_absprod_f64(int32_t a_nrows, int32_t a_ncols, const int32_t *a_colptr,
                       const int32_t *a_rowidx, const double *a_val,
                       int32_t b_nrows, int32_t b_ncols, const int32_t *b_colptr,
                       const int32_t *b_rowidx, const double *b_val,
                       const int32_t *c_colptr, const int32_t *c_rowidx,
                       double *c_abs, int32_t *c_terms) {
    int rc = check_pair(a_nrows, a_ncols, a_colptr, a_rowidx, b_nrows, b_ncols,
                        b_colptr, b_rowidx);
    if (rc) return rc;
    size_t m = (size_t)(a_nrows > 0 ? a_nrows : 1);
    double *acc = (double *)calloc(m, sizeof(double));
    int32_t *cnt = (int32_t *)calloc(m, sizeof(int32_t));
    if (!acc || !cnt) { free(acc); free(cnt); return ORACLE_ENOMEM; }
    for (int32_t j = 0; j < b_ncols; ++j) {
        for (int32_t p = b_colptr[j]; p < b_colptr[j + 1]; ++p) {
            int32_t k = b_rowidx[p];
            double bkj = b_val[p] < 0 ? -b_val[p] : b_val[p];
            for (int32_t q = a_colptr[k]; q < a_colptr[k + 1]; ++q) {
                int32_t i = a_rowidx[q];
                double aik = a_val[q] < 0 ? -a_val[q] : a_val[q];
                acc[i] += aik * bkj;
                cnt[i] += 1;
            }
        }
        for (int32_t r = c_colptr[j]; r < c_colptr[j + 1]; ++r) {
            int32_t i = c_rowidx[r];
            c_abs[r] = acc[i];
            c_terms[r] = cnt[i];
            acc[i] = 0.0;
            cnt[i] = 0;
        }
    }
    free(acc); free(cnt);
    return ORACLE_OK;
}

/* position of row i inside the sorted column j of C, or -1 */
static int32_t find_in_column(const int32_t *c_colptr, const int32_t *c_rowidx,
                              int32_t j, int32_t i) {
    int32_t lo = c_colptr[j], hi = c_colptr[j + 1];
    while (lo < hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (c_rowidx[mid] < i) lo = mid + 1;
        else hi = mid;
    }
    if (lo < c_colptr[j + 1] && c_rowidx[lo] == i) return lo;
    return -1;
}

/* row view of B's pattern: for every row k, the columns j (ascending) and the
 * positions p of the stored B(k,j) */
static int b_rows(int32_t b_nrows, int32_t b_ncols, const int32_t *b_colptr,
                  const int32_t *b_rowidx, int32_t **rowptr_out, int32_t **colj_out,
                  int32_t **pos_out) {
    int32_t nnz = b_colptr[b_ncols];
    int32_t *rowptr = (int32_t *)calloc((size_t)b_nrows + 1, sizeof(int32_t));
    int32_t *colj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    int32_t *pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    int32_t *fill = (int32_t *)calloc((size_t)b_nrows + 1, sizeof(int32_t));
    if (!rowptr || !colj || !pos || !fill) {
        free(rowptr); free(colj); free(pos); free(fill);
        return ORACLE_ENOMEM;
    }
    for (int32_t p = 0; p < nnz; ++p) rowptr[b_rowidx[p] + 1] += 1;
    for (int32_t k = 0; k < b_nrows; ++k) rowptr[k + 1] += rowptr[k];
    for (int32_t j = 0; j < b_ncols; ++j) /* columns visited in ascending order */
        for (int32_t p = b_colptr[j]; p < b_colptr[j + 1]; ++p) {
            int32_t k = b_rowidx[p];
            int32_t at = rowptr[k] + fill[k]++;
            colj[at] = j;
            pos[at] = p;
        }
    free(fill);
    *rowptr_out = rowptr; *colj_out = colj; *pos_out = pos;
    return ORACLE_OK;
}

#define BACKWARD_BODY(T)                                                              \
    int rc = check_pair(a_nrows, a_ncols, a_colptr, a_rowidx, b_nrows, b_ncols,       \
                        b_colptr, b_rowidx);                                          \
    if (rc) return rc;                                                                \
    if (db_val) {                                                                     \
        for (int32_t j = 0; j < b_ncols; ++j)                                         \
            for (int32_t p = b_colptr[j]; p < b_colptr[j + 1]; ++p) {                 \
                int32_t k = b_rowidx[p];                                              \
                T acc = (T)0;                                                         \
                for (int32_t q = a_colptr[k]; q < a_colptr[k + 1]; ++q) {             \
                    int32_t at = find_in_column(c_colptr, c_rowidx, j, a_rowidx[q]);  \
                    if (at < 0) return ORACLE_EBADCSC;                                \
                    acc = acc + a_val[q] * g_val[at];                                 \
                }                                                                     \
                db_val[p] = acc;                                                      \
            }                                                                         \
    }                                                                                 \
    if (da_val) {                                                                     \
        int32_t *rowptr, *colj, *pos;                                                 \
        rc = b_rows(b_nrows, b_ncols, b_colptr, b_rowidx, &rowptr, &colj, &pos);      \
        if (rc) return rc;                                                            \
        for (int32_t k = 0; k < a_ncols; ++k)                                         \
            for (int32_t q = a_colptr[k]; q < a_colptr[k + 1]; ++q) {                 \
                int32_t i = a_rowidx[q];                                              \
                T acc = (T)0;                                                         \
                for (int32_t r = rowptr[k]; r < rowptr[k + 1]; ++r) {                 \
                    int32_t at = find_in_column(c_colptr, c_rowidx, colj[r], i);      \
                    if (at < 0) { rc = ORACLE_EBADCSC; break; }                       \
                    acc = acc + g_val[at] * b_val[pos[r]];                            \
                }                                                                     \
                da_val[q] = acc;                                                      \
            }                                                                         \
        free(rowptr); free(colj); free(pos);                                          \
    }                                                                                 \
    return rc;

int oracle_backward_f64(int32_t a_nrows, int32_t a_ncols, const int32_t *a_colptr,
                        const int32_t *a_rowidx, const double *a_val,
                        int32_t b_nrows, int32_t b_ncols, const int32_t *b_colptr,
                        const int32_t *b_rowidx, const double *b_val,
                        const int32_t *c_colptr, const int32_t *c_rowidx,
                        const double *g_val, double *da_val, double *db_val) {
    BACKWARD_BODY(double)
}

int oracle_backward_f32(int32_t a_nrows, int32_t a_ncols, const int32_t *a_colptr,
                        const int32_t *a_rowidx, const float *a_val,
                        int32_t b_nrows, int32_t b_ncols, const int32_t *b_colptr,
                        const int32_t *b_rowidx, const float *b_val,
                        const int32_t *c_colptr, const int32_t *c_rowidx,
                        const float *g_val, float *da_val, float *db_val) {
    BACKWARD_BODY(float)
}

int oracle_sort_columns(int32_t n, const int64_t *op, int32_t *perm) {
    /* stable insertion of each column index behind all columns with a
     * greater or equal Op: a plain stable sort by decreasing Op */
    for (int32_t j = 0; j < n; ++j) perm[j] = j;
    /* merge sort for O(n log n) on large n, kept stable */
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!tmp) return ORACLE_ENOMEM;
    for (int32_t width = 1; width < n; width *= 2) {
        for (int32_t lo = 0; lo < n; lo += 2 * width) {
            int32_t mid = lo + width < n ? lo + width : n;
            int32_t hi = lo + 2 * width < n ? lo + 2 * width : n;
            int32_t a = lo, b = mid, o = lo;
            while (a < mid && b < hi) {
                /* take from the left run unless the right one is strictly larger */
                if (op[perm[b]] > op[perm[a]]) tmp[o++] = perm[b++];
                else tmp[o++] = perm[a++];
            }
            while (a < mid) tmp[o++] = perm[a++];
            while (b < hi) tmp[o++] = perm[b++];
        }
        memcpy(perm, tmp, sizeof(int32_t) * (size_t)n);
    }
    free(tmp);
    return ORACLE_OK;
}

int oracle_blocking(int32_t n, const int64_t *op_sorted, int32_t bmin, int32_t bmax,
                    int32_t *starts, int32_t *nblocks) {
    if (bmin < 1 || bmax < bmin) return ORACLE_EBADCSC;
    int32_t nb = 0;
    int32_t j = 0; /* columns already processed */
    while (j < n) {
        starts[nb++] = j;
        /* 1. start with bmin columns j .. j + bmin - 1 (clamped to n) */
        int32_t j2 = j + bmin < n ? j + bmin : n;
        /* 2. grow while the next column has the block's (first, largest) Op;
         * 3. stop at j + bmax or n */
        while (j2 < n && j2 < j + bmax && op_sorted[j2] == op_sorted[j]) ++j2;
        j = j2;
    }
    starts[nb] = n;
    *nblocks = nb;
    return ORACLE_OK;
}

int64_t oracle_hash_size(int64_t maxop) {
    if (maxop <= 0) return 0;
    int64_t h = 1;
    while (h <= maxop) h *= 2; /* smallest power of two strictly above maxop */
    return h;
}

/* Columns of C are independent (Section 2.1): each thread takes whole
 * columns and runs Algorithm 1 on them with SPA arrays of its own. Two
 * sweeps, as in the single-threaded pair: the distinct rows of every column
 * (its SPA flags), a prefix sum into the column pointers, then the values. */
int oracle_spgemm_f64_parallel(int32_t a_nrows, int32_t a_ncols, const int32_t *a_colptr,
                               const int32_t *a_rowidx, const double *a_val,
                               int32_t b_nrows, int32_t b_ncols, const int32_t *b_colptr,
                               const int32_t *b_rowidx, const double *b_val,
                               int32_t *c_colptr, int64_t *nnz_cap, int32_t *c_rowidx,
                               double *c_val, int32_t nthreads, int32_t *threads_used) {
    int rc = check_pair(a_nrows, a_ncols, a_colptr, a_rowidx, b_nrows, b_ncols,
                        b_colptr, b_rowidx);
    if (rc) return rc;
    size_t m = (size_t)(a_nrows > 0 ? a_nrows : 1);
    int32_t *count = (int32_t *)malloc(sizeof(int32_t) * (size_t)(b_ncols > 0 ? b_ncols : 1));
    if (!count) return ORACLE_ENOMEM;
    int failed = 0, used = 1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
#ifdef _OPENMP
#pragma omp single
        used = omp_get_num_threads();
#endif
        unsigned char *flag = (unsigned char *)calloc(m, 1);
        int32_t *touched = (int32_t *)malloc(m * sizeof(int32_t));
        if (!flag || !touched) {
#pragma omp atomic write
            failed = 1;
        } else {
#pragma omp for schedule(dynamic, 256)
            for (int32_t j = 0; j < b_ncols; ++j) {
                int32_t counter = 0;
                for (int32_t p = b_colptr[j]; p < b_colptr[j + 1]; ++p) {
                    int32_t k = b_rowidx[p];
                    for (int32_t q = a_colptr[k]; q < a_colptr[k + 1]; ++q) {
                        int32_t i = a_rowidx[q];
                        if (!flag[i]) { flag[i] = 1; touched[counter++] = i; }
                    }
                }
                for (int32_t r = 0; r < counter; ++r) flag[touched[r]] = 0;
                count[j] = counter;
            }
        }
        free(flag);
        free(touched);
    }
    if (failed) { free(count); return ORACLE_ENOMEM; }
    int64_t total = 0;
    c_colptr[0] = 0;
    for (int32_t j = 0; j < b_ncols; ++j) {
        total += count[j];
        if (total > 2147483647LL) { free(count); return ORACLE_EOVERFLOW; }
        c_colptr[j + 1] = (int32_t)total;
    }
    free(count);
    if (total > *nnz_cap) { *nnz_cap = total; return ORACLE_EOVERFLOW; }
    *nnz_cap = total;
#pragma omp parallel
    {
        double *spa_values = (double *)calloc(m, sizeof(double));
        unsigned char *spa_flags = (unsigned char *)calloc(m, 1);
        int32_t *spa_indices = (int32_t *)malloc(m * sizeof(int32_t));
        if (!spa_values || !spa_flags || !spa_indices) {
#pragma omp atomic write
            failed = 1;
        } else {
#pragma omp for schedule(dynamic, 256)
            for (int32_t j = 0; j < b_ncols; ++j) {
                int32_t counter = 0;
                for (int32_t p = b_colptr[j]; p < b_colptr[j + 1]; ++p) {
                    int32_t k = b_rowidx[p];
                    double bkj = b_val[p];
                    for (int32_t q = a_colptr[k]; q < a_colptr[k + 1]; ++q) {
                        int32_t i = a_rowidx[q];
                        double tmp_val = a_val[q] * bkj;
                        spa_values[i] = spa_values[i] + tmp_val;
                        if (spa_flags[i] == 0) {
                            spa_flags[i] = 1;
                            spa_indices[counter++] = i;
                        }
                    }
                }
                qsort(spa_indices, (size_t)counter, sizeof(int32_t), cmp_i32);
                for (int32_t r = 0; r < counter; ++r) {
                    int32_t i = spa_indices[r];
                    c_rowidx[c_colptr[j] + r] = i;
                    c_val[c_colptr[j] + r] = spa_values[i];
                    spa_values[i] = 0.0;
                    spa_flags[i] = 0;
                }
            }
        }
        free(spa_values);
        free(spa_flags);
        free(spa_indices);
    }
    *threads_used = used;
    return failed ? ORACLE_ENOMEM : ORACLE_OK;
}
