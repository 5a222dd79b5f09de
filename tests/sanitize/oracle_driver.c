/* Driver for a sanitizer build of the oracle (test infrastructure): every
 * oracle entry point on seeded random inputs of many shapes (empty matrices
 * and columns, one row, long columns, rectangular operands, shuffled rows),
 * with every output array allocated to exactly the size the header states, so
 * that AddressSanitizer and UBSan see any access or arithmetic outside it.
 * Also checks that the parallel product equals the single-threaded one and
 * that malformed inputs are refused. Exit status 0 on success. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static uint64_t next_u64(void) { /* splitmix64 */
    uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
static int32_t below(int32_t n) { return n <= 0 ? 0 : (int32_t)(next_u64() % (uint64_t)n); }
static double unit(void) { return (double)(next_u64() >> 11) * (2.0 / 9007199254740992.0) - 1.0; }

typedef struct {
    int32_t m, n, nnz;
    int32_t *cp, *ri;
    double *v;
    float *vf;
} mat;

/* m x n with column j holding min(m, z_j) distinct rows in random order */
static mat random_mat(int32_t m, int32_t n, int32_t zmax) {
    mat a;
    a.m = m;
    a.n = n;
    a.cp = malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t *z = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    a.cp[0] = 0;
    for (int32_t j = 0; j < n; ++j) {
        z[j] = below(zmax + 1);
        if (z[j] > m) z[j] = m;
        a.cp[j + 1] = a.cp[j] + z[j];
    }
    a.nnz = a.cp[n];
    a.ri = malloc(sizeof(int32_t) * (size_t)(a.nnz > 0 ? a.nnz : 1));
    a.v = malloc(sizeof(double) * (size_t)(a.nnz > 0 ? a.nnz : 1));
    a.vf = malloc(sizeof(float) * (size_t)(a.nnz > 0 ? a.nnz : 1));
    char *used = calloc((size_t)(m > 0 ? m : 1), 1);
    for (int32_t j = 0; j < n; ++j) {
        for (int32_t p = a.cp[j]; p < a.cp[j + 1]; ++p) {
            int32_t r;
            do r = below(m); while (used[r]);
            used[r] = 1;
            a.ri[p] = r;
            a.v[p] = unit();
            a.vf[p] = (float)a.v[p];
        }
        for (int32_t p = a.cp[j]; p < a.cp[j + 1]; ++p) used[a.ri[p]] = 0;
    }
    free(used);
    free(z);
    return a;
}

static void free_mat(mat *a) {
    free(a->cp);
    free(a->ri);
    free(a->v);
    free(a->vf);
}

static int fail(const char *what, int rc) {
    fprintf(stderr, "oracle driver: %s failed (%d)\n", what, rc);
    return 1;
}

static int one_case(int32_t m, int32_t k, int32_t n, int32_t za, int32_t zb) {
    mat a = random_mat(m, k, za), b = random_mat(k, n, zb);
    int rc;
    if ((rc = oracle_check_csc(a.m, a.n, a.cp, a.ri)) || (rc = oracle_check_csc(b.m, b.n, b.cp, b.ri)))
        return fail("check_csc", rc);
    int64_t *op = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if ((rc = oracle_opcount(k, a.cp, n, b.cp, b.ri, op))) return fail("opcount", rc);
    int32_t *ccp = malloc(sizeof(int32_t) * (size_t)(n + 1));
    if ((rc = oracle_symbolic(m, k, a.cp, a.ri, k, n, b.cp, b.ri, ccp))) return fail("symbolic", rc);
    const int32_t nnz = ccp[n];
    const size_t sz = (size_t)(nnz > 0 ? nnz : 1);
    int32_t *cri = malloc(sizeof(int32_t) * sz), *cri2 = malloc(sizeof(int32_t) * sz);
    double *cv = malloc(sizeof(double) * sz), *cv2 = malloc(sizeof(double) * sz);
    float *cvf = malloc(sizeof(float) * sz);
    if ((rc = oracle_spgemm_f64(m, k, a.cp, a.ri, a.v, k, n, b.cp, b.ri, b.v, ccp, cri, cv)))
        return fail("spgemm_f64", rc);
    if ((rc = oracle_spgemm_f32(m, k, a.cp, a.ri, a.vf, k, n, b.cp, b.ri, b.vf, ccp, cri2, cvf)))
        return fail("spgemm_f32", rc);
    double *cabs = malloc(sizeof(double) * sz);
    int32_t *cterms = malloc(sizeof(int32_t) * sz);
    if ((rc = oracle_absprod_f64(m, k, a.cp, a.ri, a.v, k, n, b.cp, b.ri, b.v, ccp, cri, cabs, cterms)))
        return fail("absprod", rc);
    double *g = malloc(sizeof(double) * sz), *da = malloc(sizeof(double) * (size_t)(a.nnz + 1)),
           *db = malloc(sizeof(double) * (size_t)(b.nnz + 1));
    float *gf = malloc(sizeof(float) * sz), *daf = malloc(sizeof(float) * (size_t)(a.nnz + 1)),
          *dbf = malloc(sizeof(float) * (size_t)(b.nnz + 1));
    for (int32_t i = 0; i < nnz; ++i) {
        g[i] = unit();
        gf[i] = (float)g[i];
    }
    if ((rc = oracle_backward_f64(m, k, a.cp, a.ri, a.v, k, n, b.cp, b.ri, b.v, ccp, cri, g, da, db)))
        return fail("backward_f64", rc);
    if ((rc = oracle_backward_f32(m, k, a.cp, a.ri, a.vf, k, n, b.cp, b.ri, b.vf, ccp, cri, gf, daf, dbf)))
        return fail("backward_f32", rc);
    /* the parallel product equals the single-threaded one */
    int32_t *pcp = malloc(sizeof(int32_t) * (size_t)(n + 1));
    int64_t cap = nnz;
    int32_t used = 0;
    if ((rc = oracle_spgemm_f64_parallel(m, k, a.cp, a.ri, a.v, k, n, b.cp, b.ri, b.v, pcp, &cap,
                                         cri2, cv2, 3, &used)))
        return fail("spgemm_f64_parallel", rc);
    if (memcmp(pcp, ccp, sizeof(int32_t) * (size_t)(n + 1)) || memcmp(cri2, cri, sizeof(int32_t) * (size_t)nnz) ||
        memcmp(cv2, cv, sizeof(double) * (size_t)nnz))
        return fail("parallel equals single-threaded", -1);
    /* Section 3.1 planning steps on the Op counts */
    int32_t *perm = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t *ops = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int32_t *starts = malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t nb = 0;
    if ((rc = oracle_sort_columns(n, op, perm))) return fail("sort_columns", rc);
    for (int32_t j = 0; j < n; ++j) ops[j] = op[perm[j]];
    if ((rc = oracle_blocking(n, ops, 1 + below(8), 8 + below(64), starts, &nb))) return fail("blocking", rc);
    for (int32_t j = 0; j < n; ++j) (void)oracle_hash_size(ops[j]);
    free(op); free(ccp); free(cri); free(cri2); free(cv); free(cv2); free(cvf); free(cabs);
    free(cterms); free(g); free(da); free(db); free(gf); free(daf); free(dbf); free(pcp);
    free(perm); free(ops); free(starts);
    free_mat(&a);
    free_mat(&b);
    return 0;
}

int main(void) {
    /* shapes: empty, one row, one column, rectangular, dense-ish, long columns */
    static const int32_t shapes[][5] = {
        {0, 0, 0, 0, 0}, {1, 1, 1, 1, 1}, {1, 40, 7, 1, 40}, {5, 0, 9, 3, 0}, {7, 5, 0, 3, 3},
        {64, 64, 64, 8, 8}, {300, 120, 250, 12, 20}, {1000, 1000, 50, 40, 300}, {37, 91, 13, 37, 91},
        {2000, 30, 400, 2000, 30}};
    for (unsigned s = 0; s < sizeof(shapes) / sizeof(shapes[0]); ++s)
        for (int rep = 0; rep < 4; ++rep)
            if (one_case(shapes[s][0], shapes[s][1], shapes[s][2], shapes[s][3], shapes[s][4])) return 1;
    for (int rep = 0; rep < 200; ++rep)
        if (one_case(1 + below(60), below(60), below(60), below(12), below(12))) return 1;
    /* malformed inputs are refused, not read out of bounds */
    int32_t cp_bad[3] = {0, 3, 2}, ri_ok[3] = {0, 1, 2}, ri_bad[2] = {0, 9}, cp2[3] = {0, 1, 2};
    int32_t ri_rep[2] = {1, 1}, cp_rep[2] = {0, 2};
    if (oracle_check_csc(4, 2, cp_bad, ri_ok) == 0) return fail("decreasing colptr refused", 0);
    if (oracle_check_csc(4, 2, cp2, ri_bad) == 0) return fail("row out of range refused", 0);
    if (oracle_check_csc(4, 1, cp_rep, ri_rep) == 0) return fail("repeated row refused", 0);
    printf("oracle driver: ok\n");
    return 0;
}
