/*
 * Reference (oracle) sparse matrix product C = A * B on CSR inputs.
 *
 * TEST INFRASTRUCTURE.  This file is the plain, slow, obviously correct CPU
 * definition that the GPU path is checked against.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg load it.  It shares no code,
 * header, table or constant with the GPU library, and the GPU library never
 * calls it.
 *
 * What it computes (paper Section III-A, Algorithm 1 "row-by-row formulation of
 * SpGEMM" and the text that follows it):
 *   - rows of C are produced one at a time, one per row of A;
 *   - for a row i of A only the rows k of B named by the column indices of row
 *     i are visited ("selective streaming" of B);
 *   - every matching pair forms one partial product a_ik * b_kj;
 *   - partial products that share a column j are merged by summation into one
 *     entry C[i,j], and the row's entries are emitted in ascending column order.
 * This reaches exactly the plain definition
 *     pattern(C) = { (i,j) : exists k with A[i,k] and B[k,j] stored },
 *     C[i,j]     = sum_k A[i,k] * B[k,j],
 * so the oracle is that definition written out with a dense accumulator.
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - structural entries are kept even when their sum cancels to zero
 *     (the algorithm emits every column of the column set COLB);
 *   - the column set and partial-product list are reset for every row;
 *   - stored entries are iterated as given, so a column repeated inside a row
 *     of A (or B) contributes once per stored copy (CSR entries add);
 *   - arithmetic is IEEE binary64: each product is rounded once, then added to
 *     the running sum of its column in the order the products are generated
 *     (A row stored order, then B row stored order), the first product of a
 *     column initialising it.  The build compiles with -ffp-contract=off so no
 *     multiply-add is fused.  FP32 inputs are promoted to binary64 by the
 *     caller before the call; that product is exact.
 *   - alongside each value the oracle returns S_ij = sum_k |a_ik * b_kj|, the
 *     scale against which a reordered floating-point sum is judged.
 *
 * Threads: rows are independent; with nthreads > 1 the requested rows are
 * split statically and each thread owns its accumulators, so per-row
 * arithmetic (and therefore every bit of the result) is unchanged.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int cmp_int32(const void* x, const void* y) {
    int32_t a = *(const int32_t*)x, b = *(const int32_t*)y;
    return (a > b) - (a < b);
}

typedef struct {
    int64_t* mark;    /* mark[j] == stamp  <=> column j already in the current row */
    int64_t stamp;    /* bumped once per row, so a row listed twice is still fresh */
    double* acc;      /* running sum of products with column j */
    double* sabs;     /* running sum of |product| with column j */
    int32_t* touched; /* the row's column set, in first-seen order */
} scratch_t;

static int scratch_init(scratch_t* s, int64_t n, int with_values) {
    memset(s, 0, sizeof(*s));
    size_t nn = (size_t)(n > 0 ? n : 1);
    s->mark = (int64_t*)malloc(nn * sizeof(int64_t));
    s->touched = (int32_t*)malloc(nn * sizeof(int32_t));
    if (with_values) {
        s->acc = (double*)malloc(nn * sizeof(double));
        s->sabs = (double*)malloc(nn * sizeof(double));
    }
    if (!s->mark || !s->touched || (with_values && (!s->acc || !s->sabs))) return -1;
    for (size_t j = 0; j < nn; ++j) s->mark[j] = -1;
    s->stamp = -1;
    return 0;
}

static void scratch_free(scratch_t* s) {
    free(s->mark); free(s->touched); free(s->acc); free(s->sabs);
}

/* One row of C: returns the number of distinct columns; counts products. */
static int64_t row_symbolic(int64_t i, const int64_t* a_rp, const int32_t* a_col,
                            const int64_t* b_rp, const int32_t* b_col,
                            scratch_t* s, int64_t* products) {
    int64_t count = 0, prod = 0, stamp = ++s->stamp;
    for (int64_t p = a_rp[i]; p < a_rp[i + 1]; ++p) {
        int32_t k = a_col[p];                       /* row of B that matches */
        for (int64_t q = b_rp[k]; q < b_rp[k + 1]; ++q) {
            int32_t j = b_col[q];
            if (s->mark[j] != stamp) { s->mark[j] = stamp; ++count; }
            ++prod;
        }
    }
    *products = prod;
    return count;
}

static int64_t row_numeric(int64_t i, const int64_t* a_rp, const int32_t* a_col,
                           const double* a_val, const int64_t* b_rp, const int32_t* b_col,
                           const double* b_val, scratch_t* s,
                           int32_t* out_col, double* out_val, double* out_sabs) {
    int64_t count = 0, stamp = ++s->stamp;
    for (int64_t p = a_rp[i]; p < a_rp[i + 1]; ++p) {
        int32_t k = a_col[p];
        double a = a_val[p];
        for (int64_t q = b_rp[k]; q < b_rp[k + 1]; ++q) {
            int32_t j = b_col[q];
            double prod = a * b_val[q];             /* one rounded multiply */
            if (s->mark[j] != stamp) {
                s->mark[j] = stamp;
                s->acc[j] = prod;
                s->sabs[j] = fabs(prod);
                s->touched[count++] = j;
            } else {
                s->acc[j] = s->acc[j] + prod;       /* one rounded add */
                s->sabs[j] = s->sabs[j] + fabs(prod);
            }
        }
    }
    qsort(s->touched, (size_t)count, sizeof(int32_t), cmp_int32);
    for (int64_t t = 0; t < count; ++t) {
        int32_t j = s->touched[t];
        out_col[t] = j;
        out_val[t] = s->acc[j];
        if (out_sabs) out_sabs[t] = s->sabs[j];
    }
    return count;
}

/*
 * Pattern pass over the rows listed in rows[0..nrows): nnz_out[r] = number of
 * distinct columns of C's row rows[r]; prod_out[r] = number of partial products.
 * Returns 0, or -1 when scratch memory cannot be allocated.
 */
int oracle_spgemm_count(int64_t b_cols,
                        const int64_t* a_rp, const int32_t* a_col,
                        const int64_t* b_rp, const int32_t* b_col,
                        const int64_t* rows, int64_t nrows,
                        int64_t* nnz_out, int64_t* prod_out, int nthreads) {
    int failed = 0;
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel num_threads(nthreads) reduction(| : failed)
    {
        scratch_t s;
        int ok = scratch_init(&s, b_cols, 0) == 0;
        if (!ok) failed = 1;
        /* every thread reaches the work-sharing loop, even without scratch */
#pragma omp for schedule(static)
        for (int64_t r = 0; r < nrows; ++r) {
            int64_t pr = 0;
            if (!ok) continue;
            nnz_out[r] = row_symbolic(rows[r], a_rp, a_col, b_rp, b_col, &s, &pr);
            prod_out[r] = pr;
        }
        scratch_free(&s);
    }
    return failed ? -1 : 0;
}

/*
 * Value pass: for each listed row writes its columns (ascending), values and
 * per-entry scale S_ij starting at offsets[r] of the output arrays.  c_sabs may
 * be NULL.  Returns 0, or -1 on allocation failure or when a row's entry count
 * disagrees with the offsets (a corrupted call).
 */
int oracle_spgemm_fill(int64_t b_cols,
                       const int64_t* a_rp, const int32_t* a_col, const double* a_val,
                       const int64_t* b_rp, const int32_t* b_col, const double* b_val,
                       const int64_t* rows, int64_t nrows, const int64_t* offsets,
                       int32_t* c_col, double* c_val, double* c_sabs, int nthreads) {
    int failed = 0;
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel num_threads(nthreads) reduction(| : failed)
    {
        scratch_t s;
        int ok = scratch_init(&s, b_cols, 1) == 0;
        if (!ok) failed = 1;
#pragma omp for schedule(static)
        for (int64_t r = 0; r < nrows; ++r) {
            int64_t o = offsets[r];
            if (!ok) continue;
            int64_t cnt = row_numeric(rows[r], a_rp, a_col, a_val, b_rp, b_col, b_val, &s,
                                      c_col + o, c_val + o, c_sabs ? c_sabs + o : NULL);
            if (cnt != offsets[r + 1] - o) failed = 1;
        }
        scratch_free(&s);
    }
    return failed ? -1 : 0;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
