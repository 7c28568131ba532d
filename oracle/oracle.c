/*
 * oracle.c -- the FP64 reference for sparse-times-dense multiplication.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link
 * or call this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header or constant with the GPU
 * library.
 *
 * What it computes (NeutronSparse, Sec. 5.1, "AIV-based SpMM execution"):
 * every output row i is the sum, over the stored entries p of row i of the
 * sparse A, of the value v_p times row col_p of the dense B -- the
 * gather-then-accumulate definition of SpMM.  The matrix-engine form of the
 * same section computes the identical sum with the zeros of a tile included,
 * so a single definition covers both paths:
 *
 *     C*[i][j] = sum_{p = rowptr[i]}^{rowptr[i+1]-1} v_p * B[col_p][j]
 *
 * evaluated serially in double precision, row by row, entries in CSR order,
 * j innermost.  Inputs stored as f32, bf16 or f16 are widened to double
 * exactly (all three are subsets of binary64).  Duplicate column indices add;
 * an empty row gives zeros.
 *
 * It also returns S[i][j] = sum_p |v_p| * |B[col_p][j]|, the scale that the
 * normalised error metric divides by.
 *
 * The threaded variant splits rows statically over POSIX threads; each row is
 * still summed in the same serial order, so the bits do not depend on the
 * thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <pthread.h>

enum { ORC_F32 = 0, ORC_BF16 = 1, ORC_F16 = 2, ORC_F64 = 3 };

/* IEEE binary16 -> double, written from the format's definition:
 * 1 sign bit, 5 exponent bits (bias 15), 10 fraction bits; exponent 0 encodes
 * zero and subnormals (fraction * 2^-24), exponent 31 encodes inf / NaN. */
static double half_to_double(uint16_t h)
{
    int sign = (h >> 15) & 1;
    int e = (h >> 10) & 0x1f;
    int f = h & 0x3ff;
    double v;
    if (e == 0)
        v = ldexp((double)f, -24);
    else if (e == 31)
        v = f ? NAN : INFINITY;
    else
        v = ldexp((double)(f | 0x400), e - 25);
    return sign ? -v : v;
}

/* bfloat16 is the upper half of a binary32: widen by appending 16 zero bits. */
static double bf16_to_double(uint16_t b)
{
    uint32_t u = (uint32_t)b << 16;
    float f;
    memcpy(&f, &u, sizeof f);
    return (double)f;
}

static inline double load_elem(const void *base, int64_t idx, int dtype)
{
    switch (dtype) {
    case ORC_F32: return (double)((const float *)base)[idx];
    case ORC_BF16: return bf16_to_double(((const uint16_t *)base)[idx]);
    case ORC_F16: return half_to_double(((const uint16_t *)base)[idx]);
    default: return ((const double *)base)[idx];
    }
}

double oracle_widen(const void *base, int64_t idx, int dtype)
{
    return load_elem(base, idx, dtype);
}

typedef struct {
    int64_t n;
    const int64_t *rowptr;
    const int32_t *colidx;
    const void *vals;
    int val_dtype;
    const void *B;
    int b_dtype;
    int64_t ldb;
    const int64_t *rows; /* output row r of this call is A's row rows[r] (or r) */
    int64_t r0, r1;      /* range of output rows this worker owns */
    double *C;           /* (r1 - r0) rows of n, row stride n */
    double *S;           /* nullable */
} job_t;

static void spmm_rows(const job_t *j)
{
    for (int64_t r = j->r0; r < j->r1; ++r) {
        int64_t i = j->rows ? j->rows[r] : r;
        double *crow = j->C + r * j->n;
        double *srow = j->S ? j->S + r * j->n : NULL;
        for (int64_t c = 0; c < j->n; ++c) crow[c] = 0.0;
        if (srow)
            for (int64_t c = 0; c < j->n; ++c) srow[c] = 0.0;
        for (int64_t p = j->rowptr[i]; p < j->rowptr[i + 1]; ++p) {
            double v = load_elem(j->vals, p, j->val_dtype);
            int64_t brow = (int64_t)j->colidx[p] * j->ldb;
            for (int64_t c = 0; c < j->n; ++c) {
                double b = load_elem(j->B, brow + c, j->b_dtype);
                crow[c] += v * b;
                if (srow) srow[c] += fabs(v) * fabs(b);
            }
        }
    }
}

static void *worker(void *arg)
{
    spmm_rows((const job_t *)arg);
    return NULL;
}

/*
 * C (nrows x n, row-major, stride n) receives rows `rows[0..nrows)` of A*B, or
 * rows 0..nrows-1 when `rows` is NULL.  S (same shape) is optional.
 * Returns 0, or -1 when a thread cannot be started.
 */
int oracle_spmm(int64_t nrows, int64_t n, const int64_t *rowptr, const int32_t *colidx,
                const void *vals, int val_dtype, const void *B, int b_dtype, int64_t ldb,
                const int64_t *rows, double *C, double *S, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > nrows) nthreads = nrows > 0 ? (int)nrows : 1;
    job_t base = {n, rowptr, colidx, vals, val_dtype, B, b_dtype, ldb, rows, 0, nrows, C, S};
    if (nthreads == 1) {
        spmm_rows(&base);
        return 0;
    }
    pthread_t *tid = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    job_t *jobs = (job_t *)calloc((size_t)nthreads, sizeof(job_t));
    if (!tid || !jobs) { free(tid); free(jobs); return -1; }
    int started = 0, rc = 0;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = base;
        jobs[t].r0 = nrows * t / nthreads;
        jobs[t].r1 = nrows * (t + 1) / nthreads;
        if (pthread_create(&tid[t], NULL, worker, &jobs[t]) != 0) { rc = -1; break; }
        ++started;
    }
    for (int t = 0; t < started; ++t) pthread_join(tid[t], NULL);
    free(tid);
    free(jobs);
    return rc;
}
