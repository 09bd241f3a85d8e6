/*
 * Oracle O1: the classical matrix product in IEEE binary64.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links this file;
 * only the tests, the smoke check and the benchmark's CPU-baseline leg load it.
 *
 * C[i][j] = sum_{p=0}^{k-1} A[i][p] * B[p][j]  -- the definition of C = A*B that
 * both the classical recursion (paper, Section 2.1, F_C recurrence) and the
 * bilinear form of Equation (1) reduce to.  Every fast algorithm of the paper
 * reaches this exact value in exact arithmetic (Equation (2) substituted into
 * Equation (1), Section 2.2), so this is the reference result.
 *
 * Rounding: each product a*b is rounded, then added; p ascends.  The file is
 * compiled with -ffp-contract=off so no fused multiply-add changes that, and
 * rows are split across OpenMP threads so the result does not depend on the
 * thread count.  Row-major storage with leading dimensions (elements).
 */
#include <stdint.h>
#include <omp.h>

/* C = A * B for an m x k times k x n product. */
void oracle_gemm_f64(int64_t m, int64_t k, int64_t n,
                     const double *A, int64_t lda,
                     const double *B, int64_t ldb,
                     double *C, int64_t ldc)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        double *c = C + i * ldc;
        for (int64_t j = 0; j < n; ++j) c[j] = 0.0;
        const double *a = A + i * lda;
        for (int64_t p = 0; p < k; ++p) {
            const double aip = a[p];
            const double *b = B + p * ldb;
            for (int64_t j = 0; j < n; ++j) c[j] = c[j] + aip * b[j];
        }
    }
}

/* The same product restricted to a list of rows: Out[t][j] = (A*B)[rows[t]][j].
 * Used to check single rows of very large products. */
void oracle_gemm_rows_f64(int64_t nrows, const int64_t *rows, int64_t k, int64_t n,
                          const double *A, int64_t lda,
                          const double *B, int64_t ldb,
                          double *Out, int64_t ldo)
{
    #pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < nrows; ++t) {
        double *c = Out + t * ldo;
        for (int64_t j = 0; j < n; ++j) c[j] = 0.0;
        const double *a = A + rows[t] * lda;
        for (int64_t p = 0; p < k; ++p) {
            const double aip = a[p];
            const double *b = B + p * ldb;
            for (int64_t j = 0; j < n; ++j) c[j] = c[j] + aip * b[j];
        }
    }
}

/* Compensated variant of the row product (Ogita, Rump and Oishi, "Accurate sum
 * and dot product", SIAM J. Sci. Comput. 2005, algorithm Dot2 built from
 * TwoSum and a Dekker/Veltkamp TwoProduct).  Its result is as accurate as if
 * computed in twice the working precision, so the oracle's own rounding does
 * not mask errors of a few ulps in the product under test. */
static inline void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

static inline void split(double a, double *hi, double *lo)
{
    const double factor = 134217729.0; /* 2^27 + 1 */
    double c = factor * a;
    double h = c - (c - a);
    *hi = h;
    *lo = a - h;
}

static inline void two_prod(double a, double b, double *p, double *e)
{
    double x = a * b;
    double ah, al, bh, bl;
    split(a, &ah, &al);
    split(b, &bh, &bl);
    *e = al * bl - (((x - ah * bh) - al * bh) - ah * bl);
    *p = x;
}

void oracle_gemm_rows_dot2_f64(int64_t nrows, const int64_t *rows, int64_t k, int64_t n,
                               const double *A, int64_t lda,
                               const double *B, int64_t ldb,
                               double *Out, int64_t ldo)
{
    #pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < nrows; ++t) {
        const double *a = A + rows[t] * lda;
        for (int64_t j = 0; j < n; ++j) {
            double s = 0.0, c = 0.0;
            for (int64_t p = 0; p < k; ++p) {
                double h, r, q;
                two_prod(a[p], B[p * ldb + j], &h, &r);
                two_sum(s, h, &s, &q);
                c = c + (q + r);
            }
            Out[t * ldo + j] = s + c;
        }
    }
}

int oracle_num_threads(void)
{
    return omp_get_max_threads();
}
