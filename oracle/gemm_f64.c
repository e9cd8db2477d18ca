/*
 * FP64 reference GEMM -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is part of the oracle.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may build, load or call it; the GPU
 * product path never does.  It shares no header, helper or constant with the
 * HIP library.
 *
 * What it computes is the plain definition of the general matrix product the
 * report is about (Introduction and Background sections: C = alpha*A*B +
 * beta*C over an M x N output with a K-long inner dimension):
 *
 *     C[i][j] = alpha * sum_{k=0}^{K-1} A(i,k) * B(k,j)  +  beta * Cin[i][j]
 *
 * in IEEE double precision, with the k-sum taken in increasing k for every
 * output element, starting from 0.  With B column-major the loops are i, j, k
 * (one dot product per element, both operands walked along k); with B
 * row-major they are i, k, j (row k of B added into row i of C).  The two
 * nests are interchanges of the same definition and give every element the
 * same sequence of roundings.  No blocking, no BLAS.
 *
 * Layouts (element addressing):
 *   A row-major    A(i,k) = a[i*lda + k]      A column-major  A(i,k) = a[k*lda + i]
 *   B row-major    B(k,j) = b[k*ldb + j]      B column-major  B(k,j) = b[j*ldb + k]
 *   C row-major    C(i,j) = c[i*ldc + j]
 *
 * The beta term is skipped when beta == 0 (Cin is then never read), so a NaN
 * in an unread Cin cannot leak into the result.
 *
 * rows / nrows: when rows != NULL only the listed output rows are computed and
 * output row r of `c` holds C[rows[r]][:] (a row sample of a large product);
 * otherwise all M rows are computed.  Cin is always indexed by the true row.
 *
 * Rows are distributed over OpenMP threads; each output element is computed
 * by one thread in the fixed order above, so the result does not depend on
 * the thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_gemm_f64(int64_t M, int64_t N, int64_t K,
                    const double *a, int64_t lda, int a_col_major,
                    const double *b, int64_t ldb, int b_col_major,
                    const double *cin, int64_t ldcin,
                    double alpha, double beta,
                    double *c, int64_t ldc,
                    const int64_t *rows, int64_t nrows)
{
    if (M < 0 || N < 0 || K < 0) return -1;
    int64_t nout = rows ? nrows : M;
    if (nout < 0) return -1;
    int fail = 0;

    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nout; ++r) {
        int64_t i = rows ? rows[r] : r;
        if (i < 0 || i >= M) { fail = 1; continue; }
        double *acc = c + r * ldc;
        if (b_col_major) {
            for (int64_t j = 0; j < N; ++j) {
                const double *bcol = b + j * ldb;
                double sum = 0.0;
                for (int64_t k = 0; k < K; ++k)
                    sum += (a_col_major ? a[k * lda + i] : a[i * lda + k]) * bcol[k];
                acc[j] = sum;
            }
        } else {
            for (int64_t j = 0; j < N; ++j) acc[j] = 0.0;
            for (int64_t k = 0; k < K; ++k) {
                double aik = a_col_major ? a[k * lda + i] : a[i * lda + k];
                const double *brow = b + k * ldb;
                for (int64_t j = 0; j < N; ++j) acc[j] += aik * brow[j];
            }
        }
        if (beta != 0.0) {
            const double *crow = cin + i * ldcin;
            for (int64_t j = 0; j < N; ++j) acc[j] = alpha * acc[j] + beta * crow[j];
        } else {
            for (int64_t j = 0; j < N; ++j) acc[j] = alpha * acc[j];
        }
    }
    return fail ? -2 : 0;
}

/* Number of OpenMP threads a parallel region of this library uses. */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
