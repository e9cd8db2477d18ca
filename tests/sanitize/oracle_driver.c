/* Driver of the oracle's FP64 GEMM (oracle/gemm_f64.c), built with it under
 * AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_sanitizers.py.
 * Small-integer products, every layout, row samples, beta terms and leading
 * dimensions larger than the extent; each result is compared with a direct
 * evaluation of the definition (exact for these integers).  Exits non-zero on
 * a mismatch; the sanitizers abort on memory or undefined-behaviour errors. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_gemm_f64(int64_t M, int64_t N, int64_t K, const double *a, int64_t lda,
                    int a_col_major, const double *b, int64_t ldb, int b_col_major,
                    const double *cin, int64_t ldcin, double alpha, double beta, double *c,
                    int64_t ldc, const int64_t *rows, int64_t nrows);

static uint64_t state = 12345;
static int small_int(void) {
  state = state * 6364136223846793005ull + 1442695040888963407ull;
  return (int)((state >> 33) % 9) - 4;
}

int main(void) {
  int bad = 0;
  for (int it = 0; it < 60; ++it) {
    int64_t M = 1 + it % 7, N = 1 + (it * 3) % 5, K = it % 6;
    int ac = it & 1, bc = (it >> 1) & 1;
    int64_t lda = (ac ? M : K) + it % 3, ldb = (bc ? K : N) + it % 2, ldc = N + 1;
    if (lda < 1) lda = 1;
    if (ldb < 1) ldb = 1;
    int64_t na = (ac ? (K > 0 ? K : 1) : M) * lda, nb = (bc ? N : (K > 0 ? K : 1)) * ldb;
    double *a = malloc(sizeof(double) * (size_t)na), *b = malloc(sizeof(double) * (size_t)nb);
    double *cin = malloc(sizeof(double) * (size_t)(M * N)), *c = malloc(sizeof(double) * (size_t)(M * ldc));
    int64_t *rows = malloc(sizeof(int64_t) * (size_t)M);
    for (int64_t i = 0; i < na; ++i) a[i] = small_int();
    for (int64_t i = 0; i < nb; ++i) b[i] = small_int();
    for (int64_t i = 0; i < M * N; ++i) cin[i] = small_int();
    for (int64_t i = 0; i < M; ++i) rows[i] = M - 1 - i;
    double beta = it % 3 == 0 ? 0.0 : 0.5;
    int sampled = it % 4 == 0;
    if (oracle_gemm_f64(M, N, K, a, lda, ac, b, ldb, bc, cin, N, 2.0, beta, c, ldc,
                        sampled ? rows : NULL, sampled ? M : 0) != 0) bad++;
    for (int64_t r = 0; r < M; ++r) {
      int64_t i = sampled ? rows[r] : r;
      for (int64_t j = 0; j < N; ++j) {
        double s = 0;
        for (int64_t k = 0; k < K; ++k)
          s += (ac ? a[k * lda + i] : a[i * lda + k]) * (bc ? b[j * ldb + k] : b[k * ldb + j]);
        double want = 2.0 * s + (beta != 0 ? beta * cin[i * N + j] : 0.0);
        if (c[r * ldc + j] != want) bad++;
      }
    }
    free(a); free(b); free(cin); free(c); free(rows);
  }
  if (oracle_gemm_f64(-1, 1, 1, NULL, 1, 0, NULL, 1, 0, NULL, 1, 1.0, 0.0, NULL, 1, NULL, 0) != -1)
    bad++;
  if (bad) {
    fprintf(stderr, "%d mismatch(es)\n", bad);
    return 1;
  }
  printf("oracle driver: ok\n");
  return 0;
}
