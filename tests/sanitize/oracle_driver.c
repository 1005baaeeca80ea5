/* The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (built and
 * run by tests/test_sanitizers.py): small integer products through bqo_gemm,
 * against a product written out here from the unit table i^2 = j^2 = k^2 =
 * ijk = -1 (16 complex products, each four real ones), exact on integers. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int bqo_gemm(int64_t m, int64_t n, int64_t k, const double* const A[8], int64_t lda, const double* const B[8],
             int64_t ldb, double* const C[8], int64_t ldc);

/* e_u e_v = sgn e_w for the units 1, i, j, k. */
static const int W[4][4] = {{0, 1, 2, 3}, {1, 0, 3, 2}, {2, 3, 0, 1}, {3, 2, 1, 0}};
static const int SG[4][4] = {{1, 1, 1, 1}, {1, -1, 1, -1}, {1, -1, -1, 1}, {1, 1, -1, -1}};

int main(void) {
  int fails = 0;
  unsigned seed = 7;
  for (int t = 0; t < 40; ++t) {
    const int64_t m = 1 + t % 5, n = 1 + (t * 3) % 7, k = (t * 7) % 6;  /* k = 0 included */
    double *a[8], *b[8], *c[8], *r[8];
    for (int q = 0; q < 8; ++q) {
      a[q] = malloc(sizeof(double) * (size_t)(m * (k ? k : 1)));
      b[q] = malloc(sizeof(double) * (size_t)((k ? k : 1) * n));
      c[q] = malloc(sizeof(double) * (size_t)(m * n));
      r[q] = calloc((size_t)(m * n), sizeof(double));
      for (int64_t x = 0; x < m * k; ++x) a[q][x] = (double)((int)((seed = seed * 1103515245u + 12345u) >> 16) % 33 - 16);
      for (int64_t x = 0; x < k * n; ++x) b[q][x] = (double)((int)((seed = seed * 1103515245u + 12345u) >> 16) % 33 - 16);
    }
    for (int u = 0; u < 4; ++u)
      for (int v = 0; v < 4; ++v)
        for (int64_t i = 0; i < m; ++i)
          for (int64_t j = 0; j < n; ++j)
            for (int64_t kk = 0; kk < k; ++kk) {
              /* (a_u + i a_{u+4})(b_v + i b_{v+4}) e_u e_v */
              const double ar = a[u][i * k + kk], ai = a[u + 4][i * k + kk];
              const double br = b[v][kk * n + j], bi = b[v + 4][kk * n + j];
              const int w = W[u][v], s = SG[u][v];
              r[w][i * n + j] += s * (ar * br - ai * bi);
              r[w + 4][i * n + j] += s * (ar * bi + ai * br);
            }
    if (bqo_gemm(m, n, k, (const double* const*)a, k ? k : 1, (const double* const*)b, n, c, n) != 0) {
      ++fails;
      fprintf(stderr, "bqo_gemm rejected case %d\n", t);
    } else {
      for (int q = 0; q < 8; ++q)
        for (int64_t x = 0; x < m * n; ++x)
          if (c[q][x] != r[q][x]) {
            ++fails;
            fprintf(stderr, "case %d block %d element %lld: %g != %g\n", t, q, (long long)x, c[q][x], r[q][x]);
            q = 8;
            break;
          }
    }
    for (int q = 0; q < 8; ++q) {
      free(a[q]);
      free(b[q]);
      free(c[q]);
      free(r[q]);
    }
  }
  printf("oracle: 40 products, %d failures\n", fails);
  return fails ? 1 : 0;
}
