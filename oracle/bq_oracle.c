/*
 * Oracle: plain FP64 CPU product of matrix-valued biquaternions.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; it exists so that tests, the smoke check and the CPU
 * baseline of the benchmark have an independent answer to compare with.
 * It shares no code, header, table or helper with the HIP library.
 *
 * What it computes (Sec. II A of the paper):
 *   A matrix-valued biquaternion Q in H_C^{m x k} is  Q = S + V . q_check
 *   (eq. Q) with S, V_x, V_y, V_z complex m x k matrices and the reversed
 *   unit vector q_check = (k_check, j_check, i_check) (eq. defQ), i.e.
 *   Q = S + V_z i + V_y j + V_x k.
 *   The matrix product (eq. MatrixQMultiplication) is, element by element,
 *   (Q1 Q2)[i,j] = sum_k  q1(i,k) q2(k,j)
 *   where each term is the scalar biquaternion product of eq. QMultiplication:
 *     s  = s1 s2 - v1 . v2
 *     v  = s1 v2 + v1 s2 - v1 x v2.
 *   Written out in real arithmetic this is the 64-real-product
 *   component-wise form (16 complex products per term, Sec. III A).
 *
 * Storage (Sec. III, eqs. biquat-repres and main-biquat-eqn): eight real
 * blocks M1..M8 with unit coefficients
 *     1 : M1 + i M5     i : M2 + i M6     j : M3 + i M7     k : M4 + i M8
 * so  S = M1 + i M5,  V_z = M2 + i M6,  V_y = M3 + i M7,  V_x = M4 + i M8.
 * Each block is row-major with its own leading dimension (elements).
 *
 * Evaluation order: for each output row i, k ascends, and for each k the
 * full scalar product q1(i,k) q2(k,j) is formed and then added to C[i,j].
 * Build with -ffp-contract=off so no multiply-add is fused.  Rows are
 * split across OpenMP threads; each C[i,j] is produced by one thread in a
 * fixed order, so results do not depend on the thread count.
 *
 * Parity pins live in the CPU test-suite: quaternion unit relations,
 * associativity, the 2n x 2n complex isomorph (eq. mapping-formulas) against
 * a library complex GEMM, brute force on tiny sizes against the 2x2 Pauli
 * form (eqs. TRG-in-C, qmap1), exact integer arithmetic, the T, conj and dagger
 * anti-/homomorphisms and the trace rule.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* One complex number as a pair of reals. */
typedef struct { double re, im; } cx;

static inline cx cx_mul(cx a, cx b) {
  cx r;
  r.re = a.re * b.re - a.im * b.im;
  r.im = a.re * b.im + a.im * b.re;
  return r;
}
static inline cx cx_add(cx a, cx b) { cx r = {a.re + b.re, a.im + b.im}; return r; }
static inline cx cx_sub(cx a, cx b) { cx r = {a.re - b.re, a.im - b.im}; return r; }

/* Scalar biquaternion in scalar-vector form: s + v_x k + v_y j + v_z i. */
typedef struct { cx s, vx, vy, vz; } bq;

/* Scalar product of eq. QMultiplication. */
static inline bq bq_mul(bq p, bq q) {
  bq r;
  /* s1 s2 - v1 . v2 */
  cx dot = cx_add(cx_add(cx_mul(p.vx, q.vx), cx_mul(p.vy, q.vy)), cx_mul(p.vz, q.vz));
  r.s = cx_sub(cx_mul(p.s, q.s), dot);
  /* v1 x v2 with components (x, y, z) */
  cx crx = cx_sub(cx_mul(p.vy, q.vz), cx_mul(p.vz, q.vy));
  cx cry = cx_sub(cx_mul(p.vz, q.vx), cx_mul(p.vx, q.vz));
  cx crz = cx_sub(cx_mul(p.vx, q.vy), cx_mul(p.vy, q.vx));
  /* s1 v2 + v1 s2 - v1 x v2 */
  r.vx = cx_sub(cx_add(cx_mul(p.s, q.vx), cx_mul(p.vx, q.s)), crx);
  r.vy = cx_sub(cx_add(cx_mul(p.s, q.vy), cx_mul(p.vy, q.s)), cry);
  r.vz = cx_sub(cx_add(cx_mul(p.s, q.vz), cx_mul(p.vz, q.s)), crz);
  return r;
}

/* Read element (r, c) of a biquaternion stored as 8 real blocks. */
static inline bq bq_load(const double* const M[8], int64_t ld, int64_t r, int64_t c) {
  int64_t o = r * ld + c;
  bq q;
  q.s.re = M[0][o];  q.s.im = M[4][o];
  q.vz.re = M[1][o]; q.vz.im = M[5][o];
  q.vy.re = M[2][o]; q.vy.im = M[6][o];
  q.vx.re = M[3][o]; q.vx.im = M[7][o];
  return q;
}

int bqo_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void bqo_set_num_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

/*
 * C = A B for A in H_C^{m x k}, B in H_C^{k x n}; all 24 block pointers must
 * be valid host arrays (absent components are passed as zero blocks).
 * Returns 0 on success, -1 on a bad argument.  C must not overlap A or B.
 */
int bqo_gemm(int64_t m, int64_t n, int64_t k,
             const double* const A[8], int64_t lda,
             const double* const B[8], int64_t ldb,
             double* const C[8], int64_t ldc) {
  if (m < 0 || n < 0 || k < 0) return -1;
  if (lda < (k > 0 ? k : 1) || ldb < (n > 0 ? n : 1) || ldc < (n > 0 ? n : 1)) return -1;
  for (int c = 0; c < 8; ++c)
    if (!A[c] || !B[c] || !C[c]) return -1;

  int64_t i;
#pragma omp parallel for schedule(static)
  for (i = 0; i < m; ++i) {
    double* c0 = C[0] + i * ldc; double* c1 = C[1] + i * ldc;
    double* c2 = C[2] + i * ldc; double* c3 = C[3] + i * ldc;
    double* c4 = C[4] + i * ldc; double* c5 = C[5] + i * ldc;
    double* c6 = C[6] + i * ldc; double* c7 = C[7] + i * ldc;
    for (int64_t j = 0; j < n; ++j) {
      c0[j] = 0.0; c1[j] = 0.0; c2[j] = 0.0; c3[j] = 0.0;
      c4[j] = 0.0; c5[j] = 0.0; c6[j] = 0.0; c7[j] = 0.0;
    }
    for (int64_t kk = 0; kk < k; ++kk) {
      bq a = bq_load(A, lda, i, kk);
      for (int64_t j = 0; j < n; ++j) {
        bq t = bq_mul(a, bq_load(B, ldb, kk, j));
        c0[j] += t.s.re;  c4[j] += t.s.im;
        c1[j] += t.vz.re; c5[j] += t.vz.im;
        c2[j] += t.vy.re; c6[j] += t.vy.im;
        c3[j] += t.vx.re; c7[j] += t.vx.im;
      }
    }
  }
  return 0;
}
