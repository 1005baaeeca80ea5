// Host-only exercise of the library's argument validation under AddressSanitizer
// and UndefinedBehaviorSanitizer (built and run by tests/test_sanitizers.py; no
// GPU and no HIP call: only the entry points that validate, size and plan).
//
// Pointers are host integers standing in for device addresses; the library
// never dereferences them during validation.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>

#include "bq.h"

namespace {

std::mt19937_64 rng(20261203);

int64_t pick(std::initializer_list<int64_t> v) {
  auto it = v.begin();
  std::advance(it, rng() % v.size());
  return *it;
}

bq_matrix_t make(int64_t rows, int64_t cols, int64_t ld, uintptr_t base, unsigned mask, int64_t stride) {
  bq_matrix_t M;
  std::memset(&M, 0, sizeof M);
  for (int c = 0; c < 8; ++c)
    M.comp[c] = (mask >> c & 1) ? reinterpret_cast<double*>(base + uintptr_t(c) * uintptr_t(stride)) : nullptr;
  M.rows = rows;
  M.cols = cols;
  M.ld = ld;
  return M;
}

// a + b without signed overflow (saturates at the int64 limits).
int64_t sat_add(int64_t a, int64_t b) {
  if (b > 0 && a > INT64_MAX - b) return INT64_MAX;
  if (b < 0 && a < INT64_MIN - b) return INT64_MIN;
  return a + b;
}

int fails = 0;

void expect(bool ok, const char* what, long long i) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s (case %lld)\n", what, i);
    ++fails;
  }
}

}  // namespace

int main() {
  const int64_t dims[] = {0, 1, 2, 3, 7, 64, 65, 1000, -1, int64_t(1) << 31, int64_t(1) << 40, INT64_MAX};
  long long checked = 0;
  for (long long i = 0; i < 200000; ++i) {
    const int64_t m = dims[rng() % 12], n = dims[rng() % 12], k = dims[rng() % 12];
    const int opA = int(pick({0, 1, 2, 3, -1, 4})), opB = int(pick({0, 1, 2, 3, 7}));
    const int prec = int(pick({0, 1, 2, 3, 4, -1, 5}));
    const int slices = int(pick({0, 1, 5, 8, 9, 14, 16, 20, 21, -1}));
    const unsigned ma = unsigned(rng() & 0xFF), mb = unsigned(rng() & 0xFF);
    const bool ta = opA == 1 || opA == 3, tb = opB == 1 || opB == 3;
    const int64_t ar = ta ? k : m, ac = ta ? m : k, br = tb ? n : k, bc = tb ? k : n;
    const int64_t lda = pick({ac, sat_add(ac, 1), sat_add(ac, -1), 1, 0}), ldb = pick({bc, sat_add(bc, 3), 1});
    const int64_t ldc = pick({n, sat_add(n, 2), sat_add(n, -1)});
    const int64_t stride = pick({int64_t(1) << 32, 64, 8, 4});
    bq_matrix_t A = make(ar, ac, lda, uintptr_t(1) << 44, ma, stride);
    bq_matrix_t B = make(br, bc, ldb, uintptr_t(2) << 44, mb, stride);
    bq_matrix_t C = make(m, n, ldc, uintptr_t(3) << 44, rng() % 8 ? 0xFFu : unsigned(rng() & 0xFF), stride);
    if (rng() % 50 == 0) A.comp[rng() % 8] = reinterpret_cast<double*>((uintptr_t(1) << 44) + 4);  // misaligned
    size_t res = 0, mn = 0;
    const bq_status_t ws_st = bq_gemm_workspace_size(m, n, k, ma, mb, bq_prec_t(prec), slices, &res, &mn);
    expect(ws_st >= BQ_OK && ws_st <= BQ_ERR_ARCH, "workspace_size status in range", i);
    expect(ws_st != BQ_OK || mn <= res, "streamed minimum <= resident size", i);
    const size_t pool[] = {0, 1, mn, res, res + 4096, SIZE_MAX};
    const size_t wsb = pool[rng() % 6];
    const void* ws = rng() % 10 ? reinterpret_cast<const void*>(uintptr_t(4) << 44) : nullptr;
    const bq_status_t st = bq_gemm_check(bq_op_t(opA), bq_op_t(opB), rng() % 100 ? &A : nullptr,
                                         rng() % 100 ? &B : nullptr, &C, bq_prec_t(prec), slices, ws, wsb);
    expect(st >= BQ_OK && st <= BQ_ERR_ARCH, "check status in range", i);
    const char* d = bq_last_error_detail();
    expect(d != nullptr && std::strlen(d) < 4096, "detail text", i);
    const char* s = bq_status_string(st);
    expect(s != nullptr && std::strncmp(s, "BQ_", 3) == 0, "status string", i);
    // Whatever the arguments, a call that passes validation has a workspace
    // at least as large as the query's streamed minimum.
    if (st == BQ_OK && ws_st == BQ_OK && m > 0 && n > 0 && k > 0) expect(wsb >= mn, "OK implies enough workspace", i);
    ++checked;
  }
  for (unsigned a = 0; a < 256; ++a)
    for (unsigned b = 0; b < 256; ++b) {
      const int g = bq_plan_real_gemms(a, b);
      expect(g >= 0 && g <= 24, "plan count in 0..24", a * 256 + b);
    }
  expect(bq_plan_real_gemms(0xFF, 0xFF) == 24, "24 real GEMMs for full biquaternions", 0);
  for (int s = -3; s < 12; ++s) expect(bq_status_string(bq_status_t(s)) != nullptr, "status string", s);
  std::printf("validated %lld calls, %d failures\n", checked, fails);
  return fails ? 1 : 0;
}
