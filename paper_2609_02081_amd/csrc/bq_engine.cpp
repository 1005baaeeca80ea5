// Host engine of the bilinear biquaternion GEMM: argument validation (pure
// host code, runs before anything is enqueued), planning (bilinear scheme of
// eq. bilinearH or the component-wise form, whichever needs fewer real
// GEMMs for the active components), workspace carving and kernel launches.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <fstream>
#include <sstream>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include "bq.h"
#include "bq_internal.h"

struct TraceSlot {
  hipEvent_t start, stop;
  bq_trace_record_t rec;
};

struct bq_handle_s {
  int device;
  int cu_count;
  std::string arch;
  bool trace = false;
  std::vector<TraceSlot> pending;
  rocblas_handle rb = nullptr;  // eigensolver calls; its device memory is always the caller's workspace
  void* scratch = nullptr;      // this device's static workspace of bq_gemm_noalloc
  size_t scratch_bytes = 0;
};

namespace {

thread_local std::string g_detail = "no error";

bq_status_t fail(bq_status_t s, const std::string& msg) {
  g_detail = msg;
  return s;
}

// ---------------------------------------------------------------------------
// Quaternion unit algebra (Sec. II A): units 0..3 = 1, i, j, k with
// i^2 = j^2 = k^2 = ijk = -1.  kUnitProd[u][v] = {sign, w}: e_u e_v = sign e_w.
// ---------------------------------------------------------------------------
struct UnitProd {
  int sign;
  int w;
};
constexpr UnitProd kUnitProd[4][4] = {
    {{1, 0}, {1, 1}, {1, 2}, {1, 3}},
    {{1, 1}, {-1, 0}, {1, 3}, {-1, 2}},
    {{1, 2}, {-1, 3}, {-1, 0}, {1, 1}},
    {{1, 3}, {1, 2}, {-1, 1}, {-1, 0}},
};

// eq. bilinearH: operand pairs (unit of M, unit of N) of P1..P4, their
// weights in Q1..Q4, and the Hadamard rows of P5..P8.
constexpr int kPairs[4][2] = {{0, 0}, {3, 2}, {1, 3}, {2, 1}};
constexpr double kDirectCoef[4] = {2.0, -2.0, -2.0, -2.0};
constexpr double kHad[4][4] = {{1, 1, 1, 1}, {1, 1, -1, -1}, {1, -1, 1, -1}, {1, -1, -1, 1}};
// Q_w += kHadOut[w] * 1/4 * sum_q kHad[w][q] P_{5+q}
constexpr double kHadOut[4] = {-0.25, 0.25, 0.25, 0.25};

// op(M) of an operand (Sec. III, sign rules for T, * and dagger): the unit
// coefficient M_u (u = 1, i, j, k) becomes sgn[op][u] M_u, conjugated for *
// and dagger, transposed for T and dagger.  In the component layout these
// are the per-component signs (+,+,-,+ | +,+,-,+) for T, (+,-,+,- | -,+,-,+)
// for * and (+,-,-,- | -,+,+,+) for dagger.
constexpr double kOpUnitSign[4][4] = {
    {1.0, 1.0, 1.0, 1.0},     // N
    {1.0, 1.0, -1.0, 1.0},    // T
    {1.0, -1.0, 1.0, -1.0},   // C (*)
    {1.0, -1.0, -1.0, -1.0},  // H (dagger)
};
inline bool op_conj(bq_op_t o) { return o == BQ_OP_C || o == BQ_OP_H; }
inline bool op_trans(bq_op_t o) { return o == BQ_OP_T || o == BQ_OP_H; }

struct Cplx {
  double re, im;
};
inline Cplx cmul(Cplx a, Cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

struct Operand {
  const double* r = nullptr;  // real part (nullptr = zero)
  const double* i = nullptr;  // imaginary part (nullptr = zero)
  int64_t ld = 0;
  double s = 1.0;  // operand = r + i * s * i_part
  int combo = -1;  // >= 0: Hadamard combination q, formed into the workspace
};

struct Tgt {
  int w;
  Cplx coef;
};

struct Prod {
  Operand L, R;
  std::vector<Tgt> tgts;
};

struct Plan {
  int64_t m = 0, n = 0, k = 0;  // op(A) is m x k, op(B) k x n
  bool ta = false, tb = false;  // A stored k x m, B stored n x k (op T or H)
  bool bilinear = false;
  std::vector<Prod> prods;
  bool combA_r = false, combA_i = false, combB_r = false, combB_i = false;
  double wA[4][4] = {}, wB[4][4] = {};
  int real_gemms = 0;
};

int prod_cost(const Operand& L, const Operand& R) {
  const int lparts = (L.r != nullptr) + (L.i != nullptr);
  const int rparts = (R.r != nullptr) + (R.i != nullptr);
  if (lparts == 0 || rparts == 0) return 0;
  if (lparts == 2 && rparts == 2) return 3;
  return lparts * rparts;
}

// Placeholder pointer marking "present, formed in the workspace".
const double* const kCombo = reinterpret_cast<const double*>(uintptr_t(8));

struct Problem {
  int64_t m, n, k;
  const double* a[8];
  const double* b[8];
  int64_t lda, ldb;
  bq_op_t opA, opB;
};

Plan make_plan(const Problem& P) {
  const double sA = op_conj(P.opA) ? -1.0 : 1.0;
  const double sB = op_conj(P.opB) ? -1.0 : 1.0;
  auto usA = [&](int u) { return kOpUnitSign[P.opA][u]; };
  auto usB = [&](int u) { return kOpUnitSign[P.opB][u]; };

  // Component-wise form: 16 complex products, absent ones skipped.
  Plan cw;
  for (int u = 0; u < 4; ++u)
    for (int v = 0; v < 4; ++v) {
      Prod p;
      p.L = {P.a[u], P.a[u + 4], P.lda, sA, -1};
      p.R = {P.b[v], P.b[v + 4], P.ldb, sB, -1};
      const int c = prod_cost(p.L, p.R);
      if (c == 0) continue;
      const UnitProd up = kUnitProd[u][v];
      p.tgts.push_back({up.w, {up.sign * usA(u) * usB(v), 0.0}});
      cw.real_gemms += c;
      cw.prods.push_back(p);
    }

  // Bilinear form, eq. bilinearH.
  Plan bl;
  bl.bilinear = true;
  for (int q = 0; q < 4; ++q) {
    const int u = kPairs[q][0], v = kPairs[q][1];
    Prod p;
    p.L = {P.a[u], P.a[u + 4], P.lda, sA, -1};
    p.R = {P.b[v], P.b[v + 4], P.ldb, sB, -1};
    const int c = prod_cost(p.L, p.R);
    if (c == 0) continue;
    p.tgts.push_back({q, {kDirectCoef[q] * usA(u) * usB(v), 0.0}});
    bl.real_gemms += c;
    bl.prods.push_back(p);
  }
  bool aR = false, aI = false, bR = false, bI = false;
  for (int u = 0; u < 4; ++u) {
    aR |= P.a[u] != nullptr;
    aI |= P.a[u + 4] != nullptr;
    bR |= P.b[u] != nullptr;
    bI |= P.b[u + 4] != nullptr;
  }
  for (int q = 0; q < 4; ++q) {
    Prod p;
    p.L = {aR ? kCombo : nullptr, aI ? kCombo : nullptr, 0, sA, q};
    p.R = {bR ? kCombo : nullptr, bI ? kCombo : nullptr, 0, sB, q};
    const int c = prod_cost(p.L, p.R);
    if (c == 0) continue;
    for (int w = 0; w < 4; ++w) p.tgts.push_back({w, {kHadOut[w] * kHad[w][q], 0.0}});
    bl.real_gemms += c;
    bl.prods.push_back(p);
    for (int uu = 0; uu < 4; ++uu) {
      bl.wA[q][uu] = kHad[q][uu] * usA(uu);
      bl.wB[q][uu] = kHad[q][uu] * usB(uu);
    }
  }
  bl.combA_r = aR;
  bl.combA_i = aI;
  bl.combB_r = bR;
  bl.combB_i = bI;
  Plan& best = bl.real_gemms <= cw.real_gemms ? bl : cw;
  best.m = P.m;
  best.n = P.n;
  best.k = P.k;
  best.ta = op_trans(P.opA);
  best.tb = op_trans(P.opB);
  return best;
}

// Workspace slot of one pre-combined operand: the stored orientation (op T
// and H keep it), rows padded to whole 64-byte lines.  Sized for either
// orientation, so the workspace query needs no op.
size_t combo_slot_bytes(int64_t rows, int64_t cols) {
  return std::max(size_t(rows) * size_t((cols + 7) / 8 * 8), size_t(cols) * size_t((rows + 7) / 8 * 8)) * 8;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Arithmetic of the real GEMMs: et = -1 FP64 MFMA, else the digit type of
// the split form (0 BF16, 1 FP8, 2 INT8) with S slices, or 3 for the CRT
// form with S moduli (S = 0: chosen from k by digit_default_slices or
// crt_default_moduli).
struct Prec {
  int et = -1;
  int S = 0;
};

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// CRT form: prod(p_1..p_N) > k 2^(2b + 1), exactly (32-bit limbs), i.e. the
// moduli tell apart every integer of |P| <= k 2^(2b) with |P| < M / 2.
bool crt_carries(int N, int64_t k, int b) {
  std::vector<uint64_t> P{1};
  for (int i = 0; i < N; ++i) {
    uint64_t carry = 0;
    for (uint64_t& l : P) {
      const uint64_t t = l * uint64_t(bq::crt_modulus(i)) + carry;
      l = t & 0xffffffffu;
      carry = t >> 32;
    }
    if (carry) P.push_back(carry);
  }
  const int sh = 2 * b + 1;
  std::vector<uint64_t> R(size_t(sh / 32 + 3), 0);
  const unsigned __int128 v = (unsigned __int128)uint64_t(k) << (sh % 32);
  R[sh / 32] = uint64_t(v) & 0xffffffffu;
  R[sh / 32 + 1] = uint64_t(v >> 32) & 0xffffffffu;
  R[sh / 32 + 2] = uint64_t(v >> 64) & 0xffffffffu;
  const size_t L = std::max(P.size(), R.size());
  for (size_t i = L; i-- > 0;) {
    const uint64_t a = i < P.size() ? P[i] : 0, c = i < R.size() ? R[i] : 0;
    if (a != c) return a > c;
  }
  return false;
}

// Integer bits b of the CRT form: the largest b <= 53 the N moduli carry for
// inner dimension k (0 if none).
int crt_bits(int N, int64_t k) {
  k = std::max<int64_t>(k, 1);
  double logm = 0.0;
  for (int i = 0; i < N; ++i) logm += std::log2(double(bq::crt_modulus(i)));
  int b = std::min(53, int(std::floor((logm - 1.0 - std::log2(double(k))) / 2.0)) + 1);
  while (b > 0 && !crt_carries(N, k, b)) --b;
  return std::max(b, 0);
}

// Fewest moduli that carry 53 bits for inner dimension k.
int crt_default_moduli(int64_t k) {
  for (int N = 1; N <= bq::kMaxCrtModuli; ++N)
    if (crt_bits(N, k) >= 53) return N;
  return bq::kMaxCrtModuli;
}

// Default slice count of a digit form (slices = 0).  S digits of beta bits
// under an exponent with headroom h carry beta S - h significand bits of a
// row's (column's) largest element.  The truncation of a length-k dot
// product (the dropped digit pairs and the remainders, one term per k
// element, of random sign) grows like sqrt(k) 2^-(beta S - h) times the row
// and column maxima, so the default asks for 48 + ceil(log2(k) / 2) bits:
// 55 at k = 16384, where the sampled error of the Hermitian workload is
// about 1e-13 2^(56 - bits) (below 5e-13 at 55 bits); the fewest slices
// that carry them, capped at the digit type's maximum.
int digit_default_slices(int et, int64_t k) {
  const int lg = k > 1 ? 64 - __builtin_clzll(uint64_t(k - 1)) : 0;  // ceil(log2 k)
  const int need = 48 + (lg + 1) / 2;
  const int b = bq::slice_beta(et), h = bq::slice_head(et), smax = bq::max_slices(et);
  for (int S = 1; S <= smax; ++S)
    if (b * S - h >= need) return S;
  return smax;
}

// Slices (moduli) one real product of inner dimension k uses.
int split_count(const Prec& pr, int64_t k) {
  if (pr.S != 0 || pr.et < 0) return pr.S;
  return pr.et == 3 ? crt_default_moduli(k) : digit_default_slices(pr.et, k);
}

// Largest padded k of the CRT GEMM (k is padded to 128): kp 127^2 < 2^31
// keeps the int32 sums exact.
constexpr int64_t kCrtMaxK = 133120;

// Digit buffers of one split real product (reused by every real product).
// Row length of the CRT form's residue planes (16-byte rows).
int64_t crt_ldr(int64_t n) { return round_up(n, 16); }

// The CRT form keeps the exponents and residue planes (N x m x crt_ldr(n)
// bytes) of up to kCrtProducts real products, the real products of one
// complex product, which one reconstruction pass then combines.
struct SplitLayout {
  int64_t rows_pad, cols_pad, kp;
  int S, sets;
  int digit_sets;  // 1, or sets when every real product keeps its own digits (grouped CRT plans)
  size_t a_bytes, b_bytes, ea_bytes, eb_bytes, r_bytes;  // ea, eb, r: per set
  size_t total() const {
    return size_t(digit_sets) * (a_bytes + b_bytes) + size_t(sets) * (ea_bytes + eb_bytes + r_bytes);
  }
};

SplitLayout split_layout(const Prec& pr, int64_t m, int64_t n, int64_t k, bool grouped = false) {
  SplitLayout L{};
  const int es = pr.et == 0 ? 2 : 1;
  L.S = split_count(pr, k);
  L.sets = pr.et == 3 ? bq::kCrtProducts : 1;
  L.digit_sets = (grouped && pr.et == 3) ? L.sets : 1;
  L.rows_pad = round_up(m, pr.et == 3 ? 256 : 128);
  L.cols_pad = round_up(n, pr.et == 3 ? 256 : 64);
  L.kp = round_up(k, pr.et == 3 ? 128 : 64);
  L.a_bytes = align256(size_t(L.S) * size_t(L.rows_pad) * size_t(L.kp) * es);
  L.b_bytes = align256(size_t(L.S) * size_t(L.cols_pad) * size_t(L.kp) * es);
  L.ea_bytes = align256(size_t(L.rows_pad) * 4);
  L.eb_bytes = align256(size_t(L.cols_pad) * 4);
  L.r_bytes = pr.et == 3 ? align256(size_t(L.S) * size_t(m) * size_t(crt_ldr(n))) : 0;
  return L;
}

// Size limits of a product: each dimension below 2^31 and each matrix
// (op(A) m x k, op(B) k x n, C m x n) at most 2^40 elements (8 TiB per
// block).  Within them every workspace and address computation fits 64 bits.
constexpr int64_t kMaxDim = (int64_t(1) << 31) - 1;
constexpr int64_t kMaxElems = int64_t(1) << 40;

bool too_large(int64_t m, int64_t n, int64_t k) {
  if (m > kMaxDim || n > kMaxDim || k > kMaxDim) return true;
  auto big = [](int64_t a, int64_t b) { return a > 0 && b > kMaxElems / a; };
  return big(m, k) || big(k, n) || big(m, n);
}

// Workspace: pre-combined operands of P5..P8 (packed, ld = cols), plus the
// digit buffers of one real product in the split form.
void workspace_need(const Plan& pl, const Prec& pr, int64_t m, int64_t n, int64_t k, size_t* resident,
                    size_t* minimum, bool grouped = false) {
  *resident = 0;
  *minimum = 0;
  if (m == 0 || n == 0 || k == 0) return;
  const size_t split = pr.et >= 0 ? split_layout(pr, m, n, k, grouped).total() : 0;
  bool any = false;
  for (const Prod& p : pl.prods) any |= (p.L.combo >= 0);
  if (pl.bilinear && any) {
    const size_t a1 = align256(combo_slot_bytes(m, k));
    const size_t b1 = align256(combo_slot_bytes(k, n));
    const size_t per_q = (pl.combA_r + pl.combA_i) * a1 + (pl.combB_r + pl.combB_i) * b1;
    *resident = 4 * per_q;
    *minimum = per_q;
  }
  *resident += split;
  *minimum += split;
}

bq_status_t prec_of(bq_prec_t prec, int slices, Prec* out) {
  Prec p;
  switch (prec) {
    case BQ_PREC_FP64: p.et = -1; break;
    case BQ_PREC_SPLIT_BF16: p.et = 0; break;
    case BQ_PREC_SPLIT_FP8: p.et = 1; break;
    case BQ_PREC_SPLIT_INT8: p.et = 2; break;
    case BQ_PREC_SPLIT_INT8_CRT: p.et = 3; break;
    default: return fail(BQ_ERR_INVALID_VALUE, "unknown precision");
  }
  if (slices < 0) return fail(BQ_ERR_INVALID_VALUE, "slices must be >= 0");
  if (p.et == 3) {
    if (slices > bq::kMaxCrtModuli)
      return fail(BQ_ERR_INVALID_VALUE, "moduli above " + std::to_string(bq::kMaxCrtModuli));
    p.S = slices;
  } else if (p.et >= 0) {
    p.S = slices;  // 0: chosen from k by digit_default_slices
    if (p.S > bq::max_slices(p.et))
      return fail(BQ_ERR_INVALID_VALUE, "slices above " + std::to_string(bq::max_slices(p.et)) +
                                            " for this digit type");
  }
  *out = p;
  return BQ_OK;
}

Problem problem_of(bq_op_t opA, bq_op_t opB, const bq_matrix_t* A, const bq_matrix_t* B) {
  Problem P;
  P.m = op_trans(opA) ? A->cols : A->rows;
  P.k = op_trans(opA) ? A->rows : A->cols;
  P.n = op_trans(opB) ? B->rows : B->cols;
  for (int c = 0; c < 8; ++c) {
    P.a[c] = A->comp[c];
    P.b[c] = B->comp[c];
  }
  P.lda = A->ld;
  P.ldb = B->ld;
  P.opA = opA;
  P.opB = opB;
  return P;
}

struct Range {
  uintptr_t lo, hi;
};

bool overlaps(Range a, Range b) { return a.lo < b.hi && b.lo < a.hi; }

Range block_range(const double* p, int64_t rows, int64_t cols, int64_t ld) {
  const uintptr_t lo = reinterpret_cast<uintptr_t>(p);
  const uintptr_t bytes = (uintptr_t)(((rows - 1) * ld + cols) * 8);
  return {lo, lo + bytes};
}

bool misaligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 7u) != 0; }

// Planner log (BQ_LOG=1): one line per validated call on stderr.
bool log_enabled() {
  const char* e = std::getenv("BQ_LOG");
  return e && e[0] == '1';
}

unsigned mask_of(const bq_matrix_t* M) {
  unsigned m = 0;
  for (int c = 0; c < 8; ++c) m |= (M->comp[c] != nullptr) << c;
  return m;
}

void log_plan(const Plan& pl, const Prec& pr, bq_op_t opA, bq_op_t opB, const bq_matrix_t* A,
              const bq_matrix_t* B, bool streamed, size_t ws_used) {
  static const char* kOp = "NTCH";
  static const char* kPrec[5] = {"split_bf16", "split_fp8", "split_int8", "split_int8_crt", "?"};
  const char* prec = pr.et < 0 ? "fp64" : kPrec[std::min(pr.et, 4)];
  int nprod = 0, ncombo = 0;
  for (const Prod& p : pl.prods) {
    ++nprod;
    ncombo += p.L.combo >= 0;
  }
  std::fprintf(stderr,
               "[bq] plan m=%lld n=%lld k=%lld op=%c%c maskA=0x%02x maskB=0x%02x form=%s real_gemms=%d "
               "complex_products=%d hadamard=%d prec=%s slices=%d workspace=%s %zu B\n",
               (long long)pl.m, (long long)pl.n, (long long)pl.k, kOp[opA & 3], kOp[opB & 3], mask_of(A), mask_of(B),
               pl.bilinear ? "bilinear" : "componentwise", pl.real_gemms, nprod, ncombo, prec,
               pr.et >= 0 ? split_count(pr, pl.k) : 0, streamed ? "streamed" : "resident", ws_used);
}

// Validation shared by every entry point.  out_mask: output components the
// call writes (all of them must be non-null).
bq_status_t validate(bq_op_t opA, bq_op_t opB, const bq_matrix_t* A, const bq_matrix_t* B,
                     const bq_matrix_t* C, bq_prec_t prec, int slices, const void* ws,
                     size_t ws_bytes, unsigned out_mask, Plan* plan_out, bool* streamed, Prec* prec_out,
                     bool check_ws = true) {
  if (!A || !B || !C) return fail(BQ_ERR_INVALID_VALUE, "A, B and C must be non-null");
  auto op_ok = [](bq_op_t o) { return o == BQ_OP_N || o == BQ_OP_T || o == BQ_OP_C || o == BQ_OP_H; };
  if (!op_ok(opA) || !op_ok(opB)) return fail(BQ_ERR_INVALID_VALUE, "op must be N, T, C or H");
  Prec pr;
  if (bq_status_t ps = prec_of(prec, slices, &pr); ps != BQ_OK) return ps;
  const bq_matrix_t* M[3] = {A, B, C};
  const char* nm[3] = {"A", "B", "C"};
  for (int t = 0; t < 3; ++t) {
    if (M[t]->rows < 0 || M[t]->cols < 0)
      return fail(BQ_ERR_INVALID_VALUE, std::string(nm[t]) + ": negative dimension");
    if (M[t]->ld < std::max<int64_t>(1, M[t]->cols))
      return fail(BQ_ERR_INVALID_VALUE, std::string(nm[t]) + ": ld < max(1, cols)");
    for (int c = 0; c < 8; ++c)
      if (M[t]->comp[c] && misaligned(M[t]->comp[c]))
        return fail(BQ_ERR_INVALID_VALUE, std::string(nm[t]) + ": component not 8-byte aligned");
  }
  // Kernels keep offsets inside a tile in 32 bits: 128 rows of any leading
  // dimension must span fewer than 2^32 elements.
  for (int t = 0; t < 3; ++t)
    if (M[t]->ld > (int64_t(1) << 24))
      return fail(BQ_ERR_UNSUPPORTED, std::string(nm[t]) + ": ld above 2^24 elements is not supported");
  // op(A) is m x k, op(B) is k x n.
  const int64_t m = op_trans(opA) ? A->cols : A->rows, k = op_trans(opA) ? A->rows : A->cols;
  const int64_t kb = op_trans(opB) ? B->cols : B->rows, n = op_trans(opB) ? B->rows : B->cols;
  if (k != kb) return fail(BQ_ERR_INVALID_VALUE, "inner dimensions of op(A) and op(B) differ");
  if (C->rows != m || C->cols != n) return fail(BQ_ERR_INVALID_VALUE, "C must be rows(op(A)) x cols(op(B))");
  if (too_large(m, n, k))
    return fail(BQ_ERR_UNSUPPORTED, "a dimension above 2^31 - 1 or a matrix above 2^40 elements");
  if (pr.et == 3 && k > 0) {
    if (round_up(k, 128) > kCrtMaxK)
      return fail(BQ_ERR_UNSUPPORTED, "CRT form: k above " + std::to_string(kCrtMaxK) + " is not supported");
    if (crt_bits(split_count(pr, k), k) < 1)
      return fail(BQ_ERR_INVALID_VALUE, "CRT form: too few moduli for this inner dimension");
  }
  if (C->rows > 0 && C->cols > 0)
    for (int c = 0; c < 8; ++c)
      if ((out_mask >> c & 1) && !C->comp[c])
        return fail(BQ_ERR_INVALID_VALUE, "output component " + std::to_string(c) + " is null");
  if (check_ws && ws_bytes > 0 && !ws) return fail(BQ_ERR_INVALID_VALUE, "ws is null but ws_bytes > 0");

  Plan plan = make_plan(problem_of(opA, opB, A, B));
  size_t res = 0, mn = 0;
  workspace_need(plan, pr, m, n, k, &res, &mn);
  if (check_ws && ws_bytes < mn)
    return fail(BQ_ERR_WORKSPACE, "workspace " + std::to_string(ws_bytes) + " B < minimum " + std::to_string(mn) + " B");
  const char* fs = std::getenv("BQ_FORCE_STREAMED");
  const bool force_stream = fs && fs[0] == '1';
  const bool use_stream = check_ws && ((ws_bytes < res) || (force_stream && mn < res));

  // Aliasing: output blocks against inputs, workspace and each other.
  if (m > 0 && n > 0) {
    std::vector<Range> outs;
    for (int c = 0; c < 8; ++c)
      if (out_mask >> c & 1) outs.push_back(block_range(C->comp[c], m, n, C->ld));
    std::vector<Range> ins;
    if (k > 0) {
      for (int c = 0; c < 8; ++c) {
        if (A->comp[c]) ins.push_back(block_range(A->comp[c], A->rows, A->cols, A->ld));
        if (B->comp[c]) ins.push_back(block_range(B->comp[c], B->rows, B->cols, B->ld));
      }
    }
    const size_t used_ws = use_stream ? mn : res;
    if (check_ws && ws && used_ws > 0) {
      // The part of the workspace the plan writes must not hold an input:
      // the pre-combination and the digit splits would overwrite it before
      // the GEMMs read it.
      const uintptr_t lo = reinterpret_cast<uintptr_t>(ws);
      const Range wr{lo, lo + used_ws};
      for (const Range& r : ins)
        if (overlaps(wr, r)) return fail(BQ_ERR_ALIAS, "the workspace overlaps a component of A or B");
      ins.push_back(wr);
    }
    for (size_t i = 0; i < outs.size(); ++i) {
      for (const Range& r : ins)
        if (overlaps(outs[i], r)) return fail(BQ_ERR_ALIAS, "C overlaps an input or the workspace");
      for (size_t j = i + 1; j < outs.size(); ++j)
        if (overlaps(outs[i], outs[j])) return fail(BQ_ERR_ALIAS, "two components of C overlap");
    }
  }
  if (log_enabled()) log_plan(plan, pr, opA, opB, A, B, use_stream, check_ws ? (use_stream ? mn : res) : 0);
  if (plan_out) *plan_out = std::move(plan);
  if (streamed) *streamed = use_stream;
  if (prec_out) *prec_out = pr;
  return BQ_OK;
}

// Tile order of the single-call GEMM: each XCD takes a contiguous range of
// tiles, walked in groups of 4 tile rows (at n = 16384 and 24576 groups of
// 2 and 8 are 0.7-2 % slower, of 16 5-6 %, and without the XCD ranges the
// product is 8-10 % slower).  BQ_TILE_ORDER="xcd,group" overrides.
void tile_order(int* xcd, int* group) {
  *xcd = 1;
  *group = 4;
  const char* e = std::getenv("BQ_TILE_ORDER");
  if (!e || !*e) return;
  int a = 1, b = 4;
  if (std::sscanf(e, "%d,%d", &a, &b) == 2 && b >= 1) {
    *xcd = a != 0;
    *group = b;
  }
}

// BQ_SLICE_FLUSH = f > 0 flushes the level sums at least every f k-steps
// (never less often than exactness allows).
int slice_flush(int et, int S) {
  const int bound = bq::slice_flush_steps(et, S);
  const char* e = std::getenv("BQ_SLICE_FLUSH");
  if (!e || !*e) return bound;
  const int v = std::atoi(e);
  return v > 0 ? std::min(v, bound) : bound;
}

int tile_override() {
  const char* e = std::getenv("BQ_TILE_CONFIG");
  if (!e || !*e) return -1;
  const int v = std::atoi(e);
  return (v >= 0 && v < bq::num_tile_configs() && bq::tile_config(v).bm > 0) ? v : -1;
}

bq_status_t hip_fail(hipError_t e, const char* what) {
  return fail(BQ_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Brackets one launch with events when the handle traces.
struct Tracer {
  bq_handle_t h;
  hipStream_t s;
  TraceSlot slot{};
  bool on = false;
  Tracer(bq_handle_t hh, hipStream_t ss, int kernel, int cfg, int64_t m, int64_t n, int64_t k, double flops,
         double bytes)
      : h(hh), s(ss) {
    if (!h || !h->trace) return;
    if (hipEventCreate(&slot.start) != hipSuccess) return;
    if (hipEventCreate(&slot.stop) != hipSuccess) {
      (void)hipEventDestroy(slot.start);
      return;
    }
    slot.rec = {kernel, cfg, m, n, k, 0.0, flops, bytes};
    on = hipEventRecord(slot.start, s) == hipSuccess;
  }
  void done() {
    if (!on) return;
    if (hipEventRecord(slot.stop, s) == hipSuccess) {
      h->pending.push_back(slot);
    } else {
      (void)hipEventDestroy(slot.start);
      (void)hipEventDestroy(slot.stop);
    }
    on = false;
  }
};

// Launch arguments of one problem's CRT sequence, collected instead of
// launched (grouped CRT plans run each stage of every problem in one
// launch).  round: index of the complex product in the plan.
struct CrtRecord {
  struct Split { bq::CrtSplitItem it; int N, round; };
  struct Gemm { bq::CrtGemmItem it; int round; };
  struct Comb { bq::CrtCombineArgs c; int N, round; };
  struct Fill { double* p; int64_t rows, cols, ld; };
  std::vector<bq::CombineArgs> pre;  // Hadamard pre-combinations
  std::vector<Split> splits;
  std::vector<Gemm> gemms;
  std::vector<Comb> combs;
  std::vector<Fill> fills;
  int rounds = 0;
};

// Enqueue the plan.  Validation has passed.  With rec (CRT form only) the
// launches are recorded, not made, and every real product of a complex
// product keeps its own digit buffers.
bq_status_t execute(bq_handle_t h, const Plan& pl, const Prec& pr, const bq_matrix_t* A, const bq_matrix_t* B,
                    bq_matrix_t* C, unsigned out_mask, void* ws, bool streamed, hipStream_t s,
                    CrtRecord* rec = nullptr) {
  const int64_t m = pl.m, n = pl.n, k = pl.k;
  if (m == 0 || n == 0) return BQ_OK;
  bool touched[8] = {};
  const int cfg_override = tile_override();

  // Workspace slots for the pre-combined operands, in the operands' stored
  // orientation (rows padded to whole 64-byte lines so the GEMM takes its
  // aligned 16-byte load path).
  const int64_t kpad = round_up(k, 8), npad = round_up(n, 8), mpad = round_up(m, 8);
  const size_t a1 = align256(combo_slot_bytes(m, k));
  const size_t b1 = align256(combo_slot_bytes(k, n));
  char* wp = static_cast<char*>(ws);
  double* cA_r[4] = {};
  double* cA_i[4] = {};
  double* cB_r[4] = {};
  double* cB_i[4] = {};
  const int nslot = streamed ? 1 : 4;
  for (int q = 0; q < nslot && k > 0; ++q) {
    if (pl.combA_r) { cA_r[q] = reinterpret_cast<double*>(wp); wp += a1; }
    if (pl.combA_i) { cA_i[q] = reinterpret_cast<double*>(wp); wp += a1; }
    if (pl.combB_r) { cB_r[q] = reinterpret_cast<double*>(wp); wp += b1; }
    if (pl.combB_i) { cB_i[q] = reinterpret_cast<double*>(wp); wp += b1; }
  }
  // Digit buffers of the split form.
  SplitLayout sl{};
  void* dig_a = nullptr;
  void* dig_b = nullptr;
  int* exp_a = nullptr;
  int* exp_b = nullptr;
  int* crt_ea[bq::kCrtProducts] = {};
  int* crt_eb[bq::kCrtProducts] = {};
  signed char* crt_res[bq::kCrtProducts] = {};
  void* crt_da[bq::kCrtProducts] = {};
  void* crt_db[bq::kCrtProducts] = {};
  if (pr.et >= 0 && k > 0) {
    sl = split_layout(pr, m, n, k, rec != nullptr);
    for (int q = 0; q < sl.digit_sets; ++q) {
      crt_da[q] = wp; wp += sl.a_bytes;
      crt_db[q] = wp; wp += sl.b_bytes;
    }
    dig_a = crt_da[0];
    dig_b = crt_db[0];
    for (int q = 0; q < sl.sets; ++q) {
      crt_ea[q] = reinterpret_cast<int*>(wp); wp += sl.ea_bytes;
      crt_eb[q] = reinterpret_cast<int*>(wp); wp += sl.eb_bytes;
      crt_res[q] = reinterpret_cast<signed char*>(wp); wp += sl.r_bytes;
    }
    exp_a = crt_ea[0];
    exp_b = crt_eb[0];
  }
  const bool crt = pr.et == 3;
  const int es = pr.et == 0 ? 2 : 1;
  const int S = sl.S;  // slices, or moduli of the CRT form, for this k
  const int beta = crt ? crt_bits(S, k) : (pr.et >= 0 ? bq::slice_beta(pr.et) : 0);
  const int head = (pr.et >= 0 && !crt) ? bq::slice_head(pr.et) : 0;

  // One real product T = X Y of the split form, X = xw1 x1 + xw2 x2 (m x k),
  // Y = yw1 y1 + yw2 y2 (k x n); C_w op= cw * T for each (w, cw).
  auto split_product = [&](const double* x1, double xw1, const double* x2, double xw2, int64_t ldx,
                           const double* y1, double yw1, const double* y2, double yw2, int64_t ldy,
                           const std::vector<std::pair<int, double>>& outs) -> hipError_t {
    bq::SliceGemmArgs sg{};
    for (const auto& o : outs) {
      if (!(out_mask >> o.first & 1) || o.second == 0.0) continue;
      sg.c[sg.ntgt] = C->comp[o.first];
      sg.coef[sg.ntgt] = o.second;
      sg.mode[sg.ntgt] = touched[o.first] ? bq::TGT_ACCUM : bq::TGT_WRITE;
      touched[o.first] = true;
      ++sg.ntgt;
    }
    if (sg.ntgt == 0) return hipSuccess;
    // The left factor takes one exponent per row of op(A): along the stored
    // rows (row kernels) for N and C, along the stored columns (column
    // kernels, which also transpose the digits) for T and H; the right factor
    // the other way round.
    bq::SplitArgs xa = pl.ta ? bq::SplitArgs{x1, x2, xw1, xw2, ldx, k, m, 0, sl.rows_pad, sl.kp,
                                             sl.rows_pad * sl.kp, beta, head, 0}
                             : bq::SplitArgs{x1, x2, xw1, xw2, ldx, m, k, sl.rows_pad, 0, sl.kp,
                                             sl.rows_pad * sl.kp, beta, head, 1};
    bq::SplitArgs ya = pl.tb ? bq::SplitArgs{y1, y2, yw1, yw2, ldy, n, k, sl.cols_pad, 0, sl.kp,
                                             sl.cols_pad * sl.kp, beta, head, 1}
                             : bq::SplitArgs{y1, y2, yw1, yw2, ldy, k, n, 0, sl.cols_pad, sl.kp,
                                             sl.cols_pad * sl.kp, beta, head, 0};
    const double elems_x = double(m) * double(k), elems_y = double(k) * double(n);
    {
      Tracer tr(h, s, BQ_KERNEL_SPLIT, -1, m, k, 0, 0.0,
                elems_x * 8.0 * (x2 ? 2 : 1) * 2.0 + double(sl.rows_pad) * double(sl.kp) * S * es);
      hipError_t e = bq::launch_split(pr.et, S, xa, exp_a, dig_a, s);
      tr.done();
      if (e != hipSuccess) return e;
    }
    {
      Tracer tr(h, s, BQ_KERNEL_SPLIT, -1, k, n, 0, 0.0,
                elems_y * 8.0 * (y2 ? 2 : 1) * 2.0 + double(sl.cols_pad) * double(sl.kp) * S * es);
      hipError_t e = bq::launch_split(pr.et, S, ya, exp_b, dig_b, s);
      tr.done();
      if (e != hipSuccess) return e;
    }
    sg.a = dig_a;
    sg.b = dig_b;
    sg.slice_stride_a = sl.rows_pad * sl.kp;
    sg.slice_stride_b = sl.cols_pad * sl.kp;
    sg.kp = sl.kp;
    sg.ea = exp_a;
    sg.eb = exp_b;
    sg.m = m;
    sg.n = n;
    sg.beta = beta;
    sg.kflush = slice_flush(pr.et, S);
    sg.ldc = C->ld;
    const double pairs = double(S) * double(S + 1) / 2.0;
    Tracer tr(h, s, BQ_KERNEL_SLICE_GEMM, S, m, n, k, pairs * 2.0 * double(m) * double(n) * double(k), 0.0);
    hipError_t e = bq::launch_slice_gemm(pr.et, S, sg, s);
    tr.done();
    return e;
  };

  // CRT form: one real product T = X Y into residue set q (exponents and
  // residue planes of its INT8 GEMMs); crt_combine reconstructs it.
  const int64_t ldr = crt_ldr(n);
  int round = 0;  // complex product being enqueued (recorded launches carry it)
  auto crt_product = [&](const double* x1, const double* x2, double xw2, int64_t ldx, const double* y1,
                         const double* y2, double yw2, int64_t ldy, int q) -> hipError_t {
    bq::SplitArgs xa = pl.ta ? bq::SplitArgs{x1, x2, 1.0, xw2, ldx, k, m, 0, sl.rows_pad, sl.kp,
                                             sl.rows_pad * sl.kp, beta, 0, 0}
                             : bq::SplitArgs{x1, x2, 1.0, xw2, ldx, m, k, sl.rows_pad, 0, sl.kp,
                                             sl.rows_pad * sl.kp, beta, 0, 1};
    bq::SplitArgs ya = pl.tb ? bq::SplitArgs{y1, y2, 1.0, yw2, ldy, n, k, sl.cols_pad, 0, sl.kp,
                                             sl.cols_pad * sl.kp, beta, 0, 1}
                             : bq::SplitArgs{y1, y2, 1.0, yw2, ldy, k, n, 0, sl.cols_pad, sl.kp,
                                             sl.cols_pad * sl.kp, beta, 0, 0};
    if (rec) {
      const int dq = sl.digit_sets > 1 ? q : 0;
      rec->splits.push_back({{xa, crt_ea[q], crt_da[dq]}, S, round});
      rec->splits.push_back({{ya, crt_eb[q], crt_db[dq]}, S, round});
      rec->gemms.push_back({{{crt_da[dq], crt_db[dq], sl.rows_pad * sl.kp, sl.cols_pad * sl.kp, sl.kp, m, n,
                              crt_res[q], m * ldr, ldr},
                             S},
                            round});
      return hipSuccess;
    }
    {
      Tracer tr(h, s, BQ_KERNEL_SPLIT, -1, m, k, 0, 0.0,
                double(m) * double(k) * 8.0 * (x2 ? 2 : 1) * 2.0 + double(sl.rows_pad) * double(sl.kp) * S);
      hipError_t e = bq::launch_crt_split(S, xa, crt_ea[q], dig_a, s);
      tr.done();
      if (e != hipSuccess) return e;
    }
    {
      Tracer tr(h, s, BQ_KERNEL_SPLIT, -1, k, n, 0, 0.0,
                double(k) * double(n) * 8.0 * (y2 ? 2 : 1) * 2.0 + double(sl.cols_pad) * double(sl.kp) * S);
      hipError_t e = bq::launch_crt_split(S, ya, crt_eb[q], dig_b, s);
      tr.done();
      if (e != hipSuccess) return e;
    }
    const bq::CrtGemmArgs cg{dig_a, dig_b, sl.rows_pad * sl.kp, sl.cols_pad * sl.kp, sl.kp, m, n,
                             crt_res[q], m * ldr, ldr};
    Tracer tr(h, s, BQ_KERNEL_CRT_GEMM, S, m, n, k, double(S) * 2.0 * double(m) * double(n) * double(k), 0.0);
    hipError_t e = bq::launch_crt_gemm(S, cg, s);
    tr.done();
    return e;
  };

  auto combine = [&](bool left, int q0, int nq, int slot0) -> hipError_t {
    bq::CombineArgs ca{};
    const bq_matrix_t* X = left ? A : B;
    for (int c = 0; c < 8; ++c) ca.src[c] = X->comp[c];
    ca.lds = X->ld;
    ca.rows = X->rows;
    ca.cols = X->cols;
    ca.ldd = left ? (pl.ta ? mpad : kpad) : (pl.tb ? kpad : npad);
    ca.nq = nq;
    int nsrc = 0, ndst = 0;
    for (int c = 0; c < 8; ++c) nsrc += (ca.src[c] != nullptr);
    for (int j = 0; j < nq; ++j) {
      ca.dst_r[j] = left ? cA_r[slot0 + j] : cB_r[slot0 + j];
      ca.dst_i[j] = left ? cA_i[slot0 + j] : cB_i[slot0 + j];
      ndst += (ca.dst_r[j] != nullptr) + (ca.dst_i[j] != nullptr);
      for (int u = 0; u < 4; ++u) ca.w[j][u] = left ? pl.wA[q0 + j][u] : pl.wB[q0 + j][u];
    }
    if (rec) {
      rec->pre.push_back(ca);
      return hipSuccess;
    }
    Tracer tr(h, s, BQ_KERNEL_COMBINE, -1, ca.rows, ca.cols, 0, 0.0,
              double(nsrc + ndst) * double(ca.rows) * double(ca.cols) * 8.0);
    hipError_t e = bq::launch_combine(ca, s);
    tr.done();
    return e;
  };

  if (k > 0 && pl.bilinear && !streamed) {
    hipError_t e = combine(true, 0, 4, 0);
    if (e == hipSuccess) e = combine(false, 0, 4, 0);
    if (e != hipSuccess) return hip_fail(e, "pre-combination launch");
  }

  for (const Prod& p : pl.prods) {
    if (k == 0) break;
    if (&p != &pl.prods.front()) ++round;
    if (rec) rec->rounds = std::max(rec->rounds, round + 1);  // the longest plan of the batch
    Operand L = p.L, R = p.R;
    if (L.combo >= 0) {
      const int slot = streamed ? 0 : L.combo;
      if (streamed) {
        hipError_t e = combine(true, L.combo, 1, 0);
        if (e == hipSuccess) e = combine(false, R.combo, 1, 0);
        if (e != hipSuccess) return hip_fail(e, "pre-combination launch");
      }
      L.r = L.r ? cA_r[slot] : nullptr;
      L.i = L.i ? cA_i[slot] : nullptr;
      L.ld = pl.ta ? mpad : kpad;
      R.r = R.r ? cB_r[slot] : nullptr;
      R.i = R.i ? cB_i[slot] : nullptr;
      R.ld = pl.tb ? kpad : npad;
    }
    // Imaginary-only operands: (i s x) as a real operand x times i s.
    Cplx rot = {1.0, 0.0};
    if (!L.r && L.i) { rot = cmul(rot, {0.0, L.s}); L.r = L.i; L.i = nullptr; }
    if (!R.r && R.i) { rot = cmul(rot, {0.0, R.s}); R.r = R.i; R.i = nullptr; }
    int kind;
    if (L.i && R.i) kind = bq::KIND_GAUSS;
    else if (R.i) kind = bq::KIND_RC;
    else if (L.i) kind = bq::KIND_CR;
    else kind = bq::KIND_RR;
    const bool pr_nz = true;
    const bool pi_nz = (kind != bq::KIND_RR);

    if (pr.et >= 0) {
      // Split form: the complex product as its real products, each added into
      // C with the coefficients it carries through P_R, P_I and the targets.
      struct RealProd {
        const double *x1, *x2;
        double xw2;
        const double *y1, *y2;
        double yw2;
        double aR, aI;  // P_R += aR T, P_I += aI T
      };
      std::vector<RealProd> rps;
      const double sig = L.s * R.s;
      if (kind == bq::KIND_GAUSS) {
        rps.push_back({L.r, nullptr, 0.0, R.r, nullptr, 0.0, 1.0, -1.0});
        rps.push_back({L.i, nullptr, 0.0, R.i, nullptr, 0.0, -sig, -sig});
        rps.push_back({L.r, L.i, L.s, R.r, R.i, R.s, 0.0, 1.0});
      } else if (kind == bq::KIND_RC) {
        rps.push_back({L.r, nullptr, 0.0, R.r, nullptr, 0.0, 1.0, 0.0});
        rps.push_back({L.r, nullptr, 0.0, R.i, nullptr, 0.0, 0.0, R.s});
      } else if (kind == bq::KIND_CR) {
        rps.push_back({L.r, nullptr, 0.0, R.r, nullptr, 0.0, 1.0, 0.0});
        rps.push_back({L.i, nullptr, 0.0, R.r, nullptr, 0.0, 0.0, L.s});
      } else {
        rps.push_back({L.r, nullptr, 0.0, R.r, nullptr, 0.0, 1.0, 0.0});
      }
      if (crt) {
        // The real products of this complex product into residue sets, then
        // one reconstruction pass: target q takes sum_p coef[q][p] T_p.
        bq::CrtCombineArgs cc{};
        int slot_of[8];
        for (int w = 0; w < 8; ++w) slot_of[w] = -1;
        std::vector<int> used;
        for (size_t pi = 0; pi < rps.size(); ++pi) {
          const RealProd& rp = rps[pi];
          const int col = (int)used.size();
          bool any = false;
          for (const Tgt& t : p.tgts) {
            const Cplx c = cmul(t.coef, rot);
            const int ws[2] = {t.w, t.w + 4};
            const double vs[2] = {c.re * rp.aR - c.im * rp.aI, c.re * rp.aI + c.im * rp.aR};
            for (int u = 0; u < 2; ++u) {
              if (!(out_mask >> ws[u] & 1) || vs[u] == 0.0) continue;
              if (slot_of[ws[u]] < 0) {
                slot_of[ws[u]] = cc.ntgt;
                cc.c[cc.ntgt++] = C->comp[ws[u]];
              }
              cc.coef[slot_of[ws[u]]][col] += vs[u];
              any = true;
            }
          }
          if (any) used.push_back((int)pi);
        }
        if (cc.ntgt == 0) continue;
        for (size_t q = 0; q < used.size(); ++q) {
          const RealProd& rp = rps[used[q]];
          hipError_t e = crt_product(rp.x1, rp.x2, rp.xw2, L.ld, rp.y1, rp.y2, rp.yw2, R.ld, (int)q);
          if (e != hipSuccess) return hip_fail(e, "split-precision launch");
          cc.res[q] = crt_res[q];
          cc.ea[q] = crt_ea[q];
          cc.eb[q] = crt_eb[q];
        }
        cc.np = (int)used.size();
        for (int w = 0; w < 8; ++w) {
          if (slot_of[w] < 0) continue;
          cc.mode[slot_of[w]] = touched[w] ? bq::TGT_ACCUM : bq::TGT_WRITE;
          touched[w] = true;
        }
        cc.plane_r = m * ldr;
        cc.ldr = ldr;
        cc.m = m;
        cc.n = n;
        cc.bits = beta;
        cc.ldc = C->ld;
        if (rec) {
          rec->combs.push_back({cc, S, round});
          continue;
        }
        int rw = 0;
        for (int q = 0; q < cc.ntgt; ++q) rw += cc.mode[q] == bq::TGT_ACCUM ? 2 : 1;
        Tracer tr(h, s, BQ_KERNEL_CRT_COMBINE, S, m, n, 0, 0.0,
                  double(m) * double(n) * (double(S) * cc.np + 8.0 * rw));
        hipError_t e = bq::launch_crt_combine(S, cc, s);
        tr.done();
        if (e != hipSuccess) return hip_fail(e, "split-precision launch");
        continue;
      }
      for (const RealProd& rp : rps) {
        std::vector<std::pair<int, double>> outs;
        for (const Tgt& t : p.tgts) {
          const Cplx c = cmul(t.coef, rot);
          outs.push_back({t.w, c.re * rp.aR - c.im * rp.aI});
          outs.push_back({t.w + 4, c.re * rp.aI + c.im * rp.aR});
        }
        hipError_t e = split_product(rp.x1, 1.0, rp.x2, rp.xw2, L.ld, rp.y1, 1.0, rp.y2, rp.yw2, R.ld, outs);
        if (e != hipSuccess) return hip_fail(e, "split-precision launch");
      }
      continue;
    }

    bq::GemmArgs g{};
    g.lr = L.r; g.li = L.i; g.lda = L.ld;
    g.rr = R.r; g.ri = R.i; g.ldb = R.ld;
    g.m = m; g.n = n; g.k = k;
    g.ta = pl.ta; g.tb = pl.tb;
    g.sL = L.s; g.sR = R.s;
    g.ldc = C->ld;
    g.ntgt = 0;
    tile_order(&g.xcd_remap, &g.group_m);
    auto al16 = [](const double* q) { return q == nullptr || (reinterpret_cast<uintptr_t>(q) & 15u) == 0; };
    g.vec = (g.lda % 2 == 0) && (g.ldb % 2 == 0) && al16(g.lr) && al16(g.li) && al16(g.rr) && al16(g.ri);
    for (const Tgt& t : p.tgts) {
      const Cplx c = cmul(t.coef, rot);
      const bool out_r = (c.re != 0.0 && pr_nz) || (c.im != 0.0 && pi_nz);
      const bool out_i = (c.re != 0.0 && pi_nz) || (c.im != 0.0 && pr_nz);
      bq::Target T{};
      T.ar = c.re;
      T.ai = c.im;
      T.cr = C->comp[t.w];
      T.ci = C->comp[t.w + 4];
      const bool want_r = out_r && (out_mask >> t.w & 1);
      const bool want_i = out_i && (out_mask >> (t.w + 4) & 1);
      T.mode_r = want_r ? (touched[t.w] ? bq::TGT_ACCUM : bq::TGT_WRITE) : bq::TGT_SKIP;
      T.mode_i = want_i ? (touched[t.w + 4] ? bq::TGT_ACCUM : bq::TGT_WRITE) : bq::TGT_SKIP;
      if (want_r) touched[t.w] = true;
      if (want_i) touched[t.w + 4] = true;
      if (T.mode_r == bq::TGT_SKIP && T.mode_i == bq::TGT_SKIP) continue;
      g.tgt[g.ntgt++] = T;
    }
    if (g.ntgt == 0) continue;
    const int cfg = bq::tile_config_for(kind, cfg_override, m, n, k);
    const int nprod = kind == bq::KIND_GAUSS ? 3 : (kind == bq::KIND_RR ? 1 : 2);
    Tracer tr(h, s, kind, cfg, m, n, k, double(nprod) * 2.0 * double(m) * double(n) * double(k), 0.0);
    hipError_t e = bq::launch_cgemm(kind, g, cfg, s);
    tr.done();
    if (e != hipSuccess) return hip_fail(e, "GEMM launch");
  }
  for (int c = 0; c < 8; ++c) {
    if ((out_mask >> c & 1) && !touched[c]) {
      if (rec) {
        rec->fills.push_back({C->comp[c], m, n, C->ld});
        continue;
      }
      Tracer tr(h, s, BQ_KERNEL_FILL, -1, m, n, 0, 0.0, double(m) * double(n) * 8.0);
      hipError_t e = bq::launch_fill_zero(C->comp[c], m, n, C->ld, s);
      tr.done();
      if (e != hipSuccess) return hip_fail(e, "zero-fill launch");
    }
  }
  return BQ_OK;
}

bq_status_t check_handle(bq_handle_t h) {
  if (!h) return fail(BQ_ERR_INVALID_VALUE, "handle is null");
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (cur != h->device) {
    e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  }
  return BQ_OK;
}

bq_status_t run(bq_handle_t h, bq_op_t opA, bq_op_t opB, const bq_matrix_t* A, const bq_matrix_t* B,
                bq_matrix_t* C, bq_prec_t prec, int slices, void* ws, size_t ws_bytes, unsigned out_mask,
                bq_stream_t stream) {
  if (!h) return fail(BQ_ERR_INVALID_VALUE, "handle is null");
  Plan plan;
  Prec pr;
  bool streamed = false;
  bq_status_t st = validate(opA, opB, A, B, C, prec, slices, ws, ws_bytes, out_mask, &plan, &streamed, &pr);
  if (st != BQ_OK) return st;
  st = check_handle(h);
  if (st != BQ_OK) return st;
  return execute(h, plan, pr, A, B, C, out_mask, ws, streamed, static_cast<hipStream_t>(stream));
}

bq_matrix_t restrict_to(const bq_matrix_t* X, unsigned mask) {
  bq_matrix_t Y = *X;
  for (int c = 0; c < 8; ++c)
    if (!(mask >> c & 1)) Y.comp[c] = nullptr;
  return Y;
}

}  // namespace

extern "C" {

bq_status_t bq_create(bq_handle_t* h, int device) {
  if (!h) return fail(BQ_ERR_INVALID_VALUE, "h is null");
  *h = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (device < 0 || device >= count) return fail(BQ_ERR_INVALID_VALUE, "device out of range");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(BQ_ERR_ARCH, std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
  bq_handle_s* hh = new bq_handle_s;
  hh->device = device;
  hh->cu_count = prop.multiProcessorCount;
  hh->arch = prop.gcnArchName;
  // The eigensolver's handle lives on the same device.
  int prev = -1;
  (void)hipGetDevice(&prev);
  if ((e = hipSetDevice(device)) != hipSuccess) {
    delete hh;
    return hip_fail(e, "hipSetDevice");
  }
  const rocblas_status rs = rocblas_create_handle(&hh->rb);
  // The static workspace of bq_gemm_noalloc: its device address on this
  // device, looked up with the device current.
  const hipError_t se = bq::noalloc_scratch(device, &hh->scratch, &hh->scratch_bytes);
  if (prev >= 0) (void)hipSetDevice(prev);
  if (rs != rocblas_status_success) {
    delete hh;
    return fail(BQ_ERR_HIP, "rocblas_create_handle failed");
  }
  if (se != hipSuccess) {
    (void)rocblas_destroy_handle(hh->rb);
    delete hh;
    return hip_fail(se, "static workspace lookup");
  }
  *h = hh;
  return BQ_OK;
}

bq_status_t bq_destroy(bq_handle_t h) {
  if (h) {
    for (TraceSlot& t : h->pending) {
      (void)hipEventDestroy(t.start);
      (void)hipEventDestroy(t.stop);
    }
    if (h->rb) (void)rocblas_destroy_handle(h->rb);
  }
  delete h;
  return BQ_OK;
}

bq_status_t bq_trace_enable(bq_handle_t h, int enable) {
  if (!h) return fail(BQ_ERR_INVALID_VALUE, "handle is null");
  h->trace = enable != 0;
  return BQ_OK;
}

bq_status_t bq_trace_read(bq_handle_t h, bq_trace_record_t* recs, int cap, int* count) {
  if (!h || !count || cap < 0 || (cap > 0 && !recs)) return fail(BQ_ERR_INVALID_VALUE, "bad trace_read argument");
  const int ncopy = std::min<int>(cap, (int)h->pending.size());
  for (int i = 0; i < ncopy; ++i) {
    TraceSlot& t = h->pending[i];
    hipError_t e = hipEventSynchronize(t.stop);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.start, t.stop);
    if (e != hipSuccess) return hip_fail(e, "trace event");
    recs[i] = t.rec;
    recs[i].ms = ms;
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  h->pending.erase(h->pending.begin(), h->pending.begin() + ncopy);
  *count = ncopy;
  return BQ_OK;
}

const char* bq_status_string(bq_status_t s) {
  switch (s) {
    case BQ_OK: return "BQ_OK";
    case BQ_ERR_INVALID_VALUE: return "BQ_ERR_INVALID_VALUE";
    case BQ_ERR_UNSUPPORTED: return "BQ_ERR_UNSUPPORTED";
    case BQ_ERR_ALIAS: return "BQ_ERR_ALIAS";
    case BQ_ERR_WORKSPACE: return "BQ_ERR_WORKSPACE";
    case BQ_ERR_HIP: return "BQ_ERR_HIP";
    case BQ_ERR_ARCH: return "BQ_ERR_ARCH";
  }
  return "BQ_ERR_UNKNOWN";
}

const char* bq_last_error_detail(void) { return g_detail.c_str(); }

bq_status_t bq_gemm_workspace_size(int64_t m, int64_t n, int64_t k, unsigned maskA, unsigned maskB,
                                   bq_prec_t prec, int slices, size_t* resident_bytes, size_t* min_bytes) {
  if (m < 0 || n < 0 || k < 0) return fail(BQ_ERR_INVALID_VALUE, "negative dimension");
  if (too_large(m, n, k))
    return fail(BQ_ERR_UNSUPPORTED, "a dimension above 2^31 - 1 or a matrix above 2^40 elements");
  if (maskA > 0xFFu || maskB > 0xFFu) return fail(BQ_ERR_INVALID_VALUE, "mask has bits above 7");
  Prec pr;
  if (bq_status_t ps = prec_of(prec, slices, &pr); ps != BQ_OK) return ps;
  Problem P{};
  P.m = m; P.n = n; P.k = k;
  const double* present = kCombo;
  for (int c = 0; c < 8; ++c) {
    P.a[c] = (maskA >> c & 1) ? present : nullptr;
    P.b[c] = (maskB >> c & 1) ? present : nullptr;
  }
  P.lda = std::max<int64_t>(1, k);
  P.ldb = std::max<int64_t>(1, n);
  Plan pl = make_plan(P);
  size_t res = 0, mn = 0;
  workspace_need(pl, pr, m, n, k, &res, &mn);
  if (resident_bytes) *resident_bytes = res;
  if (min_bytes) *min_bytes = mn;
  return BQ_OK;
}

int bq_plan_real_gemms(unsigned maskA, unsigned maskB) {
  Problem P{};
  P.m = P.n = P.k = 1;
  for (int c = 0; c < 8; ++c) {
    P.a[c] = (maskA >> c & 1) ? kCombo : nullptr;
    P.b[c] = (maskB >> c & 1) ? kCombo : nullptr;
  }
  P.lda = P.ldb = 1;
  return make_plan(P).real_gemms;
}

bq_status_t bq_gemm_check(bq_op_t opA, bq_op_t opB, const bq_matrix_t* A, const bq_matrix_t* B,
                          const bq_matrix_t* C, bq_prec_t prec, int slices, const void* ws, size_t ws_bytes) {
  return validate(opA, opB, A, B, C, prec, slices, ws, ws_bytes, 0xFFu, nullptr, nullptr, nullptr);
}

bq_status_t bq_gemm(bq_handle_t h, bq_op_t opA, bq_op_t opB, const bq_matrix_t* A, const bq_matrix_t* B,
                    bq_matrix_t* C, bq_prec_t prec, int slices, void* ws, size_t ws_bytes, bq_stream_t stream) {
  return run(h, opA, opB, A, B, C, prec, slices, ws, ws_bytes, 0xFFu, stream);
}

bq_status_t bq_gemm_noalloc(bq_handle_t h, bq_op_t opA, bq_op_t opB, const bq_matrix_t* A, const bq_matrix_t* B,
                            bq_matrix_t* C, bq_prec_t prec, int slices, bq_stream_t stream) {
  if (!h) return fail(BQ_ERR_INVALID_VALUE, "handle is null");
  if (!h->scratch) return fail(BQ_ERR_HIP, "no static workspace on this device");
  const bq_status_t st = run(h, opA, opB, A, B, C, prec, slices, h->scratch, h->scratch_bytes, 0xFFu, stream);
  if (st == BQ_ERR_WORKSPACE)
    return fail(st, "bq_gemm_noalloc: " + g_detail + "; the static workspace holds " +
                        std::to_string(h->scratch_bytes) + " B");
  return st;
}

// The subalgebra entry points: bq_gemm with the inputs and the output
// restricted to the algebra's components (the others are neither read nor
// written and may be NULL).
static bq_status_t run_sub(bq_handle_t h, bq_op_t opA, bq_op_t opB, const bq_matrix_t* A, const bq_matrix_t* B,
                           bq_matrix_t* C, bq_prec_t prec, int slices, void* ws, size_t ws_bytes, unsigned mask,
                           bq_stream_t stream) {
  if (!A || !B || !C) return fail(BQ_ERR_INVALID_VALUE, "A, B and C must be non-null");
  bq_matrix_t a = restrict_to(A, mask), b = restrict_to(B, mask), c = restrict_to(C, mask);
  return run(h, opA, opB, &a, &b, &c, prec, slices, ws, ws_bytes, mask, stream);
}

bq_status_t bq_re_gemm(bq_handle_t h, bq_op_t opA, bq_op_t opB, const bq_matrix_t* A, const bq_matrix_t* B,
                       bq_matrix_t* C, bq_prec_t prec, int slices, void* ws, size_t ws_bytes, bq_stream_t stream) {
  return run_sub(h, opA, opB, A, B, C, prec, slices, ws, ws_bytes, BQ_MASK_REAL, stream);
}

bq_status_t bq_cx_gemm(bq_handle_t h, bq_op_t opA, bq_op_t opB, const bq_matrix_t* A, const bq_matrix_t* B,
                       bq_matrix_t* C, bq_prec_t prec, int slices, void* ws, size_t ws_bytes, bq_stream_t stream) {
  return run_sub(h, opA, opB, A, B, C, prec, slices, ws, ws_bytes, BQ_MASK_COMPLEX, stream);
}

bq_status_t bq_rq_gemm(bq_handle_t h, bq_op_t opA, bq_op_t opB, const bq_matrix_t* A, const bq_matrix_t* B,
                       bq_matrix_t* C, bq_prec_t prec, int slices, void* ws, size_t ws_bytes, bq_stream_t stream) {
  return run_sub(h, opA, opB, A, B, C, prec, slices, ws, ws_bytes, BQ_MASK_REAL_QUATERNION, stream);
}

}  // extern "C"

// ===========================================================================
// Batched form (grouped plans)
// ===========================================================================
struct bq_grouped_plan_s {
  bq_handle_t h = nullptr;
  int count = 0;
  Prec pr;
  std::vector<bq_problem_t> probs;
  std::vector<Plan> plans;
  std::vector<size_t> ws_off;  // FP64 and CRT: each problem's own workspace region
  size_t ws_bytes = 0;
  void* d_crt = nullptr;  // CRT: item tables of the grouped launches
  size_t crt_bytes = 0;
  bq::GemmArgs* d_prods = nullptr;
  bq::GroupedItem* d_items = nullptr;
  int* d_counter = nullptr;
  bq::CombineArgs* d_comb = nullptr;
  int64_t* d_prefix = nullptr;
  bq::CombineArgs* d_ht = nullptr;  // per-product schedule: Hadamard sums of P5..P8, one per problem
  int64_t* d_ht_prefix = nullptr;
  int nitems = 0;
  int ncomb = 0;
  int64_t total_rows = 0;
  std::vector<int> order;  // problems, largest work first
  int cfg = 0;
  int dyn = 3;  // schedule bits: 1 = device work counter (else cyclic), 2 = one launch per complex product
  std::vector<int> round_off, round_n;  // per complex product: its items after the nitems per-tile ones
  int ops = -1;  // 0..3: every problem has (ta, tb) = (ops >> 1, ops & 1); -1: they differ
  int blocks = 0;
  double flops = 0.0;
  void* bound_ws = nullptr;
  bool bound = false;
  hipStream_t cap = nullptr;
  hipGraphExec_t exec = nullptr;
  std::string tune_key;
};

namespace {

constexpr int kGroupedTile = 64;  // every grouped tile configuration is 64 x 64

void grouped_release_graph(bq_grouped_plan_t p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  p->exec = nullptr;
  p->bound = false;
}

std::string tune_cache_path() {
  const char* e = std::getenv("BQ_TUNE_CACHE");
  return e ? std::string(e) : std::string();
}

bool tune_cache_lookup(const std::string& key, int* cfg, int* dyn) {
  const std::string path = tune_cache_path();
  if (path.empty()) return false;
  std::ifstream f(path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    std::istringstream ss(line);
    std::string k;
    int c = -1, d = -1;
    if (ss >> k >> c >> d && k == key && (c == 0 || c == 6) && d >= 0 && d <= 3) {
      *cfg = c;
      *dyn = d;
      found = true;  // the last entry for a key wins
    }
  }
  return found;
}

void tune_cache_store(const std::string& key, int cfg, int dyn) {
  const std::string path = tune_cache_path();
  if (path.empty()) return;
  std::ofstream f(path, std::ios::app);
  f << key << " " << cfg << " " << dyn << "\n";
}

// Grouped CRT plans: every problem's CRT sequence recorded against its own
// workspace region (base + offset), then laid out as item tables of the
// grouped launches: the Hadamard pre-combinations of all problems, then per
// complex product (round) the exponents of every operand, the residues (one
// launch per modulus count), the residue GEMMs and the reconstructions (one
// launch per modulus count).
struct CrtLaunch {
  enum Type { PRE, EXP, SPLIT, GEMM, COMBINE } type;
  int N;
  int count;
  int64_t blocks;
  size_t items, prefix;  // byte offsets into the table buffer
};

bq_status_t crt_record(bq_grouped_plan_t p, char* base, CrtRecord* rec) {
  for (int i : p->order) {
    bq_problem_t& q = p->probs[i];
    bq_status_t st = execute(p->h, p->plans[i], p->pr, &q.A, &q.B, &q.C, 0xFFu, base + p->ws_off[i], false,
                             nullptr, rec);
    if (st != BQ_OK) return st;
  }
  return BQ_OK;
}

void crt_tables(const CrtRecord& rec, std::vector<char>* bytes, std::vector<CrtLaunch>* launches) {
  bytes->clear();
  launches->clear();
  auto put = [&](const void* src, size_t n) {
    const size_t off = align256(bytes->size());
    bytes->resize(off + n);
    if (n) std::memcpy(bytes->data() + off, src, n);
    return off;
  };
  // Items and the prefix of their block counts into the buffer; the launch
  // joins the list when it has blocks.
  auto add = [&](CrtLaunch::Type type, int N, const auto& items, auto blocks_of) {
    std::vector<int64_t> prefix;
    int64_t total = 0;
    for (const auto& it : items) {
      prefix.push_back(total);
      total += blocks_of(it);
    }
    CrtLaunch L{type, N, int(items.size()), total, 0, 0};
    L.items = put(items.data(), items.size() * sizeof(items[0]));
    L.prefix = put(prefix.data(), prefix.size() * sizeof(int64_t));
    if (L.count > 0 && L.blocks > 0) launches->push_back(L);
  };
  add(CrtLaunch::PRE, 0, rec.pre, [](const bq::CombineArgs& c) { return c.rows; });
  for (int r = 0; r < rec.rounds; ++r) {
    std::vector<CrtRecord::Split> sp;
    for (const auto& x : rec.splits)
      if (x.round == r) sp.push_back(x);
    std::stable_sort(sp.begin(), sp.end(), [](const auto& a, const auto& b) { return a.N < b.N; });
    std::vector<bq::CrtSplitItem> all;
    for (const auto& x : sp) all.push_back(x.it);
    add(CrtLaunch::EXP, 0, all, [](const bq::CrtSplitItem& it) { return bq::crt_exp_blocks(it.a); });
    for (size_t i = 0; i < sp.size();) {
      size_t j = i;
      std::vector<bq::CrtSplitItem> part;
      while (j < sp.size() && sp[j].N == sp[i].N) part.push_back(sp[j++].it);
      add(CrtLaunch::SPLIT, sp[i].N, part, [](const bq::CrtSplitItem& it) { return bq::crt_split_blocks(it.a); });
      i = j;
    }
    std::vector<bq::CrtGemmItem> gm;
    for (const auto& x : rec.gemms)
      if (x.round == r) gm.push_back(x.it);
    add(CrtLaunch::GEMM, 0, gm, [](const bq::CrtGemmItem& it) { return bq::crt_gemm_blocks(it); });
    std::vector<CrtRecord::Comb> cb;
    for (const auto& x : rec.combs)
      if (x.round == r) cb.push_back(x);
    std::stable_sort(cb.begin(), cb.end(), [](const auto& a, const auto& b) { return a.N < b.N; });
    for (size_t i = 0; i < cb.size();) {
      size_t j = i;
      std::vector<bq::CrtCombineArgs> part;
      while (j < cb.size() && cb[j].N == cb[i].N) part.push_back(cb[j++].c);
      add(CrtLaunch::COMBINE, cb[i].N, part, [](const bq::CrtCombineArgs& c) { return bq::crt_combine_blocks(c); });
      i = j;
    }
  }
  if (bytes->empty()) bytes->resize(256);
}

hipError_t crt_launch(const CrtLaunch& L, const char* d, hipStream_t s) {
  const int64_t* prefix = reinterpret_cast<const int64_t*>(d + L.prefix);
  switch (L.type) {
    case CrtLaunch::PRE:
      return bq::launch_grouped_combine(reinterpret_cast<const bq::CombineArgs*>(d + L.items), prefix, L.count,
                                        L.blocks, s);
    case CrtLaunch::EXP:
      return bq::launch_crt_exp_grouped(reinterpret_cast<const bq::CrtSplitItem*>(d + L.items), prefix, L.count,
                                        L.blocks, s);
    case CrtLaunch::SPLIT:
      return bq::launch_crt_split_grouped(L.N, reinterpret_cast<const bq::CrtSplitItem*>(d + L.items), prefix,
                                          L.count, L.blocks, s);
    case CrtLaunch::GEMM:
      return bq::launch_crt_gemm_grouped(reinterpret_cast<const bq::CrtGemmItem*>(d + L.items), prefix, L.count,
                                         L.blocks, s);
    case CrtLaunch::COMBINE:
      return bq::launch_crt_combine_grouped(L.N, reinterpret_cast<const bq::CrtCombineArgs*>(d + L.items), prefix,
                                            L.count, L.blocks, s);
  }
  return hipErrorInvalidValue;
}

// Host tables of an FP64 plan for workspace ws, copied to the device, then
// the graph [grouped pre-combination -> persistent grouped GEMM] recorded.
bq_status_t grouped_bind(bq_grouped_plan_t p, void* ws) {
  grouped_release_graph(p);
  const bool trace = p->h->trace;
  p->h->trace = false;  // no trace events inside the recorded graph
  struct Restore {
    bq_handle_t h;
    bool t;
    ~Restore() { h->trace = t; }
  } restore{p->h, trace};
  hipError_t e = hipSuccess;
  bq_status_t st = BQ_OK;
  if (p->pr.et == 3) {
    // CRT form: the grouped launches over every problem's recorded items.
    CrtRecord rec;
    st = crt_record(p, static_cast<char*>(ws), &rec);
    if (st != BQ_OK) return st;
    std::vector<char> bytes;
    std::vector<CrtLaunch> launches;
    crt_tables(rec, &bytes, &launches);
    if (bytes.size() > p->crt_bytes) return fail(BQ_ERR_INVALID_VALUE, "CRT item tables outgrew the plan");
    e = hipMemcpy(p->d_crt, bytes.data(), bytes.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "grouped table upload");
    e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    for (const CrtRecord::Fill& f : rec.fills)
      if (e == hipSuccess) e = bq::launch_fill_zero(f.p, f.rows, f.cols, f.ld, p->cap);
    for (const CrtLaunch& L : launches)
      if (e == hipSuccess) e = crt_launch(L, static_cast<const char*>(p->d_crt), p->cap);
    if (e != hipSuccess) st = hip_fail(e, "grouped CRT launch");
  } else if (p->pr.et >= 0) {
    e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    // Split forms: every problem's split-precision sequence, one after another
    // on the capture stream, sharing the workspace.
    for (int i = 0; i < p->count && st == BQ_OK; ++i) {
      bq_problem_t& q = p->probs[p->order[i]];
      st = execute(p->h, p->plans[p->order[i]], p->pr, &q.A, &q.B, &q.C, 0xFFu, ws, false, p->cap);
    }
  } else {
    // One launch per complex product (schedule bit 2): the Hadamard
    // products P5..P8 go first and write their P into the problem's
    // workspace, one pass forms the Hadamard sums S_w = sum_q H[w][q] P_{5+q}
    // in place (the 4 x 4 combination of the pre-combination kernel), and
    // the direct products P1..P4 write C_w = c_w P_w + s_w S_w once: C is
    // never read, against four read-modify-writes of all eight C blocks
    // when each Hadamard product adds into C.
    const bool defer = (p->dyn & 2) != 0;
    std::vector<bq::CombineArgs> comb, ht;
    std::vector<int64_t> prefix, ht_prefix;
    std::vector<bq::GemmArgs> prods(size_t(p->count) * 8);
    int64_t rows = 0, ht_rows = 0;
    for (int pi = 0; pi < p->count; ++pi) {
      const bq_problem_t& q = p->probs[pi];
      const Plan& pl = p->plans[pi];
      const int64_t m = pl.m, n = pl.n, k = pl.k;  // shapes of op(A), op(B)
      char* wp = static_cast<char*>(ws) + p->ws_off[pi];
      const int64_t kpad = round_up(k, 8), npad = round_up(n, 8), mpad = round_up(m, 8);
      const size_t a1 = align256(combo_slot_bytes(m, k)), b1 = align256(combo_slot_bytes(k, n));
      double *cAr[4], *cAi[4], *cBr[4], *cBi[4];
      for (int c = 0; c < 4; ++c) {
        cAr[c] = reinterpret_cast<double*>(wp); wp += a1;
        cAi[c] = reinterpret_cast<double*>(wp); wp += a1;
        cBr[c] = reinterpret_cast<double*>(wp); wp += b1;
        cBi[c] = reinterpret_cast<double*>(wp); wp += b1;
      }
      for (int side = 0; side < 2; ++side) {
        bq::CombineArgs ca{};
        const bq_matrix_t& X = side == 0 ? q.A : q.B;
        for (int c = 0; c < 8; ++c) ca.src[c] = X.comp[c];
        ca.lds = X.ld;
        ca.rows = X.rows;  // the stored orientation (op T / H keep it)
        ca.cols = X.cols;
        ca.ldd = side == 0 ? (pl.ta ? mpad : kpad) : (pl.tb ? kpad : npad);
        ca.nq = 4;
        for (int j = 0; j < 4; ++j) {
          ca.dst_r[j] = side == 0 ? cAr[j] : cBr[j];
          ca.dst_i[j] = side == 0 ? cAi[j] : cBi[j];
          for (int u = 0; u < 4; ++u) ca.w[j][u] = side == 0 ? pl.wA[j][u] : pl.wB[j][u];
        }
        prefix.push_back(rows);
        rows += ca.rows;
        comb.push_back(ca);
      }
      // Hadamard products' P (deferred schedule): 4 complex blocks after the
      // pre-combined operands, rows of npad doubles.
      const size_t p1 = align256(size_t(m) * size_t(npad) * 8);
      double *Pr[4], *Pi[4];
      for (int c = 0; c < 4; ++c) {
        Pr[c] = reinterpret_cast<double*>(wp); wp += p1;
        Pi[c] = reinterpret_cast<double*>(wp); wp += p1;
      }
      // A problem defers its Hadamard sums when it runs all eight complex
      // products of the bilinear form: P1..P4 in slots 0..3, P5..P8 in 4..7.
      const int np = int(pl.prods.size());
      bool full = defer && pl.bilinear && np == 8;
      for (int j = 0; full && j < 8; ++j) full = pl.prods[j].L.combo == (j < 4 ? -1 : j - 4);
      double had_coef[4] = {0.0, 0.0, 0.0, 0.0};  // s_w: C_w gets s_w S_w
      if (full) {
        bq::CombineArgs h{};
        for (int u = 0; u < 4; ++u) {
          h.src[u] = Pr[u];
          h.src[u + 4] = Pi[u];
          h.dst_r[u] = Pr[u];
          h.dst_i[u] = Pi[u];
          for (int w = 0; w < 4; ++w) h.w[w][u] = kHad[w][u];
        }
        h.lds = h.ldd = npad;
        h.rows = m;
        h.cols = n;
        h.nq = 4;
        ht_prefix.push_back(ht_rows);
        ht_rows += m;
        ht.push_back(h);
        for (int j = 4; j < 8; ++j)
          for (const Tgt& t : pl.prods[j].tgts) had_coef[t.w] = t.coef.re / kHad[t.w][j - 4];
      }
      // Slots in launch order: with one launch per slot, slots 4..7 run
      // first; WRITE / ACCUM of each C block follow that order.
      static constexpr int kSeq[8] = {0, 1, 2, 3, 4, 5, 6, 7};
      static constexpr int kDeferSeq[8] = {4, 5, 6, 7, 0, 1, 2, 3};
      const int* seq = defer ? kDeferSeq : kSeq;
      bool touched[8] = {};
      for (int si = 0; si < 8; ++si) {
        const int qi = seq[si];
        if (qi >= np) continue;
        const Prod& pd = pl.prods[qi];
        Operand L = pd.L, R = pd.R;
        const int combo = L.combo;
        if (L.combo >= 0) {
          L.r = cAr[L.combo]; L.i = cAi[L.combo]; L.ld = pl.ta ? mpad : kpad;
          R.r = cBr[R.combo]; R.i = cBi[R.combo]; R.ld = pl.tb ? kpad : npad;
        }
        bq::GemmArgs g{};
        g.lr = L.r; g.li = L.i; g.lda = L.ld;
        g.rr = R.r; g.ri = R.i; g.ldb = R.ld;
        g.m = m; g.n = n; g.k = k;
        g.ta = pl.ta; g.tb = pl.tb;
        g.sL = L.s; g.sR = R.s;
        g.ldc = q.C.ld;
        g.ldadd = npad;
        g.xcd_remap = 0;
        g.group_m = 1;
        auto al16 = [](const double* x) { return (reinterpret_cast<uintptr_t>(x) & 15u) == 0; };
        g.vec = (g.lda % 2 == 0) && (g.ldb % 2 == 0) && al16(g.lr) && al16(g.li) && al16(g.rr) && al16(g.ri);
        if (full && combo >= 0) {
          // P of a Hadamard product into the workspace, written once.
          bq::Target T{};
          T.ar = 1.0;
          T.cr = Pr[combo];
          T.ci = Pi[combo];
          T.mode_r = T.mode_i = bq::TGT_WRITE;
          g.tgt[g.ntgt++] = T;
          g.ldc = npad;
        } else {
          for (const Tgt& t : pd.tgts) {
            bq::Target T{};
            T.ar = t.coef.re;
            T.ai = t.coef.im;
            T.cr = q.C.comp[t.w];
            T.ci = q.C.comp[t.w + 4];
            T.mode_r = touched[t.w] ? bq::TGT_ACCUM : bq::TGT_WRITE;
            T.mode_i = touched[t.w + 4] ? bq::TGT_ACCUM : bq::TGT_WRITE;
            touched[t.w] = touched[t.w + 4] = true;
            if (full) {  // direct product: the only writer of C_w, plus s_w S_w
              T.sr = Pr[t.w];
              T.si = Pi[t.w];
              T.sc = had_coef[t.w];
            }
            g.tgt[g.ntgt++] = T;
          }
        }
        prods[size_t(pi) * 8 + qi] = g;
      }
    }
    // Buffer-resource loads when every product's operand tiles allow them.
    int buf = 1;
    for (const bq::GemmArgs& g : prods)
      if (g.m > 0 && !bq::grouped_spans_fit(p->cfg, g.ta, g.tb, g.lda, g.ldb)) buf = 0;
    // Tables go to the device before recording (a synchronous copy may not
    // run while this thread records a graph).
    e = hipMemcpy(p->d_prods, prods.data(), prods.size() * sizeof(bq::GemmArgs), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(p->d_comb, comb.data(), comb.size() * sizeof(bq::CombineArgs), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(p->d_prefix, prefix.data(), prefix.size() * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess && !ht.empty())
      e = hipMemcpy(p->d_ht, ht.data(), ht.size() * sizeof(bq::CombineArgs), hipMemcpyHostToDevice);
    if (e == hipSuccess && !ht.empty())
      e = hipMemcpy(p->d_ht_prefix, ht_prefix.data(), ht_prefix.size() * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "grouped table upload");
    e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    e = bq::launch_grouped_combine(p->d_comb, p->d_prefix, p->ncomb, rows, p->cap);
    if (defer) {
      // Hadamard products (rounds 4..7), their sums, then the direct products.
      auto round = [&](int q) {
        if (e == hipSuccess && p->round_n[q] > 0)
          e = bq::launch_grouped(p->cfg, p->dyn & 1, p->ops, buf, p->d_prods, p->d_items + p->nitems + p->round_off[q],
                                 p->round_n[q], p->d_counter, p->blocks, p->cap);
      };
      for (int q = 4; q < 8; ++q) round(q);
      if (e == hipSuccess) e = bq::launch_grouped_combine(p->d_ht, p->d_ht_prefix, int(ht.size()), ht_rows, p->cap);
      for (int q = 0; q < 4; ++q) round(q);
    } else if (e == hipSuccess) {
      e = bq::launch_grouped(p->cfg, p->dyn & 1, p->ops, buf, p->d_prods, p->d_items, p->nitems, p->d_counter,
                             p->blocks, p->cap);
    }
    if (e != hipSuccess) st = hip_fail(e, "grouped launch");
  }
  hipGraph_t graph = nullptr;
  hipError_t e2 = hipStreamEndCapture(p->cap, &graph);
  if (st != BQ_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
  e2 = hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e2 != hipSuccess) return hip_fail(e2, "hipGraphInstantiate");
  p->bound_ws = ws;
  p->bound = true;
  return BQ_OK;
}

bq_status_t grouped_check_ws(bq_grouped_plan_t p, void* ws, size_t ws_bytes) {
  if (ws_bytes < p->ws_bytes)
    return fail(BQ_ERR_WORKSPACE, "workspace " + std::to_string(ws_bytes) + " B < " + std::to_string(p->ws_bytes) + " B");
  if (p->ws_bytes > 0 && !ws) return fail(BQ_ERR_INVALID_VALUE, "ws is null");
  // the workspace must not overlap any problem's operands
  if (ws && p->ws_bytes > 0) {
    const Range w{reinterpret_cast<uintptr_t>(ws), reinterpret_cast<uintptr_t>(ws) + p->ws_bytes};
    for (const bq_problem_t& q : p->probs) {
      const bq_matrix_t* M[3] = {&q.A, &q.B, &q.C};
      for (const bq_matrix_t* X : M)
        if (X->rows > 0 && X->cols > 0)
          for (int c = 0; c < 8; ++c)
            if (X->comp[c] && overlaps(w, block_range(X->comp[c], X->rows, X->cols, X->ld)))
              return fail(BQ_ERR_ALIAS, "workspace overlaps a problem's matrix");
    }
  }
  return BQ_OK;
}

}  // namespace

extern "C" {

bq_status_t bq_grouped_plan_create(bq_handle_t h, int count, const bq_problem_t* problems, bq_prec_t prec, int slices,
                                   bq_grouped_plan_t* plan) {
  if (!plan) return fail(BQ_ERR_INVALID_VALUE, "plan is null");
  *plan = nullptr;
  if (!h) return fail(BQ_ERR_INVALID_VALUE, "handle is null");
  if (count < 0 || (count > 0 && !problems)) return fail(BQ_ERR_INVALID_VALUE, "bad problem list");
  Prec pr;
  if (bq_status_t ps = prec_of(prec, slices, &pr); ps != BQ_OK) return ps;
  std::vector<Plan> plans(count);
  std::vector<size_t> offs(count, 0);
  size_t total_ws = 0;
  std::vector<std::pair<Range, int>> outs, ins;  // (range, problem)
  double flops = 0.0;
  for (int i = 0; i < count; ++i) {
    const bq_problem_t& q = problems[i];
    Plan pl;
    bool streamed = false;
    Prec dummy;
    bq_status_t st = validate(q.opA, q.opB, &q.A, &q.B, &q.C, prec, slices, nullptr, 0, 0xFFu, &pl, &streamed,
                              &dummy, false);
    if (st != BQ_OK) return fail(st, "problem " + std::to_string(i) + ": " + g_detail);
    const int64_t m = pl.m, n = pl.n, k = pl.k;
    if (pr.et < 0) {
      for (int c = 0; c < 8; ++c)
        if (!q.A.comp[c] || !q.B.comp[c])
          return fail(BQ_ERR_UNSUPPORTED, "problem " + std::to_string(i) +
                                              ": FP64 batched plans need all 16 input components");
      if (m == 0 || n == 0 || k == 0)
        return fail(BQ_ERR_UNSUPPORTED, "problem " + std::to_string(i) + ": FP64 batched plans need m, n, k > 0");
    }
    size_t res = 0, mn = 0;
    workspace_need(pl, pr, m, n, k, &res, &mn, pr.et == 3);
    if (pr.et < 0) res += 8 * align256(size_t(m) * size_t(round_up(n, 8)) * 8);  // the Hadamard products' P
    if (pr.et < 0 || pr.et == 3) {
      offs[i] = total_ws;
      total_ws += res;
    } else {
      total_ws = std::max(total_ws, res);
    }
    flops += double(pl.real_gemms) * 2.0 * double(m) * double(n) * double(k);
    plans[i] = pl;
    if (m > 0 && n > 0) {
      for (int c = 0; c < 8; ++c) {
        if (q.C.comp[c]) outs.push_back({block_range(q.C.comp[c], m, n, q.C.ld), i});
        if (k > 0) {
          if (q.A.comp[c]) ins.push_back({block_range(q.A.comp[c], q.A.rows, q.A.cols, q.A.ld), i});
          if (q.B.comp[c]) ins.push_back({block_range(q.B.comp[c], q.B.rows, q.B.cols, q.B.ld), i});
        }
      }
    }
  }
  // Problems run concurrently: no C may overlap any other matrix of any problem.
  {
    std::vector<std::pair<Range, int>> all;  // second: -1 input, else output index
    for (auto& r : ins) all.push_back({r.first, -1});
    for (size_t j = 0; j < outs.size(); ++j) all.push_back({outs[j].first, int(j)});
    std::sort(all.begin(), all.end(), [](const auto& a, const auto& b) { return a.first.lo < b.first.lo; });
    uintptr_t reach = 0;
    bool reach_out = false;
    for (size_t j = 0; j < all.size(); ++j) {
      const bool is_out = all[j].second >= 0;
      if (j > 0 && all[j].first.lo < reach && (is_out || reach_out))
        return fail(BQ_ERR_ALIAS, "a C block overlaps another matrix of the batch");
      if (all[j].first.hi > reach) {
        reach = all[j].first.hi;
        reach_out = is_out;
      } else if (is_out) {
        reach_out = true;
      }
    }
  }
  bq_status_t st = check_handle(h);
  if (st != BQ_OK) return st;

  auto* p = new bq_grouped_plan_s;
  p->h = h;
  p->count = count;
  p->pr = pr;
  p->probs.assign(problems, problems + count);
  p->plans = std::move(plans);
  p->ws_off = std::move(offs);
  p->ws_bytes = total_ws;
  p->flops = flops;
  p->order.resize(count);
  for (int i = 0; i < count; ++i) p->order[i] = i;
  auto work = [&](int i) {
    const Plan& pl = p->plans[i];
    return double(pl.m) * double(pl.n) * double(pl.k);
  };
  std::stable_sort(p->order.begin(), p->order.end(), [&](int a, int b) { return work(a) > work(b); });
  p->blocks = 2 * std::max(1, h->cu_count);
  for (int i = 0; i < count; ++i) {
    const int o = 2 * int(p->plans[i].ta) + int(p->plans[i].tb);
    p->ops = (i == 0 || p->ops == o) ? o : -1;
  }

  std::ostringstream key;
  key << h->arch << ":" << h->cu_count << ":" << pr.et << ":" << pr.S << ":";
  uint64_t hash = 1469598103934665603ull;
  for (int i : p->order) {
    const Plan& pl = p->plans[i];
    const int64_t d[3] = {pl.m, pl.n, pl.k};
    for (int64_t x : d) {
      hash ^= uint64_t(x);
      hash *= 1099511628211ull;
    }
  }
  key << std::hex << hash;
  p->tune_key = key.str();
  (void)tune_cache_lookup(p->tune_key, &p->cfg, &p->dyn);

  hipError_t e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
  if (e == hipSuccess && pr.et < 0 && count > 0) {
    // Items of both schedules: (problem, tile) running the problem's complex
    // products in turn, then per complex product q the (problem, tile) items
    // of q alone (one launch each, so concurrent blocks share q's operands).
    std::vector<bq::GroupedItem> items;
    for (int i : p->order) {
      const int tm = int((p->plans[i].m + kGroupedTile - 1) / kGroupedTile);
      const int tn = int((p->plans[i].n + kGroupedTile - 1) / kGroupedTile);
      for (int a = 0; a < tm; ++a)
        for (int b = 0; b < tn; ++b) items.push_back({i * 8, int(p->plans[i].prods.size()), a, b});
    }
    p->nitems = int(items.size());
    for (int q = 0; q < 8; ++q) {
      p->round_off.push_back(int(items.size()) - p->nitems);
      for (int i : p->order) {
        if (q >= int(p->plans[i].prods.size())) continue;
        const int tm = int((p->plans[i].m + kGroupedTile - 1) / kGroupedTile);
        const int tn = int((p->plans[i].n + kGroupedTile - 1) / kGroupedTile);
        for (int a = 0; a < tm; ++a)
          for (int b = 0; b < tn; ++b) items.push_back({i * 8 + q, 1, a, b});
      }
      p->round_n.push_back(int(items.size()) - p->nitems - p->round_off.back());
    }
    p->ncomb = 2 * count;
    e = hipMalloc(&p->d_prods, sizeof(bq::GemmArgs) * size_t(count) * 8);
    if (e == hipSuccess) e = hipMalloc(&p->d_items, sizeof(bq::GroupedItem) * items.size());
    if (e == hipSuccess) e = hipMalloc(&p->d_counter, 256);
    if (e == hipSuccess) e = hipMalloc(&p->d_comb, sizeof(bq::CombineArgs) * size_t(p->ncomb));
    if (e == hipSuccess) e = hipMalloc(&p->d_prefix, sizeof(int64_t) * size_t(p->ncomb));
    if (e == hipSuccess) e = hipMalloc(&p->d_ht, sizeof(bq::CombineArgs) * size_t(count));
    if (e == hipSuccess) e = hipMalloc(&p->d_ht_prefix, sizeof(int64_t) * size_t(count));
    if (e == hipSuccess)
      e = hipMemcpy(p->d_items, items.data(), sizeof(bq::GroupedItem) * items.size(), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess && pr.et == 3 && count > 0) {
    // Table sizes do not depend on the workspace address: record against a
    // stand-in base once to size the device buffer.
    CrtRecord rec;
    st = crt_record(p, reinterpret_cast<char*>(uintptr_t(1) << 20), &rec);
    if (st != BQ_OK) {
      bq_grouped_plan_destroy(p);
      return st;
    }
    std::vector<char> bytes;
    std::vector<CrtLaunch> launches;
    crt_tables(rec, &bytes, &launches);
    p->crt_bytes = bytes.size();
    p->nitems = int(rec.gemms.size());
    e = hipMalloc(&p->d_crt, p->crt_bytes);
  }
  if (e != hipSuccess) {
    bq_grouped_plan_destroy(p);
    return hip_fail(e, "grouped plan setup");
  }
  *plan = p;
  return BQ_OK;
}

bq_status_t bq_grouped_plan_workspace_size(bq_grouped_plan_t plan, size_t* bytes) {
  if (!plan || !bytes) return fail(BQ_ERR_INVALID_VALUE, "null argument");
  *bytes = plan->ws_bytes;
  return BQ_OK;
}

bq_status_t bq_grouped_plan_info(bq_grouped_plan_t plan, int* tile_config, int* dynamic_schedule, int* work_items) {
  if (!plan) return fail(BQ_ERR_INVALID_VALUE, "plan is null");
  if (tile_config) *tile_config = plan->cfg;
  if (dynamic_schedule) *dynamic_schedule = plan->dyn;
  if (work_items) *work_items = plan->nitems;
  return BQ_OK;
}

bq_status_t bq_grouped_plan_launch(bq_grouped_plan_t plan, void* ws, size_t ws_bytes, bq_stream_t stream) {
  if (!plan) return fail(BQ_ERR_INVALID_VALUE, "plan is null");
  bq_status_t st = grouped_check_ws(plan, ws, ws_bytes);
  if (st != BQ_OK) return st;
  st = check_handle(plan->h);
  if (st != BQ_OK) return st;
  if (plan->count == 0) return BQ_OK;
  if (!plan->bound || plan->bound_ws != ws) {
    st = grouped_bind(plan, ws);
    if (st != BQ_OK) return st;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  Tracer tr(plan->h, s, BQ_KERNEL_GROUPED, plan->pr.et >= 0 ? plan->pr.S : plan->cfg, plan->count, plan->nitems, 0,
            plan->flops, 0.0);
  hipError_t e = hipGraphLaunch(plan->exec, s);
  tr.done();
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return BQ_OK;
}

bq_status_t bq_grouped_plan_autotune(bq_grouped_plan_t plan, void* ws, size_t ws_bytes, bq_stream_t stream) {
  if (!plan) return fail(BQ_ERR_INVALID_VALUE, "plan is null");
  bq_status_t st = grouped_check_ws(plan, ws, ws_bytes);
  if (st != BQ_OK) return st;
  if (plan->pr.et >= 0 || plan->count == 0) return BQ_OK;
  st = check_handle(plan->h);
  if (st != BQ_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(BQ_ERR_HIP, "hipEventCreate");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(BQ_ERR_HIP, "hipEventCreate");
  }
  const int cfgs[2] = {0, 6};
  float best = 1e30f;
  int best_cfg = plan->cfg, best_dyn = plan->dyn;
  for (int c : cfgs) {
    for (int d : {3, 2, 1, 0}) {
      plan->cfg = c;
      plan->dyn = d;
      st = grouped_bind(plan, ws);
      if (st != BQ_OK) break;
      hipError_t e = hipGraphLaunch(plan->exec, s);  // warm-up
      if (e == hipSuccess) e = hipEventRecord(e0, s);
      for (int r = 0; r < 3 && e == hipSuccess; ++r) e = hipGraphLaunch(plan->exec, s);
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        st = hip_fail(e, "autotune");
        break;
      }
      if (ms < best) {
        best = ms;
        best_cfg = c;
        best_dyn = d;
      }
    }
    if (st != BQ_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  plan->cfg = best_cfg;
  plan->dyn = best_dyn;
  grouped_release_graph(plan);
  if (st != BQ_OK) return st;
  tune_cache_store(plan->tune_key, best_cfg, best_dyn);
  return grouped_bind(plan, ws);
}

bq_status_t bq_grouped_plan_destroy(bq_grouped_plan_t plan) {
  if (!plan) return BQ_OK;
  grouped_release_graph(plan);
  if (plan->cap) (void)hipStreamDestroy(plan->cap);
  if (plan->d_prods) (void)hipFree(plan->d_prods);
  if (plan->d_items) (void)hipFree(plan->d_items);
  if (plan->d_counter) (void)hipFree(plan->d_counter);
  if (plan->d_comb) (void)hipFree(plan->d_comb);
  if (plan->d_prefix) (void)hipFree(plan->d_prefix);
  if (plan->d_ht) (void)hipFree(plan->d_ht);
  if (plan->d_ht_prefix) (void)hipFree(plan->d_ht_prefix);
  if (plan->d_crt) (void)hipFree(plan->d_crt);
  delete plan;
  return BQ_OK;
}

}  // extern "C"

// ===========================================================================
// Hermitian eigenproblem (diagonalization through the complex isomorph)
// ===========================================================================
namespace {

// Weights of the isomorph's quadrants Z11, Z12, Z21, Z22 over c1..c8
// (eq. mapping-formulas read backwards: Z = M+ + M-, E = c1 + i c2,
// F = c3 + i c4, G = -c6 + i c5, H = -c8 + i c7).
constexpr double kIsoRe[4][8] = {{1, 0, 0, 0, 0, -1, 0, 0},
                                 {0, 0, 1, 0, 0, 0, 0, -1},
                                 {0, 0, -1, 0, 0, 0, 0, -1},
                                 {1, 0, 0, 0, 0, 1, 0, 0}};
constexpr double kIsoIm[4][8] = {{0, 1, 0, 0, 1, 0, 0, 0},
                                 {0, 0, 0, 1, 0, 0, 1, 0},
                                 {0, 0, 0, 1, 0, 0, -1, 0},
                                 {0, -1, 0, 0, 1, 0, 0, 0}};

enum HeevCase { HEEV_FULL, HEEV_BLOCKS, HEEV_BLOCKS_EQUAL, HEEV_BLOCKS_CONJ, HEEV_ANTI_J, HEEV_ANTI_K, HEEV_ANTI_JK };

// Anti-diagonal with j and k together: the singular value decomposition of
// Z12 (BQ_HEEV_JK=full takes the full problem instead, for comparison), by
// divide and conquer (BQ_SVD=gesvd: bidiagonal QR).
bool heev_jk_svd() {
  const char* e = std::getenv("BQ_HEEV_JK");
  return !(e && std::strcmp(e, "full") == 0);
}
bool heev_use_gesvd() {
  const char* e = std::getenv("BQ_SVD");
  return e && std::strcmp(e, "gesvd") == 0;
}

HeevCase heev_case(unsigned mask) {
  auto has = [&](int c) { return (mask >> c & 1) != 0; };  // c: 0-based component
  const bool jk = has(2) || has(3) || has(6) || has(7);
  const bool field = has(0) || has(1) || has(4) || has(5);
  if (!jk) {
    if (!has(1) && !has(5)) return HEEV_BLOCKS_EQUAL;  // Z11 = Z22 = c1 + i c5
    if (!has(4) && !has(5)) return HEEV_BLOCKS_CONJ;   // Z22 = conj(Z11), Z11 = c1 + i c2
    return HEEV_BLOCKS;
  }
  if (!field) {
    if (!has(3) && !has(7)) return HEEV_ANTI_J;  // j only: a = i
    if (!has(2) && !has(6)) return HEEV_ANTI_K;  // k only: a = 1
    if (heev_jk_svd()) return HEEV_ANTI_JK;      // j and k: SVD of Z12
  }
  return HEEV_FULL;
}

struct HeevLayout {
  int64_t order = 0;  // order of each eigensolve (or of the SVD)
  int solves = 0;
  size_t z = 0, x1 = 0, x2 = 0, d1 = 0, d2 = 0, e = 0, info = 0, src = 0, scratch = 0, u = 0, vh = 0;
  size_t scratch_bytes = 0, total = 0;
  bool z_in_ws = false;
};

// Eigensolver scratch for one solve (rocBLAS device-memory size query: the
// call returns before touching its pointers, which only need to be non-null).
bool heev_scratch(rocblas_handle rb, int64_t order, bool vectors, size_t* bytes) {
  *bytes = 0;
  if (order == 0) return true;
  if (rocblas_start_device_memory_size_query(rb) != rocblas_status_success) return false;
  auto* fake_c = reinterpret_cast<rocblas_double_complex*>(uintptr_t(256));
  auto* fake_d = reinterpret_cast<double*>(uintptr_t(256));
  auto* fake_i = reinterpret_cast<rocblas_int*>(uintptr_t(256));
  (void)rocsolver_zheevd(rb, vectors ? rocblas_evect_original : rocblas_evect_none, rocblas_fill_lower,
                         (rocblas_int)order, fake_c, (rocblas_int)order, fake_d, fake_d, fake_i);
  return rocblas_stop_device_memory_size_query(rb, bytes) == rocblas_status_success;
}

// The same for the singular value decomposition of one n x n block.
bool svd_scratch(rocblas_handle rb, int64_t n, bool vectors, size_t* bytes) {
  *bytes = 0;
  if (n == 0) return true;
  if (rocblas_start_device_memory_size_query(rb) != rocblas_status_success) return false;
  auto* fake_c = reinterpret_cast<rocblas_double_complex*>(uintptr_t(256));
  auto* fake_d = reinterpret_cast<double*>(uintptr_t(256));
  auto* fake_i = reinterpret_cast<rocblas_int*>(uintptr_t(256));
  const rocblas_svect sv = vectors ? rocblas_svect_singular : rocblas_svect_none;
  const rocblas_int ni = (rocblas_int)n, ld = vectors ? ni : 1;
  if (heev_use_gesvd())
    (void)rocsolver_zgesvd(rb, sv, sv, ni, ni, fake_c, ni, fake_d, fake_c, ld, fake_c, ld, fake_d,
                           rocblas_outofplace, fake_i);
  else
    (void)rocsolver_zgesdd(rb, sv, sv, ni, ni, fake_c, ni, fake_d, fake_c, ld, fake_c, ld, fake_i);
  return rocblas_stop_device_memory_size_query(rb, bytes) == rocblas_status_success;
}

bool heev_layout(rocblas_handle rb, int64_t n, unsigned mask, bool vectors, HeevLayout* L) {
  const HeevCase hc = heev_case(mask);
  HeevLayout l;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += align256(bytes);
    return at;
  };
  const size_t cplx = 16;
  if (hc == HEEV_FULL) {
    l.order = 2 * n;
    l.solves = 1;
    l.z_in_ws = !vectors;  // with vectors the isomorph is built in V and solved in place
    if (l.z_in_ws) l.z = take(size_t(l.order) * size_t(l.order) * cplx);
  } else if (hc == HEEV_ANTI_JK) {
    l.order = n;
    l.solves = 1;
    l.x1 = take(size_t(n) * size_t(n) * cplx);
    l.d1 = take(size_t(n) * 8);
    if (vectors) {
      l.u = take(size_t(n) * size_t(n) * cplx);
      l.vh = take(size_t(n) * size_t(n) * cplx);
      l.src = take(size_t(2 * n) * 8);
    }
  } else {
    l.order = n;
    l.solves = hc == HEEV_BLOCKS ? 2 : 1;
    l.x1 = take(size_t(n) * size_t(n) * cplx);
    if (l.solves == 2) l.x2 = take(size_t(n) * size_t(n) * cplx);
    l.d1 = take(size_t(n) * 8);
    if (l.solves == 2) l.d2 = take(size_t(n) * 8);
    if (vectors) l.src = take(size_t(2 * n) * 8);
  }
  l.e = take(size_t(std::max<int64_t>(l.order, 1)) * 8);
  l.info = take(2 * sizeof(int));
  if (hc == HEEV_ANTI_JK ? !svd_scratch(rb, n, vectors, &l.scratch_bytes)
                         : !heev_scratch(rb, l.order, vectors, &l.scratch_bytes))
    return false;
  l.scratch = take(l.scratch_bytes);
  l.total = off;
  *L = l;
  return true;
}

}  // namespace

extern "C" {

bq_status_t bq_heev_workspace_size(bq_handle_t h, int64_t n, unsigned mask, int want_vectors, size_t* bytes) {
  if (!bytes) return fail(BQ_ERR_INVALID_VALUE, "bytes is null");
  *bytes = 0;
  if (bq_status_t st = check_handle(h); st != BQ_OK) return st;
  if (n < 0) return fail(BQ_ERR_INVALID_VALUE, "negative dimension");
  if (mask > 0xFFu) return fail(BQ_ERR_INVALID_VALUE, "mask has bits above 7");
  if (2 * n > INT32_MAX) return fail(BQ_ERR_UNSUPPORTED, "2n above the eigensolver's 32-bit order");
  if (n == 0) return BQ_OK;
  HeevLayout L;
  if (!heev_layout(h->rb, n, mask, want_vectors != 0, &L)) return fail(BQ_ERR_HIP, "eigensolver size query failed");
  *bytes = L.total;
  return BQ_OK;
}

bq_status_t bq_heev(bq_handle_t h, const bq_matrix_t* A, double* w, double* V, int64_t ldv, int* info, void* ws,
                    size_t ws_bytes, bq_stream_t stream) {
  if (!A) return fail(BQ_ERR_INVALID_VALUE, "A is null");
  if (A->rows != A->cols) return fail(BQ_ERR_INVALID_VALUE, "A must be square");
  const int64_t n = A->rows, N = 2 * n;
  if (n < 0) return fail(BQ_ERR_INVALID_VALUE, "negative dimension");
  if (A->ld < std::max<int64_t>(1, n)) return fail(BQ_ERR_INVALID_VALUE, "A: ld < max(1, cols)");
  for (int c = 0; c < 8; ++c)
    if (A->comp[c] && misaligned(A->comp[c])) return fail(BQ_ERR_INVALID_VALUE, "A: component not 8-byte aligned");
  if (N > INT32_MAX) return fail(BQ_ERR_UNSUPPORTED, "2n above the eigensolver's 32-bit order");
  if (n > 0 && !w) return fail(BQ_ERR_INVALID_VALUE, "w is null");
  if (V && ldv < std::max<int64_t>(1, N)) return fail(BQ_ERR_INVALID_VALUE, "ldv < 2n");
  if (V && ldv > INT32_MAX) return fail(BQ_ERR_UNSUPPORTED, "ldv above the eigensolver's 32-bit range");
  if (ws_bytes > 0 && !ws) return fail(BQ_ERR_INVALID_VALUE, "ws is null but ws_bytes > 0");
  if (bq_status_t st = check_handle(h); st != BQ_OK) return st;
  if (n == 0) return BQ_OK;
  const unsigned mask = mask_of(A);
  const HeevCase hc = heev_case(mask);
  const bool vectors = V != nullptr;
  HeevLayout L;
  if (!heev_layout(h->rb, n, mask, vectors, &L)) return fail(BQ_ERR_HIP, "eigensolver size query failed");
  if (ws_bytes < L.total)
    return fail(BQ_ERR_WORKSPACE, "workspace " + std::to_string(ws_bytes) + " B < " + std::to_string(L.total) + " B");
  // Outputs against the input and the workspace.
  {
    std::vector<Range> ins;
    for (int c = 0; c < 8; ++c)
      if (A->comp[c]) ins.push_back(block_range(A->comp[c], n, n, A->ld));
    const uintptr_t wl = reinterpret_cast<uintptr_t>(ws);
    if (L.total > 0) ins.push_back({wl, wl + L.total});
    std::vector<Range> outs = {{reinterpret_cast<uintptr_t>(w), reinterpret_cast<uintptr_t>(w) + uintptr_t(N) * 8}};
    if (V) {
      const uintptr_t v0 = reinterpret_cast<uintptr_t>(V);
      outs.push_back({v0, v0 + (uintptr_t(N - 1) * uintptr_t(ldv) + uintptr_t(N)) * 16});
    }
    if (info) outs.push_back({reinterpret_cast<uintptr_t>(info), reinterpret_cast<uintptr_t>(info) + sizeof(int)});
    for (size_t i = 0; i < outs.size(); ++i) {
      for (const Range& r : ins)
        if (overlaps(outs[i], r)) return fail(BQ_ERR_ALIAS, "an output overlaps A or the workspace");
      for (size_t j = i + 1; j < outs.size(); ++j)
        if (overlaps(outs[i], outs[j])) return fail(BQ_ERR_ALIAS, "two outputs overlap");
    }
  }

  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  auto at = [&](size_t off) { return reinterpret_cast<void*>(base + off); };
  if (rocblas_set_stream(h->rb, s) != rocblas_status_success) return fail(BQ_ERR_HIP, "rocblas_set_stream failed");
  if (rocblas_set_workspace(h->rb, at(L.scratch), L.scratch_bytes) != rocblas_status_success)
    return fail(BQ_ERR_HIP, "rocblas_set_workspace failed");
  double* E = static_cast<double*>(at(L.e));
  int* inf = static_cast<int*>(at(L.info));
  const rocblas_evect ev = vectors ? rocblas_evect_original : rocblas_evect_none;
  const double in_bytes = double(__builtin_popcount(mask)) * double(n) * double(n) * 8.0;

  auto map = [&](int quadrant, Cplx scale, int64_t R, double* out, int64_t ldo) -> hipError_t {
    bq::HeevMapArgs a{};
    for (int c = 0; c < 8; ++c) a.src[c] = A->comp[c];
    a.lds = A->ld;
    a.n = n;
    a.R = R;
    for (int q = 0; q < 4; ++q) {
      const int src_q = R == N ? q : quadrant;
      for (int c = 0; c < 8; ++c) {
        // (scale) * (re + i im) per component weight
        const double wr = kIsoRe[src_q][c], wi = kIsoIm[src_q][c];
        a.wr[q][c] = scale.re * wr - scale.im * wi;
        a.wi[q][c] = scale.re * wi + scale.im * wr;
      }
    }
    a.out = out;
    a.ldo = ldo;
    Tracer tr(h, s, BQ_KERNEL_HEEV_MAP, -1, R, R, 0, 0.0, in_bytes + double(R) * double(R) * 16.0);
    hipError_t e = bq::launch_heev_map(a, s);
    tr.done();
    return e;
  };
  auto solve = [&](double* Z, int64_t ld, double* D, int* inf_out) -> bq_status_t {
    Tracer tr(h, s, BQ_KERNEL_HEEV_SOLVE, vectors ? 1 : 0, L.order, L.order, 0, 0.0, 0.0);
    const rocblas_status rs = rocsolver_zheevd(h->rb, ev, rocblas_fill_lower, (rocblas_int)L.order,
                                               reinterpret_cast<rocblas_double_complex*>(Z), (rocblas_int)ld, D, E,
                                               inf_out);
    tr.done();
    if (rs != rocblas_status_success)
      return fail(BQ_ERR_HIP, std::string("rocsolver_zheevd: ") + rocblas_status_to_string(rs));
    return BQ_OK;
  };

  hipError_t e = hipSuccess;
  if (hc == HEEV_FULL) {
    double* Z = vectors ? V : static_cast<double*>(at(L.z));
    const int64_t ldz = vectors ? ldv : N;
    if ((e = map(0, {1.0, 0.0}, N, Z, ldz)) != hipSuccess) return hip_fail(e, "isomorph launch");
    if (bq_status_t st = solve(Z, ldz, w, inf); st != BQ_OK) return st;
    if (info && (e = bq::launch_heev_info(inf, nullptr, info, s)) != hipSuccess) return hip_fail(e, "info launch");
    return BQ_OK;
  }

  double* X1 = static_cast<double*>(at(L.x1));
  double* X2 = L.solves == 2 ? static_cast<double*>(at(L.x2)) : nullptr;
  double* D1 = static_cast<double*>(at(L.d1));
  double* D2 = L.solves == 2 ? static_cast<double*>(at(L.d2)) : nullptr;
  int64_t* src = vectors ? static_cast<int64_t*>(at(L.src)) : nullptr;
  bq::HeevAsmArgs asmb{};
  asmb.n = n;
  asmb.ldx = n;
  asmb.src = src;
  asmb.V = V;
  asmb.ldv = ldv;
  const double r2 = 1.0 / std::sqrt(2.0);
  double s1 = 1.0, s2 = 1.0;
  int rev = 0;
  const double* list2 = nullptr;
  if (hc == HEEV_ANTI_JK) {
    // Z = [[0, Z12], [Z12^H, 0]], Z12 = U S V^H: with G = V U^H,
    // U_G = [[I, I], [G, -G]] / sqrt 2 gives U_G^H Z U_G = diag(U S U^H, -U S U^H),
    // so the eigenvalues are +-s and the eigenvectors [u; +-v] / sqrt 2.  The
    // map of the lower block Z21 is read by the solver as Z21^H = Z12 =
    // Ux S Vx^H, so u = Ux[:, i] and v = Vx[:, i] (row i of Vx^H, conjugated).
    if ((e = map(2, {1.0, 0.0}, n, X1, n)) != hipSuccess) return hip_fail(e, "reduced block launch");
    auto* Ux = vectors ? static_cast<double*>(at(L.u)) : nullptr;
    auto* VxH = vectors ? static_cast<double*>(at(L.vh)) : nullptr;
    const rocblas_svect sv = vectors ? rocblas_svect_singular : rocblas_svect_none;
    const rocblas_int ni = (rocblas_int)n, ld = vectors ? ni : 1;
    auto* Xc = reinterpret_cast<rocblas_double_complex*>(X1);
    auto* Uc = reinterpret_cast<rocblas_double_complex*>(vectors ? Ux : X1);
    auto* Vc = reinterpret_cast<rocblas_double_complex*>(vectors ? VxH : X1);
    {
      Tracer tr(h, s, BQ_KERNEL_HEEV_SOLVE, vectors ? 3 : 2, n, n, 0, 0.0, 0.0);
      const rocblas_status rs =
          heev_use_gesvd() ? rocsolver_zgesvd(h->rb, sv, sv, ni, ni, Xc, ni, D1, Uc, ld, Vc, ld, E, rocblas_outofplace, inf)
                           : rocsolver_zgesdd(h->rb, sv, sv, ni, ni, Xc, ni, D1, Uc, ld, Vc, ld, inf);
      tr.done();
      if (rs != rocblas_status_success)
        return fail(BQ_ERR_HIP, std::string("rocsolver singular value decomposition: ") + rocblas_status_to_string(rs));
    }
    // -s (list 1: S is descending, so -S ascends) and +s (list 2: S reversed).
    s1 = -1.0;
    list2 = D1;
    s2 = 1.0;
    rev = 1;
    for (int l = 0; l < 2; ++l) {
      asmb.xt[l] = Ux;
      asmb.ct[l][0] = r2;
      asmb.xb[l] = VxH;
      asmb.rows_b[l] = 1;
      asmb.conj_b[l] = 1;
      asmb.cb[l][0] = l == 0 ? -r2 : r2;
    }
    asmb.rev2 = 1;
  } else if (hc == HEEV_ANTI_J || hc == HEEV_ANTI_K) {
    // U^dagger Z U = diag(a Z12, -a Z12) with U = [[I, I], [a I, -a I]] / sqrt(2).
    const Cplx a = hc == HEEV_ANTI_J ? Cplx{0.0, 1.0} : Cplx{1.0, 0.0};
    if ((e = map(1, a, n, X1, n)) != hipSuccess) return hip_fail(e, "reduced block launch");
    if (bq_status_t st = solve(X1, n, D1, inf); st != BQ_OK) return st;
    list2 = D1;
    s2 = -1.0;
    rev = 1;
    // mu: [x; a x] / sqrt 2, -mu: [x; -a x] / sqrt 2
    asmb.xt[0] = asmb.xb[0] = asmb.xt[1] = asmb.xb[1] = X1;
    asmb.ct[0][0] = asmb.ct[1][0] = r2;
    asmb.cb[0][0] = r2 * a.re;
    asmb.cb[0][1] = r2 * a.im;
    asmb.cb[1][0] = -r2 * a.re;
    asmb.cb[1][1] = -r2 * a.im;
    asmb.rev2 = 1;
  } else {
    if ((e = map(0, {1.0, 0.0}, n, X1, n)) != hipSuccess) return hip_fail(e, "block launch");
    if (bq_status_t st = solve(X1, n, D1, inf); st != BQ_OK) return st;
    asmb.xt[0] = X1;
    asmb.ct[0][0] = 1.0;
    if (hc == HEEV_BLOCKS) {
      if ((e = map(3, {1.0, 0.0}, n, X2, n)) != hipSuccess) return hip_fail(e, "block launch");
      if (bq_status_t st = solve(X2, n, D2, inf + 1); st != BQ_OK) return st;
      list2 = D2;
      asmb.xb[1] = X2;
    } else {
      list2 = D1;  // Z22 = Z11, or conj(Z11): same eigenvalues
      asmb.xb[1] = X1;
      asmb.conj_b[1] = hc == HEEV_BLOCKS_CONJ;
    }
    asmb.cb[1][0] = 1.0;
  }
  {
    Tracer tr(h, s, BQ_KERNEL_HEEV_ASSEMBLE, -1, N, vectors ? N : 0, 0, 0.0,
              double(N) * 24.0 + (vectors ? double(N) * double(N) * 16.0 * 2.0 : 0.0));
    e = bq::launch_heev_merge(D1, n, s1, list2, n, s2, rev, w, src, s);
    if (e == hipSuccess && vectors) e = bq::launch_heev_assemble(asmb, s);
    tr.done();
    if (e != hipSuccess) return hip_fail(e, "eigenvalue merge / vector assembly launch");
  }
  if (info && (e = bq::launch_heev_info(inf, L.solves == 2 ? inf + 1 : nullptr, info, s)) != hipSuccess)
    return hip_fail(e, "info launch");
  return BQ_OK;
}

}  // extern "C"
