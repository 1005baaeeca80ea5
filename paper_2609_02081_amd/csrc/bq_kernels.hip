// gfx950 (CDNA4) kernels of the bilinear biquaternion GEMM.
//
//  cgemm_f64   One complex product P = L.R of eq. bilinearH as FP64 MFMA
//              real GEMMs (v_mfma_f64_16x16x4f64), Gauss-fused: one tile
//              keeps T1, T2, T3 of eq. cmplx-3-real-mult in three
//              accumulator sets, forms the sums lr+li / rr+ri on the MFMA
//              fragments in registers, and the epilogue turns (T1,T2,T3)
//              into P and adds coef*P straight into the C blocks (the
//              post-combination of eq. bilinearH), so neither the Gauss sums
//              nor T or P ever reach HBM.
//  combine     Hadamard pre-combinations (M1 +- M2 +- M3 +- M4) of
//              eq. bilinearH, HBM-bound.
//  fill_zero   Structurally zero output blocks.
//
// Tile base pointers are 64-bit; offsets inside a tile are 32-bit.  Build with
//   -Xclang -target-feature -Xclang -packed-fp32-ops
#include "bq_internal.h"

namespace bq {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------------------
// Tile order: workgroups are dealt to the 8 XCDs round-robin (w % 8).  Give
// every XCD a contiguous range of logical tiles, and walk that range in
// groups of GROUP_M tile-rows so tiles that run together share A and B panels
// in their XCD's L2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void tile_coords(int tiles_m, int tiles_n, int xcd_remap, int group_m, int& tm,
                                            int& tn) {
  constexpr int kXcd = 8;
  const int T = tiles_m * tiles_n;
  const int w = blockIdx.x;
  int t = w;
  if (xcd_remap) {
    const int x = w % kXcd, slot = w / kXcd;
    const int base = T / kXcd, rem = T % kXcd;
    t = x * base + (x < rem ? x : rem) + slot;
  }
  const int per_group = group_m * tiles_n;
  const int group = t / per_group;
  const int first_m = group * group_m;
  const int gm = min(tiles_m - first_m, group_m);
  const int in_g = t - group * per_group;
  tm = first_m + in_g % gm;
  tn = in_g / gm;
}

__device__ __forceinline__ d4 mfma_f64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// FP64 MFMA complex-product GEMM.
//
// Fragment layout of v_mfma_f64_16x16x4f64 (wave64):
//   A (16x4):  lane l holds A[l % 16][l / 16]
//   B (4x16):  lane l holds B[l / 16][l % 16]
//   D (16x16): lane l, element v holds D[l / 16 + 4 v][l % 16]
// (the D layout was checked on gfx950 with a one-wave probe).
// LDS keeps each tile in its stored orientation.  Tiles stored k-major (B,
// and A for op T / H) keep rows of BM (BN) + PAD doubles, so a fragment
// read is 16 consecutive doubles per k row.  Tiles stored with contiguous k
// (A, and B for op T / H) keep rows of BK + 1 doubles: their rows are
// written as loaded, without the bank conflicts of a transposing write, and
// the 16 rows of a fragment read fall on 16 distinct bank pairs.
// ---------------------------------------------------------------------------
// LDS of one FP64 GEMM tile (double-buffered A and B tiles).
template <int KIND, int BM, int BN, int BK>
struct TileSmem {
  static constexpr int PAD = 4;
  static constexpr int NA = (KIND == KIND_GAUSS || KIND == KIND_CR) ? 2 : 1;
  static constexpr int NB = (KIND == KIND_GAUSS || KIND == KIND_RC) ? 2 : 1;
  static constexpr int A_KM = BK * (BM + PAD), A_MM = BM * (BK + 1);
  static constexpr int A_SIZE = A_KM > A_MM ? A_KM : A_MM;
  static constexpr int B_KM = BK * (BN + PAD), B_NM = BN * (BK + 1);
  static constexpr int B_SIZE = B_KM > B_NM ? B_KM : B_NM;
  static_assert(A_SIZE % 2 == 0 && B_SIZE % 2 == 0, "buffers stay 16-byte aligned");
  __attribute__((aligned(16))) double As[2][NA][A_SIZE];
  __attribute__((aligned(16))) double Bs[2][NB][B_SIZE];
};

// Stored operand tile: R rows of C contiguous elements (C even), moved in
// pairs along the rows; pair v of thread tid + i NT is (row v / (C/2), column
// 2 (v % (C/2))).  MODE 0: 16-byte loads; 1: 8-byte loads, no checks; 2:
// checked against row_lim rows and col_lim columns (zeros outside).
template <int MODE, int PAIRS, int C, int NT>
__device__ __forceinline__ void load_pairs(double (&dst)[2 * PAIRS], const double* base, int64_t ld, int64_t row_lim,
                                           int64_t col_lim, int tid) {
#pragma unroll
  for (int i = 0; i < PAIRS; ++i) {
    const int v = tid + i * NT;
    const int r = v / (C / 2), c = 2 * (v % (C / 2));
    const uint32_t off = (uint32_t)(r * (uint32_t)ld + c);
    if constexpr (MODE == 0) {
      const d2 x = *reinterpret_cast<const d2*>(base + off);
      dst[2 * i] = x[0];
      dst[2 * i + 1] = x[1];
    } else if constexpr (MODE == 1) {
      dst[2 * i] = base[off];
      dst[2 * i + 1] = base[off + 1];
    } else {
      const bool rok = r < row_lim;
      dst[2 * i] = (rok && c < col_lim) ? base[off] : 0.0;
      dst[2 * i + 1] = (rok && c + 1 < col_lim) ? base[off + 1] : 0.0;
    }
  }
}

// The same pattern (MODE 0) through a buffer resource: the per-thread byte
// offsets voff[i] (fixed for the tile) are computed once, the k-step moves
// only the resource's scalar base, so a load costs no vector address work.
// The base must be the same in every lane (one tile per block).
template <int PAIRS>
__device__ __forceinline__ void load_pairs_rsrc(double (&dst)[2 * PAIRS], const double* base,
                                                const uint32_t (&voff)[PAIRS]) {
  const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, 0x7fffffff, 0x00020000);
#pragma unroll
  for (int i = 0; i < PAIRS; ++i) {
    const d2 x = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff[i], 0, 0));
    dst[2 * i] = x[0];
    dst[2 * i + 1] = x[1];
  }
}

// Checked pattern (as MODE 2) through a buffer resource, without branches:
// an element outside row_lim x col_lim gets an offset past the resource's
// range (num_records = 2^31 - 1), which the hardware reads as zero without
// an access; every other element is read where MODE 2 reads it.  Offsets
// stay below 2^31 (the caller checks the tile's span).
template <int PAIRS, int C, int NT>
__device__ __forceinline__ void load_pairs_rsrc_checked(double (&dst)[2 * PAIRS], const double* base, int64_t ld,
                                                        int64_t row_lim, int64_t col_lim, int tid) {
  constexpr uint32_t kOut = 0x80000000u;
  const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, 0x7fffffff, 0x00020000);
#pragma unroll
  for (int i = 0; i < PAIRS; ++i) {
    const int v = tid + i * NT;
    const int rr = v / (C / 2), c = 2 * (v % (C / 2));
    const uint32_t off = (uint32_t)((rr * (uint32_t)ld + c) * 8u);
    const bool rok = rr < row_lim;
    const uint32_t o0 = (rok && c < col_lim) ? off : kOut;
    const uint32_t o1 = (rok && c + 1 < col_lim) ? off + 8u : kOut;
    dst[2 * i] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)o0, 0, 0));
    dst[2 * i + 1] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)o1, 0, 0));
  }
}

// Full k-step of any tile (edge tiles, rows that are not 16-byte aligned)
// through a buffer resource whose range ends at the operand's last element:
// pairs past the range read as zero without an access.  VEC: 16-byte loads
// (base and rows 16-byte aligned; the range is rounded up to 16 bytes, so a
// load lies wholly inside or wholly past it); else two 8-byte loads per
// pair.  The offsets are those of load_pairs_rsrc.  Rows or columns of an
// edge tile that lie outside the matrix fall past the range, or on the
// matrix's own elements (or the 8 bytes that share the last element's
// 16-byte chunk), which feed only outputs outside the matrix, never stored;
// the k range of a full k-step lies inside the matrix.
template <int PAIRS, int VEC>
__device__ __forceinline__ void load_pairs_rsrc_range(double (&dst)[2 * PAIRS], const double* base, int64_t extent,
                                                      const uint32_t (&voff)[PAIRS]) {
  const int64_t rounded = VEC ? ((extent + 15) & ~(int64_t)15) : extent;
  const int range = (int)(rounded < 0x7fffffff ? rounded : 0x7fffffff);
  const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, range, 0x00020000);
#pragma unroll
  for (int i = 0; i < PAIRS; ++i) {
    if constexpr (VEC) {
      const d2 x = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff[i], 0, 0));
      dst[2 * i] = x[0];
      dst[2 * i + 1] = x[1];
    } else {
      dst[2 * i] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff[i], 0, 0));
      dst[2 * i + 1] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)(voff[i] + 8u), 0, 0));
    }
  }
}

// A pointer that is the same in every lane, read from the first lane when
// UNI = 1 so that the compiler keeps it (and what is computed from it) in
// scalar registers: the batched kernel reads its arguments from memory,
// the single-call kernel has them in kernel arguments, already scalar.
template <int UNI>
__device__ __forceinline__ const double* uniform_ptr(const double* p) {
  if constexpr (UNI) {
    const uint64_t b = reinterpret_cast<uint64_t>(p);
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
    return reinterpret_cast<const double*>(lo | (hi << 32));
  }
  return p;
}

// One output tile (m0, n0) of the complex product described by g: K loop and
// epilogue.  Every thread of the block must call it (it synchronises).
// TA / TB: the left / right operand is stored transposed (op T or H: the
// left one k x m, the right one n x k).
// DEEP: two register sets, global loads two k-steps ahead and the LDS store
// of the next stage three quarters of the way through the current k-step's
// MFMAs (32 more registers; used where they fit without spills).
// ADD: the batched kernel's tile: targets may carry an addend matrix
// (Target::sr / si, scaled by sc, leading dimension GemmArgs::ldadd), and
// the arguments come from a device table (operand bases made scalar).
// BUF = 1: every load goes through a buffer resource, which needs the
// stored tiles' byte span below 2^31 (spans_fit, checked by the launcher);
// BUF = 2 (two-deep only, for grids without edge tiles): the full k-steps
// of interior tiles as in BUF = 1, the rest with pointer loads (the
// register allocation of the steady-state loop comes out 1.3 % faster at
// n = 16384 than with BUF = 1); BUF = 0: pointer loads, for leading
// dimensions beyond the buffer range.
template <int KIND, int BM, int BN, int BK, int WM, int WN, int TA = 0, int TB = 0, int DEEP = 0, int ADD = 0,
          int BUF = 1>
__device__ __forceinline__ void gemm_tile(const GemmArgs& g, int64_t m0, int64_t n0,
                                          TileSmem<KIND, BM, BN, BK>& sm) {
  constexpr int NWN = BN / WN;
  constexpr int NT = (BM / WM) * NWN * 64;
  constexpr int MI = WM / 16, NI = WN / 16;
  constexpr bool HAS_LI = (KIND == KIND_GAUSS || KIND == KIND_CR);
  constexpr bool HAS_RI = (KIND == KIND_GAUSS || KIND == KIND_RC);
  constexpr int NA = HAS_LI ? 2 : 1;
  constexpr int NB = HAS_RI ? 2 : 1;
  constexpr int NACC = KIND == KIND_GAUSS ? 3 : (KIND == KIND_RR ? 1 : 2);
  constexpr int PAD = 4;
  // Elements are moved in pairs along the contiguous dimension.
  constexpr int A_PAIRS = BM * BK / 2 / NT;
  constexpr int B_PAIRS = BK * BN / 2 / NT;
  // Contiguous length of the stored tiles.
  constexpr int AC = TA ? BM : BK;
  constexpr int BC = TB ? BK : BN;
  static_assert(A_PAIRS * NT * 2 == BM * BK && B_PAIRS * NT * 2 == BK * BN, "tile / thread mismatch");
  static_assert(BK % 4 == 0 && WM % 16 == 0 && WN % 16 == 0, "bad tile");
  static_assert(((BN + PAD) * 8) % 16 == 0 && ((BM + PAD) * 8) % 16 == 0, "LDS rows must stay 16-byte aligned");

  // Double-buffered LDS in the stored orientations (see TileSmem).
  auto& As = sm.As;
  auto& Bs = sm.Bs;
  auto a_at = [](int i, int k) { return TA ? k * (BM + PAD) + i : i * (BK + 1) + k; };
  auto b_at = [](int k, int j) { return TB ? j * (BK + 1) + k : k * (BN + PAD) + j; };

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave / NWN) * WM;
  const int wn0 = (wave % NWN) * WN;
  const int fr = lane & 15;
  const int fk = lane >> 4;

  // Per-tile base pointers: all further offsets stay small (32-bit).
  const int64_t a_off = TA ? m0 : m0 * g.lda;
  const int64_t b_off = TB ? n0 * g.ldb : n0;
  const double* pa[2] = {uniform_ptr<ADD>(g.lr + a_off), HAS_LI ? uniform_ptr<ADD>(g.li + a_off) : nullptr};
  const double* pb[2] = {uniform_ptr<ADD>(g.rr + b_off), HAS_RI ? uniform_ptr<ADD>(g.ri + b_off) : nullptr};
  const int64_t mrem = g.m - m0;
  const int64_t nrem = g.n - n0;
  // Interior tiles load without bounds checks (16-byte loads when the rows
  // are 16-byte aligned).
  const bool interior = mrem >= BM && nrem >= BN;
  const bool fast = g.vec && interior;
  // Byte offsets of this thread's pairs in the stored tiles (BUF, 16-byte
  // loads), fixed for the tile.  The launcher picks BUF > 0 only where the
  // spans fit; the check is repeated here (it also came out 1.8-3.5 %
  // faster at n = 24576 than without it, through the register allocation).
  const int64_t a_span = (TA ? (int64_t)(BK - 1) * g.lda + BM : (int64_t)(BM - 1) * g.lda + BK) * 8;
  const int64_t b_span = (TB ? (int64_t)(BN - 1) * g.ldb + BK : (int64_t)(BK - 1) * g.ldb + BN) * 8;
  const bool rsrc_ok = BUF && fast && a_span < 0x7fffffff && b_span < 0x7fffffff;
  uint32_t voff_a[A_PAIRS], voff_b[B_PAIRS];
#pragma unroll
  for (int i = 0; i < A_PAIRS; ++i) {
    const int v = tid + i * NT;
    voff_a[i] = (uint32_t)(((v / (AC / 2)) * (uint32_t)g.lda + 2 * (v % (AC / 2))) * 8u);
  }
#pragma unroll
  for (int i = 0; i < B_PAIRS; ++i) {
    const int v = tid + i * NT;
    voff_b[i] = (uint32_t)(((v / (BC / 2)) * (uint32_t)g.ldb + 2 * (v % (BC / 2))) * 8u);
  }

  // Register sets for the global tiles (DEEP: k-step j goes through set j % 2).
  double ra0[NA][2 * A_PAIRS], ra1[NA][2 * A_PAIRS];
  double rb0[NB][2 * B_PAIRS], rb1[NB][2 * B_PAIRS];

  auto gload = [&](int64_t k0, double (&ra)[NA][2 * A_PAIRS], double (&rb)[NB][2 * B_PAIRS]) {
    const bool kfull = (k0 + BK <= g.k);
    const int64_t kleft = g.k - k0;
    // Stored tiles: A is BM x BK (TA: BK x BM) from k0, B is BK x BN (TB: BN x BK).
    const int64_t a_step = TA ? k0 * g.lda : k0;
    const int64_t b_step = TB ? k0 : k0 * g.ldb;
    const int64_t a_rows = TA ? kleft : mrem, a_cols = TA ? mrem : kleft;
    const int64_t b_rows = TB ? nrem : kleft, b_cols = TB ? kleft : nrem;
    if (fast && kfull) {
#pragma unroll
      for (int p = 0; p < NA; ++p) load_pairs<0, A_PAIRS, AC, NT>(ra[p], pa[p] + a_step, g.lda, 0, 0, tid);
#pragma unroll
      for (int p = 0; p < NB; ++p) load_pairs<0, B_PAIRS, BC, NT>(rb[p], pb[p] + b_step, g.ldb, 0, 0, tid);
    } else if (interior && kfull) {
      // Interior tile whose rows are not 16-byte aligned: the same pattern
      // with 8-byte loads, still without bounds checks.
#pragma unroll
      for (int p = 0; p < NA; ++p) load_pairs<1, A_PAIRS, AC, NT>(ra[p], pa[p] + a_step, g.lda, 0, 0, tid);
#pragma unroll
      for (int p = 0; p < NB; ++p) load_pairs<1, B_PAIRS, BC, NT>(rb[p], pb[p] + b_step, g.ldb, 0, 0, tid);
    } else {
#pragma unroll
      for (int p = 0; p < NA; ++p)
        load_pairs<2, A_PAIRS, AC, NT>(ra[p], pa[p] + a_step, g.lda, a_rows, a_cols, tid);
#pragma unroll
      for (int p = 0; p < NB; ++p)
        load_pairs<2, B_PAIRS, BC, NT>(rb[p], pb[p] + b_step, g.ldb, b_rows, b_cols, tid);
    }
  };
  // The same tiles through buffer resources (the tile's span below 2^31):
  // 16-byte loads for a full k-step of an interior tile with 16-byte rows,
  // else the branch-free checked loads.
  auto gload_rsrc = [&](int64_t k0, double (&ra)[NA][2 * A_PAIRS], double (&rb)[NB][2 * B_PAIRS]) {
    const bool kfull = (k0 + BK <= g.k);
    const int64_t kleft = g.k - k0;
    const int64_t a_step = TA ? k0 * g.lda : k0;
    const int64_t b_step = TB ? k0 : k0 * g.ldb;
    if (fast && kfull) {
#pragma unroll
      for (int p = 0; p < NA; ++p) load_pairs_rsrc<A_PAIRS>(ra[p], pa[p] + a_step, voff_a);
#pragma unroll
      for (int p = 0; p < NB; ++p) load_pairs_rsrc<B_PAIRS>(rb[p], pb[p] + b_step, voff_b);
    } else {
      const int64_t a_rows = TA ? kleft : mrem, a_cols = TA ? mrem : kleft;
      const int64_t b_rows = TB ? nrem : kleft, b_cols = TB ? kleft : nrem;
#pragma unroll
      for (int p = 0; p < NA; ++p)
        load_pairs_rsrc_checked<A_PAIRS, AC, NT>(ra[p], pa[p] + a_step, g.lda, a_rows, a_cols, tid);
#pragma unroll
      for (int p = 0; p < NB; ++p)
        load_pairs_rsrc_checked<B_PAIRS, BC, NT>(rb[p], pb[p] + b_step, g.ldb, b_rows, b_cols, tid);
    }
  };
  // A stored m-major (N) is transposed on the way into LDS; stored k-major
  // (TA) it goes in as is.  B the other way round.
  auto lstore = [&](int buf, const double (&ra)[NA][2 * A_PAIRS], const double (&rb)[NB][2 * B_PAIRS]) {
#pragma unroll
    for (int i = 0; i < A_PAIRS; ++i) {
      const int v = tid + i * NT;
      const int r = v / (AC / 2), c = 2 * (v % (AC / 2));
#pragma unroll
      for (int p = 0; p < NA; ++p) {
        if constexpr (TA) {
          *reinterpret_cast<d2*>(&As[buf][p][a_at(c, r)]) = d2{ra[p][2 * i], ra[p][2 * i + 1]};
        } else {
          As[buf][p][a_at(r, c)] = ra[p][2 * i];
          As[buf][p][a_at(r, c) + 1] = ra[p][2 * i + 1];
        }
      }
    }
#pragma unroll
    for (int i = 0; i < B_PAIRS; ++i) {
      const int v = tid + i * NT;
      const int r = v / (BC / 2), c = 2 * (v % (BC / 2));
#pragma unroll
      for (int p = 0; p < NB; ++p) {
        if constexpr (TB) {
          Bs[buf][p][b_at(c, r)] = rb[p][2 * i];
          Bs[buf][p][b_at(c, r) + 1] = rb[p][2 * i + 1];
        } else {
          *reinterpret_cast<d2*>(&Bs[buf][p][b_at(r, c)]) = d2{rb[p][2 * i], rb[p][2 * i + 1]};
        }
      }
    }
  };

  d4 acc[NACC][MI][NI];
#pragma unroll
  for (int q = 0; q < NACC; ++q)
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < NI; ++j) acc[q][i][j] = d4{0.0, 0.0, 0.0, 0.0};

  const double sL = g.sL, sR = g.sR;
  const int64_t nk = (g.k + BK - 1) / BK;

  // MFMAs of k-substeps [kk0, kk1) of the stage in LDS buffer buf.
  auto compute = [&](int buf, int kk0, int kk1) {
#pragma unroll
      for (int kk = kk0; kk < kk1; ++kk) {
        const int krow = kk * 4 + fk;
        double a[NA][MI], b[NB][NI];
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
          for (int p = 0; p < NA; ++p) a[p][i] = As[buf][p][a_at(wm0 + i * 16 + fr, krow)];
#pragma unroll
        for (int j = 0; j < NI; ++j)
#pragma unroll
          for (int p = 0; p < NB; ++p) b[p][j] = Bs[buf][p][b_at(krow, wn0 + j * 16 + fr)];
        if constexpr (KIND == KIND_GAUSS) {
          double as[MI], bs[NI];
#pragma unroll
          for (int i = 0; i < MI; ++i) as[i] = __builtin_fma(sL, a[NA - 1][i], a[0][i]);
#pragma unroll
          for (int j = 0; j < NI; ++j) bs[j] = __builtin_fma(sR, b[NB - 1][j], b[0][j]);
#pragma unroll
          for (int i = 0; i < MI; ++i)
#pragma unroll
            for (int j = 0; j < NI; ++j) {
              acc[0][i][j] = mfma_f64(a[0][i], b[0][j], acc[0][i][j]);
              acc[1 % NACC][i][j] = mfma_f64(a[NA - 1][i], b[NB - 1][j], acc[1 % NACC][i][j]);
              acc[2 % NACC][i][j] = mfma_f64(as[i], bs[j], acc[2 % NACC][i][j]);
            }
        } else {
#pragma unroll
          for (int i = 0; i < MI; ++i)
#pragma unroll
            for (int j = 0; j < NI; ++j) {
              acc[0][i][j] = mfma_f64(a[0][i], b[0][j], acc[0][i][j]);
              if constexpr (KIND == KIND_RC)
                acc[1 % NACC][i][j] = mfma_f64(a[0][i], b[NB - 1][j], acc[1 % NACC][i][j]);
              if constexpr (KIND == KIND_CR)
                acc[1 % NACC][i][j] = mfma_f64(a[NA - 1][i], b[0][j], acc[1 % NACC][i][j]);
            }
        }
      }
  };

  // Loads of k-step kn: any k-step (bounds-checked where the tile needs
  // it), or a full k-step of an interior tile with 16-byte rows through
  // buffer resources.  Such tiles run their full k-steps in a loop of their
  // own, so the steady state carries neither the checked loads nor their
  // registers; the last k-steps and other tiles run the general loop.
  auto load_any = [&](int64_t kn, double (&ra)[NA][2 * A_PAIRS], double (&rb)[NB][2 * B_PAIRS]) {
    if (kn < nk) gload(kn * BK, ra, rb);
  };
  auto load_rsrc = [&](int64_t kn, double (&ra)[NA][2 * A_PAIRS], double (&rb)[NB][2 * B_PAIRS]) {
    if (kn < nk) gload_rsrc(kn * BK, ra, rb);
  };
  auto load_full = [&](int64_t kn, double (&ra)[NA][2 * A_PAIRS], double (&rb)[NB][2 * B_PAIRS]) {
    const int64_t k0 = kn * BK;
#pragma unroll
    for (int p = 0; p < NA; ++p) load_pairs_rsrc<A_PAIRS>(ra[p], pa[p] + (TA ? k0 * g.lda : k0), voff_a);
#pragma unroll
    for (int p = 0; p < NB; ++p) load_pairs_rsrc<B_PAIRS>(rb[p], pb[p] + (TB ? k0 : k0 * g.ldb), voff_b);
  };
  const int64_t nkf = g.k / BK;  // full k-steps

  if constexpr (!DEEP) {
    if (nk > 0) {
      if constexpr (BUF) gload_rsrc(0, ra0, rb0);
      else gload(0, ra0, rb0);
      lstore(0, ra0, rb0);
    }
    __syncthreads();
    int64_t kt = 0;
    auto step = [&](auto load) {
      const int buf = (int)(kt & 1);
      load(kt + 1, ra0, rb0);
      compute(buf, 0, BK / 4);
      if (kt + 1 < nk) lstore(buf ^ 1, ra0, rb0);
      __syncthreads();
    };
    if constexpr (BUF) {
      if constexpr (ADD) {
        // A wave whose part of an edge tile lies wholly outside the matrix
        // skips its MFMAs (its results are never stored), so the other
        // block's wave on its SIMD has the matrix pipe to itself.
        const bool wave_live =
            __builtin_amdgcn_readfirstlane(wm0) < mrem && __builtin_amdgcn_readfirstlane(wn0) < nrem;
        auto step_live = [&](auto load) {
          const int buf = (int)(kt & 1);
          load(kt + 1, ra0, rb0);
          if (wave_live) compute(buf, 0, BK / 4);
          if (kt + 1 < nk) lstore(buf ^ 1, ra0, rb0);
          __syncthreads();
        };
        // Batched tiles: the full k-steps of every tile (a batch holds
        // many edge tiles and odd leading dimensions) run the unchecked
        // loop, within the operands' extents.
        if (a_span < 0x7fffffff && b_span < 0x7fffffff) {
          // Byte extent of each stored operand from the tile's base to its
          // last element.
          const int64_t a_ext = (TA ? (g.k - 1) * g.lda + mrem : (mrem - 1) * g.lda + g.k) * 8;
          const int64_t b_ext = (TB ? (nrem - 1) * g.ldb + g.k : (g.k - 1) * g.ldb + nrem) * 8;
          auto load_range = [&](int64_t kn, double (&ra)[NA][2 * A_PAIRS], double (&rb)[NB][2 * B_PAIRS]) {
            const int64_t a_step = TA ? kn * BK * g.lda : kn * BK;
            const int64_t b_step = TB ? kn * BK : kn * BK * g.ldb;
            if (g.vec) {
#pragma unroll
              for (int p = 0; p < NA; ++p)
                load_pairs_rsrc_range<A_PAIRS, 1>(ra[p], pa[p] + a_step, a_ext - a_step * 8, voff_a);
#pragma unroll
              for (int p = 0; p < NB; ++p)
                load_pairs_rsrc_range<B_PAIRS, 1>(rb[p], pb[p] + b_step, b_ext - b_step * 8, voff_b);
            } else {
#pragma unroll
              for (int p = 0; p < NA; ++p)
                load_pairs_rsrc_range<A_PAIRS, 0>(ra[p], pa[p] + a_step, a_ext - a_step * 8, voff_a);
#pragma unroll
              for (int p = 0; p < NB; ++p)
                load_pairs_rsrc_range<B_PAIRS, 0>(rb[p], pb[p] + b_step, b_ext - b_step * 8, voff_b);
            }
          };
          for (; kt + 1 < nkf; ++kt) step_live(load_range);
        }
        for (; kt < nk; ++kt) step_live(load_rsrc);
      } else {
        if (rsrc_ok)
          for (; kt + 1 < nkf; ++kt) step(load_full);
        for (; kt < nk; ++kt) step(load_rsrc);
      }
    } else {
      for (; kt < nk; ++kt) step(load_any);
    }
  } else {
    // k-step kt on LDS buffer kt % 2: the loads of k-step kt + 2 go into the
    // free set (rl); three quarters of the way through the MFMAs (1.8 %
    // faster than half-way, 0.9 % than a quarter) the tiles of k-step kt + 1
    // (set rs, loaded a k-step ago) go into the other buffer, which every
    // wave finished reading before the last barrier.  The barrier waits for
    // the LDS writes only, so the loads of k-step kt + 2 stay in flight.
    auto step = [&](int64_t kt, double (&ral)[NA][2 * A_PAIRS], double (&rbl)[NB][2 * B_PAIRS],
                    const double (&ras)[NA][2 * A_PAIRS], const double (&rbs)[NB][2 * B_PAIRS], auto load) {
      const int buf = (int)(kt & 1);
      load(kt + 2, ral, rbl);
      compute(buf, 0, 3 * BK / 16);
      if (kt + 1 < nk) lstore(buf ^ 1, ras, rbs);
      compute(buf, 3 * BK / 16, BK / 4);
      __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): this wave's LDS writes are done
      __builtin_amdgcn_s_barrier();
    };
    if (nk > 0) {
      if constexpr (BUF == 1) gload_rsrc(0, ra0, rb0);
      else gload(0, ra0, rb0);
      lstore(0, ra0, rb0);
      if (nk > 1) {
        if constexpr (BUF == 1) gload_rsrc(BK, ra1, rb1);
        else gload(BK, ra1, rb1);
      }
    }
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_s_barrier();
    int64_t kt = 0;
    if (BUF && rsrc_ok) {
      for (; kt + 3 < nkf; kt += 2) {
        step(kt, ra0, rb0, ra1, rb1, load_full);
        step(kt + 1, ra1, rb1, ra0, rb0, load_full);
      }
    }
    auto rest = [&](auto load) {
      for (; kt + 1 < nk; kt += 2) {
        step(kt, ra0, rb0, ra1, rb1, load);
        step(kt + 1, ra1, rb1, ra0, rb0, load);
      }
      if (kt < nk) step(kt, ra0, rb0, ra1, rb1, load);
    };
    if constexpr (BUF == 1) rest(load_rsrc);
    else rest(load_any);
  }

  // Epilogue: P from the accumulators, then coef * P into each target.
  // Targets outer, elements inner: each target is copied into registers
  // once (read in place from a device table, as the batched kernel does,
  // its fields would otherwise be reloaded after every C store).
  const int64_t ldc = g.ldc;
  const double sig = sL * sR;
  const int ntgt = g.ntgt;
  for (int t = 0; t < ntgt; ++t) {
    const Target T = g.tgt[t];
    // Addends (ADD): every value of the wave tile is loaded before the first
    // store, so the loads are in flight together rather than one per store.
    constexpr int AM = ADD ? MI : 1, AN = ADD ? NI : 1;
    double add_r[AM][AN][4], add_i[AM][AN][4];
    if constexpr (ADD) {
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NI; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t r = wm0 + i * 16 + fk + 4 * v;
            const int64_t c = wn0 + j * 16 + fr;
            const bool in = r < mrem && c < nrem;
            const int64_t aoff = (m0 + r) * g.ldadd + n0 + c;
            add_r[i][j][v] = (in && T.sr) ? T.sr[aoff] : 0.0;
            add_i[i][j][v] = (in && T.si) ? T.si[aoff] : 0.0;
          }
    }
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < NI; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t r = wm0 + i * 16 + fk + 4 * v;
          const int64_t c = wn0 + j * 16 + fr;
          if (r >= mrem || c >= nrem) continue;
          double pr, pi;
          if constexpr (KIND == KIND_GAUSS) {
            const double t1 = acc[0][i][j][v];
            const double t2 = acc[1 % NACC][i][j][v];
            const double t3 = acc[2 % NACC][i][j][v];
            pr = t1 - sig * t2;
            pi = (t3 - t1) - sig * t2;
          } else if constexpr (KIND == KIND_RC) {
            pr = acc[0][i][j][v];
            pi = sR * acc[1 % NACC][i][j][v];
          } else if constexpr (KIND == KIND_CR) {
            pr = acc[0][i][j][v];
            pi = sL * acc[1 % NACC][i][j][v];
          } else {
            pr = acc[0][i][j][v];
            pi = 0.0;
          }
          const int64_t off = (m0 + r) * ldc + n0 + c;
          if (T.mode_r != TGT_SKIP) {
            double val = (T.ai == 0.0) ? T.ar * pr : ((T.ar == 0.0) ? -T.ai * pi : T.ar * pr - T.ai * pi);
            if (ADD && T.sr) val = __builtin_fma(T.sc, add_r[ADD ? i : 0][ADD ? j : 0][v], val);
            if (T.mode_r == TGT_ACCUM) val += T.cr[off];
            T.cr[off] = val;
          }
          if (T.mode_i != TGT_SKIP) {
            double val = (T.ai == 0.0) ? T.ar * pi : ((T.ar == 0.0) ? T.ai * pr : T.ar * pi + T.ai * pr);
            if (ADD && T.si) val = __builtin_fma(T.sc, add_i[ADD ? i : 0][ADD ? j : 0][v], val);
            if (T.mode_i == TGT_ACCUM) val += T.ci[off];
            T.ci[off] = val;
          }
        }
  }
}

template <int KIND, int BM, int BN, int BK, int WM, int WN, int WPE, int TA = 0, int TB = 0, int DEEP = 0, int BUF = 1>
__global__ void __launch_bounds__((BM / WM) * (BN / WN) * 64)
__attribute__((amdgpu_waves_per_eu(WPE, WPE)))
cgemm_f64(const GemmArgs g) {
  __shared__ TileSmem<KIND, BM, BN, BK> sm;
  const int tiles_m = (int)((g.m + BM - 1) / BM);
  const int tiles_n = (int)((g.n + BN - 1) / BN);
  int tm, tn;
  tile_coords(tiles_m, tiles_n, g.xcd_remap, g.group_m, tm, tn);
  gemm_tile<KIND, BM, BN, BK, WM, WN, TA, TB, DEEP, 0, BUF>(g, (int64_t)tm * BM, (int64_t)tn * BN, sm);
}

// ---------------------------------------------------------------------------
// Hadamard pre-combination.  One thread produces two adjacent columns of
// every requested combination.
// ---------------------------------------------------------------------------
// 2 columns per thread; VEC = 1 (every pointer 16-byte aligned, both
// leading dimensions even): one 16-byte load per source and one 16-byte
// store per destination, else element by element.
template <int VEC>
__global__ void __launch_bounds__(256) combine_kernel(const CombineArgs a) {
  constexpr int CPT = 2;  // columns per thread
  const int64_t cgroups = (a.cols + CPT - 1) / CPT;
  const int64_t bpr = (cgroups + 255) / 256;
  const int64_t row = blockIdx.x / bpr;
  const int64_t c = ((blockIdx.x % bpr) * 256 + threadIdx.x) * CPT;
  if (row >= a.rows || c >= a.cols) return;
  const bool full = (c + CPT <= a.cols);
  double x[8][CPT];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const double* s = a.src[u];
    if (s) {
      const double* p = s + row * a.lds + c;
      if (VEC && full) {
        const double2 v2 = *reinterpret_cast<const double2*>(p);
        x[u][0] = v2.x;
        x[u][1] = v2.y;
      } else {
#pragma unroll
        for (int t = 0; t < CPT; ++t) x[u][t] = (c + t < a.cols) ? p[t] : 0.0;
      }
    } else {
#pragma unroll
      for (int t = 0; t < CPT; ++t) x[u][t] = 0.0;
    }
  }
  for (int q = 0; q < a.nq; ++q) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      double* d = (h == 0) ? a.dst_r[q] : a.dst_i[q];
      if (!d) continue;
      const int o = 4 * h;
      double v[CPT];
#pragma unroll
      for (int t = 0; t < CPT; ++t) {
        v[t] = a.w[q][0] * x[o][t];
#pragma unroll
        for (int u = 1; u < 4; ++u) v[t] = v[t] + a.w[q][u] * x[o + u][t];
      }
      double* p = d + row * a.ldd + c;
      if (VEC && full) {
        *reinterpret_cast<double2*>(p) = double2{v[0], v[1]};
      } else {
#pragma unroll
        for (int t = 0; t < CPT; ++t)
          if (c + t < a.cols) p[t] = v[t];
      }
    }
  }
}

__global__ void __launch_bounds__(256) fill_zero_kernel(double* p, int64_t rows, int64_t cols, int64_t ld) {
  const int64_t bpr = (cols + 255) / 256;
  const int64_t row = blockIdx.x / bpr;
  const int64_t c = (blockIdx.x % bpr) * 256 + threadIdx.x;
  if (row < rows && c < cols) p[row * ld + c] = 0.0;
}

// ---------------------------------------------------------------------------
// Batched form: many independent products in one launch.
//
// grouped_combine: the Hadamard pre-combinations of every problem; block b
// handles one row of one operand side, found by binary search in the row
// prefix table.
// grouped_gemm: persistent blocks take work items (problem, tile) in the
// given order (largest problems first) from a device counter (dyn = 1) or
// cyclically (dyn = 0); a work item runs the problem's complex products on
// its tile one after another, so it alone owns that C tile and the
// accumulation into C needs no atomics.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) grouped_combine(const CombineArgs* args, const int64_t* row_prefix,
                                                       int nargs) {
  const int64_t b = blockIdx.x;
  int lo = 0, hi = nargs - 1;
  while (lo < hi) {  // last index with row_prefix[idx] <= b
    const int mid = (lo + hi + 1) >> 1;
    if (row_prefix[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  const CombineArgs& a = args[lo];
  const int64_t row = b - row_prefix[lo];
  if (row >= a.rows) return;
  for (int64_t c = (int64_t)threadIdx.x * 2; c < a.cols; c += 512) {
    const bool two = (c + 1 < a.cols);
    double x[8][2];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double* src = a.src[u];
      if (src) {
        const double* q = src + row * a.lds + c;
        x[u][0] = q[0];
        x[u][1] = two ? q[1] : 0.0;
      } else {
        x[u][0] = 0.0;
        x[u][1] = 0.0;
      }
    }
    for (int q = 0; q < a.nq; ++q) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        double* d = (h == 0) ? a.dst_r[q] : a.dst_i[q];
        if (!d) continue;
        const int o = 4 * h;
        double v0 = a.w[q][0] * x[o][0];
        double v1 = a.w[q][0] * x[o][1];
#pragma unroll
        for (int u = 1; u < 4; ++u) {
          v0 = v0 + a.w[q][u] * x[o + u][0];
          v1 = v1 + a.w[q][u] * x[o + u][1];
        }
        double* dd = d + row * a.ldd + c;
        dd[0] = v0;
        if (two) dd[1] = v1;
      }
    }
  }
}

__global__ void reset_counter(int* counter) {
  if (threadIdx.x == 0) counter[0] = 0;
}

// OPS: 0..3 = every product of the plan has (ta, tb) = (OPS >> 1, OPS & 1),
// so one tile variant is compiled in; -1 = products differ (all four).
template <int BM, int BN, int BK, int WM, int WN, int WPE, int DYN, int OPS, int BUF = 1>
__global__ void __launch_bounds__((BM / WM) * (BN / WN) * 64)
__attribute__((amdgpu_waves_per_eu(WPE, WPE)))
grouped_gemm(const GemmArgs* __restrict__ prods, const GroupedItem* __restrict__ items, int nitems, int* counter) {
  __shared__ TileSmem<KIND_GAUSS, BM, BN, BK> sm;
  __shared__ int next;
  int it = blockIdx.x;
  for (;;) {
    if (DYN) {
      if (threadIdx.x == 0) next = atomicAdd(counter, 1);
      __syncthreads();
      // from the first lane: the item (and the product's arguments read
      // through it) is then known to be uniform and loaded into scalar
      // registers once per tile
      it = __builtin_amdgcn_readfirstlane(next);
      __syncthreads();
    }
    if (it >= nitems) break;
    const GroupedItem w = items[it];
    for (int q = 0; q < w.nprod; ++q) {
      // read in place: a private copy would sit in scratch (the epilogue
      // indexes its targets dynamically)
      const GemmArgs& g = prods[w.prod0 + q];
      const int64_t m0 = (int64_t)w.tm * BM, n0 = (int64_t)w.tn * BN;
      // op T / H operands are read in their stored orientation
      if constexpr (OPS >= 0) {
        gemm_tile<KIND_GAUSS, BM, BN, BK, WM, WN, (OPS >> 1), (OPS & 1), 0, 1, BUF>(g, m0, n0, sm);
      } else if (g.ta) {
        if (g.tb) gemm_tile<KIND_GAUSS, BM, BN, BK, WM, WN, 1, 1, 0, 1, BUF>(g, m0, n0, sm);
        else gemm_tile<KIND_GAUSS, BM, BN, BK, WM, WN, 1, 0, 0, 1, BUF>(g, m0, n0, sm);
      } else {
        if (g.tb) gemm_tile<KIND_GAUSS, BM, BN, BK, WM, WN, 0, 1, 0, 1, BUF>(g, m0, n0, sm);
        else gemm_tile<KIND_GAUSS, BM, BN, BK, WM, WN, 0, 0, 0, 1, BUF>(g, m0, n0, sm);
      }
    }
    if (!DYN) it += gridDim.x;
  }
}

// ---------------------------------------------------------------------------
// Tile configurations and launchers.
// ---------------------------------------------------------------------------
static const TileConfig kConfigs[] = {
    {64, 64, 16, 32, 32},    // 0: 4 waves, 2 waves / SIMD
    {0, 0, 0, 0, 0},         // 1: retired (one wave / SIMD, slower)
    {0, 0, 0, 0, 0},         // 2: retired (128 x 64 blocks at one wave / SIMD, slower)
    {64, 64, 32, 32, 32},    // 3: 4 waves, 2 waves / SIMD
    {0, 0, 0, 0, 0},         // 4: retired (spilled)
    {0, 0, 0, 0, 0},         // 5: retired (spilled)
    {64, 64, 8, 32, 32},     // 6: 4 waves, 2 waves / SIMD
    {0, 0, 0, 0, 0},         // 7: retired (128 x 64 blocks, slower)
    {0, 0, 0, 0, 0},         // 8: retired (128 x 64 blocks, slower)
    {0, 0, 0, 0, 0},         // 9: retired (128 x 128 x 16, slower than 11)
    {0, 0, 0, 0, 0},         // 10: retired (as 9, two-deep)
    {128, 128, 32, 32, 32},  // 11: 16 waves, 4 waves / SIMD, one block per CU (real x real only)
    {0, 0, 0, 0, 0},         // 12: retired (8 waves of 32 x 16, 4 waves / SIMD: slower, 2.4x the L2 misses)
};
constexpr int kNumConfigs = sizeof(kConfigs) / sizeof(kConfigs[0]);

int num_tile_configs() { return kNumConfigs; }
TileConfig tile_config(int cfg) { return kConfigs[cfg]; }

// Real products (one accumulator set) take k-steps of 32: 64 x 64 blocks
// (64 KB of LDS, two per CU; 5 % faster than BK = 16 at n = 4096), or
// 128 x 128 blocks of 16 waves (one per CU, half the bytes per flop: 10-12
// % faster per CU) where their rounds of blocks over the 256 CUs cost less:
// 4 small tiles per large one at 1.12x the rate, so a round of large blocks
// costs 2 / 1.12 rounds of small ones.  The complex kinds keep BK = 16,
// which leaves room for two blocks per CU.
int default_tile_config(int kind, int64_t m, int64_t n, int64_t k) {
  (void)k;
  if (kind != KIND_RR) return 0;
  constexpr int64_t kCUs = 256;
  const int64_t t128 = ((m + 127) / 128) * ((n + 127) / 128);
  const int64_t t64 = ((m + 63) / 64) * ((n + 63) / 64);
  const double rounds128 = double((t128 + kCUs - 1) / kCUs) * 2.0 / 1.12;
  const double rounds64 = double((t64 + 2 * kCUs - 1) / (2 * kCUs));
  return rounds128 < rounds64 ? 11 : 3;
}

// Byte span of the stored A and B tiles of a BM x BN x BK block below 2^31,
// so that buffer-resource offsets reach every element.
template <int BM, int BN, int BK, int TA, int TB>
static bool spans_fit(int64_t lda, int64_t ldb) {
  const int64_t a = (TA ? (int64_t)(BK - 1) * lda + BM : (int64_t)(BM - 1) * lda + BK) * 8;
  const int64_t b = (TB ? (int64_t)(BN - 1) * ldb + BK : (int64_t)(BK - 1) * ldb + BN) * 8;
  return a < 0x7fffffff && b < 0x7fffffff;
}

bool grouped_spans_fit(int cfg, int ta, int tb, int64_t lda, int64_t ldb) {
  if (cfg == 6) {
    if (ta) return tb ? spans_fit<64, 64, 8, 1, 1>(lda, ldb) : spans_fit<64, 64, 8, 1, 0>(lda, ldb);
    return tb ? spans_fit<64, 64, 8, 0, 1>(lda, ldb) : spans_fit<64, 64, 8, 0, 0>(lda, ldb);
  }
  if (ta) return tb ? spans_fit<64, 64, 16, 1, 1>(lda, ldb) : spans_fit<64, 64, 16, 1, 0>(lda, ldb);
  return tb ? spans_fit<64, 64, 16, 0, 1>(lda, ldb) : spans_fit<64, 64, 16, 0, 0>(lda, ldb);
}

// Leading dimensions too large for buffer offsets take the 64 x 64 x 16
// block with pointer loads.
template <int KIND, int BM, int BN, int BK, int WM, int WN, int WPE, int TA = 0, int TB = 0, int DEEP = 0>
static hipError_t launch_one(const GemmArgs& g, hipStream_t s) {
  if (!spans_fit<BM, BN, BK, TA, TB>(g.lda, g.ldb)) {
    const int64_t tiles = ((g.m + 63) / 64) * ((g.n + 63) / 64);
    if (tiles <= 0) return hipSuccess;
    if (tiles > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((cgemm_f64<KIND, 64, 64, 16, 32, 32, 2, TA, TB, 0, 0>), dim3((unsigned)tiles), dim3(256), 0, s,
                       g);
    return hipGetLastError();
  }
  const int64_t tm = (g.m + BM - 1) / BM, tn = (g.n + BN - 1) / BN;
  const int64_t tiles = tm * tn;
  if (tiles <= 0) return hipSuccess;
  if (tiles > 0x7fffffff) return hipErrorInvalidValue;
  constexpr int NT = (BM / WM) * (BN / WN) * 64;
  if constexpr (DEEP) {
    if (g.m % BM == 0 && g.n % BN == 0) {
      hipLaunchKernelGGL((cgemm_f64<KIND, BM, BN, BK, WM, WN, WPE, TA, TB, DEEP, 2>), dim3((unsigned)tiles), dim3(NT), 0,
                         s, g);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((cgemm_f64<KIND, BM, BN, BK, WM, WN, WPE, TA, TB, DEEP>), dim3((unsigned)tiles), dim3(NT), 0, s, g);
  return hipGetLastError();
}

// Complex kinds take configuration 0 (64 x 64 x 16), real products 3
// (64 x 64 x 32) or 11 (128 x 128 x 32); tile_config_for maps a request to
// one of these, and the launcher refuses any other.
template <int KIND>
static hipError_t launch_kind(const GemmArgs& g, int cfg, hipStream_t s) {
  // Transposed operands (op T or H) run the 64 x 64 x 16 tile.
  if (g.ta || g.tb) {
    if (g.ta && g.tb) return launch_one<KIND, 64, 64, 16, 32, 32, 2, 1, 1>(g, s);
    if (g.ta) return launch_one<KIND, 64, 64, 16, 32, 32, 2, 1, 0>(g, s);
    return launch_one<KIND, 64, 64, 16, 32, 32, 2, 0, 1>(g, s);
  }
  const int64_t tiles = ((g.m + 63) / 64) * ((g.n + 63) / 64);
  if constexpr (KIND == KIND_RR) {
    // 128 x 128 blocks: one A and one B tile in LDS (135 KB), one block per CU.
    if (cfg == 11) return launch_one<KIND, 128, 128, 32, 32, 32, 4>(g, s);
    if (cfg != 3) return hipErrorInvalidValue;
    // Large products take the two-deep pipeline, as the complex ones do.
    if (g.k >= 1024 && tiles >= 1024) return launch_one<KIND, 64, 64, 32, 32, 32, 2, 0, 0, 1>(g, s);
    return launch_one<KIND, 64, 64, 32, 32, 32, 2>(g, s);
  } else {
    if (cfg != 0) return hipErrorInvalidValue;
    // Large complex products take the two-deep pipeline (1 % faster at
    // n = 16384); short k loops and small grids do better without it.
    if constexpr (KIND == KIND_GAUSS) {
      if (g.k >= 1024 && tiles >= 1024) return launch_one<KIND, 64, 64, 16, 32, 32, 2, 0, 0, 1>(g, s);
    }
    return launch_one<KIND, 64, 64, 16, 32, 32, 2>(g, s);
  }
}

int tile_config_for(int kind, int requested, int64_t m, int64_t n, int64_t k) {
  if (kind != KIND_RR) return 0;
  return (requested == 3 || requested == 11) ? requested : default_tile_config(kind, m, n, k);
}

hipError_t launch_cgemm(int kind, const GemmArgs& g, int cfg, hipStream_t s) {
  switch (kind) {
    case KIND_GAUSS: return launch_kind<KIND_GAUSS>(g, cfg, s);
    case KIND_RC: return launch_kind<KIND_RC>(g, cfg, s);
    case KIND_CR: return launch_kind<KIND_CR>(g, cfg, s);
    case KIND_RR: return launch_kind<KIND_RR>(g, cfg, s);
    default: return hipErrorInvalidValue;
  }
}

template <int BM, int BN, int BK, int WM, int WN, int WPE, int OPS>
static hipError_t launch_grouped_ops(const GemmArgs* prods, const GroupedItem* items, int nitems, int* counter,
                                     int dyn, int blocks, hipStream_t s) {
  constexpr int NT = (BM / WM) * (BN / WN) * 64;
  if (dyn) {
    hipLaunchKernelGGL(reset_counter, dim3(1), dim3(64), 0, s, counter);
    hipLaunchKernelGGL((grouped_gemm<BM, BN, BK, WM, WN, WPE, 1, OPS>), dim3(blocks), dim3(NT), 0, s, prods, items,
                       nitems, counter);
  } else {
    hipLaunchKernelGGL((grouped_gemm<BM, BN, BK, WM, WN, WPE, 0, OPS>), dim3(blocks), dim3(NT), 0, s, prods, items,
                       nitems, counter);
  }
  return hipGetLastError();
}

template <int BM, int BN, int BK, int WM, int WN, int WPE>
static hipError_t launch_grouped_cfg(const GemmArgs* prods, const GroupedItem* items, int nitems, int* counter,
                                     int dyn, int ops, int blocks, hipStream_t s) {
  switch (ops) {
    case 0: return launch_grouped_ops<BM, BN, BK, WM, WN, WPE, 0>(prods, items, nitems, counter, dyn, blocks, s);
    case 1: return launch_grouped_ops<BM, BN, BK, WM, WN, WPE, 1>(prods, items, nitems, counter, dyn, blocks, s);
    case 2: return launch_grouped_ops<BM, BN, BK, WM, WN, WPE, 2>(prods, items, nitems, counter, dyn, blocks, s);
    case 3: return launch_grouped_ops<BM, BN, BK, WM, WN, WPE, 3>(prods, items, nitems, counter, dyn, blocks, s);
    default: return launch_grouped_ops<BM, BN, BK, WM, WN, WPE, -1>(prods, items, nitems, counter, dyn, blocks, s);
  }
}

hipError_t launch_grouped(int cfg, int dyn, int ops, int buf, const GemmArgs* prods, const GroupedItem* items,
                          int nitems, int* counter, int blocks, hipStream_t s) {
  if (!buf) {
    // Leading dimensions too large for buffer offsets: pointer loads, the
    // kernel with every tile variant, 64 x 64 x 16 blocks.
    constexpr int NT = 256;
    if (dyn) {
      hipLaunchKernelGGL(reset_counter, dim3(1), dim3(64), 0, s, counter);
      hipLaunchKernelGGL((grouped_gemm<64, 64, 16, 32, 32, 2, 1, -1, 0>), dim3(blocks), dim3(NT), 0, s, prods, items,
                         nitems, counter);
    } else {
      hipLaunchKernelGGL((grouped_gemm<64, 64, 16, 32, 32, 2, 0, -1, 0>), dim3(blocks), dim3(NT), 0, s, prods, items,
                         nitems, counter);
    }
    return hipGetLastError();
  }
  switch (cfg) {
    case 0: return launch_grouped_cfg<64, 64, 16, 32, 32, 2>(prods, items, nitems, counter, dyn, ops, blocks, s);
    case 6: return launch_grouped_cfg<64, 64, 8, 32, 32, 2>(prods, items, nitems, counter, dyn, ops, blocks, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_grouped_combine(const CombineArgs* args, const int64_t* row_prefix, int nargs, int64_t total_rows,
                                  hipStream_t s) {
  if (total_rows <= 0) return hipSuccess;
  if (total_rows > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(grouped_combine, dim3((unsigned)total_rows), dim3(256), 0, s, args, row_prefix, nargs);
  return hipGetLastError();
}

hipError_t launch_combine(const CombineArgs& a, hipStream_t s) {
  if (a.rows <= 0 || a.cols <= 0) return hipSuccess;
  auto al16 = [](const double* p) { return p == nullptr || (reinterpret_cast<uintptr_t>(p) & 15u) == 0; };
  bool vec = (a.lds % 2 == 0) && (a.ldd % 2 == 0);
  for (int u = 0; u < 8; ++u) vec = vec && al16(a.src[u]);
  for (int q = 0; q < a.nq; ++q) vec = vec && al16(a.dst_r[q]) && al16(a.dst_i[q]);
  const int64_t bpr = ((a.cols + 1) / 2 + 255) / 256;
  const int64_t blocks = bpr * a.rows;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (vec) hipLaunchKernelGGL(combine_kernel<1>, dim3((unsigned)blocks), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(combine_kernel<0>, dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fill_zero(double* p, int64_t rows, int64_t cols, int64_t ld, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  const int64_t blocks = ((cols + 255) / 256) * rows;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, rows, cols, ld);
  return hipGetLastError();
}

}  // namespace bq
