// Split-precision real GEMM (Ozaki-style) for gfx950.
//
// A real FP64 product T = X Y (X m x k, Y k x n) is computed from
// low-precision slices:
//   * every row i of X gets a power-of-two exponent e_i (the frexp exponent
//     of its largest magnitude, plus h), every column j of Y an exponent f_j;
//   * x_ij 2^-e_i in (-2^-h, 2^-h) is written as S signed digits,
//     q_1 = rint(2^b y), y_1 = y - q_1 2^-b, q_s = rint(2^{bs} y_{s-1}), ...
//     so x = 2^e_i (sum_s q_s 2^{-bs} + remainder), |q_1| <= 2^{b-h},
//     |q_s| <= 2^{b-1}; the digits are small integers, exact in BF16 (b = 7,
//     h = 0), OCP FP8 E4M3 (b = 4, h = 0) or INT8 (b = 7, h = 1: one bit of
//     headroom keeps the leading digit inside a signed byte);
//   * T_ij = 2^{e_i + f_j} sum_{d = 2}^{S+1} 2^{-bd} sum_{s + t = d} (Q_s R_t)_ij
//     (pairs with s + t > S + 1 are dropped).
// Each level d is accumulated by MFMA in FP32 (BF16/FP8) or int32 (INT8)
// over as many k-steps as keep every partial sum an exact integer (the bound
// is in slice_flush_steps), then added, scaled by 2^{-bd}, into FP64
// accumulators.  Only the splitting, the exponent scaling and the level
// accumulation are FP64.
#include <limits.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "bq_split_common.h"

namespace bq {

// Exponents: e[r] = max over the reduced dimension of frexp exponents
// (rows of the left operand, columns of the right one).  exps must hold
// INT_MIN beforehand.  Block: 256 threads.
__global__ void __launch_bounds__(256) split_exp_left(const SplitArgs a, int* exps) {
  // grid.x = rows, grid.y = chunks of 2048 columns
  const int64_t r = blockIdx.x;
  const int64_t c0 = (int64_t)blockIdx.y * 2048;
  int e = INT_MIN;
  for (int j = threadIdx.x; j < 2048; j += 256) {
    const int64_t c = c0 + j;
    if (c < a.cols) e = max(e, exp_of(operand_value(a, r * a.ld + c)));
  }
  if (!exp_special(e)) e += a.head;
  for (int o = 32; o > 0; o >>= 1) e = max(e, __shfl_xor(e, o));
  __shared__ int red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0) {
    e = max(max(red[0], red[1]), max(red[2], red[3]));
    if (e != INT_MIN) atomicMax(&exps[r], e);
  }
}

__global__ void __launch_bounds__(256) split_exp_right(const SplitArgs a, int* exps, int64_t chunk) {
  // grid.x = column blocks of 64, grid.y = row chunks of `chunk` rows;
  // thread: one column, every 4th row of the chunk.
  const int64_t c = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  const int64_t r0 = (int64_t)blockIdx.y * chunk + (threadIdx.x >> 6);
  int e = INT_MIN;
  if (c < a.cols)
    for (int64_t r = r0; r < a.rows && r < (int64_t)(blockIdx.y + 1) * chunk; r += 4)
      e = max(e, exp_of(operand_value(a, r * a.ld + c)));
  __shared__ int red[256];
  red[threadIdx.x] = e;
  __syncthreads();
  if (threadIdx.x < 64) {
    e = max(max(red[threadIdx.x], red[threadIdx.x + 64]), max(red[threadIdx.x + 128], red[threadIdx.x + 192]));
    if (c < a.cols && e != INT_MIN) atomicMax(&exps[c], exp_special(e) ? e : e + a.head);
  }
}

__global__ void __launch_bounds__(256) fill_int(int* p, int64_t n, int v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

// Digits of one element: q[0..S-1] from x and its row/column exponent.
template <int S>
__device__ __forceinline__ void digits(double x, int e, int beta, float* q) {
  double y = exp_special(e) ? 0.0 : ldexp(x, -e);
#pragma unroll
  for (int s = 1; s <= S; ++s) {
    const double d = rint(ldexp(y, beta * s));
    q[s - 1] = (float)d;
    y = y - ldexp(d, -beta * s);
  }
}

// Small integer (|q| <= 256) to BF16 bits: exact truncation of the FP32 bits.
__device__ __forceinline__ unsigned short to_bf16(float q) {
  return (unsigned short)(__float_as_uint(q) >> 16);
}

// INT8 digits (beta 7, one bit of headroom) are stored as two's-complement
// bytes (|q| <= 64).
// Small integer (|q| <= 16) to OCP FP8 E4M3 bits.
__device__ __forceinline__ unsigned char to_e4m3(float qf) {
  int q = (int)qf;
  const unsigned char s = q < 0 ? 0x80 : 0;
  q = q < 0 ? -q : q;
  if (q == 0) return 0;
  const int E = 31 - __clz(q);
  const int mant = ((q << 3) >> E) & 7;
  return (unsigned char)(s | ((E + 7) << 3) | mant);
}

// Left operand: digits D[s][r][kk] (kk < kp, rows < rows_pad; zero padding).
// Thread: 8 consecutive kk of one row.  grid.x = rows_pad, grid.y = kp / 2048.
template <int ET, int S>
__global__ void __launch_bounds__(256) split_digits_left(const SplitArgs a, const int* exps, void* out) {
  const int64_t r = blockIdx.x;
  const int64_t kk0 = (int64_t)blockIdx.y * 2048 + threadIdx.x * 8;
  if (kk0 >= a.kp) return;
  const int e = (r < a.rows) ? exps[r] : INT_MIN;
  float q[8][S];
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int64_t c = kk0 + t;
    const double x = (r < a.rows && c < a.cols) ? operand_value(a, r * a.ld + c) : 0.0;
    digits<S>(x, e, a.beta, q[t]);
  }
  constexpr int ES = ET == 0 ? 2 : 1;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int64_t o = (int64_t)s * a.slice_stride * ES + digit_offset(a.tiled, r, kk0 * ES, a.kp * ES);
    if constexpr (ET == 0) {
      i4v v;
#pragma unroll
      for (int t = 0; t < 4; ++t)
        v[t] = (int)to_bf16(q[2 * t][s]) | ((int)to_bf16(q[2 * t + 1][s]) << 16);
      *reinterpret_cast<i4v*>(static_cast<unsigned char*>(out) + o) = v;
    } else if constexpr (ET == 2) {
      i2v v;
#pragma unroll
      for (int t = 0; t < 2; ++t)
        v[t] = (int)(unsigned char)(signed char)q[4 * t][s] | ((int)(unsigned char)(signed char)q[4 * t + 1][s] << 8) |
               ((int)(unsigned char)(signed char)q[4 * t + 2][s] << 16) |
               ((int)(unsigned char)(signed char)q[4 * t + 3][s] << 24);
      *reinterpret_cast<i2v*>(static_cast<unsigned char*>(out) + o) = v;
    } else {
      i2v v;
#pragma unroll
      for (int t = 0; t < 2; ++t)
        v[t] = (int)to_e4m3(q[4 * t][s]) | ((int)to_e4m3(q[4 * t + 1][s]) << 8) |
               ((int)to_e4m3(q[4 * t + 2][s]) << 16) | ((int)to_e4m3(q[4 * t + 3][s]) << 24);
      *reinterpret_cast<i2v*>(static_cast<unsigned char*>(out) + o) = v;
    }
  }
}

// Right operand (k x n, row-major): digits stored transposed, D[s][c][kk].
// Block: a 64 (kk) x 64 (c) tile through LDS.  grid.x = cols_pad / 64,
// grid.y = kp / 64.
template <int ET, int S>
__global__ void __launch_bounds__(256) split_digits_right(const SplitArgs a, const int* exps, void* out) {
  constexpr int ES = ET == 0 ? 2 : 1;
  __shared__ __attribute__((aligned(16))) unsigned char tile[S][64][64 * ES + 16];
  const int64_t c0 = (int64_t)blockIdx.x * 64;
  const int64_t k0 = (int64_t)blockIdx.y * 64;
  const int tc = threadIdx.x & 63;
  const int64_t c = c0 + tc;
  const int e = (c < a.cols) ? exps[c] : INT_MIN;
  for (int rr = threadIdx.x >> 6; rr < 64; rr += 4) {
    const int64_t kk = k0 + rr;
    const double x = (c < a.cols && kk < a.rows) ? operand_value(a, kk * a.ld + c) : 0.0;
    float q[S];
    digits<S>(x, e, a.beta, q);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if constexpr (ET == 0)
        *reinterpret_cast<unsigned short*>(&tile[s][tc][rr * 2]) = to_bf16(q[s]);
      else if constexpr (ET == 2)
        tile[s][tc][rr] = (unsigned char)(signed char)q[s];
      else
        tile[s][tc][rr] = to_e4m3(q[s]);
    }
  }
  __syncthreads();
  // Write: row c of slice s gets 64 * ES contiguous bytes; 16-byte pieces.
  constexpr int PIECES = 64 * ES / 16;  // 8 (bf16) or 4 (fp8)
  for (int w = threadIdx.x; w < S * 64 * PIECES; w += 256) {
    const int s = w / (64 * PIECES);
    const int rem = w % (64 * PIECES);
    const int cc = rem / PIECES, p = rem % PIECES;
    const i4v v = *reinterpret_cast<const i4v*>(&tile[s][cc][p * 16]);
    const int64_t o = digit_offset(a.tiled, c0 + cc, k0 * ES + p * 16, a.kp * ES);
    *reinterpret_cast<i4v*>(static_cast<unsigned char*>(out) + (int64_t)s * a.slice_stride * ES + o) = v;
  }
}

// ---------------------------------------------------------------------------
// Slice GEMM.  A 128 x 64 block tile (8 waves of 32 x 32, or 4 waves of
// 64 x 32 for many slices), one MFMA k-step per LDS stage.  LDS holds all S slices of the A and B
// tiles of that k-step; 16-byte (BF16, INT8) or 8-byte (FP8) chunks are
// XOR-swizzled per row so fragment reads are free of bank conflicts.
//
// MFMA layouts (checked with one-wave probes on gfx950):
//   A: lane l holds row l % 16, k = E (l / 16) .. +E-1   (E elements/lane)
//   B: lane l holds column l % 16, same k
//   D: lane l, element v holds row 4 (l / 16) + v, column l % 16.
// ---------------------------------------------------------------------------
template <int ET>
struct SliceTraits;
template <>
struct SliceTraits<0> {  // BF16 digits, v_mfma_f32_16x16x32_bf16
  static constexpr int ES = 1 * 2, KSTEP = 32, CH = 16, BETA = 7;
  typedef bf16x8 frag_t;
  typedef f4 acc_t;
  __device__ static acc_t mfma(frag_t a, frag_t b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct SliceTraits<2> {  // INT8 digits, v_mfma_i32_16x16x64_i8 (exact int32 sums)
  static constexpr int ES = 1, KSTEP = 64, CH = 16, BETA = 7;
  typedef i4v frag_t;
  typedef i4v acc_t;
  __device__ static acc_t mfma(frag_t a, frag_t b, acc_t c) {
    return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
  }
};

constexpr double pow2neg(int e) { return 1.0 / (double)(1ull << e); }

// Output of one wave tile (16 MI x 16 NI at rows r0.., columns c0..):
// exponent scaling, then coef * T into every target block.
template <int MI, int NI>
__device__ __forceinline__ void store_tile(const SliceGemmArgs& g, const d4s (&acc)[MI][NI], int64_t r0, int64_t c0,
                                           int fr, int fg) {
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = r0 + i * 16 + 4 * fg + v;
        const int64_t c = c0 + j * 16 + fr;
        if (r >= g.m || c >= g.n) continue;
        const int ea = g.ea[r], eb = g.eb[c];
        const double t = exp_scaled(acc[i][j][v], ea, eb, 0);
        const int64_t off = r * g.ldc + c;
        for (int q = 0; q < g.ntgt; ++q) {
          double val = g.coef[q] * t;
          if (g.mode[q] == TGT_ACCUM) val += g.c[q][off];
          g.c[q][off] = val;
        }
      }
}



template <int ET, int S, int WM, int MI, int CACHE_B, int NSTAGE, int WPE, int PERSIST>
__global__ void __launch_bounds__(WM * 2 * 64) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
slice_gemm(const SliceGemmArgs g) {
  typedef SliceTraits<ET> Tr;
  typedef typename Tr::frag_t frag_t;
  typedef typename Tr::acc_t acc_t;
  constexpr int ES = Tr::ES, BK = Tr::KSTEP, CH = Tr::CH, BETA = Tr::BETA;
  constexpr int NT = WM * 2 * 64;
  constexpr int NI = 2;                // wave tile: (16 MI) x 32
  constexpr int BM = 16 * MI * WM, BN = 64;
  constexpr int ROWB = BK * ES;        // bytes per tile row: 64 (BF16, INT8) or 32 (FP8)
  constexpr int NCH = ROWB / CH;       // chunks per row: 4
  constexpr int A_BYTES = S * BM * ROWB;
  constexpr int B_BYTES = S * BN * ROWB;
  constexpr int STAGE = A_BYTES + B_BYTES;
  constexpr int A_LD_TOTAL = A_BYTES / 16;  // 16-byte pieces per k-step
  constexpr int A_LD = (A_LD_TOTAL + NT - 1) / NT;
  constexpr int B_LD_TOTAL = B_BYTES / 16;
  constexpr int B_LD = (B_LD_TOTAL + NT - 1) / NT;
  static_assert(NCH == 4, "four chunks per row");
  __shared__ __attribute__((aligned(16))) unsigned char lds[NSTAGE * STAGE];

  const int tiles_m = (int)((g.m + BM - 1) / BM);
  const int tiles_n = (int)((g.n + BN - 1) / BN);
  // XCD-aware grouped tile order (as in the FP64 GEMM).
  int tm, tn;
  slice_tile_coords(tiles_m, tiles_n, tm, tn);
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave >> 1) * 16 * MI, wn0 = (wave & 1) * 32;
  const int fr = lane & 15, fg = lane >> 4;

  // Byte offset of chunk ch of row r (swizzled).
  auto swz = [](int r, int ch) { return r * ROWB + swz_chunk<CH>(r, ch) * CH; };

  // Global -> LDS staging.  Piece v = tid + i NT of a k-step covers 16 bytes
  // of row r of slice s.  With PPR pieces per row and NT a multiple of PPR
  // and of 16 rows, the per-lane part of every address is the same for all
  // i (row tid / PPR, piece tid % PPR) and the rest is wave-uniform.
  constexpr int PPR = ROWB / 16;                 // pieces per row: 4 or 2
  constexpr int RPP = NT / PPR;                  // rows covered by one pass i
  static_assert(RPP % 16 == 0, "swizzle needs whole 16-row groups per pass");
  static_assert((RPP <= BM ? BM % RPP : RPP % BM) == 0 && (RPP <= BN ? BN % RPP : RPP % BN) == 0, "pass shape");
  const int lr = tid / PPR, lp = tid % PPR;
  // Lane part of the global offset for a tile of R rows (a pass may span
  // several slices when it covers more rows than the tile has).
  auto g_lane = [&](int R, int64_t slice_stride) -> int64_t {
    return ((int64_t)(lr / R) * slice_stride + (int64_t)(lr % R) * g.kp) * ES + lp * 16;
  };
  const int64_t ga_lane = g_lane(BM, g.slice_stride_a);
  const int64_t gb_lane = g_lane(BN, g.slice_stride_b);
  // LDS position of (linear row lr, piece lp); the swizzle depends only on
  // row bits 1..3, which whole-pass and whole-slice offsets (multiples of 16
  // rows) leave unchanged.
  const int l_lane_a = CH == 16 ? swz(lr, lp) : swz(lr, 2 * lp);
  const int l_lane_a2 = CH == 16 ? 0 : swz(lr, 2 * lp + 1);  // second 8-byte half (FP8 only)
  const unsigned char* ga = static_cast<const unsigned char*>(g.a) + m0 * g.kp * ES;
  const unsigned char* gb = static_cast<const unsigned char*>(g.b) + n0 * g.kp * ES;
  i4v ra[A_LD], rb[B_LD];
  // Pass i of a tile of R rows starts at slice s, row r0.
  auto pass_of = [&](int i, int R, int& s, int& r0) {
    const int row_lin = i * RPP;
    s = row_lin / R;
    r0 = row_lin % R;
  };
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < A_LD; ++i) {
      if (A_LD_TOTAL % NT == 0 || i * NT + tid < A_LD_TOTAL) {
        int s, r0;
        pass_of(i, BM, s, r0);
        const unsigned char* base = ga + (s * g.slice_stride_a + (int64_t)r0 * g.kp + k0) * ES;
        ra[i] = *reinterpret_cast<const i4v*>(base + ga_lane);
      }
    }
#pragma unroll
    for (int i = 0; i < B_LD; ++i) {
      if (B_LD_TOTAL % NT == 0 || i * NT + tid < B_LD_TOTAL) {
        int s, r0;
        pass_of(i, BN, s, r0);
        const unsigned char* base = gb + (s * g.slice_stride_b + (int64_t)r0 * g.kp + k0) * ES;
        rb[i] = *reinterpret_cast<const i4v*>(base + gb_lane);
      }
    }
  };
  auto put = [&](unsigned char* base, i4v x) {
    if constexpr (CH == 16) {
      *reinterpret_cast<i4v*>(base + l_lane_a) = x;
    } else {
      *reinterpret_cast<i2v*>(base + l_lane_a) = i2v{x[0], x[1]};
      *reinterpret_cast<i2v*>(base + l_lane_a2) = i2v{x[2], x[3]};
    }
  };
  auto lstore = [&](int st) {
    unsigned char* base = lds + st * STAGE;
#pragma unroll
    for (int i = 0; i < A_LD; ++i) {
      if (A_LD_TOTAL % NT == 0 || i * NT + tid < A_LD_TOTAL) {
        int s, r0;
        pass_of(i, BM, s, r0);
        put(base + s * BM * ROWB + r0 * ROWB, ra[i]);
      }
    }
#pragma unroll
    for (int i = 0; i < B_LD; ++i) {
      if (B_LD_TOTAL % NT == 0 || i * NT + tid < B_LD_TOTAL) {
        int s, r0;
        pass_of(i, BN, s, r0);
        put(base + A_BYTES + s * BN * ROWB + r0 * ROWB, rb[i]);
      }
    }
  };

  d4s acc[MI][NI];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j) acc[i][j] = d4s{0.0, 0.0, 0.0, 0.0};

  // Level sums (PERSIST): level d = s + t in lvl[d - 2].
  acc_t lvl[PERSIST ? S : 1][MI][NI];
#pragma unroll
  for (int d = 0; d < (PERSIST ? S : 1); ++d)
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < NI; ++j) lvl[d][i][j] = acc_t{0, 0, 0, 0};
  int since = 0;

  const int64_t nk = g.kp / BK;
  gload(0);
  lstore(0);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int st = NSTAGE == 2 ? (int)(kt & 1) : 0;
    if (kt + 1 < nk) gload((kt + 1) * BK);
    const unsigned char* base = lds + st * STAGE;
    if constexpr (PERSIST) {
      // Every B fragment of the k-step stays in registers; the A fragments
      // of one slice at a time.  Level sums live across k-steps.
      frag_t fbc[S][NI];
#pragma unroll
      for (int t = 0; t < S; ++t)
#pragma unroll
        for (int j = 0; j < NI; ++j)
          fbc[t][j] = *reinterpret_cast<const frag_t*>(base + A_BYTES + t * BN * ROWB + swz(wn0 + j * 16 + fr, fg));
#pragma unroll
      for (int s = 1; s <= S; ++s) {
        frag_t fa[MI];
#pragma unroll
        for (int i = 0; i < MI; ++i)
          fa[i] = *reinterpret_cast<const frag_t*>(base + (s - 1) * BM * ROWB + swz(wm0 + i * 16 + fr, fg));
#pragma unroll
        for (int t = 1; t <= S + 1 - s; ++t)
#pragma unroll
          for (int i = 0; i < MI; ++i)
#pragma unroll
            for (int j = 0; j < NI; ++j) lvl[s + t - 2][i][j] = Tr::mfma(fa[i], fbc[t - 1][j], lvl[s + t - 2][i][j]);
      }
      if (++since == g.kflush || kt + 1 == nk) {
        since = 0;
#pragma unroll
        for (int d = 2; d <= S + 1; ++d) {
          const double sc = pow2neg(BETA * d);
#pragma unroll
          for (int i = 0; i < MI; ++i)
#pragma unroll
            for (int j = 0; j < NI; ++j) {
#pragma unroll
              for (int v = 0; v < 4; ++v)
                acc[i][j][v] = __builtin_fma((double)lvl[d - 2][i][j][v], sc, acc[i][j][v]);
              lvl[d - 2][i][j] = acc_t{0, 0, 0, 0};
            }
        }
      }
    } else {
      frag_t fa[S][MI];
      frag_t fbc[CACHE_B ? S : 1][NI];
  #pragma unroll
      for (int s = 0; s < S; ++s) {
  #pragma unroll
        for (int i = 0; i < MI; ++i)
          fa[s][i] = *reinterpret_cast<const frag_t*>(base + s * BM * ROWB + swz(wm0 + i * 16 + fr, fg));
        if constexpr (CACHE_B) {
  #pragma unroll
          for (int j = 0; j < NI; ++j)
            fbc[s][j] = *reinterpret_cast<const frag_t*>(base + A_BYTES + s * BN * ROWB + swz(wn0 + j * 16 + fr, fg));
        }
      }
      // Levels d = 2 .. S+1.  The MFMAs of level d are issued while the sums of
      // level d-1 are flushed into FP64 (two accumulator sets), so the flush's
      // VALU work overlaps the matrix pipe; scheduling barriers between levels
      // keep register use bounded.
      acc_t lv[2][MI][NI];
      auto flush = [&](const acc_t (&x)[MI][NI], int d) {
        const double sc = pow2neg(BETA * d);
  #pragma unroll
        for (int i = 0; i < MI; ++i)
  #pragma unroll
          for (int j = 0; j < NI; ++j)
  #pragma unroll
            for (int v = 0; v < 4; ++v) acc[i][j][v] = __builtin_fma((double)x[i][j][v], sc, acc[i][j][v]);
      };
  #pragma unroll
      for (int d = 2; d <= S + 1; ++d) {
        __builtin_amdgcn_sched_barrier(0);
        const int cur = d & 1;
  #pragma unroll
        for (int i = 0; i < MI; ++i)
  #pragma unroll
          for (int j = 0; j < NI; ++j) lv[cur][i][j] = acc_t{0, 0, 0, 0};
  #pragma unroll
        for (int s = 1; s < d; ++s) {
          const int t = d - s;
          if (s > S || t > S) continue;
          frag_t fb[NI];
  #pragma unroll
          for (int j = 0; j < NI; ++j) {
            if constexpr (CACHE_B)
              fb[j] = fbc[t - 1][j];
            else
              fb[j] = *reinterpret_cast<const frag_t*>(base + A_BYTES + (t - 1) * BN * ROWB + swz(wn0 + j * 16 + fr, fg));
          }
  #pragma unroll
          for (int i = 0; i < MI; ++i)
  #pragma unroll
            for (int j = 0; j < NI; ++j) lv[cur][i][j] = Tr::mfma(fa[s - 1][i], fb[j], lv[cur][i][j]);
        }
        if (d > 2) flush(lv[cur ^ 1], d - 1);
      }
      __builtin_amdgcn_sched_barrier(0);
      flush(lv[(S + 1) & 1], S + 1);
    }
    if (NSTAGE == 1) __syncthreads();
    if (kt + 1 < nk) lstore(NSTAGE == 2 ? (st ^ 1) : 0);
    __syncthreads();
  }

  store_tile<MI, NI>(g, acc, m0 + wm0, n0 + wn0, fr, fg);
}

// ---------------------------------------------------------------------------
// Slice GEMM with direct global -> LDS loads (BF16 and INT8 digits: rows of
// 64 bytes in 16-byte chunks, digits in the tiled layout).  64 x 64 block
// tile, 4 waves of 32 x 32, one wave per SIMD.  Per k-step every thread
// copies 16 bytes of each A and each B slice tile straight into LDS
// (buffer_load_dwordx4 ... lds: lane l of a wave writes bytes 16 l .. 16 l +
// 15 after the wave's LDS base); the tiles are stored in LDS order, so the
// copy is contiguous on both sides.  Two LDS stages: the loads of k-step kt + 1 are issued
// during the MFMAs of k-step kt, one after each slice pair until all are
// out.  Pairs run level by level (d = s + t = 2 .. S + 1); level d needs
// only the new fragments of slice d - 1, read from LDS one level ahead.
// Level sums stay in registers across k-steps and go to FP64 every
// g.kflush k-steps.
// ---------------------------------------------------------------------------
template <int ET, int S>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
slice_gemm_dma(const SliceGemmArgs g) {
  typedef SliceTraits<ET> Tr;
  typedef typename Tr::frag_t frag_t;
  typedef typename Tr::acc_t acc_t;
  constexpr int ES = Tr::ES, BK = Tr::KSTEP, BETA = Tr::BETA;
  static_assert(Tr::CH == 16 && BK * ES == 64, "rows of four 16-byte chunks");
  constexpr int BM = 64, BN = 64, ROWB = 64, MI = 2, NI = 2;
  constexpr int SLICE = BM * ROWB;  // 4 KB per slice tile (A and B alike)
  constexpr int A_BYTES = S * SLICE;
  constexpr int STAGE = 2 * A_BYTES;
  static_assert(2 * STAGE <= 160 * 1024, "two stages must fit LDS");
  __shared__ __attribute__((aligned(16))) unsigned char lds[2 * STAGE];

  const int tiles_m = (int)((g.m + BM - 1) / BM);
  const int tiles_n = (int)((g.n + BN - 1) / BN);
  int tm, tn;
  slice_tile_coords(tiles_m, tiles_n, tm, tn);
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave >> 1) * 32, wn0 = (wave & 1) * 32;
  const int fr = lane & 15, fg = lane >> 4;

  // Loads: the digits are tiled (slice_tile_offset), so the tile of slice s
  // for k-step kt is 4 KB contiguous, already in LDS order; thread tid copies
  // its bytes 16 tid .. 16 tid + 15.  Buffer loads with one resource per
  // slice and block row (column) tile: its nk tiles, so any offset past them
  // would read zeros rather than another tile.
  const int64_t nk = g.kp / BK;
  const unsigned char* ga = static_cast<const unsigned char*>(g.a) + (int64_t)tm * nk * 4096;
  const unsigned char* gb = static_cast<const unsigned char*>(g.b) + (int64_t)tn * nk * 4096;
  const int64_t sa = g.slice_stride_a * ES, sb = g.slice_stride_b * ES;
  const int nrec = (int)(uint32_t)(nk * 4096);  // num_records is unsigned
  const int voff = tid * 16;
  const int wave_lds = wave * 64 * 16;
  // Load number q (0 .. 2S-1) of k-step kt into stage st: A slice q / 2 or
  // B slice q / 2.
  auto dma = [&](int q, int64_t kt, int st) {
    const int sl = q >> 1;
    const unsigned char* base = (q & 1) ? gb + sl * sb : ga + sl * sa;
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, nrec, 0x00020000);
    unsigned char* dst = lds + st * STAGE + ((q & 1) ? A_BYTES : 0) + sl * SLICE + wave_lds;
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_void_ptr)dst, 16, voff, (int)(kt * 4096), 0, 0);
  };
  auto frag = [&](const unsigned char* tile, int row) {
    return *reinterpret_cast<const frag_t*>(tile + row * ROWB + swz_chunk<16>(row, fg) * 16);
  };

  d4s acc[MI][NI];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j) acc[i][j] = d4s{0.0, 0.0, 0.0, 0.0};

#pragma unroll
  for (int q = 0; q < 2 * S; ++q) dma(q, 0, 0);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  for (int64_t k0 = 0; k0 < nk; k0 += g.kflush) {
    const int64_t k1 = min(nk, k0 + (int64_t)g.kflush);
    acc_t lvl[S][MI][NI];
#pragma unroll
    for (int d = 0; d < S; ++d)
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NI; ++j) lvl[d][i][j] = acc_t{0, 0, 0, 0};
    for (int64_t kt = k0; kt < k1; ++kt) {
      const int st = (int)(kt & 1);
      // The last k-step reloads itself into the idle stage (never read), so
      // the loads need no branch.
      const int64_t knext = kt + 1 < nk ? kt + 1 : kt;
      const unsigned char* ta = lds + st * STAGE;
      const unsigned char* tb = ta + A_BYTES;
      frag_t fa[S][MI], fb[S][NI];
#pragma unroll
      for (int i = 0; i < MI; ++i) fa[0][i] = frag(ta, wm0 + i * 16 + fr);
#pragma unroll
      for (int j = 0; j < NI; ++j) fb[0][j] = frag(tb, wn0 + j * 16 + fr);
      int q = 0;  // loads of the next k-step issued so far
#pragma unroll
      for (int d = 2; d <= S + 1; ++d) {
        // Fragments of slice d (needed from level d + 1 on), one level ahead.
        if (d <= S) {
#pragma unroll
          for (int i = 0; i < MI; ++i) fa[d - 1][i] = frag(ta + (d - 1) * SLICE, wm0 + i * 16 + fr);
#pragma unroll
          for (int j = 0; j < NI; ++j) fb[d - 1][j] = frag(tb + (d - 1) * SLICE, wn0 + j * 16 + fr);
        }
#pragma unroll
        for (int s = 1; s < d; ++s) {
          const int t = d - s;
#pragma unroll
          for (int i = 0; i < MI; ++i)
#pragma unroll
            for (int j = 0; j < NI; ++j)
              lvl[d - 2][i][j] = Tr::mfma(fa[s - 1][i], fb[t - 1][j], lvl[d - 2][i][j]);
          if (q < 2 * S) dma(q++, knext, st ^ 1);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
#pragma unroll
      for (; q < 2 * S; ++q) dma(q, knext, st ^ 1);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
    }
#pragma unroll
    for (int d = 2; d <= S + 1; ++d) {
      const double sc = pow2neg(BETA * d);
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NI; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[i][j][v] = __builtin_fma((double)lvl[d - 2][i][j][v], sc, acc[i][j][v]);
    }
  }

  store_tile<MI, NI>(g, acc, m0 + wm0, n0 + wn0, fr, fg);
}

// ---------------------------------------------------------------------------
// Slice GEMM on the 32 x 32 MFMA shapes (BF16: v_mfma_f32_32x32x16_bf16,
// INT8: v_mfma_i32_32x32x32_i8; checked with one-wave probes: A lane l holds
// row l % 32, k = 16 (l / 32) bytes on; B the same per column; D lane l,
// element v holds row 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32).  A k-step
// is 32 bytes of each digit row, so a 128 x 64 block of 8 waves (32 x 32 each,
// two waves per SIMD) keeps two LDS stages of S slices within 160 KB and
// moves a quarter fewer bytes per MFMA than the 64 x 64 block.  Digits in the
// tiled layout of 32-byte rows; per k-step a stage holds S A tiles (128 rows,
// two 64-row tiles) and S B tiles (64 rows), copied straight into LDS in 1 KB
// pieces, wave w taking pieces w, w + 8, ...  Level sums as in
// slice_gemm_dma.
// ---------------------------------------------------------------------------
typedef int i16v __attribute__((ext_vector_type(16)));
typedef float f16v __attribute__((ext_vector_type(16)));


template <int ET>
struct SliceTraits32;
template <>
struct SliceTraits32<0> {
  static constexpr int ES = 2, BETA = SliceTraits<0>::BETA;
  typedef bf16x8 frag_t;
  typedef f16v acc_t;
  __device__ static acc_t mfma(frag_t a, frag_t b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct SliceTraits32<2> {
  static constexpr int ES = 1, BETA = SliceTraits<2>::BETA;
  typedef i4v frag_t;
  typedef i16v acc_t;
  __device__ static acc_t mfma(frag_t a, frag_t b, acc_t c) {
    return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
  }
};

// Output of one 32 x 32 wave tile at (r0, c0): exponent scaling, then
// coef * T into every target block.
__device__ __forceinline__ void store_tile32(const SliceGemmArgs& g, const double (&acc)[16], int64_t r0, int64_t c0,
                                             int lane) {
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int64_t r = r0 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    const int64_t c = c0 + (lane & 31);
    if (r >= g.m || c >= g.n) continue;
    const int ea = g.ea[r], eb = g.eb[c];
    const double t = exp_scaled(acc[v], ea, eb, 0);
    const int64_t off = r * g.ldc + c;
    for (int q = 0; q < g.ntgt; ++q) {
      double val = g.coef[q] * t;
      if (g.mode[q] == TGT_ACCUM) val += g.c[q][off];
      g.c[q][off] = val;
    }
  }
}

template <int ET, int S>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
slice_gemm_x32(const SliceGemmArgs g) {
  typedef SliceTraits32<ET> Tr;
  typedef typename Tr::frag_t frag_t;
  typedef typename Tr::acc_t acc_t;
  constexpr int ES = Tr::ES, BETA = Tr::BETA;
  constexpr int BM = 128, BN = 64, RB = 32, TILE = 64 * RB;  // 2 KB per 64-row tile
  constexpr int A_SLICE = BM * RB, B_SLICE = BN * RB;
  constexpr int A_BYTES = S * A_SLICE;
  constexpr int STAGE = A_BYTES + S * B_SLICE;
  constexpr int PIECES = STAGE / 1024;  // 6 S
  // Three stages when they fit: the loads of k-step kt + 2 go out while kt
  // is computed, so a load has two k-steps to land.
  constexpr int NST = 3 * STAGE <= 160 * 1024 ? 3 : 2;
  // Every wave issues the same number of loads per stage (the last ones
  // repeat a piece of its own: the same bytes to the same place), so the
  // wait for a stage is one immediate count.
  constexpr int NPW = (PIECES + 7) / 8;
  static_assert(2 * STAGE <= 160 * 1024, "two stages must fit LDS");
  __shared__ __attribute__((aligned(16))) unsigned char lds[NST * STAGE];

  const int tiles_m = (int)((g.m + BM - 1) / BM);
  const int tiles_n = (int)((g.n + BN - 1) / BN);
  int tm, tn;
  slice_tile_coords(tiles_m, tiles_n, tm, tn);
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: one buffer resource per load
  const int wm0 = (wave >> 1) * 32, wn0 = (wave & 1) * 32;
  const int fr = lane & 31, fg = lane >> 5;

  const int64_t nk = g.kp * ES / RB;
  const int64_t run = nk * TILE;  // bytes of one 64-row tile's k-run
  const unsigned char* ga = static_cast<const unsigned char*>(g.a) + (int64_t)(2 * tm) * run;
  const unsigned char* gb = static_cast<const unsigned char*>(g.b) + (int64_t)tn * run;
  const int64_t sa = g.slice_stride_a * ES, sb = g.slice_stride_b * ES;
  const int nrec_a = (int)(uint32_t)(2 * run), nrec_b = (int)(uint32_t)run;  // num_records is unsigned
  // 1 KB piece p of a stage: A slice p / 4, quarter p % 4 (64-row tile
  // (p % 4) / 2, half p % 2); then B slice (p - 4S) / 2, half p % 2.
  auto dma = [&](int p, int64_t kt, int st) {
    const unsigned char* base;
    int nrec, voff, loff;
    if (p < 4 * S) {
      const int sl = p >> 2, q = p & 3;
      base = ga + sl * sa;
      nrec = nrec_a;
      voff = (int)((q >> 1) * run) + (q & 1) * 1024 + lane * 16;
      loff = sl * A_SLICE + q * 1024;
    } else {
      const int pb = p - 4 * S, sl = pb >> 1;
      base = gb + sl * sb;
      nrec = nrec_b;
      voff = (pb & 1) * 1024 + lane * 16;
      loff = A_BYTES + sl * B_SLICE + (pb & 1) * 1024;
    }
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, nrec, 0x00020000);
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_void_ptr)(lds + st * STAGE + loff), 16, voff,
                                             (int)(kt * TILE), 0, 0);
  };
  auto piece = [&](int i) {
    const int p = wave + 8 * i;
    return p < PIECES ? p : wave;
  };
  auto frag = [&](const unsigned char* tile, int row) {
    return *reinterpret_cast<const frag_t*>(tile + row * RB + swz_chunk32(row, fg) * 16);
  };

  double acc[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.0;

#pragma unroll
  for (int i = 0; i < NPW; ++i) dma(piece(i), 0, 0);
  if constexpr (NST == 3) {
#pragma unroll
    for (int i = 0; i < NPW; ++i) dma(piece(i), nk > 1 ? 1 : 0, 1);
    wait_vm<NPW>();
  } else {
    wait_vm<0>();
  }
  block_sync();
  for (int64_t k0 = 0; k0 < nk; k0 += g.kflush) {
    const int64_t k1 = min(nk, k0 + (int64_t)g.kflush);
    acc_t lvl[S];
#pragma unroll
    for (int d = 0; d < S; ++d)
#pragma unroll
      for (int v = 0; v < 16; ++v) lvl[d][v] = 0;
    for (int64_t kt = k0; kt < k1; ++kt) {
      const int st = (int)(kt % NST);
      const int sn = NST == 3 ? (st == 0 ? 2 : st - 1) : (st ^ 1);  // stage of k-step kt + NST - 1
      // Past the end the last k-step is reloaded into a stage nobody reads.
      const int64_t knext = kt + NST - 1 < nk ? kt + NST - 1 : nk - 1;
      const unsigned char* ta = lds + st * STAGE;
      const unsigned char* tb = ta + A_BYTES;
      frag_t fb[S];
#pragma unroll
      for (int t = 0; t < S; ++t) fb[t] = frag(tb + t * B_SLICE, wn0 + fr);
      frag_t fa = frag(ta, wm0 + fr);
      int q = 0;  // loads of k-step kt + NST - 1 issued so far
#pragma unroll
      for (int s = 1; s <= S; ++s) {
        frag_t fa_next = fa;
        if (s < S) fa_next = frag(ta + s * A_SLICE, wm0 + fr);
#pragma unroll
        for (int t = 1; t <= S + 1 - s; ++t) {
          lvl[s + t - 2] = Tr::mfma(fa, fb[t - 1], lvl[s + t - 2]);
          if (q < NPW) {
            dma(piece(q), knext, sn);
            ++q;
          }
          __builtin_amdgcn_sched_barrier(0);
        }
        fa = fa_next;
      }
      for (; q < NPW; ++q) dma(piece(q), knext, sn);
      // Stage kt + 1 is complete once at most this k-step's loads are out.
      wait_vm<NST == 3 ? NPW : 0>();
      block_sync();
    }
#pragma unroll
    for (int d = 2; d <= S + 1; ++d) {
      const double sc = pow2neg(BETA * d);
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[v] = __builtin_fma((double)lvl[d - 2][v], sc, acc[v]);
    }
  }
  // No load may still be writing this block's LDS when it ends.
  wait_vm<0>();

  store_tile32(g, acc, m0 + wm0, n0 + wn0, lane);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_split_exponents(const SplitArgs& a, int* exps, hipStream_t st) {
  const int64_t nexp = a.left ? a.rows_pad : a.cols_pad;
  hipLaunchKernelGGL(fill_int, dim3((unsigned)((nexp + 255) / 256)), dim3(256), 0, st, exps, nexp, INT_MIN);
  if (a.left)
    hipLaunchKernelGGL(split_exp_left, dim3((unsigned)a.rows, (unsigned)((a.cols + 2047) / 2048)), dim3(256), 0,
                       st, a, exps);
  else {
    // Row chunks of up to 1024 rows, shorter where the columns alone give
    // a small grid (about 2048 blocks, chunks of at least 64 rows).
    const int64_t cb = (a.cols + 63) / 64;
    const int64_t want = std::min((a.rows + 63) / 64, (2048 + cb - 1) / cb);
    const int64_t chunks = std::max((a.rows + 1023) / 1024, std::max<int64_t>(want, 1));
    const int64_t chunk = ((a.rows + chunks - 1) / chunks + 3) / 4 * 4;
    hipLaunchKernelGGL(split_exp_right, dim3((unsigned)cb, (unsigned)((a.rows + chunk - 1) / chunk)), dim3(256), 0,
                       st, a, exps, chunk);
  }
  return hipGetLastError();
}

template <int ET, int S>
static hipError_t launch_split_s(const SplitArgs& a, int* exps, void* out, hipStream_t st) {
  if (hipError_t e = launch_split_exponents(a, exps, st); e != hipSuccess) return e;
  if (a.left)
    hipLaunchKernelGGL((split_digits_left<ET, S>), dim3((unsigned)a.rows_pad, (unsigned)((a.kp + 2047) / 2048)),
                       dim3(256), 0, st, a, exps, out);
  else
    hipLaunchKernelGGL((split_digits_right<ET, S>), dim3((unsigned)(a.cols_pad / 64), (unsigned)(a.kp / 64)),
                       dim3(256), 0, st, a, exps, out);
  return hipGetLastError();
}

// Block shapes, all with 32 x 32 wave tiles:
//   variant 0: 8 waves (128 x 64 outputs), 2 waves/SIMD, B fragments read
//              from LDS for every slice pair, levels flushed every k-step;
//   variant 1: 4 waves (64 x 64 outputs), 1 wave/SIMD, every A and B
//              fragment of the k-step cached in registers, levels flushed
//              every k-step;
//   variant 2: as variant 1, with the level sums kept across k-steps and
//              flushed to FP64 every slice_flush_steps k-steps;
//   variant 3: slice_gemm_dma (BF16, INT8);
//   variant 4: slice_gemm_x32 (BF16, INT8).
template <int ET, int S, int V>
static hipError_t launch_slice_v(const SliceGemmArgs& g, hipStream_t st) {
  typedef SliceTraits<ET> Tr;
  constexpr int WM = V == 0 ? 4 : 2, CACHE_B = V == 0 ? 0 : 1, WPE = V == 0 ? 2 : 1, PERSIST = V == 2 ? 1 : 0;
  constexpr int BM = 32 * WM;
  constexpr int STAGE = S * (BM + 64) * Tr::KSTEP * Tr::ES;
  constexpr int NSTAGE = 2 * STAGE <= 160 * 1024 ? 2 : 1;
  static_assert(STAGE <= 160 * 1024, "slice tile does not fit LDS");
  const int64_t tiles = ((g.m + BM - 1) / BM) * ((g.n + 63) / 64);
  if (tiles <= 0) return hipSuccess;
  if (tiles > 0x7fffffff || g.kflush < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL((slice_gemm<ET, S, WM, 2, CACHE_B, NSTAGE, WPE, PERSIST>), dim3((unsigned)tiles),
                     dim3(WM * 2 * 64), 0, st, g);
  return hipGetLastError();
}

// Default: the direct-to-LDS shape for BF16 and INT8 digits.  FP8 digits
// have one shape, slice_gemm_f8 (variant 5, bq_split_f8.hip).
int default_slice_variant(int et, int S) {
  (void)S;
  return et == 1 ? 5 : 3;
}

int resolve_slice_variant(int et, int S, int variant) {
  if (et == 1) return 5;
  if (variant < 0 || variant > 4) return default_slice_variant(et, S);
  if (variant == 4 && S > 8) return 3;  // the 32 x 32 shape is built up to 8 slices
  if (variant == 0 && S > 6) return default_slice_variant(et, S);
  return variant;
}

int slice_variant_tiled(int variant) { return (variant == 3 || variant == 5) ? 1 : (variant == 4 ? 2 : 0); }

template <int ET, int S>
static hipError_t launch_slice_s(const SliceGemmArgs& g, int variant, hipStream_t st) {
  variant = resolve_slice_variant(ET, S, variant);
  if (variant == 0) {
    if constexpr (S <= 6) return launch_slice_v<ET, S, 0>(g, st);
    else return hipErrorInvalidValue;
  }
  if (variant == 2) return launch_slice_v<ET, S, 2>(g, st);
  if (variant == 4) {
    if constexpr (S <= 8) {
      const int64_t tiles = ((g.m + 127) / 128) * ((g.n + 63) / 64);
      if (tiles <= 0) return hipSuccess;
      if (tiles > 0x7fffffff || g.kflush < 1) return hipErrorInvalidValue;
      hipLaunchKernelGGL((slice_gemm_x32<ET, S>), dim3((unsigned)tiles), dim3(512), 0, st, g);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  if (variant == 3) {
    const int64_t tiles = ((g.m + 63) / 64) * ((g.n + 63) / 64);
    if (tiles <= 0) return hipSuccess;
    if (tiles > 0x7fffffff || g.kflush < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL((slice_gemm_dma<ET, S>), dim3((unsigned)tiles), dim3(256), 0, st, g);
    return hipGetLastError();
  }
  return launch_slice_v<ET, S, 1>(g, st);
}

int slice_block_rows(int et, int S) {
  (void)et;
  (void)S;
  return 128;  // digit rows are padded to 128, a multiple of both shapes
}

int slice_kstep(int et) {
  return et == 0 ? SliceTraits<0>::KSTEP : (et == 1 ? 64 : SliceTraits<2>::KSTEP);
}
int slice_beta(int et) { return et == 0 ? SliceTraits<0>::BETA : (et == 1 ? f8_beta() : SliceTraits<2>::BETA); }
int slice_head(int et) { return et == 0 ? 0 : (et == 1 ? f8_head() : 1); }

// Level sums stay exact while every partial sum is an integer below 2^24
// (FP32) or 2^31 (int32).  Digit bounds: |q_1| <= 2^{b-h}, |q_s| <= 2^{b-1};
// a level d = s + t has at most d - 1 <= S pairs.  With h = 1 every digit is
// within 2^{b-1}, so per k element |level| <= 2^{2b-2} S; with h = 0 the two
// pairs holding a leading digit count twice: |level| <= 2^{2b-2} (S + 3).
int slice_flush_steps(int et, int S) {
  const int b = slice_beta(et);
  const double per_k = std::ldexp(1.0, 2 * b - 2) * (slice_head(et) ? S : S + 3);
  const double lim = et == 2 ? 2147483647.0 : 16777216.0;
  const int64_t kmax = (int64_t)(lim / per_k);
  const int64_t steps = kmax / slice_kstep(et);
  return (int)std::max<int64_t>(1, std::min<int64_t>(steps, 1 << 20));
}

#define BQ_SPLIT_CASES(ET, X) \
  X(ET, 1) X(ET, 2) X(ET, 3) X(ET, 4) X(ET, 5) X(ET, 6) X(ET, 7) X(ET, 8)
#define BQ_SPLIT_CASES_MORE(X) \
  X(1, 9) X(1, 10) X(1, 11) X(1, 12) X(1, 13) X(2, 9)

hipError_t launch_split(int et, int S, const SplitArgs& a, int* exps, void* out, hipStream_t st) {
#define X(E, SS) \
  if (et == E && S == SS) return launch_split_s<E, SS>(a, exps, out, st);
  BQ_SPLIT_CASES(0, X)
  BQ_SPLIT_CASES(1, X)
  BQ_SPLIT_CASES(2, X)
  BQ_SPLIT_CASES_MORE(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_slice_gemm(int et, int S, int variant, const SliceGemmArgs& g, hipStream_t st) {
  if (et == 1) return launch_slice_gemm_f8(S, g, st);
#define X(E, SS) \
  if (et == E && S == SS) return launch_slice_s<E, SS>(g, variant, st);
  BQ_SPLIT_CASES(0, X)
  BQ_SPLIT_CASES(2, X)
  X(2, 9)
#undef X
  return hipErrorInvalidValue;
}



int max_slices(int et) { return et == 0 ? 8 : (et == 1 ? 13 : 9); }

}  // namespace bq
