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
//     h = 0), OCP FP8 E4M3 (b = 5, h = 1: every digit within 16) or INT8
//     (b = 7, h = 1: one bit of headroom keeps the leading digit inside a
//     signed byte);
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
    const int64_t o = (int64_t)s * a.slice_stride * ES + digit_offset(r, kk0 * ES, a.kp * ES);
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
    const int64_t o = digit_offset(c0 + cc, k0 * ES + p * 16, a.kp * ES);
    *reinterpret_cast<i4v*>(static_cast<unsigned char*>(out) + (int64_t)s * a.slice_stride * ES + o) = v;
  }
}

// ---------------------------------------------------------------------------
// Slice GEMM (BF16 and INT8 digits; FP8 digits: bq_split_f8.hip).
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

// 2^-e for 0 <= e <= 126 (levels reach e = b (S + 1) = 70): two shifts of at
// most 63 bits each, so no shift reaches the width of the operand.
constexpr double pow2neg(int e) {
  return (1.0 / (double)(1ull << (e / 2))) * (1.0 / (double)(1ull << (e - e / 2)));
}

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

  // Loads: the digits are tiled (digit_offset), so the tile of slice s
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

template <int ET, int S>
static hipError_t launch_slice_s(const SliceGemmArgs& g, hipStream_t st) {
  const int64_t tiles = ((g.m + 63) / 64) * ((g.n + 63) / 64);
  if (tiles <= 0) return hipSuccess;
  if (tiles > 0x7fffffff || g.kflush < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL((slice_gemm_dma<ET, S>), dim3((unsigned)tiles), dim3(256), 0, st, g);
  return hipGetLastError();
}

int slice_block_rows(int et, int S) {
  (void)et;
  (void)S;
  return 128;  // digit rows are padded to 128, a multiple of every block's rows
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

hipError_t launch_slice_gemm(int et, int S, const SliceGemmArgs& g, hipStream_t st) {
  if (et == 1) return launch_slice_gemm_f8(S, g, st);
#define X(E, SS) \
  if (et == E && S == SS) return launch_slice_s<E, SS>(g, st);
  BQ_SPLIT_CASES(0, X)
  BQ_SPLIT_CASES(2, X)
  X(2, 9)
#undef X
  return hipErrorInvalidValue;
}



int max_slices(int et) { return et == 0 ? 8 : (et == 1 ? 13 : 9); }

}  // namespace bq
