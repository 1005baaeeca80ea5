// CRT-based split form of one real product (Ozaki scheme II,
// integer-modular), for gfx950.
//
// A real product T = X Y: every row of X (column of Y) gets its frexp
// exponent e (f), the scaled integers X' = rint(x 2^(b - e)) (|X'| <= 2^b,
// b <= 53, exact in FP64) are written as symmetric residues modulo N odd,
// pairwise coprime moduli p_i <= 255 (one signed byte each), every modulus
// is one exact INT8 GEMM with int32 sums (|sum| <= k 127^2 < 2^31), its
// result reduced to a residue again, and P = X'Y' is recovered from its
// residues r_i by the Chinese remainder theorem: P = sum_i r_i c_i - q M
// with M = p_1 ... p_N, c_i = (M / p_i) ((M / p_i)^-1 mod p_i) and q the
// integer nearest to sum_i r_i (c_i / M).  The bound |P| <= k 2^(2b) <
// 2^127 lets that sum run in 128-bit wraparound integers, so P is exact;
// it is rounded to FP64 once and T = P 2^(e + f - 2b) is the correctly
// rounded product of the scaled integers.  N moduli with M > 2 k 2^(2b)
// carry b bits.
#include <limits.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <vector>

#include "bq_split_common.h"

namespace bq {

constexpr int kCrtModuli[kMaxCrtModuli] = {255, 253, 251, 247, 241, 239, 233, 229, 227, 223,
                                           211, 199, 197, 193, 191, 181, 179, 173, 167, 163};

// 2^18 and 2^36 modulo each p_i: the weights of the 18-bit limbs of X'.
struct CrtTables {
  int w18[kMaxCrtModuli];
  int w36[kMaxCrtModuli];
};
constexpr CrtTables make_crt_tables() {
  CrtTables t{};
  for (int i = 0; i < kMaxCrtModuli; ++i) {
    t.w18[i] = (int)((1ll << 18) % kCrtModuli[i]);
    t.w36[i] = (int)((1ll << 36) % kCrtModuli[i]);
  }
  return t;
}
constexpr CrtTables kCrtW = make_crt_tables();

// Symmetric residue of t (|t| < 2^31) modulo an odd p: [-(p-1)/2, (p-1)/2].
// For a p known at compile time (the division becomes a multiplication).
__device__ __forceinline__ int sym_mod(int t, int p) {
  t %= p;
  const int h = (p - 1) >> 1;
  return t > h ? t - p : (t < -h ? t + p : t);
}

// The same for a p known at run time: q = rint(t / p) in FP64 is exact (t / p
// is never within 1 / (2 p) of a half-integer for odd p, far above the
// rounding error), and t - q p is formed exactly by one fma.
__device__ __forceinline__ int sym_mod_rt(int t, double p, double inv_p) {
  const double td = (double)t;
  return (int)__builtin_fma(-rint(td * inv_p), p, td);
}

// Residues of one element: X' = rint(x 2^(b - e)) (|X'| <= 2^53) as 18-bit
// limbs a2 2^36 + a1 2^18 + a0 (a0, a1 in [0, 2^18), |a2| <= 2^17), so
// a2 (2^36 mod p) + a1 (2^18 mod p) + a0 stays below 2^27 and one reduction
// per modulus is left; p and the weights are constants once unrolled.
template <int N>
__device__ __forceinline__ void crt_residues(double x, int e, int b, signed char* r) {
  const double y = exp_special(e) ? 0.0 : rint(ldexp(x, b - e));
  const int64_t xi = (int64_t)y;
  const int a0 = (int)(xi & 0x3ffff);
  const int a1 = (int)((xi >> 18) & 0x3ffff);
  const int a2 = (int)(xi >> 36);
#pragma unroll
  for (int i = 0; i < N; ++i) r[i] = (signed char)sym_mod(a2 * kCrtW.w36[i] + a1 * kCrtW.w18[i] + a0, kCrtModuli[i]);
}

// Left factor: residue planes R[i][row][kk] in the tiled 64-byte layout.
// Thread: 2 consecutive kk of one row, so a wave reads 1 KB of the row and
// writes 128 contiguous bytes of each plane.  grid.x = rows_pad,
// grid.y = kp / 512.
template <int N>
__device__ __forceinline__ void crt_split_left_at(const SplitArgs& a, const int* exps, void* out, int64_t r,
                                                  int64_t kk) {
  if (kk >= a.kp) return;
  const int e = (r < a.rows) ? exps[r] : INT_MIN;
  signed char q[2][N];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int64_t c = kk + t;
    const double x = (r < a.rows && c < a.cols) ? operand_value(a, r * a.ld + c) : 0.0;
    crt_residues<N>(x, e, a.beta, q[t]);
  }
  const int64_t o = digit_offset(r, kk, a.kp);
#pragma unroll
  for (int i = 0; i < N; ++i)
    *reinterpret_cast<unsigned short*>(static_cast<unsigned char*>(out) + (int64_t)i * a.slice_stride + o) =
        (unsigned short)((unsigned char)q[0][i] | ((unsigned)(unsigned char)q[1][i] << 8));
}

template <int N>
__global__ void __launch_bounds__(256) crt_split_left(const SplitArgs a, const int* exps, void* out) {
  crt_split_left_at<N>(a, exps, out, blockIdx.x, (int64_t)blockIdx.y * 512 + threadIdx.x * 2);
}

// Right factor (k x n): residues stored transposed, R[i][col][kk].  Thread:
// one column and 16 consecutive kk (one 16-byte chunk of each plane),
// consecutive lanes on consecutive columns, so every row read is coalesced
// and no LDS transpose is needed.  grid.x = cols_pad / 64, grid.y = kp / 64.
template <int N>
__device__ __forceinline__ void crt_split_right_block(const SplitArgs& a, const int* exps, void* out, int64_t bx,
                                                      int64_t by) {
  const int64_t c = bx * 64 + (threadIdx.x & 63);
  const int64_t k0 = by * 64 + (threadIdx.x >> 6) * 16;
  const int e = (c < a.cols) ? exps[c] : INT_MIN;
  i4v q[N];
#pragma unroll
  for (int i = 0; i < N; ++i) q[i] = i4v{0, 0, 0, 0};
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int64_t kk = k0 + t;
    const double x = (c < a.cols && kk < a.rows) ? operand_value(a, kk * a.ld + c) : 0.0;
    signed char d[N];
    crt_residues<N>(x, e, a.beta, d);
#pragma unroll
    for (int i = 0; i < N; ++i) q[i][t >> 2] |= (int)(unsigned char)d[i] << (8 * (t & 3));
  }
  const int64_t o = digit_offset(c, k0, a.kp);
#pragma unroll
  for (int i = 0; i < N; ++i)
    *reinterpret_cast<i4v*>(static_cast<unsigned char*>(out) + (int64_t)i * a.slice_stride + o) = q[i];
}

template <int N>
__global__ void __launch_bounds__(256) crt_split_right(const SplitArgs a, const int* exps, void* out) {
  crt_split_right_block<N>(a, exps, out, blockIdx.x, blockIdx.y);
}

// Exponents of one operand without atomics (grouped launches): a row-kernel
// operand takes one block per row, a column-kernel operand one block per 64
// columns over all its rows; every block writes its exponents once.
__device__ __forceinline__ void crt_exp_block(const SplitArgs& a, int* exps, int64_t b, int* red) {
  int e = INT_MIN;
  if (a.left) {
    const int64_t r = b;
    for (int64_t c = threadIdx.x; c < a.cols; c += 256) e = max(e, exp_of(operand_value(a, r * a.ld + c)));
    for (int o = 32; o > 0; o >>= 1) e = max(e, __shfl_xor(e, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
      e = max(max(red[0], red[1]), max(red[2], red[3]));
      exps[r] = exp_special(e) ? e : e + a.head;
    }
  } else {
    const int64_t c = b * 64 + (threadIdx.x & 63);
    if (c < a.cols)
      for (int64_t r = threadIdx.x >> 6; r < a.rows; r += 4) e = max(e, exp_of(operand_value(a, r * a.ld + c)));
    red[threadIdx.x] = e;
    __syncthreads();
    if (threadIdx.x < 64 && c < a.cols) {
      e = max(max(red[threadIdx.x], red[threadIdx.x + 64]), max(red[threadIdx.x + 128], red[threadIdx.x + 192]));
      exps[c] = exp_special(e) ? e : e + a.head;
    }
  }
}

// One INT8 GEMM per modulus (blockIdx.y): residue planes of X (rows padded
// to 256) and Y (columns padded to 256) in the tiled 64-byte layout, a 128 x
// 128 block of 4 waves (64 x 64 each, 16 v_mfma_i32_16x16x64_i8 per k-step),
// four LDS stages filled straight from global memory three k-steps ahead,
// every wave moving 4 of the stage's 16 KB.  The int32 result is reduced to
// its symmetric residue and stored as a byte plane R[i][row][col].
constexpr int kCrtGemmLds = 4 * 4 * 64 * 64;  // four stages of two A and two B 4 KB tiles

__device__ __forceinline__ void crt_gemm_block(const CrtGemmArgs& g, int tm, int tn, int mod, unsigned char* lds) {
  constexpr int BM = 128, BN = 128, ROWB = 64, TILE = 64 * ROWB;  // 4 KB per 64-row tile
  constexpr int STAGE = 4 * TILE;                                  // two A tiles, two B tiles
  constexpr int NST = 4, NPW = 4;
  static_assert(NST * STAGE == kCrtGemmLds, "LDS size");
  const int p = kCrtModuli[mod];
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm0 = (wave >> 1) * 64, wn0 = (wave & 1) * 64;
  const int fr = lane & 15, fg = lane >> 4;

  const int64_t nk = g.kp / ROWB;
  const int64_t run = nk * TILE;
  const unsigned char* ga = static_cast<const unsigned char*>(g.a) + mod * g.plane_a + (int64_t)(2 * tm) * run;
  const unsigned char* gb = static_cast<const unsigned char*>(g.b) + mod * g.plane_b + (int64_t)(2 * tn) * run;
  const int nrec = (int)(uint32_t)(2 * run);
  // 1 KB piece q of a stage: q < 8 A (tile q / 4, quarter q % 4), else B.
  auto dma = [&](int q, int64_t kt, int st) {
    const int side = q >> 3, t = (q >> 2) & 1, quarter = q & 3;
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc((void*)(side ? gb : ga), (short)0, nrec, 0x00020000);
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_void_ptr)(lds + st * STAGE + q * 1024), 16,
                                             (int)(t * run) + quarter * 1024 + lane * 16, (int)(kt * TILE), 0, 0);
  };
  auto frag = [&](const unsigned char* base, int row) {
    return *reinterpret_cast<const i4v*>(base + row * ROWB + swz_chunk<16>(row & 63, fg) * 16);
  };

  i4v acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = i4v{0, 0, 0, 0};

  // Prologue: k-steps 0..NST-2 (past the end: the last one again).
#pragma unroll
  for (int s = 0; s < NST - 1; ++s)
#pragma unroll
    for (int i = 0; i < NPW; ++i) dma(wave * NPW + i, s < nk ? s : nk - 1, s);
  wait_vm<(NST - 2) * NPW>();
  block_sync();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int st = (int)(kt % NST);
    const int sn = (int)((kt + NST - 1) % NST);
    const int64_t knext = kt + NST - 1 < nk ? kt + NST - 1 : nk - 1;
    const unsigned char* ta = lds + st * STAGE;
    const unsigned char* tb = ta + 2 * TILE;
    i4v fa[4], fb[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) fa[i] = frag(ta, wm0 + i * 16 + fr);
#pragma unroll
    for (int j = 0; j < 4; ++j) fb[j] = frag(tb, wn0 + j * 16 + fr);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[i], fb[j], acc[i][j], 0, 0, 0);
      dma(wave * NPW + i, knext, sn);
      __builtin_amdgcn_sched_barrier(0);
    }
    // Stage kt + 1 is complete once at most the loads of the last two
    // k-steps (kt + NST - 2, kt + NST - 1) are still out.
    wait_vm<(NST - 2) * NPW>();
    block_sync();
  }
  wait_vm<0>();
  __builtin_amdgcn_s_waitcnt(0xC07F);
  block_sync();

  // Residues into a 128 x 128 byte tile in LDS (rows of OUT_LD bytes), then
  // 16-byte row stores (columns up to ldr, a multiple of 16).
  constexpr int OUT_LD = BN + 16;
  static_assert(BM * OUT_LD <= kCrtGemmLds, "output tile fits the stages");
  const double pd = (double)p, inv_p = 1.0 / pd;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        lds[(wm0 + i * 16 + 4 * fg + v) * OUT_LD + wn0 + j * 16 + fr] =
            (unsigned char)sym_mod_rt(acc[i][j][v], pd, inv_p);
  __syncthreads();
  signed char* out = g.out + (int64_t)mod * g.plane_r;
  for (int w = tid; w < BM * (BN / 16); w += 256) {
    const int r = w / (BN / 16), ch = w % (BN / 16);
    const int64_t grow = m0 + r, gcol = n0 + ch * 16;
    if (grow < g.m && gcol < g.ldr)
      *reinterpret_cast<i4v*>(out + grow * g.ldr + gcol) = *reinterpret_cast<const i4v*>(lds + r * OUT_LD + ch * 16);
  }
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
crt_gemm(const CrtGemmArgs g) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[kCrtGemmLds];
  const int tiles_m = (int)((g.m + 127) / 128);
  const int tiles_n = (int)((g.n + 127) / 128);
  int tm, tn;
  slice_tile_coords(tiles_m, tiles_n, tm, tn);
  crt_gemm_block(g, tm, tn, blockIdx.y, lds);
}

// The same GEMM for large products: a 256 x 256 block of 4 waves (128 x 128
// each: 8 x 8 v_mfma_i32_16x16x64_i8 per k-step, accumulators in AGPRs), so
// each k-step moves 32 KB into LDS for 2^23 multiply-adds, half the bytes
// per MFMA of the 128 x 128 block.  Four LDS stages of 32 KB filled straight
// from global memory three k-steps ahead (8 KB per wave per k-step, one 1 KB
// piece after each row of MFMAs); the fragments of k-step kt + 1 are read
// from LDS into a second register set while the MFMAs of k-step kt run.
// The int32 results are reduced to residues, gathered as a 256 x 256 byte
// tile in LDS and stored as 16-byte rows.
template <int NST>  // LDS stages; 4 measured faster than 5
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
crt_gemm_256(const CrtGemmArgs g) {
  constexpr int BM = 256, BN = 256, ROWB = 64, TILE = 64 * ROWB;  // 4 KB per 64-row tile
  constexpr int STAGE = 8 * TILE;                                  // four A tiles, four B tiles
  constexpr int NPW = 8;
  static_assert(NST >= 4 && NST * STAGE <= 160 * 1024, "stages fit LDS");
  constexpr int OUT_LD = BN + 16;
  static_assert(BM * OUT_LD <= NST * STAGE, "the residue tile fits the stages");
  __shared__ __attribute__((aligned(16))) unsigned char lds[NST * STAGE];
  const int mod = blockIdx.y;
  const int p = kCrtModuli[mod];

  const int tiles_m = (int)((g.m + BM - 1) / BM);
  const int tiles_n = (int)((g.n + BN - 1) / BN);
  int tm, tn;
  slice_tile_coords(tiles_m, tiles_n, tm, tn);
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm0 = (wave >> 1) * 128, wn0 = (wave & 1) * 128;
  const int fr = lane & 15, fg = lane >> 4;

  const int64_t nk = g.kp / ROWB;
  const int64_t run = nk * TILE;
  const unsigned char* ga = static_cast<const unsigned char*>(g.a) + mod * g.plane_a + (int64_t)(4 * tm) * run;
  const unsigned char* gb = static_cast<const unsigned char*>(g.b) + mod * g.plane_b + (int64_t)(4 * tn) * run;
  const int nrec = (int)(uint32_t)(4 * run);
  const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc((void*)ga, (short)0, nrec, 0x00020000);
  const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc((void*)gb, (short)0, nrec, 0x00020000);
  // 1 KB piece q of a stage: q < 16 A (tile q / 4, quarter q % 4), else B.
  auto dma = [&](int q, int64_t kt, int st) {
    const int t = (q >> 2) & 3, quarter = q & 3;
    __builtin_amdgcn_raw_ptr_buffer_load_lds(q >= 16 ? rb : ra, (lds_void_ptr)(lds + st * STAGE + q * 1024), 16,
                                             (int)(t * run) + quarter * 1024 + lane * 16, (int)(kt * TILE), 0, 0);
  };
  auto frag = [&](const unsigned char* base, int row) {
    return *reinterpret_cast<const i4v*>(base + row * ROWB + swz_chunk<16>(row & 63, fg) * 16);
  };
  auto read_frags = [&](int st, i4v(&fa)[8], i4v(&fb)[8]) {
    const unsigned char* ta = lds + st * STAGE;
    const unsigned char* tb = ta + 4 * TILE;
#pragma unroll
    for (int i = 0; i < 8; ++i) fa[i] = frag(ta, wm0 + i * 16 + fr);
#pragma unroll
    for (int j = 0; j < 8; ++j) fb[j] = frag(tb, wn0 + j * 16 + fr);
  };

  i4v acc[8][8];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[i][j] = i4v{0, 0, 0, 0};

  // One k-step: fa, fb hold its fragments; na, nb receive those of kt + 1
  // (for kt + 1 = nk, stale LDS bytes that are never used).  Stage kt + 1 is
  // complete once only the loads of k-steps kt + 2 .. kt + NST - 2 are out;
  // after the barrier every wave holds the fragments of k-step kt, so stage
  // (kt - 1) % NST is free for k-step kt + NST - 1.
  auto step = [&](int64_t kt, i4v(&fa)[8], i4v(&fb)[8], i4v(&na)[8], i4v(&nb)[8]) {
    wait_vm<(NST - 3) * NPW>();
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): fa, fb have landed
    block_sync();
    read_frags((int)((kt + 1) % NST), na, nb);
    const int64_t knext = kt + NST - 1 < nk ? kt + NST - 1 : nk - 1;
    const int sn = (int)((kt + NST - 1) % NST);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[i], fb[j], acc[i][j], 0, 0, 0);
      dma(wave * NPW + i, knext, sn);
      __builtin_amdgcn_sched_barrier(0);
    }
  };

  // Prologue: k-steps 0..NST-2 (past the end: the last one again); the
  // fragments of k-step 0.
#pragma unroll
  for (int s = 0; s < NST - 1; ++s)
#pragma unroll
    for (int i = 0; i < NPW; ++i) dma(wave * NPW + i, s < nk ? s : nk - 1, s);
  wait_vm<(NST - 2) * NPW>();
  block_sync();
  i4v xa[8], xb[8], ya[8], yb[8];
  read_frags(0, xa, xb);
  // nk is even (k padded to 128).
  for (int64_t kt = 0; kt < nk; kt += 2) {
    step(kt, xa, xb, ya, yb);
    step(kt + 1, ya, yb, xa, xb);
  }
  wait_vm<0>();
  __builtin_amdgcn_s_waitcnt(0xC07F);
  block_sync();

  // Residues into a byte tile (rows of OUT_LD bytes), then 16-byte stores.
  const double pd = (double)p, inv_p = 1.0 / pd;
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        lds[(wm0 + i * 16 + 4 * fg + v) * OUT_LD + wn0 + j * 16 + fr] =
            (unsigned char)sym_mod_rt(acc[i][j][v], pd, inv_p);
  __syncthreads();
  signed char* out = g.out + (int64_t)mod * g.plane_r;
  for (int w = tid; w < BM * (BN / 16); w += 256) {
    const int r = w / (BN / 16), ch = w % (BN / 16);
    const int64_t grow = m0 + r, gcol = n0 + ch * 16;
    if (grow < g.m && gcol < g.ldr)
      *reinterpret_cast<i4v*>(out + grow * g.ldr + gcol) = *reinterpret_cast<const i4v*>(lds + r * OUT_LD + ch * 16);
  }
}

// |P| rounded to FP64 once (round to nearest even): the leading 64 bits
// with every lower bit folded into a sticky bit, converted as two exact
// 32-bit halves joined by one fma.
__device__ __forceinline__ double u128_to_double(unsigned __int128 u) {
  const uint64_t hi = (uint64_t)(u >> 64);
  int sh = 0;
  uint64_t top = (uint64_t)u;
  if (hi != 0) {
    sh = 64 - __builtin_clzll(hi);
    const unsigned __int128 rest = u & ((((unsigned __int128)1) << sh) - 1);
    top = (uint64_t)(u >> sh) | (uint64_t)(rest != 0);
  }
  const double d = __builtin_fma((double)(uint32_t)(top >> 32), 4294967296.0, (double)(uint32_t)top);
  return ldexp(d, sh);
}

// P_p from its residues, T_p = P_p 2^(e + f - 2b) for the np real
// products, sum_p coef[q][p] T_p into every target.  Thread: 4 consecutive
// columns of one row (one 32-bit load per residue plane); grid.x = rows *
// ceil(cols / 1024).  The 128-bit sum runs in FP64 over 32-bit parts of c_i
// and M: x_j = sum_i r_i c_ij - q M_j stays an integer below 2^45, so every
// fma is exact; the carries are then moved up (floor and fma, exact) until
// each part lies in [0, 2^32), the carry out of the top part being the
// reduction modulo 2^128.  The parts and c_i / M are staged in LDS and read
// as broadcasts.
constexpr int kCombineCols = 4;
constexpr int kGroupedCombineCols = 2;  // fewer registers per thread, more waves for small products

struct CrtLds {
  double cpart[kMaxCrtModuli][4];
  double frac[kMaxCrtModuli];
  double mpart[4];
};

template <int N, int CC>
__device__ __forceinline__ void crt_values(const CrtCombineArgs& g, const CrtLds& K, const signed char* res,
                                           int64_t off, double (&out)[CC]) {
  double x[CC][4];
  double s[CC];
#pragma unroll
  for (int e = 0; e < CC; ++e) {
    s[e] = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) x[e][j] = 0.0;
  }
#pragma unroll
  for (int i = 0; i < N; ++i) {
    static_assert(CC == 2 || CC == 4, "one 16- or 32-bit load per plane");
    const signed char* src = res + (int64_t)i * g.plane_r + off;
    const uint32_t w = CC == 4 ? *reinterpret_cast<const uint32_t*>(src) : *reinterpret_cast<const uint16_t*>(src);
    const double fr = K.frac[i];
#pragma unroll
    for (int e = 0; e < CC; ++e) {
      const double v = (double)(int)(signed char)(w >> (8 * e));
      s[e] = __builtin_fma(v, fr, s[e]);
#pragma unroll
      for (int j = 0; j < 4; ++j) x[e][j] = __builtin_fma(v, K.cpart[i][j], x[e][j]);
    }
  }
  unsigned __int128 Mu = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) Mu |= (unsigned __int128)(uint32_t)K.mpart[j] << (32 * j);
  const __int128 M = (__int128)Mu;
  constexpr double two32 = 4294967296.0, inv32 = 1.0 / 4294967296.0;
#pragma unroll
  for (int e = 0; e < CC; ++e) {
    const double q = rint(s[e]);
    uint32_t limb[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      double y = __builtin_fma(-q, K.mpart[j], x[e][j]);
      const double f = floor(y * inv32);
      y = __builtin_fma(-f, two32, y);
      if (j < 3) x[e][j + 1] += f;
      limb[j] = (uint32_t)y;
    }
    const unsigned __int128 P = ((unsigned __int128)(((uint64_t)limb[3] << 32) | limb[2]) << 64) |
                                (((uint64_t)limb[1] << 32) | limb[0]);
    __int128 Ps = (__int128)P;
    if (N <= 16) {
      // M < 2^125: an estimate of q one off leaves P - M or P + M, both in range.
      const __int128 half = (M - 1) >> 1;
      if (Ps > half) Ps -= M;
      else if (Ps < -half) Ps += M;
    }
    const bool neg = Ps < 0;
    const double a = u128_to_double((unsigned __int128)(neg ? -Ps : Ps));
    out[e] = neg ? -a : a;
  }
}

// Constants of the first N moduli into LDS (every thread calls it).
template <int N>
__device__ __forceinline__ void crt_stage_consts(CrtLds& K, const double (&cpart)[kMaxCrtModuli][4],
                                                 const double (&frac)[kMaxCrtModuli], const double (&mpart)[4]) {
  for (int t = threadIdx.x; t < N * 4; t += 256) K.cpart[t / 4][t % 4] = cpart[t / 4][t % 4];
  for (int t = threadIdx.x; t < N; t += 256) K.frac[t] = frac[t];
  if (threadIdx.x < 4) K.mpart[threadIdx.x] = mpart[threadIdx.x];
  __syncthreads();
}

// Columns c0 .. c0 + CC - 1 of row r of the reconstruction of one complex
// product.
template <int N, int CC = kCombineCols>
__device__ __forceinline__ void crt_combine_at(const CrtCombineArgs& g, const CrtLds& K, int64_t r, int64_t c0) {
  if (r >= g.m || c0 >= g.n) return;
  double t[kCrtProducts][CC];
#pragma unroll
  for (int p = 0; p < kCrtProducts; ++p) {
#pragma unroll
    for (int e = 0; e < CC; ++e) t[p][e] = 0.0;
    if (p < g.np) {
      crt_values<N, CC>(g, K, g.res[p], r * g.ldr + c0, t[p]);
      const int ea = g.ea[p][r];
#pragma unroll
      for (int e = 0; e < CC; ++e) {
        const int eb = (c0 + e < g.n) ? g.eb[p][c0 + e] : INT_MIN;
        t[p][e] = exp_special(ea) || exp_special(eb) ? exp_scaled(0.0, ea, eb, 0)
                                                      : ldexp(t[p][e], ea + eb - 2 * g.bits);
      }
    }
  }
  // Per target, its pointer, coefficients and mode go to registers before
  // any store (the arguments may sit in a device table the compiler cannot
  // tell apart from C).
  const int ntgt = g.ntgt, np = g.np;
  const int64_t n = g.n;
  for (int q = 0; q < ntgt; ++q) {
    double* cq = g.c[q] + r * g.ldc;
    double w[kCrtProducts];
#pragma unroll
    for (int p = 0; p < kCrtProducts; ++p) w[p] = g.coef[q][p];
    const bool accum = g.mode[q] == TGT_ACCUM;
#pragma unroll
    for (int e = 0; e < CC; ++e) {
      if (c0 + e >= n) continue;
      // zero coefficients are skipped, as the products they would scale
      double val = 0.0;
      bool any = false;
#pragma unroll
      for (int p = 0; p < kCrtProducts; ++p) {
        if (p < np && w[p] != 0.0) {
          val = any ? __builtin_fma(w[p], t[p][e], val) : w[p] * t[p][e];
          any = true;
        }
      }
      if (accum) val += cq[c0 + e];
      cq[c0 + e] = val;
    }
  }
}

template <int N>
__global__ void __launch_bounds__(256) crt_combine(const CrtCombineArgs g) {
  __shared__ CrtLds K;
  crt_stage_consts<N>(K, g.cpart, g.frac, g.mpart);
  const int64_t bpr = (g.n + 256 * kCombineCols - 1) / (256 * kCombineCols);
  crt_combine_at<N>(g, K, blockIdx.x / bpr, (blockIdx.x % bpr) * (256 * kCombineCols) + threadIdx.x * kCombineCols);
}

// ---------------------------------------------------------------------------
// Grouped forms: one launch over the items of many problems.
// ---------------------------------------------------------------------------
// The Chinese remainder constants of one modulus count (filled on the host).
struct CrtConsts {
  double cpart[kMaxCrtModuli][4];
  double frac[kMaxCrtModuli];
  double mpart[4];
};

// Last item whose first block is at or before block b.
__device__ __forceinline__ int crt_find_item(const int64_t* prefix, int count, int64_t b) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ void __launch_bounds__(256) crt_exp_grouped(const CrtSplitItem* items, const int64_t* prefix, int count) {
  __shared__ int red[256];
  const int64_t b = blockIdx.x;
  const int i = crt_find_item(prefix, count, b);
  crt_exp_block(items[i].a, items[i].exps, b - prefix[i], red);
}

template <int N>
__global__ void __launch_bounds__(256) crt_split_grouped(const CrtSplitItem* items, const int64_t* prefix, int count) {
  const int64_t b = blockIdx.x;
  const int i = crt_find_item(prefix, count, b);
  const CrtSplitItem& it = items[i];
  const int64_t local = b - prefix[i];
  if (it.a.left) {
    // thread: one pair of kk of one row, pairs of consecutive rows packed
    // into the block (padding rows are left alone: their GEMM rows are
    // never stored)
    const int64_t pairs = it.a.kp / 2;
    const int64_t q = local * 256 + threadIdx.x;
    const int64_t r = q / pairs;
    if (r >= it.a.rows) return;
    crt_split_left_at<N>(it.a, it.exps, it.out, r, (q % pairs) * 2);
  } else {
    const int64_t nky = it.a.kp / 64;
    crt_split_right_block<N>(it.a, it.exps, it.out, local / nky, local % nky);
  }
}

// Item blocks run modulus by modulus, tiles row by row within a modulus.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
crt_gemm_grouped(const CrtGemmItem* items, const int64_t* prefix, int count) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[kCrtGemmLds];
  const int64_t b = blockIdx.x;
  const int i = crt_find_item(prefix, count, b);
  const CrtGemmArgs& g = items[i].g;
  const int tiles_n = (int)((g.n + 127) / 128);
  const int64_t tiles = ((g.m + 127) / 128) * tiles_n;
  const int64_t local = b - prefix[i];
  const int t = (int)(local % tiles);
  crt_gemm_block(g, t / tiles_n, t % tiles_n, (int)(local / tiles), lds);
}

template <int N>
__global__ void __launch_bounds__(256) crt_combine_grouped(const CrtCombineArgs* items, const int64_t* prefix,
                                                           int count, const CrtConsts k) {
  __shared__ CrtLds K;
  crt_stage_consts<N>(K, k.cpart, k.frac, k.mpart);
  const int64_t b = blockIdx.x;
  const int i = crt_find_item(prefix, count, b);
  // thread: one pair of columns; the pairs of consecutive rows packed into
  // the block
  const CrtCombineArgs& g = items[i];
  const int64_t qpr = (g.n + kGroupedCombineCols - 1) / kGroupedCombineCols;
  const int64_t q = (b - prefix[i]) * 256 + threadIdx.x;
  crt_combine_at<N, kGroupedCombineCols>(g, K, q / qpr, (q % qpr) * kGroupedCombineCols);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <int N>
static hipError_t launch_crt_split_n(const SplitArgs& a, int* exps, void* out, hipStream_t st) {
  if (hipError_t e = launch_split_exponents(a, exps, st); e != hipSuccess) return e;
  if (a.left)
    hipLaunchKernelGGL((crt_split_left<N>), dim3((unsigned)a.rows_pad, (unsigned)((a.kp + 511) / 512)),
                       dim3(256), 0, st, a, exps, out);
  else
    hipLaunchKernelGGL((crt_split_right<N>), dim3((unsigned)(a.cols_pad / 64), (unsigned)(a.kp / 64)), dim3(256), 0,
                       st, a, exps, out);
  return hipGetLastError();
}

// Chinese remainder constants of the first N moduli, exact (base-2^32
// big integers): c_i = M_i (M_i^-1 mod p_i) with M_i = M / p_i and M, kept
// modulo 2^128 as four 32-bit parts (exact in FP64), and c_i / M in FP64.

static std::vector<uint32_t> big_mul(std::vector<uint32_t> v, uint32_t x) {
  uint64_t carry = 0;
  for (uint32_t& l : v) {
    const uint64_t t = uint64_t(l) * x + carry;
    l = uint32_t(t);
    carry = t >> 32;
  }
  if (carry) v.push_back(uint32_t(carry));
  return v;
}

static std::vector<uint32_t> big_div(const std::vector<uint32_t>& v, uint32_t x) {  // exact division
  std::vector<uint32_t> q(v.size());
  uint64_t rem = 0;
  for (size_t i = v.size(); i-- > 0;) {
    const uint64_t cur = (rem << 32) | v[i];
    q[i] = uint32_t(cur / x);
    rem = cur % x;
  }
  return q;
}

static uint32_t big_mod(const std::vector<uint32_t>& v, uint32_t x) {
  uint64_t rem = 0;
  for (size_t i = v.size(); i-- > 0;) rem = ((rem << 32) | v[i]) % x;
  return uint32_t(rem);
}

static long double big_value(const std::vector<uint32_t>& v) {
  long double d = 0.0L;
  for (size_t i = v.size(); i-- > 0;) d = d * 4294967296.0L + (long double)v[i];
  return d;
}

static CrtConsts make_crt_consts(int N) {
  CrtConsts t{};
  std::vector<uint32_t> M{1};
  for (int i = 0; i < N; ++i) M = big_mul(M, uint32_t(kCrtModuli[i]));
  const long double Md = big_value(M);
  auto part = [](const std::vector<uint32_t>& v, int j) -> double {
    return size_t(j) < v.size() ? double(v[size_t(j)]) : 0.0;
  };
  for (int j = 0; j < 4; ++j) t.mpart[j] = part(M, j);
  for (int i = 0; i < N; ++i) {
    const uint32_t p = uint32_t(kCrtModuli[i]);
    const std::vector<uint32_t> Mi = big_div(M, p);
    const uint32_t a = big_mod(Mi, p);
    uint32_t inv = 1;  // a^-1 mod p by search (p < 256)
    while ((uint64_t(a) * inv) % p != 1) ++inv;
    const std::vector<uint32_t> ci = big_mul(Mi, inv);
    for (int j = 0; j < 4; ++j) t.cpart[i][j] = part(ci, j);
    t.frac[i] = (double)(big_value(ci) / Md);
  }
  return t;
}

template <int N>
static hipError_t launch_crt_combine_n(CrtCombineArgs g, hipStream_t st) {
  const int64_t blocks = g.m * ((g.n + 256 * kCombineCols - 1) / (256 * kCombineCols));
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffff || (g.ldr % kCombineCols) != 0) return hipErrorInvalidValue;
  static const CrtConsts k = make_crt_consts(N);
  std::copy(&k.cpart[0][0], &k.cpart[0][0] + kMaxCrtModuli * 4, &g.cpart[0][0]);
  std::copy(k.frac, k.frac + kMaxCrtModuli, g.frac);
  std::copy(k.mpart, k.mpart + 4, g.mpart);
  hipLaunchKernelGGL((crt_combine<N>), dim3((unsigned)blocks), dim3(256), 0, st, g);
  return hipGetLastError();
}

#define BQ_CRT_CASES(X) \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) X(19) X(20)

hipError_t launch_crt_split(int N, const SplitArgs& a, int* exps, void* out, hipStream_t st) {
#define X(NN) \
  if (N == NN) return launch_crt_split_n<NN>(a, exps, out, st);
  BQ_CRT_CASES(X)
#undef X
  return hipErrorInvalidValue;
}

// Block shape of the residue GEMMs: 256 x 256 once the grid holds two
// blocks per CU (the larger block halves the bytes per MFMA), else 128 x 128
// for more blocks on small products.  BQ_CRT_TILE=128 or 256 overrides.
int crt_gemm_tile(int N, int64_t m, int64_t n) {
  const char* e = std::getenv("BQ_CRT_TILE");
  if (e && std::atoi(e) == 128) return 128;
  if (e && std::atoi(e) == 256) return 256;
  const int64_t big = ((m + 255) / 256) * ((n + 255) / 256) * N;
  return big >= 512 ? 256 : 128;
}

hipError_t launch_crt_gemm(int N, const CrtGemmArgs& g, hipStream_t st) {
  if (g.m <= 0 || g.n <= 0 || N <= 0) return hipSuccess;
  if (N > kMaxCrtModuli || (g.ldr & 15) != 0) return hipErrorInvalidValue;
  if (crt_gemm_tile(N, g.m, g.n) == 256) {
    if (g.kp % 128 != 0) return hipErrorInvalidValue;  // the loop takes k-steps in pairs
    const int64_t tiles = ((g.m + 255) / 256) * ((g.n + 255) / 256);
    if (tiles > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(crt_gemm_256<4>, dim3((unsigned)tiles, (unsigned)N), dim3(256), 0, st, g);
  } else {
    const int64_t tiles = ((g.m + 127) / 128) * ((g.n + 127) / 128);
    if (tiles > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(crt_gemm, dim3((unsigned)tiles, (unsigned)N), dim3(256), 0, st, g);
  }
  return hipGetLastError();
}

hipError_t launch_crt_combine(int N, const CrtCombineArgs& g, hipStream_t st) {
#define X(NN) \
  if (N == NN) return launch_crt_combine_n<NN>(g, st);
  BQ_CRT_CASES(X)
#undef X
  return hipErrorInvalidValue;
}

int crt_modulus(int i) { return (i >= 0 && i < kMaxCrtModuli) ? kCrtModuli[i] : 0; }

int64_t crt_combine_blocks(const CrtCombineArgs& c) {
  return (c.m * ((c.n + kGroupedCombineCols - 1) / kGroupedCombineCols) + 255) / 256;
}

hipError_t launch_crt_exp_grouped(const CrtSplitItem* items, const int64_t* prefix, int count, int64_t blocks,
                                  hipStream_t st) {
  if (count <= 0 || blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(crt_exp_grouped, dim3((unsigned)blocks), dim3(256), 0, st, items, prefix, count);
  return hipGetLastError();
}

template <int N>
static hipError_t launch_crt_split_grouped_n(const CrtSplitItem* items, const int64_t* prefix, int count,
                                             int64_t blocks, hipStream_t st) {
  hipLaunchKernelGGL((crt_split_grouped<N>), dim3((unsigned)blocks), dim3(256), 0, st, items, prefix, count);
  return hipGetLastError();
}

hipError_t launch_crt_split_grouped(int N, const CrtSplitItem* items, const int64_t* prefix, int count,
                                    int64_t blocks, hipStream_t st) {
  if (count <= 0 || blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
#define X(NN) \
  if (N == NN) return launch_crt_split_grouped_n<NN>(items, prefix, count, blocks, st);
  BQ_CRT_CASES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_crt_gemm_grouped(const CrtGemmItem* items, const int64_t* prefix, int count, int64_t blocks,
                                   hipStream_t st) {
  if (count <= 0 || blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(crt_gemm_grouped, dim3((unsigned)blocks), dim3(256), 0, st, items, prefix, count);
  return hipGetLastError();
}

template <int N>
static hipError_t launch_crt_combine_grouped_n(const CrtCombineArgs* items, const int64_t* prefix, int count,
                                               int64_t blocks, hipStream_t st) {
  static const CrtConsts k = make_crt_consts(N);
  hipLaunchKernelGGL((crt_combine_grouped<N>), dim3((unsigned)blocks), dim3(256), 0, st, items, prefix, count, k);
  return hipGetLastError();
}

hipError_t launch_crt_combine_grouped(int N, const CrtCombineArgs* items, const int64_t* prefix, int count,
                                      int64_t blocks, hipStream_t st) {
  if (count <= 0 || blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
#define X(NN) \
  if (N == NN) return launch_crt_combine_grouped_n<NN>(items, prefix, count, blocks, st);
  BQ_CRT_CASES(X)
#undef X
  return hipErrorInvalidValue;
}

}  // namespace bq
