// Split-precision real GEMM with OCP FP8 E4M3 digits on CDNA4's FP8 matrix
// rate (v_mfma_scale_f32_32x32x64_f8f6f4, unit scales).
//
// Digits: beta = 5 with one bit of exponent headroom (h = 1): the scaled
// element lies in (-1/2, 1/2), so every digit is an integer in [-16, 16],
// all exactly representable in E4M3 (four significant bits, 16 = 2^4).  S
// digits carry 5 S - 1 bits of a row's largest element.
//
// Block: a 64 x 64 output tile, 4 waves of 32 x 32 (one MFMA per slice pair
// and 64-deep k-step), one wave per SIMD.  Digits are in the tiled layout of
// 64-byte rows (digit_offset): the 64 rows x one k-step of a
// slice are 4 KB contiguous, already in LDS order, and move straight into LDS
// (buffer_load_dwordx4 ... lds, thread tid copying bytes 16 tid .. 16 tid +
// 15 of each tile).
//
// Per k-step every wave reads the B fragments of all S slices into registers
// (8 VGPRs each) and streams the A fragments one slice at a time; level d =
// s + t accumulates in FP32 (AGPRs) across k-steps while the sums stay exact
// integers and then goes to FP64 scaled by 2^-5d.  LDS: the B tiles of one
// k-step (S x 4 KB) and two stages of A tiles (2 x S x 4 KB): once every wave
// has its B fragments (after the MFMAs of the first A slice, which consume
// them all), the loads of the next k-step go out, B into the B tiles and A
// into the idle A stage, and have the rest of the k-step to land.
#include <limits.h>

#include "bq_split_common.h"

namespace bq {

namespace {

typedef int i8x __attribute__((ext_vector_type(8)));
typedef float f16x __attribute__((ext_vector_type(16)));

constexpr int kF8Beta = 5;
constexpr int kF8Head = 1;

// 2^-e for 0 <= e <= 126 (level scales reach 2^-70, beyond one 64-bit
// shift): two shifts of at most 63, no recursion, folded to a constant.
constexpr double pow2neg(int e) {
  return (1.0 / (double)(1ull << (e / 2))) * (1.0 / (double)(1ull << (e - e / 2)));
}

__device__ __forceinline__ f16x mfma_f8(i8x a, i8x b, f16x c) {
  // Formats 0, 0: both operands E4M3; scales 127 (E8M0 2^0): plain products.
  return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
}

// Output of one 32 x 32 wave tile at (r0, c0): exponent scaling, then
// coef * T into every target block.  D layout of the 32 x 32 MFMA shapes:
// lane l, element v holds row 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32.
__device__ __forceinline__ void store_tile_f8(const SliceGemmArgs& g, const double (&acc)[16], int64_t r0,
                                              int64_t c0, int lane) {
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int64_t r = r0 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    const int64_t c = c0 + (lane & 31);
    if (r >= g.m || c >= g.n) continue;
    const double t = exp_scaled(acc[v], g.ea[r], g.eb[c], 0);
    const int64_t off = r * g.ldc + c;
    for (int q = 0; q < g.ntgt; ++q) {
      double val = g.coef[q] * t;
      if (g.mode[q] == TGT_ACCUM) val += g.c[q][off];
      g.c[q][off] = val;
    }
  }
}

template <int S>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
slice_gemm_f8(const SliceGemmArgs g) {
  constexpr int BM = 64, BN = 64, ROWB = 64;
  constexpr int SLICE = BM * ROWB;         // 4 KB per slice tile
  constexpr int A_STAGE = S * SLICE;
  constexpr int B_OFF = 2 * A_STAGE;       // B tiles after the two A stages
  static_assert(3 * A_STAGE <= 160 * 1024, "two A stages and one B stage must fit LDS");
  __shared__ __attribute__((aligned(16))) unsigned char lds[3 * A_STAGE];

  const int tiles_m = (int)((g.m + BM - 1) / BM);
  const int tiles_n = (int)((g.n + BN - 1) / BN);
  int tm, tn;
  slice_tile_coords(tiles_m, tiles_n, tm, tn);
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm0 = (wave >> 1) * 32, wn0 = (wave & 1) * 32;
  const int fr = lane & 31, fh = lane >> 5;  // fragment row (column) and k half

  // One buffer resource per slice and block row (column) tile covering its
  // nk tiles, as in the other direct-to-LDS slice GEMMs.
  const int64_t nk = g.kp / 64;
  const unsigned char* ga = static_cast<const unsigned char*>(g.a) + (int64_t)tm * nk * SLICE;
  const unsigned char* gb = static_cast<const unsigned char*>(g.b) + (int64_t)tn * nk * SLICE;
  const int64_t sa = g.slice_stride_a, sb = g.slice_stride_b;
  const int nrec = (int)(uint32_t)(nk * SLICE);
  const int voff = tid * 16;
  const int wave_lds = wave * 64 * 16;
  auto dma = [&](const unsigned char* base, int64_t kt, unsigned char* dst) {
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, nrec, 0x00020000);
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_void_ptr)(dst + wave_lds), 16, voff, (int)(kt * SLICE), 0, 0);
  };
  auto load_step = [&](int64_t kt, int astage) {
#pragma unroll
    for (int s = 0; s < S; ++s) dma(gb + s * sb, kt, lds + B_OFF + s * SLICE);
#pragma unroll
    for (int s = 0; s < S; ++s) dma(ga + s * sa, kt, lds + astage * A_STAGE + s * SLICE);
  };
  // Fragment of a 32-row (column) strip: lane l takes row row0 + l % 32,
  // bytes 32 (l / 32) .. + 31 of its 64-byte row (chunks 2 fh, 2 fh + 1 at
  // their swizzled positions).  A and B use the same k order, so the MFMA
  // pairs byte j of A's lane with byte j of B's: the dot product is exact
  // whatever order the hardware assigns to k inside a lane.
  auto frag = [&](const unsigned char* tile, int row0) {
    const int row = row0 + fr;
    const unsigned char* p = tile + row * ROWB;
    const i4v lo = *reinterpret_cast<const i4v*>(p + swz_chunk<16>(row, 2 * fh) * 16);
    const i4v hi = *reinterpret_cast<const i4v*>(p + swz_chunk<16>(row, 2 * fh + 1) * 16);
    return i8x{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
  };

  double acc[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.0;

  load_step(0, 0);
  wait_vm<0>();
  block_sync();
  int64_t kt = 0;
  for (int64_t k0 = 0; k0 < nk; k0 += g.kflush) {
    const int64_t k1 = min(nk, k0 + (int64_t)g.kflush);
    f16x lvl[S];
#pragma unroll
    for (int d = 0; d < S; ++d)
#pragma unroll
      for (int v = 0; v < 16; ++v) lvl[d][v] = 0.f;
    for (kt = k0; kt < k1; ++kt) {
      const int st = (int)(kt & 1);
      const unsigned char* ta = lds + st * A_STAGE;
      const unsigned char* tb = lds + B_OFF;
      i8x fb[S];
#pragma unroll
      for (int t = 0; t < S; ++t) fb[t] = frag(tb + t * SLICE, wn0);
      i8x fa = frag(ta, wm0);
      i8x fa_next = S > 1 ? frag(ta + SLICE, wm0) : fa;
      // First A slice: pairs (1, t) for every t, levels 2 .. S + 1.  They
      // read every B fragment, so afterwards the B tiles are free.
#pragma unroll
      for (int t = 1; t <= S; ++t) lvl[t - 1] = mfma_f8(fa, fb[t - 1], lvl[t - 1]);
      // Every wave holds its B fragments (lgkmcnt(0)): the next k-step's
      // tiles go to the B tiles and the other A stage, which every wave
      // finished reading before the barrier that closed the last k-step.
      // (The last k-step reloads its own tiles into the B tiles, which every
      // wave has read, and the idle A stage: no branch, so the MFMAs above
      // stay ahead of the barrier.)
      __builtin_amdgcn_sched_barrier(0);
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
      block_sync();
      load_step(kt + 1 < nk ? kt + 1 : kt, st ^ 1);
#pragma unroll
      for (int s = 2; s <= S; ++s) {
        fa = fa_next;
        if (s < S) fa_next = frag(ta + s * SLICE, wm0);
#pragma unroll
        for (int t = 1; t <= S + 1 - s; ++t) lvl[s + t - 2] = mfma_f8(fa, fb[t - 1], lvl[s + t - 2]);
      }
      // The next k-step's tiles have landed (this wave's loads, then every
      // wave's at the barrier), and every wave is done with this A stage.
      wait_vm<0>();
      block_sync();
    }
#pragma unroll
    for (int d = 2; d <= S + 1; ++d) {
      constexpr int kMaxLevel = S + 1;
      static_assert(kF8Beta * kMaxLevel <= 126, "level scale range");
      const double sc = pow2neg(kF8Beta * d);
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[v] = __builtin_fma((double)lvl[d - 2][v], sc, acc[v]);
    }
  }

  store_tile_f8(g, acc, m0 + wm0, n0 + wn0, lane);
}

}  // namespace

int f8_beta() { return kF8Beta; }
int f8_head() { return kF8Head; }

template <int S>
static hipError_t launch_f8_s(const SliceGemmArgs& g, hipStream_t st) {
  const int64_t tiles = ((g.m + 63) / 64) * ((g.n + 63) / 64);
  if (tiles <= 0) return hipSuccess;
  if (tiles > 0x7fffffff || g.kflush < 1 || g.kp % 64 != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL((slice_gemm_f8<S>), dim3((unsigned)tiles), dim3(256), 0, st, g);
  return hipGetLastError();
}

hipError_t launch_slice_gemm_f8(int S, const SliceGemmArgs& g, hipStream_t st) {
  switch (S) {
    case 1: return launch_f8_s<1>(g, st);
    case 2: return launch_f8_s<2>(g, st);
    case 3: return launch_f8_s<3>(g, st);
    case 4: return launch_f8_s<4>(g, st);
    case 5: return launch_f8_s<5>(g, st);
    case 6: return launch_f8_s<6>(g, st);
    case 7: return launch_f8_s<7>(g, st);
    case 8: return launch_f8_s<8>(g, st);
    case 9: return launch_f8_s<9>(g, st);
    case 10: return launch_f8_s<10>(g, st);
    case 11: return launch_f8_s<11>(g, st);
    case 12: return launch_f8_s<12>(g, st);
    case 13: return launch_f8_s<13>(g, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace bq
