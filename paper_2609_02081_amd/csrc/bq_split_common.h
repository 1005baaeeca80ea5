// Device helpers shared by the split-form kernels (bq_split.hip, bq_crt.hip):
// vector types, the split operand, the tiled digit layout, the XCD-aware
// tile order and the explicit wait / barrier primitives of the pipelined
// kernels.
#pragma once

#include <limits.h>

#include "bq_internal.h"

namespace bq {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4s __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i4v __attribute__((ext_vector_type(4)));
typedef int i2v __attribute__((ext_vector_type(2)));

// Value of the split operand: w1 * s1 + w2 * s2 (s2 may be absent).  The
// FP64 path forms its Gauss sums with the same single rounding.
__device__ __forceinline__ double operand_value(const SplitArgs& a, int64_t off) {
  const double x = a.s1[off];
  return a.s2 ? __builtin_fma(a.w2, a.s2[off], a.w1 * x) : a.w1 * x;
}

// Row / column exponent markers: INT_MIN for an all-zero row or column (its
// digits are zero and so is its part of the product), kExpNonFinite for one
// holding a NaN or an infinity (it wins every max; its digits are zero and
// its part of the product is NaN, as in the FP64 path).
constexpr int kExpNonFinite = INT_MAX;

__device__ __forceinline__ bool exp_special(int e) { return e == INT_MIN || e == kExpNonFinite; }

__device__ __forceinline__ int exp_of(double x) {
  if (!__builtin_isfinite(x)) return kExpNonFinite;
  int e;
  (void)frexp(x, &e);
  return x == 0.0 ? INT_MIN : e;
}

// Scale of a product element with row exponent ea and column exponent eb.
__device__ __forceinline__ double exp_scaled(double v, int ea, int eb, int shift) {
  if (ea == kExpNonFinite || eb == kExpNonFinite) return __builtin_nan("");
  if (ea == INT_MIN || eb == INT_MIN) return 0.0;
  return ldexp(v, ea + eb + shift);
}

// Chunk position of logical chunk ch in tile row r (rows of 4 chunks).
// 16-byte chunks (rows of 64 bytes): a 16-byte LDS access is served 8 lanes
// at a time over 32 banks (128 bytes); a fragment read has 8 lanes on 8
// consecutive rows at one logical chunk, and rows 2j, 2j + 1 share a
// 128-byte bank line offset by 64 bytes, so even rows must take 4 distinct
// positions, and odd rows too: position = ch ^ f(r) with f built from row
// bits 1..3.  8-byte chunks (rows of 32 bytes): 16 lanes per access on 16
// consecutive rows; rows r and r + 4 share banks, so f = bits 2..3.
template <int CH>
__device__ __forceinline__ int swz_chunk(int r, int ch) {
  if constexpr (CH == 16) return ch ^ ((((r >> 1) ^ (r >> 3)) & 1) | ((r >> 1) & 2));
  else return ch ^ ((r >> 2) & 3);
}

// Tiled digit layout (direct-to-LDS slice and residue GEMMs): within one
// slice, the 64 rows x one k-step (64 bytes per row) of row tile rt, k-step
// kt form one 4 KB block at (rt * nk + kt) * 4096, stored in the LDS order
// (row r at r * 64, logical 16-byte chunk ch at the swizzled position), so
// that a straight copy lands the tile ready for fragment reads.  Byte
// offset of the digit at (row r, byte b of the row) in one slice whose rows
// hold row_bytes.
__device__ __forceinline__ int64_t digit_offset(int64_t r, int64_t byte_in_row, int64_t row_bytes) {
  constexpr int RB = 64;
  const int64_t nk = row_bytes / RB, kt = byte_in_row / RB;
  const int rr = (int)(r & 63), b = (int)(byte_in_row % RB);
  return ((r >> 6) * nk + kt) * (64 * RB) + rr * RB + swz_chunk<16>(rr, b >> 4) * 16 + (b & 15);
}

// Block -> output tile, XCD-aware and grouped by 8 tile rows (as in the
// FP64 GEMM): consecutive block ids land on different XCDs, so each XCD
// gets a contiguous run of tiles.
__device__ __forceinline__ void slice_tile_coords(int tiles_m, int tiles_n, int& tm, int& tn) {
  const int T = tiles_m * tiles_n, w = blockIdx.x;
  const int x = w % 8, slot = w / 8, base = T / 8, rem = T % 8;
  const int t = x * base + (x < rem ? x : rem) + slot;
  const int per_group = 8 * tiles_n, group = t / per_group, first_m = group * 8;
  const int gm = min(tiles_m - first_m, 8), in_g = t - group * per_group;
  tm = first_m + in_g % gm;
  tn = in_g / gm;
}

// LDS destination of the direct global -> LDS buffer loads.
typedef __attribute__((address_space(3))) void* lds_void_ptr;

// Workgroup barrier without the memory fence of __syncthreads (which would
// wait for every load in flight, prefetches included): the kernels order
// their LDS traffic themselves (wait_vm before, fragment reads consumed
// before the barrier).
__device__ __forceinline__ void block_sync() {
  __builtin_amdgcn_sched_barrier(0);
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_sched_barrier(0);
}

// s_waitcnt vmcnt(N): wait until at most N vector-memory loads are pending.
#define BQ_WAIT_VM_CASE(K) \
  else if constexpr (N == K) asm volatile("s_waitcnt vmcnt(" #K ")" ::: "memory");
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N <= 31, "vmcnt range used here");
  if constexpr (N == 0) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  BQ_WAIT_VM_CASE(1) BQ_WAIT_VM_CASE(2) BQ_WAIT_VM_CASE(3) BQ_WAIT_VM_CASE(4) BQ_WAIT_VM_CASE(5)
  BQ_WAIT_VM_CASE(6) BQ_WAIT_VM_CASE(7) BQ_WAIT_VM_CASE(8) BQ_WAIT_VM_CASE(9) BQ_WAIT_VM_CASE(10)
  BQ_WAIT_VM_CASE(11) BQ_WAIT_VM_CASE(12) BQ_WAIT_VM_CASE(13) BQ_WAIT_VM_CASE(14) BQ_WAIT_VM_CASE(15)
  BQ_WAIT_VM_CASE(16) BQ_WAIT_VM_CASE(17) BQ_WAIT_VM_CASE(18) BQ_WAIT_VM_CASE(19) BQ_WAIT_VM_CASE(20)
  BQ_WAIT_VM_CASE(21) BQ_WAIT_VM_CASE(22) BQ_WAIT_VM_CASE(23) BQ_WAIT_VM_CASE(24) BQ_WAIT_VM_CASE(25)
  BQ_WAIT_VM_CASE(26) BQ_WAIT_VM_CASE(27) BQ_WAIT_VM_CASE(28) BQ_WAIT_VM_CASE(29) BQ_WAIT_VM_CASE(30)
  BQ_WAIT_VM_CASE(31)
}
#undef BQ_WAIT_VM_CASE

}  // namespace bq
