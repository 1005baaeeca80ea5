// Internal interfaces between the host engine (bq_engine.cpp) and the
// gfx950 kernels (bq_kernels.hip).  Not part of the public C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bq {

// Which real products one complex product L.R needs (Sec. III A).
//   GAUSS: L = lr + i sL li, R = rr + i sR ri.  Three products
//          T1 = lr rr, T2 = li ri, T3 = (lr + sL li)(rr + sR ri)
//          give P_R = T1 - sL sR T2 and P_I = T3 - T1 - sL sR T2
//          (eq. cmplx-3-real-mult with the conjugation signs folded in).
//   RC:    L real, R complex:  P_R = lr rr, P_I = sR lr ri.
//   CR:    L complex, R real:  P_R = lr rr, P_I = sL li rr.
//   RR:    both real:          P_R = lr rr, P_I = 0.
enum Kind : int { KIND_GAUSS = 0, KIND_RC = 1, KIND_CR = 2, KIND_RR = 3 };

enum TargetMode : int { TGT_SKIP = 0, TGT_WRITE = 1, TGT_ACCUM = 2 };

// One output quaternion unit w receives coef * P:
//   C_w     (=cr)  op=  ar * P_R - ai * P_I
//   C_{w+4} (=ci)  op=  ar * P_I + ai * P_R
struct Target {
  double* cr;
  double* ci;
  double ar, ai;
  int mode_r, mode_i;
};

constexpr int kMaxTargets = 4;

struct GemmArgs {
  const double* lr;
  const double* li;
  int64_t lda;
  const double* rr;
  const double* ri;
  int64_t ldb;
  int64_t m, n, k;
  double sL, sR;
  int ntgt;
  int vec;  // 1: lda, ldb even and operand bases 16-byte aligned
  Target tgt[kMaxTargets];
  int64_t ldc;
  int xcd_remap;  // 1: deal contiguous tile ranges to the 8 XCDs
  int group_m;    // tile-rows per group of the grouped tile order (>= 1)
};

// Linear combinations of quaternion components (the Hadamard rows of
// eq. bilinearH, with operand signs folded in):
//   dst_r[q] = sum_u w[q][u] src[u],  dst_i[q] = sum_u w[q][u] src[u + 4].
// src[c] == nullptr is a zero component; dst pointers may be nullptr (skip).
struct CombineArgs {
  const double* src[8];
  int64_t lds;
  double* dst_r[4];
  double* dst_i[4];
  int64_t ldd;
  double w[4][4];
  int nq;
  int pad_;
  int64_t rows, cols;
};

struct TileConfig {
  int bm, bn, bk, wm, wn;
};

// Launchers (bq_kernels.hip).  Return hipSuccess or the launch error.
hipError_t launch_cgemm(int kind, const GemmArgs& g, int cfg, hipStream_t s);
hipError_t launch_combine(const CombineArgs& a, hipStream_t s);
hipError_t launch_fill_zero(double* p, int64_t rows, int64_t cols, int64_t ld, hipStream_t s);
int num_tile_configs();
TileConfig tile_config(int cfg);
int default_tile_config(int kind, int64_t m, int64_t n, int64_t k);

}  // namespace bq
