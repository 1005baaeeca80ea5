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
//   C_w     (=cr)  op=  ar * P_R - ai * P_I  [+ sc * sr]
//   C_{w+4} (=ci)  op=  ar * P_I + ai * P_R  [+ sc * si]
// sr, si (may be null): an addend block pair with leading dimension
// GemmArgs::ldadd (the batched form's Hadamard sums, added by the direct
// products' epilogue so that C is written once and never read).
struct Target {
  double* cr;
  double* ci;
  double ar, ai;
  int mode_r, mode_i;
  const double* sr;
  const double* si;
  double sc;
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
  int ta, tb;     // 1: lr/li stored k x m (lda along m), rr/ri stored n x k (ldb along k)
  int64_t ldadd;  // leading dimension of the targets' addend blocks
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

// One real FP64 operand to be split into low-precision digit slices:
// value = w1 * s1 + w2 * s2 (s2 may be null), row-major with leading
// dimension ld.  left: the operand is the left factor (m x k, one exponent
// per row, digits D[s][row][kk]); otherwise the right factor (k x n, one
// exponent per column, digits stored transposed, D[s][col][kk]).
struct SplitArgs {
  const double* s1;
  const double* s2;
  double w1, w2;
  int64_t ld;
  int64_t rows, cols;          // source shape
  int64_t rows_pad, cols_pad;  // left: rows padded to 128; right: cols padded to 64
  int64_t kp;                  // reduced dimension padded to 64 (zero digits)
  int64_t slice_stride;        // elements between consecutive slices
  int beta;                    // digit width in bits
  int head;                    // exponent headroom: row/column exponent = frexp exponent + head
  int left;
};

constexpr int kMaxSliceTargets = 8;

// T = X Y from digit slices; coef[q] * T is stored (TGT_WRITE) or added
// (TGT_ACCUM) into c[q] (m x n, leading dimension ldc).
struct SliceGemmArgs {
  const void* a;  // left digits  [S][rows_pad][kp]
  const void* b;  // right digits [S][cols_pad][kp]
  int64_t slice_stride_a, slice_stride_b, kp;
  const int* ea;  // row exponents of the left operand
  const int* eb;  // column exponents of the right operand
  int64_t m, n;
  int beta;
  int kflush;  // k-steps whose level sums stay exact before they go to FP64
  int ntgt;
  double* c[kMaxSliceTargets];
  double coef[kMaxSliceTargets];
  int mode[kMaxSliceTargets];
  int64_t ldc;
};

// Work item of the batched form: tile (tm, tn) of one problem, whose complex
// products are prods[prod0 .. prod0 + nprod).
struct GroupedItem {
  int prod0;
  int nprod;
  int tm, tn;
};

// CRT-based split form (bq_crt.hip): residue planes and their GEMMs.
constexpr int kMaxCrtModuli = 20;
struct CrtGemmArgs {
  const void* a;  // residues of X: [N][rows_pad (256)][kp], tiled 64-byte layout
  const void* b;  // residues of Y: [N][cols_pad (256)][kp], same
  int64_t plane_a, plane_b;  // bytes between modulus planes
  int64_t kp;
  int64_t m, n;
  signed char* out;  // result residues [N][m][ldr], ldr a multiple of 16
  int64_t plane_r, ldr;
};
// Up to kCrtProducts real products T_p of one complex product (the Gauss
// form has three), each from its own residue planes and exponents; target q
// gets sum_p coef[q][p] T_p, written or added once.
constexpr int kCrtProducts = 3;
struct CrtCombineArgs {
  int np;
  const signed char* res[kCrtProducts];
  const int* ea[kCrtProducts];
  const int* eb[kCrtProducts];
  int64_t plane_r, ldr;
  int64_t m, n;
  int bits;
  int ntgt;
  double* c[kMaxSliceTargets];
  double coef[kMaxSliceTargets][kCrtProducts];
  int mode[kMaxSliceTargets];
  int64_t ldc;
  // Filled by the launcher: Chinese remainder constants of the N moduli.
  double cpart[kMaxCrtModuli][4];  // c_i modulo 2^128 as four 32-bit parts, low first
  double frac[kMaxCrtModuli];      // c_i / M
  double mpart[4];                 // M modulo 2^128, the same way
};

// Complex linear map of the 8 components into an R x R complex buffer
// (heev_map_kernel): quadrant q (R = 2n: 0..3 = 11, 12, 21, 22; R = n: 0).
struct HeevMapArgs {
  const double* src[8];
  int64_t lds;
  int64_t n, R;
  double wr[4][8], wi[4][8];
  double* out;  // interleaved complex, row-major, stored conjugated
  int64_t ldo;  // complex elements
};

// Eigenvector assembly (heev_assemble_kernel): lists 0 and 1 of the merge.
struct HeevAsmArgs {
  int64_t n;
  const double* xt[2];  // top-half source per list (column-major n x n complex) or null
  const double* xb[2];  // bottom-half source per list or null
  int64_t ldx;
  double ct[2][2], cb[2][2];  // complex coefficients (re, im)
  int conj_t[2], conj_b[2];
  int rows_t[2], rows_b[2];   // vector j is row j of the source (not column j)
  const int64_t* src;
  int rev2;
  double* V;
  int64_t ldv;
};

struct TileConfig {
  int bm, bn, bk, wm, wn;
};

// Device address and size of this device's static workspace of
// bq_gemm_noalloc (bq_noalloc.hip); looked up once per device.
hipError_t noalloc_scratch(int device, void** ptr, size_t* bytes);

// Launchers (bq_kernels.hip).  Return hipSuccess or the launch error.
hipError_t launch_cgemm(int kind, const GemmArgs& g, int cfg, hipStream_t s);
hipError_t launch_combine(const CombineArgs& a, hipStream_t s);
hipError_t launch_fill_zero(double* p, int64_t rows, int64_t cols, int64_t ld, hipStream_t s);
int num_tile_configs();
TileConfig tile_config(int cfg);
int default_tile_config(int kind, int64_t m, int64_t n, int64_t k);
// The configuration a single product runs: the request where it suits the
// kind (3 or 11 for real products; complex kinds always take 0), else the
// default.
int tile_config_for(int kind, int requested, int64_t m, int64_t n, int64_t k);
// Batched form (complex x complex products only).  cfg: 0 or 6 (tile
// configurations above); dyn: 1 = device work counter, 0 = cyclic; ops:
// 0..3 when every product has (ta, tb) = (ops >> 1, ops & 1) (one tile
// variant compiled in), -1 when they differ.
hipError_t launch_grouped(int cfg, int dyn, int ops, int buf, const GemmArgs* prods, const GroupedItem* items,
                          int nitems, int* counter, int blocks, hipStream_t s);
// Whether a batched product's operand tiles (tile configuration cfg, ops
// ta / tb) can be read through buffer resources (buf = 1 above).
bool grouped_spans_fit(int cfg, int ta, int tb, int64_t lda, int64_t ldb);
hipError_t launch_grouped_combine(const CombineArgs* args, const int64_t* row_prefix, int nargs, int64_t total_rows,
                                  hipStream_t s);
// Split-precision kernels (bq_split.hip, bq_split_f8.hip).  et: 0 = BF16
// digits (beta 7), 1 = OCP FP8 E4M3 digits (beta 5, headroom 1), 2 = INT8
// digits (beta 7, headroom 1).
hipError_t launch_split(int et, int S, const SplitArgs& a, int* exps, void* out, hipStream_t s);
// Row (a.left) or column exponents of a split operand into exps.
hipError_t launch_split_exponents(const SplitArgs& a, int* exps, hipStream_t s);
hipError_t launch_slice_gemm(int et, int S, const SliceGemmArgs& g, hipStream_t s);
// FP8 digits (bq_split_f8.hip): beta 5, headroom 1, 1..13 slices.
hipError_t launch_slice_gemm_f8(int S, const SliceGemmArgs& g, hipStream_t s);
int f8_beta();
int f8_head();
int max_slices(int et);
int slice_block_rows(int et, int S);  // rows of a slice-GEMM block tile (128 or 64)
int slice_kstep(int et);              // k per MFMA step (32 or 64)
int slice_beta(int et);
int slice_head(int et);
int slice_flush_steps(int et, int S);  // k-steps per exact level accumulation
hipError_t launch_crt_split(int N, const SplitArgs& a, int* exps, void* out, hipStream_t s);  // a.beta = bits
hipError_t launch_crt_gemm(int N, const CrtGemmArgs& g, hipStream_t s);
hipError_t launch_crt_combine(int N, const CrtCombineArgs& g, hipStream_t s);
int crt_modulus(int i);

// Grouped CRT launches (batched plans): every launch covers a list of items
// of many problems; item i owns blocks [prefix[i], prefix[i + 1]) of a 1-D
// grid, and a block finds its item by binary search in prefix.
//   exponents: one operand per item (CrtSplitItem), crt_exp_blocks blocks;
//   residues:  the same items, crt_split_blocks blocks (all items one N);
//   GEMM:      one real product per item, 128 x 128 tiles x moduli;
//   combine:   one complex product per item (all items one N).
struct CrtSplitItem {
  SplitArgs a;
  int* exps;
  void* out;
};
struct CrtGemmItem {
  CrtGemmArgs g;
  int nmod;
};
inline int64_t crt_exp_blocks(const SplitArgs& a) { return a.left ? a.rows : (a.cols + 63) / 64; }
// Residues of the rows (columns) an operand has; the padding rows (columns)
// only feed GEMM results that are never stored.
inline int64_t crt_split_blocks(const SplitArgs& a) {
  return a.left ? (a.rows * (a.kp / 2) + 255) / 256 : ((a.cols + 63) / 64) * (a.kp / 64);
}
inline int64_t crt_gemm_blocks(const CrtGemmItem& it) {
  return ((it.g.m + 127) / 128) * ((it.g.n + 127) / 128) * it.nmod;
}
int64_t crt_combine_blocks(const CrtCombineArgs& c);
hipError_t launch_crt_exp_grouped(const CrtSplitItem* items, const int64_t* prefix, int count, int64_t blocks,
                                  hipStream_t s);
hipError_t launch_crt_split_grouped(int N, const CrtSplitItem* items, const int64_t* prefix, int count,
                                    int64_t blocks, hipStream_t s);
hipError_t launch_crt_gemm_grouped(const CrtGemmItem* items, const int64_t* prefix, int count, int64_t blocks,
                                   hipStream_t s);
hipError_t launch_crt_combine_grouped(int N, const CrtCombineArgs* items, const int64_t* prefix, int count,
                                      int64_t blocks, hipStream_t s);
// Hermitian eigenproblem kernels (bq_heev.hip).
hipError_t launch_heev_map(const HeevMapArgs& a, hipStream_t s);
hipError_t launch_heev_merge(const double* x1, int64_t n1, double s1, const double* x2, int64_t n2, double s2, int rev,
                             double* w, int64_t* src, hipStream_t s);
hipError_t launch_heev_assemble(const HeevAsmArgs& a, hipStream_t s);
hipError_t launch_heev_info(const int* a, const int* b, int* out, hipStream_t s);

}  // namespace bq
