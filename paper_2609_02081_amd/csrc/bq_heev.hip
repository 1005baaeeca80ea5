// Kernels of the Hermitian biquaternion eigenproblem (gfx950): the complex
// isomorph of eq. mapping-formulas (or one of its blocks, for the reduced
// problems of the Hadamard transformation for diagonalization), the merge of
// two ascending eigenvalue lists, and the eigenvector assembly.  The
// eigensolves and singular value decompositions themselves are rocSOLVER
// calls made by the engine.
#include "bq_internal.h"

namespace bq {

// out (R x R complex, interleaved re/im doubles, row-major with leading
// dimension ldo complex elements): quadrant q = (row / n) * 2 + col / n of
// size n holds sum_c wr[q][c] M_c + i sum_c wi[q][c] M_c, stored
// conjugated.  The map of a Hermitian A is Hermitian, so the conjugated
// row-major buffer read column-major (as the eigensolver reads it) is the
// map itself.  One thread per element; consecutive threads walk a row.
__global__ void __launch_bounds__(256) heev_map_kernel(const HeevMapArgs a) {
  const int64_t bpr = (a.R + 255) / 256;
  const int64_t r = blockIdx.x / bpr;
  const int64_t c = (blockIdx.x % bpr) * 256 + threadIdx.x;
  if (r >= a.R || c >= a.R) return;
  const int qr = r >= a.n, qc = c >= a.n;
  const int q = qr * 2 + qc;
  const int64_t off = (r - qr * a.n) * a.lds + (c - qc * a.n);
  double re = 0.0, im = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const double* s = a.src[k];
    if (!s) continue;
    const double wr = a.wr[q][k], wi = a.wi[q][k];
    if (wr == 0.0 && wi == 0.0) continue;
    const double x = s[off];
    re = __builtin_fma(wr, x, re);
    im = __builtin_fma(wi, x, im);
  }
  double* o = a.out + 2 * (r * a.ldo + c);
  o[0] = re;
  o[1] = -im;
}

// Ascending merge of list 1 (y1[i] = s1 * x1[i], ascending) and list 2
// (y2[j] = s2 * x2[rev ? n2 - 1 - j : j], ascending).  Element i of list 1
// goes to rank i + #{j : y2[j] < y1[i]}, element j of list 2 to
// j + #{i : y1[i] <= y2[j]}: every rank is taken once, ties keep list 1
// first.  src[rank] = i (list 1) or n1 + j (list 2).
__device__ __forceinline__ int64_t count_less(const double* x, int64_t n, double s, int rev, double v, bool or_equal) {
  int64_t lo = 0, hi = n;  // first index whose value is > v (or >= v)
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    const double y = s * x[rev ? n - 1 - mid : mid];
    if (or_equal ? (y <= v) : (y < v)) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__global__ void __launch_bounds__(256) heev_merge_kernel(const double* x1, int64_t n1, double s1, const double* x2,
                                                         int64_t n2, double s2, int rev, double* w, int64_t* src) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < n1) {
    const double v = s1 * x1[t];
    const int64_t rank = t + count_less(x2, n2, s2, rev, v, false);
    w[rank] = v;
    if (src) src[rank] = t;
  } else if (t < n1 + n2) {
    const int64_t j = t - n1;
    const double v = s2 * x2[rev ? n2 - 1 - j : j];
    const int64_t rank = j + count_less(x1, n1, s1, 0, v, true);
    w[rank] = v;
    if (src) src[rank] = t;
  }
}

// V (2n x 2n complex, column-major, leading dimension ldv): column o takes
// list l = (src[o] >= n) and its index; list 2 indexes run reversed when
// rev2.  Rows 0..n-1 are ct[l] * (conj_t[l] ? conj : id)(xt[l][:, col]),
// or of row col of xt[l] when rows_t[l]; rows n..2n-1 likewise from xb[l];
// a null matrix gives zeros.  X matrices are the solver's: column-major
// n x n complex, leading dimension ldx.
__global__ void __launch_bounds__(256) heev_assemble_kernel(const HeevAsmArgs a) {
  const int64_t N = 2 * a.n;
  const int64_t bpc = (N + 255) / 256;
  const int64_t o = blockIdx.x / bpc;
  const int64_t r = (blockIdx.x % bpc) * 256 + threadIdx.x;
  if (o >= N || r >= N) return;
  const int64_t s = a.src[o];
  const int l = s >= a.n;
  int64_t col = s - l * a.n;
  if (l == 1 && a.rev2) col = a.n - 1 - col;
  const bool top = r < a.n;
  const int64_t rr = top ? r : r - a.n;
  const double* X = top ? a.xt[l] : a.xb[l];
  double re = 0.0, im = 0.0;
  if (X) {
    const int by_rows = top ? a.rows_t[l] : a.rows_b[l];
    const double* x = X + 2 * (by_rows ? rr * a.ldx + col : col * a.ldx + rr);
    const double xr = x[0];
    const double xi = (top ? a.conj_t[l] : a.conj_b[l]) ? -x[1] : x[1];
    const double cr = top ? a.ct[l][0] : a.cb[l][0];
    const double ci = top ? a.ct[l][1] : a.cb[l][1];
    re = cr * xr - ci * xi;
    im = cr * xi + ci * xr;
  }
  double* v = a.V + 2 * (o * a.ldv + r);
  v[0] = re;
  v[1] = im;
}

__global__ void heev_info_kernel(const int* a, const int* b, int* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int x = a ? a[0] : 0;
    if (b) x = max(x, b[0]);
    out[0] = x;
  }
}

hipError_t launch_heev_map(const HeevMapArgs& a, hipStream_t s) {
  if (a.R <= 0) return hipSuccess;
  const int64_t blocks = a.R * ((a.R + 255) / 256);
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(heev_map_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_heev_merge(const double* x1, int64_t n1, double s1, const double* x2, int64_t n2, double s2, int rev,
                             double* w, int64_t* src, hipStream_t s) {
  const int64_t total = n1 + n2;
  if (total <= 0) return hipSuccess;
  const int64_t blocks = (total + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(heev_merge_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x1, n1, s1, x2, n2, s2, rev, w,
                     src);
  return hipGetLastError();
}

hipError_t launch_heev_assemble(const HeevAsmArgs& a, hipStream_t s) {
  const int64_t N = 2 * a.n;
  if (N <= 0) return hipSuccess;
  const int64_t blocks = N * ((N + 255) / 256);
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(heev_assemble_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_heev_info(const int* a, const int* b, int* out, hipStream_t s) {
  hipLaunchKernelGGL(heev_info_kernel, dim3(1), dim3(64), 0, s, a, b, out);
  return hipGetLastError();
}

}  // namespace bq
