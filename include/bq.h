/*
 * bq.h -- C-ABI of the MI355X (gfx950) bilinear biquaternion GEMM library.
 *
 * Operation (paper Sec. II A, eq. MatrixQMultiplication; Sec. III A,
 * eq. bilinearH with eq. cmplx-3-real-mult): C = op(A) . op(B) for
 * matrix-valued biquaternions A in H_C^{m x k}, B in H_C^{k x n}, computed by
 * the bilinear scheme (8 complex products formed with Gauss's three real
 * products each: 24 real GEMMs for full biquaternions) or, when the active
 * components make it cheaper (Sec. III A, last paragraph), by the
 * component-wise form with absent terms omitted.
 *
 * Layout (Sec. III, eqs. biquat-repres and main-biquat-eqn): a biquaternion
 * matrix is eight real FP64 blocks
 *     comp[0..7] = [M1..M8] = [E_R, E_I, F_R, F_I, G_I, -G_R, H_I, -H_R]
 * so the coefficient of unit 1 is comp[0] + i comp[4], of i comp[1] + i comp[5],
 * of j comp[2] + i comp[6], of k comp[3] + i comp[7].  Every block is
 * row-major with the same leading dimension ld (elements, ld >= cols) and
 * lives in device memory of the handle's GPU.  All offsets are 64-bit.
 *
 * Ownership: the caller owns A, B, C and any workspace; they must stay valid
 * until the work enqueued on the stream has finished.  The library keeps no
 * pointer after a call returns.
 *
 * Errors: every argument check is synchronous host code and runs before
 * anything is enqueued; on any error nothing is enqueued and C is untouched.
 * Faults inside kernels surface at the caller's next stream synchronisation.
 * Calls are asynchronous with respect to the host.
 *
 * Threading: a handle is not thread-safe; use one handle per host thread.
 */
#ifndef BQ_H
#define BQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The enumerations below travel as 32-bit integers.  C++ gives them int as
 * their fixed underlying type, so any integer a C caller passes is a value
 * the library can read and reject (BQ_ERR_INVALID_VALUE) rather than an
 * out-of-range enumeration value. */
#ifdef __cplusplus
#define BQ_ENUM(tag) enum tag : int
#else
#define BQ_ENUM(tag) enum tag
#endif

typedef BQ_ENUM(bq_status_e) {
  BQ_OK = 0,
  BQ_ERR_INVALID_VALUE = 1, /* null/negative/mismatched argument            */
  BQ_ERR_UNSUPPORTED = 2,   /* valid request the library does not implement */
  BQ_ERR_ALIAS = 3,         /* C overlaps A, B, the workspace or itself, or
                               the workspace overlaps A or B                 */
  BQ_ERR_WORKSPACE = 4,     /* workspace smaller than the minimum plan       */
  BQ_ERR_HIP = 5,           /* a HIP runtime call failed                     */
  BQ_ERR_ARCH = 6           /* device is not gfx950                          */
} bq_status_t;

/* op(X): N = as stored, T = biquaternion transpose, C = complex conjugate,
 * H = Hermitian conjugate (Sec. III, sign rules for T, *, dagger).
 * For T and H the stored matrix is the transpose: op(A) is m x k when A is
 * stored k x m (A.rows = k, A.cols = m), op(B) is k x n when B is stored
 * n x k.  T and H read the transposed tiles straight from the stored layout
 * (no copy); the sign rules are folded into the pre-combination and the
 * combination weights. */
typedef BQ_ENUM(bq_op_e) { BQ_OP_N = 0, BQ_OP_T = 1, BQ_OP_C = 2, BQ_OP_H = 3 } bq_op_t;

/* Arithmetic of the real GEMMs.  FP64: FP64 MFMA.  The split forms (an
 * Ozaki-style scheme; the paper itself uses FP64 throughout, Sec. III A)
 * write every FP64 operand as `slices` signed integer digits of beta bits
 * under a power-of-two exponent per row (left operand) or column (right
 * operand), multiply digit slices on low-precision MFMA with exact FP32
 * (BF16, FP8) or int32 (INT8) sums, keep the slice pairs with s + t <=
 * slices + 1, and accumulate and rescale in FP64.  Digit types: BF16
 * (beta 7, slices 1..8), OCP FP8 E4M3 (beta 5 with one bit of exponent
 * headroom h, so every digit lies in [-16, 16], exact in E4M3; slices
 * 1..13), INT8 (beta 7 with h = 1, so the leading digit fits a signed byte;
 * slices 1..9).  S digits carry beta S - h significand bits of a row's
 * (column's) largest element; slices = 0 picks the fewest slices that carry
 * 48 + ceil(log2(k) / 2) bits for the call's k (the truncation of a
 * length-k dot product grows like sqrt(k)), capped at the maximum: at
 * k = 16384 BF16 8, FP8 12, INT8 8 slices.
 * SPLIT_INT8_CRT is the integer-modular form (Ozaki scheme II): every row of
 * the left factor (column of the right) is scaled by a power of two to b-bit
 * integers (b <= 53, one rounding per element), the exact integer product is
 * carried as `slices` residues modulo the fixed odd pairwise coprime moduli
 * 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 211, 199, 197, 193, 191,
 * 181, 179, 173, 167, 163 (first `slices` of them), one exact INT8 GEMM with
 * int32 sums per modulus, and recovered by the Chinese remainder theorem in
 * mixed radix with an FP64 evaluation.  b is the largest value <= 53 with
 * p_1 ... p_N > 2 k 2^(2b); slices 1..20, 0 = the fewest moduli that give
 * b = 53 for the call's k (16 at k = 16384), and an explicit count that gives
 * b = 0 is BQ_ERR_INVALID_VALUE.  k is limited to 133120 (int32 sums stay
 * exact).  The Hadamard and Gauss pre-combinations and the post-combination
 * stay FP64. */
typedef BQ_ENUM(bq_prec_e) {
  BQ_PREC_FP64 = 0,
  BQ_PREC_SPLIT_BF16 = 1,
  BQ_PREC_SPLIT_FP8 = 2,
  BQ_PREC_SPLIT_INT8 = 3,
  BQ_PREC_SPLIT_INT8_CRT = 4
} bq_prec_t;

typedef struct bq_handle_s* bq_handle_t;
typedef void* bq_stream_t; /* a hipStream_t; NULL = the null stream */

/* One matrix-valued biquaternion.  For an input, comp[c] == NULL means the
 * component is identically zero (an "absent" component).  For an output of
 * bq_gemm all eight pointers are required. */
typedef struct {
  double* comp[8];
  int64_t rows;
  int64_t cols;
  int64_t ld;
} bq_matrix_t;

/* Component masks: bit c set <=> comp[c] active. */
#define BQ_MASK_FULL 0xFFu
#define BQ_MASK_REAL_QUATERNION 0x0Fu
#define BQ_MASK_COMPLEX 0x11u
#define BQ_MASK_REAL 0x01u

/* Create a handle bound to HIP device `device` (BQ_ERR_ARCH if it is not
 * gfx950, BQ_ERR_HIP if the runtime call fails).  *h receives the handle. */
bq_status_t bq_create(bq_handle_t* h, int device);
bq_status_t bq_destroy(bq_handle_t h);

/* Static text for a status code (never NULL). */
const char* bq_status_string(bq_status_t s);
/* Text of the last failure detected by this host thread (never NULL).  It
 * takes no handle: failures are detected before a handle exists (bq_create)
 * and by the handle-free calls (bq_gemm_check, bq_gemm_workspace_size), and
 * a handle serves one host thread anyway, so the text is kept per thread. */
const char* bq_last_error_detail(void);

/* Workspace for bq_gemm.  *resident_bytes lets every pre-combined operand
 * stay in memory at once; *min_bytes is the least the streamed plan needs
 * (pre-combinations formed one product at a time).  Either output pointer
 * may be NULL.  maskA/maskB as in BQ_MASK_*.  m, n, k are the shapes of
 * op(A) (m x k) and op(B) (k x n); the sizes hold for every op.  The sizes
 * depend on the shapes, masks and precision only (not on the device), so
 * the query takes no handle and a caller can size memory before creating
 * one. */
bq_status_t bq_gemm_workspace_size(int64_t m, int64_t n, int64_t k,
                                   unsigned maskA, unsigned maskB,
                                   bq_prec_t prec, int slices,
                                   size_t* resident_bytes, size_t* min_bytes);

/* Host-only validation of a bq_gemm call (no HIP call is made): returns what
 * bq_gemm would return for these arguments before enqueueing anything.
 * With BQ_LOG=1 in the environment, every validated call (this one and
 * bq_gemm) prints its plan on stderr: shape, ops, masks, bilinear or
 * component-wise form, real GEMMs, precision, slices, resident or streamed
 * workspace. */
bq_status_t bq_gemm_check(bq_op_t opA, bq_op_t opB, const bq_matrix_t* A,
                          const bq_matrix_t* B, const bq_matrix_t* C,
                          bq_prec_t prec, int slices, const void* ws,
                          size_t ws_bytes);

/* C <- op(A) op(B), C is m x n, op(A) m x k, op(B) k x n.
 * ws: device workspace (may be NULL when bq_gemm_workspace_size gives 0);
 * with ws_bytes >= resident size the resident plan runs, otherwise with
 * ws_bytes >= min size the streamed plan, otherwise BQ_ERR_WORKSPACE.
 * m == 0 or n == 0: no-op.  k == 0: C = 0.  Each of m, n, k must be below
 * 2^31 and each of op(A), op(B), C at most 2^40 elements, every ld at most
 * 2^24 (BQ_ERR_UNSUPPORTED otherwise).
 * Components of C that are structurally zero for the given input masks are
 * written as 0.  `slices` is used by the split forms (0 = default). */
bq_status_t bq_gemm(bq_handle_t h, bq_op_t opA, bq_op_t opB,
                    const bq_matrix_t* A, const bq_matrix_t* B, bq_matrix_t* C,
                    bq_prec_t prec, int slices, void* ws, size_t ws_bytes,
                    bq_stream_t stream);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  bq_gemm
 * with the workspace taken from a static device array of
 * BQ_NOALLOC_SCRATCH_BYTES bytes that the library holds on each GPU it runs
 * on until the process ends (its address is looked up once per device by
 * bq_create); the call allocates nothing.  The resident plan runs when its
 * workspace fits the array, else the streamed one; a product that needs
 * more than the array returns BQ_ERR_WORKSPACE (nothing enqueued).  Square
 * FP64 biquaternion products fit up to n = 1448 resident, n = 2896
 * streamed.  Every call on a GPU shares that GPU's array: calls that
 * overlap on one GPU (other streams, threads or handles) race, so the
 * caller serialises them.  No part of the array has to start at zero (every
 * kernel writes what it later reads), so nothing is cleared between calls.
 * Other arguments, conventions and errors as for bq_gemm. */
#define BQ_NOALLOC_SCRATCH_BYTES (256u << 20)
bq_status_t bq_gemm_noalloc(bq_handle_t h, bq_op_t opA, bq_op_t opB, const bq_matrix_t* A,
                            const bq_matrix_t* B, bq_matrix_t* C, bq_prec_t prec, int slices,
                            bq_stream_t stream);

/* Subalgebra special cases (Sec. III A: real, complex and real-quaternion
 * matrices embedded in H_C).  The arguments and conventions of bq_gemm (op
 * sign rules of Sec. III, precision, slices, workspace sized by
 * bq_gemm_workspace_size with the algebra's mask for both operands); only
 * the named components of A, B and C are read or written, the rest may be
 * NULL (a NULL named input component is zero).
 *   bq_re_gemm: comp[0]                     (1 real GEMM)
 *   bq_cx_gemm: comp[0] + i comp[4]         (3 real GEMMs, Gauss)
 *   bq_rq_gemm: comp[0..3] (real quaternion, 8 real GEMMs, bilinear) */
bq_status_t bq_re_gemm(bq_handle_t h, bq_op_t opA, bq_op_t opB, const bq_matrix_t* A,
                       const bq_matrix_t* B, bq_matrix_t* C, bq_prec_t prec, int slices,
                       void* ws, size_t ws_bytes, bq_stream_t stream);
bq_status_t bq_cx_gemm(bq_handle_t h, bq_op_t opA, bq_op_t opB, const bq_matrix_t* A,
                       const bq_matrix_t* B, bq_matrix_t* C, bq_prec_t prec, int slices,
                       void* ws, size_t ws_bytes, bq_stream_t stream);
bq_status_t bq_rq_gemm(bq_handle_t h, bq_op_t opA, bq_op_t opB, const bq_matrix_t* A,
                       const bq_matrix_t* B, bq_matrix_t* C, bq_prec_t prec, int slices,
                       void* ws, size_t ws_bytes, bq_stream_t stream);

/* Number of real GEMMs the planner runs for these masks (the paper's counts:
 * 24 full, 8 real quaternion, 3 complex, 1 real).  Host only. */
int bq_plan_real_gemms(unsigned maskA, unsigned maskB);

/* ---------------------------------------------------------------------------
 * Batched form: many independent products C_p = op(A_p) op(B_p) of
 * different sizes in one plan, run as one graph.  FP64: a pre-combination
 * launch for every problem, then persistent launches whose blocks take
 * (problem, 64 x 64 tile) work items, largest problems first: either one
 * launch whose items run the problem's eight complex products on their tile
 * in turn, or one launch per complex product (the autotuner picks); in the
 * latter the Hadamard products P5..P8 go first and write their P into the
 * problem's workspace, one launch forms their Hadamard sums, and the direct
 * products P1..P4 write each C block once (FP64 workspace per problem: the
 * pre-combined operands plus 8 blocks of m x round_up(n, 8) doubles).  CRT
 * form: per complex product, one launch for each stage over every problem
 * (exponents, residues, residue GEMMs, reconstruction; stages split by
 * modulus count where that differs); each problem keeps its own workspace
 * region (its pre-combinations and the residues of three real products),
 * so the plan's workspace is the sum over the problems, and every result
 * equals the single call's bit for bit.  The
 * digit-slice forms replay every problem's sequence in one graph.
 *
 * Pointers in the problems are baked into the plan: A, B, C of every problem
 * must stay valid (and C must not overlap any A, B or other C) until the
 * plan is destroyed.  FP64 plans need full biquaternions (all 16 input
 * components present); others return BQ_ERR_UNSUPPORTED.  Every op is
 * taken, per problem (T and H read the stored matrices, as in bq_gemm).
 * Plan creation allocates the plan's device tables (hipMalloc, once);
 * launching allocates nothing.  A plan is bound to the workspace pointer of
 * its first launch: a later launch with another pointer re-records the graph.
 * Calls on one plan must not overlap.
 * ------------------------------------------------------------------------- */
typedef struct {
  bq_op_t opA, opB;
  bq_matrix_t A, B, C;
} bq_problem_t;

typedef struct bq_grouped_plan_s* bq_grouped_plan_t;

bq_status_t bq_grouped_plan_create(bq_handle_t h, int count, const bq_problem_t* problems, bq_prec_t prec,
                                   int slices, bq_grouped_plan_t* plan);
/* Device workspace one launch needs (bytes). */
bq_status_t bq_grouped_plan_workspace_size(bq_grouped_plan_t plan, size_t* bytes);
/* Autotuner: times every candidate tile configuration and work schedule of
 * the FP64 plan on the given workspace and stream (synchronising it), keeps
 * the fastest, and records it in the cache file named by BQ_TUNE_CACHE (if
 * set) under a key of device architecture, CU count, precision and problem
 * sizes; a later plan with the same key reads it back at creation.  For the
 * split forms it returns BQ_OK without changes. */
bq_status_t bq_grouped_plan_autotune(bq_grouped_plan_t plan, void* ws, size_t ws_bytes, bq_stream_t stream);
bq_status_t bq_grouped_plan_launch(bq_grouped_plan_t plan, void* ws, size_t ws_bytes, bq_stream_t stream);
/* Chosen tile configuration, schedule (bit 0: blocks take work items from a
 * device counter, else cyclically; bit 1: one launch per complex product)
 * and work items (FP64: tiles; CRT: real products). */
bq_status_t bq_grouped_plan_info(bq_grouped_plan_t plan, int* tile_config, int* dynamic_schedule, int* work_items);
bq_status_t bq_grouped_plan_destroy(bq_grouped_plan_t plan);

/* ---------------------------------------------------------------------------
 * Diagonalization of a Hermitian matrix-valued biquaternion (Sec. III and the
 * Hadamard transformation for diagonalization in the implementation section):
 * A (n x n, A^dagger = A, i.e. components c1 and c6..c8 symmetric, c2..c5
 * antisymmetric) is mapped to its complex Hermitian isomorph
 *   Z(A) = [[Z11, Z12], [Z21, Z22]]  (2n x 2n; eq. mapping-formulas read
 *   backwards, M = M+ + M-):
 *   Z11 = (c1 - c6) + i (c2 + c5),   Z12 = (c3 - c8) + i (c4 + c7),
 *   Z21 = -(c3 + c8) + i (c4 - c7),  Z22 = (c1 + c6) + i (c5 - c2),
 * whose eigenvalues and eigenvectors are returned.  The components present
 * select the work:
 *   - no j or k components (c3, c4, c7, c8 absent): Z is block diagonal; the
 *     two n x n blocks are solved separately, once when Z22 = Z11 (c2, c6
 *     absent) or Z22 = conj(Z11) (c5, c6 absent);
 *   - j and k only (c1, c2, c5, c6 absent) with pure j (c3, c7) or pure k
 *     (c4, c8): Z is block anti-diagonal and the Hadamard-type transform
 *     U = [[I, I], [a I, -a I]] / sqrt(2) (a = i for pure j, a = 1 for pure
 *     k) makes it diag(a Z12, -a Z12): one n x n solve, eigenvalues +-mu;
 *   - j and k only with both present: with the singular value decomposition
 *     Z12 = U S V^dagger and G = V U^dagger, U_G = [[I, I], [G, -G]] / sqrt(2)
 *     makes Z diag(U S U^dagger, -U S U^dagger): one n x n SVD, eigenvalues
 *     +-s, eigenvectors [u; +-v] / sqrt(2);
 *   - otherwise one 2n x 2n solve.
 * The complex Hermitian eigensolver is rocSOLVER's zheevd and the SVD its
 * zgesdd (library calls); the mapping, the reduction, the eigenvalue merge
 * and the eigenvector assembly are this library's kernels.
 *
 * w:    device, 2n doubles: eigenvalues in ascending order.
 * V:    device or NULL: eigenvectors of Z(A) as columns, 2n x 2n complex
 *       (interleaved re, im doubles), column-major with leading dimension
 *       ldv >= 2n complex elements: Z(A) V = V diag(w), V^dagger V = I.
 * info: device int or NULL: 0 on success, > 0 if an eigensolve or the SVD
 *       did not converge (written asynchronously, like w and V).
 * Only the part of A the isomorph's lower triangle comes from is read; A
 * is taken to be Hermitian, not checked.  n == 0 is a no-op.  Errors as for
 * bq_gemm (validation first, nothing enqueued on error); the workspace is
 * the caller's, the eigensolver's scratch included (no allocation). */
bq_status_t bq_heev_workspace_size(bq_handle_t h, int64_t n, unsigned mask, int want_vectors,
                                   size_t* bytes);
bq_status_t bq_heev(bq_handle_t h, const bq_matrix_t* A, double* w, double* V, int64_t ldv, int* info,
                    void* ws, size_t ws_bytes, bq_stream_t stream);

/* Launch tracing (measurement support, not part of the product semantics).
 * While enabled, every kernel the handle enqueues is bracketed by a pair of
 * HIP events recorded on the same stream.  bq_trace_read waits for the
 * recorded events, copies up to `cap` records (oldest first), removes them
 * and sets *count to the number copied.  `flops` and `bytes` are the
 * algorithmic work of the launch: 2 m n k per real product for a GEMM,
 * the bytes read plus written for a pre-combination or zero fill. */
typedef BQ_ENUM(bq_kernel_e) {
  BQ_KERNEL_GEMM_GAUSS = 0, /* complex x complex, 3 real products    */
  BQ_KERNEL_GEMM_RC = 1,    /* real x complex, 2 real products       */
  BQ_KERNEL_GEMM_CR = 2,    /* complex x real, 2 real products       */
  BQ_KERNEL_GEMM_RR = 3,    /* real x real, 1 real product           */
  BQ_KERNEL_COMBINE = 10,   /* Hadamard pre-combination              */
  BQ_KERNEL_FILL = 11,      /* zero fill of a structurally zero block */
  BQ_KERNEL_SPLIT = 12,     /* exponents + digit slices of one operand */
  BQ_KERNEL_SLICE_GEMM = 13, /* one real product from digit slices;
                               flops = pairs * 2 m n k, config = slices */
  BQ_KERNEL_GROUPED = 14,    /* one launch of a batched plan (whole graph);
                               flops = executed real-GEMM flops of all problems */
  BQ_KERNEL_CRT_GEMM = 15,   /* the INT8 GEMMs of one real product in the CRT
                               form; flops = moduli * 2 m n k, config = moduli */
  BQ_KERNEL_CRT_COMBINE = 16, /* residues -> FP64 product -> targets; bytes
                               read + written */
  BQ_KERNEL_HEEV_MAP = 20,   /* isomorph (or reduced block) of a Hermitian
                               biquaternion; bytes read + written */
  BQ_KERNEL_HEEV_SOLVE = 21, /* one complex Hermitian eigensolve (zheevd);
                               m = n = its order, config = 1 with vectors */
  BQ_KERNEL_HEEV_ASSEMBLE = 22 /* eigenvalue merge + eigenvector assembly */
} bq_kernel_t;

typedef struct {
  int kernel; /* bq_kernel_t */
  int config; /* tile configuration of a GEMM launch, else -1 */
  int64_t m, n, k;
  double ms;
  double flops;
  double bytes;
} bq_trace_record_t;

bq_status_t bq_trace_enable(bq_handle_t h, int enable);
bq_status_t bq_trace_read(bq_handle_t h, bq_trace_record_t* recs, int cap, int* count);

#ifdef __cplusplus
}
#endif

#endif /* BQ_H */
