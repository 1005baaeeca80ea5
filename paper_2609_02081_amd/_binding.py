"""ctypes binding of libbq.so: argument marshalling only.

Every arithmetic step runs in the HIP library.  Tensors are torch float64
device tensors shaped (8, rows, cols) (or lists of 8 tensors / None); torch
only provides the memory, the workspace allocation and the current stream.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libbq.so")

OPS = {"N": 0, "T": 1, "C": 2, "H": 3}
PRECS = {"fp64": 0, "split_bf16": 1, "split_fp8": 2, "split_int8": 3, "split_int8_crt": 4}
STATUS = {0: "BQ_OK", 1: "BQ_ERR_INVALID_VALUE", 2: "BQ_ERR_UNSUPPORTED", 3: "BQ_ERR_ALIAS",
          4: "BQ_ERR_WORKSPACE", 5: "BQ_ERR_HIP", 6: "BQ_ERR_ARCH"}

FULL, REAL_QUAT, COMPLEX, REAL = 0xFF, 0x0F, 0x11, 0x01


class BqMatrix(ctypes.Structure):
    _fields_ = [("comp", ctypes.c_void_p * 8), ("rows", ctypes.c_int64),
                ("cols", ctypes.c_int64), ("ld", ctypes.c_int64)]


class BqProblem(ctypes.Structure):
    _fields_ = [("opA", ctypes.c_int), ("opB", ctypes.c_int), ("A", BqMatrix), ("B", BqMatrix), ("C", BqMatrix)]


class BqTraceRecord(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int), ("config", ctypes.c_int), ("m", ctypes.c_int64),
                ("n", ctypes.c_int64), ("k", ctypes.c_int64), ("ms", ctypes.c_double),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]


KERNEL_NAMES = {0: "gemm_gauss", 1: "gemm_rc", 2: "gemm_cr", 3: "gemm_rr", 10: "combine", 11: "fill",
                12: "split", 13: "slice_gemm", 14: "grouped", 15: "crt_gemm",
                16: "crt_combine", 20: "heev_map", 21: "heev_solve",
                22: "heev_assemble"}


class BqError(RuntimeError):
    def __init__(self, code: int, detail: str):
        super().__init__(f"{STATUS.get(code, code)}: {detail}")
        self.code = code
        self.detail = detail


_lib = None

# (name, restype, argtypes) of every symbol declared in include/bq.h
_M = ctypes.POINTER(BqMatrix)
_SIGS = [
    ("bq_create", ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int]),
    ("bq_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("bq_status_string", ctypes.c_char_p, [ctypes.c_int]),
    ("bq_last_error_detail", ctypes.c_char_p, []),
    ("bq_gemm_workspace_size", ctypes.c_int,
     [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint, ctypes.c_uint, ctypes.c_int,
      ctypes.c_int, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
    ("bq_gemm_check", ctypes.c_int,
     [ctypes.c_int, ctypes.c_int, _M, _M, _M, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t]),
    ("bq_gemm", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _M, _M, _M, ctypes.c_int, ctypes.c_int,
      ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    ("bq_gemm_noalloc", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _M, _M, _M, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]),
    ("bq_re_gemm", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _M, _M, _M, ctypes.c_int, ctypes.c_int,
      ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    ("bq_cx_gemm", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _M, _M, _M, ctypes.c_int, ctypes.c_int,
      ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    ("bq_rq_gemm", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _M, _M, _M, ctypes.c_int, ctypes.c_int,
      ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    ("bq_plan_real_gemms", ctypes.c_int, [ctypes.c_uint, ctypes.c_uint]),
    ("bq_grouped_plan_create", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(BqProblem), ctypes.c_int, ctypes.c_int,
      ctypes.POINTER(ctypes.c_void_p)]),
    ("bq_grouped_plan_workspace_size", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]),
    ("bq_grouped_plan_autotune", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    ("bq_grouped_plan_launch", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    ("bq_grouped_plan_info", ctypes.c_int,
     [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    ("bq_grouped_plan_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("bq_heev_workspace_size", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]),
    ("bq_heev", ctypes.c_int,
     [ctypes.c_void_p, _M, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
      ctypes.c_size_t, ctypes.c_void_p]),
    ("bq_trace_enable", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    ("bq_trace_read", ctypes.c_int,
     [ctypes.c_void_p, ctypes.POINTER(BqTraceRecord), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
]


def lib():
    """Load libbq.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().bq_last_error_detail().decode()


def check(code: int) -> None:
    if code != 0:
        raise BqError(code, last_error())


_handles: dict[int, ctypes.c_void_p] = {}


def handle(device: int = 0) -> ctypes.c_void_p:
    h = _handles.get(device)
    if h is None:
        h = ctypes.c_void_p()
        check(lib().bq_create(ctypes.byref(h), device))
        _handles[device] = h
    return h


def _is_tensor(x) -> bool:
    return hasattr(x, "data_ptr") and hasattr(x, "stride")


def matrix(X, mask: int = FULL, rows=None, cols=None) -> BqMatrix:
    """BqMatrix over a (8, rows, cols) tensor or a list of 8 (rows, cols)
    tensors / None.  Components outside `mask` (or None) are passed as absent."""
    M = BqMatrix()
    comps = list(X) if not _is_tensor(X) else [X[c] for c in range(8)]
    if len(comps) != 8:
        raise ValueError("a biquaternion matrix has 8 components")
    ref = next((c for c in comps if c is not None), None)
    if ref is None:
        if rows is None or cols is None:
            raise ValueError("all components absent: give rows and cols")
        M.rows, M.cols, M.ld = rows, cols, max(1, cols)
        return M
    M.rows, M.cols = ref.shape
    M.ld = ref.stride(0) if ref.shape[0] > 1 else max(1, ref.shape[1])
    if ref.numel() == 0:
        # nothing is read or written: the layout does not matter
        M.ld = max(1, ref.shape[1])
        for c, t in enumerate(comps):
            present = t is not None and (mask >> c & 1) and t.data_ptr() != 0
            M.comp[c] = t.data_ptr() if present else None
        return M
    for c, t in enumerate(comps):
        if t is None or not (mask >> c & 1):
            M.comp[c] = None
            continue
        if t.shape != ref.shape or (t.shape[0] > 1 and t.stride(0) != M.ld) or t.stride(1) != 1:
            raise ValueError("components must share shape and row-major layout")
        M.comp[c] = t.data_ptr()
    return M


def _stream(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _on(stream):
    """Context in which temporaries (workspace, outputs) are allocated: the
    caller's stream when one is given, so that torch's caching allocator
    hands their memory to later work only in that stream's order."""
    import contextlib

    import torch

    return torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()


def workspace_size(m, n, k, mask_a=FULL, mask_b=FULL, prec="fp64", slices=0):
    res = ctypes.c_size_t()
    mn = ctypes.c_size_t()
    check(lib().bq_gemm_workspace_size(m, n, k, mask_a, mask_b, PRECS[prec], slices,
                                       ctypes.byref(res), ctypes.byref(mn)))
    return res.value, mn.value


def heev_workspace_size(n, mask=FULL, vectors=True, device=0) -> int:
    out = ctypes.c_size_t()
    check(lib().bq_heev_workspace_size(handle(device), n, mask, int(bool(vectors)), ctypes.byref(out)))
    return out.value


def heev(A, *, mask=FULL, vectors=True, workspace=None, stream=None):
    """Eigenvalues (2n, ascending) and optionally eigenvectors of the complex
    isomorph of the Hermitian biquaternion A (8, n, n): returns (w, V, info)
    with V (2n, 2n) complex128 whose columns are the eigenvectors (None
    without vectors) and info a device int tensor (0 = converged)."""
    import torch

    Am = matrix(A, mask)
    n = Am.rows
    dev = (A if _is_tensor(A) else next(t for t in A if t is not None)).device
    with _on(stream):
        w = torch.empty(2 * n, dtype=torch.float64, device=dev)
        info = torch.zeros(1, dtype=torch.int32, device=dev)
        V = None
        if vectors:
            # column-major 2n x 2n complex = row-major storage of V^T
            Vt = torch.empty((2 * n, 2 * n), dtype=torch.complex128, device=dev)
        need = heev_workspace_size(n, _mask_of(Am), vectors, dev.index or 0)
        if workspace is None:
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    check(lib().bq_heev(handle(dev.index or 0), ctypes.byref(Am), ctypes.c_void_p(w.data_ptr()),
                        ctypes.c_void_p(Vt.data_ptr()) if vectors else None, 2 * n,
                        ctypes.c_void_p(info.data_ptr()), ctypes.c_void_p(workspace.data_ptr()),
                        workspace.numel() * workspace.element_size(), _stream(stream)))
    if vectors:
        V = Vt.transpose(0, 1)
    return w, V, info


def plan_real_gemms(mask_a=FULL, mask_b=FULL) -> int:
    return lib().bq_plan_real_gemms(mask_a, mask_b)


def bq_gemm(A, B, C=None, *, opA="N", opB="N", mask_a=FULL, mask_b=FULL, prec="fp64", slices=0,
            workspace=None, streamed=False, stream=None):
    """C = op(A) op(B) on the current device; returns C (8, m, n) float64."""
    import torch

    Am = matrix(A, mask_a)
    Bm = matrix(B, mask_b)
    # op T and H take the stored matrix transposed
    m, k = (Am.cols, Am.rows) if opA in ("T", "H") else (Am.rows, Am.cols)
    n = Bm.rows if opB in ("T", "H") else Bm.cols
    dev = (A if _is_tensor(A) else next(t for t in A if t is not None)).device
    res, mn = workspace_size(m, n, k, _mask_of(Am), _mask_of(Bm), prec, slices)
    with _on(stream):
        if C is None:
            C = torch.empty((8, m, n), dtype=torch.float64, device=dev)
        if workspace is None:
            need = mn if streamed else res
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    Cm = matrix(C)
    ws_bytes = workspace.numel() * workspace.element_size()
    if streamed:
        ws_bytes = min(ws_bytes, mn)
    check(lib().bq_gemm(handle(dev.index or 0), OPS[opA], OPS[opB], ctypes.byref(Am), ctypes.byref(Bm),
                        ctypes.byref(Cm), PRECS[prec], slices, ctypes.c_void_p(workspace.data_ptr()),
                        ws_bytes, _stream(stream)))
    return C


NOALLOC_SCRATCH_BYTES = 256 << 20


def bq_gemm_noalloc(A, B, C, *, opA="N", opB="N", mask_a=FULL, mask_b=FULL, prec="fp64", slices=0, stream=None):
    """C = op(A) op(B) into the caller's C (8, m, n), with the library's static
    workspace: neither the library nor this function allocates device memory."""
    Am = matrix(A, mask_a)
    Bm = matrix(B, mask_b)
    Cm = matrix(C)
    dev = (C if _is_tensor(C) else next(t for t in C if t is not None)).device
    check(lib().bq_gemm_noalloc(handle(dev.index or 0), OPS[opA], OPS[opB], ctypes.byref(Am), ctypes.byref(Bm),
                                ctypes.byref(Cm), PRECS[prec], slices, _stream(stream)))
    return C


def _mask_of(M: BqMatrix) -> int:
    return sum(1 << c for c in range(8) if M.comp[c])


def _sub_gemm(name, mask, comps_a, comps_b, comps_c, opA, opB, prec, slices, workspace, stream):
    """Shared marshalling of the subalgebra entry points: 8-slot component
    lists with the algebra's components in place, the rest None."""
    import torch

    Am, Bm, Cm = matrix(comps_a, mask), matrix(comps_b, mask), matrix(comps_c, mask)
    dev = next(t for t in comps_c if t is not None).device
    m, k = (Am.cols, Am.rows) if opA in ("T", "H") else (Am.rows, Am.cols)
    n = Bm.rows if opB in ("T", "H") else Bm.cols
    if workspace is None:
        res, _ = workspace_size(m, n, k, mask, mask, prec, slices)
        with _on(stream):
            workspace = torch.empty(max(res, 1), dtype=torch.uint8, device=dev)
    check(getattr(lib(), name)(handle(dev.index or 0), OPS[opA], OPS[opB], ctypes.byref(Am), ctypes.byref(Bm),
                               ctypes.byref(Cm), PRECS[prec], slices, ctypes.c_void_p(workspace.data_ptr()),
                               workspace.numel() * workspace.element_size(), _stream(stream)))


def re_gemm(A, B, C, opA="N", opB="N", prec="fp64", slices=0, workspace=None, stream=None):
    """A, B, C: (rows, cols) real tensors (component 1 alone)."""
    z = [None] * 7
    _sub_gemm("bq_re_gemm", REAL, [A] + z, [B] + z, [C] + z, opA, opB, prec, slices, workspace, stream)
    return C


def cx_gemm(A, B, C, opA="N", opB="N", prec="fp64", slices=0, workspace=None, stream=None):
    """A, B, C: (re, im) pairs of real tensors (components 1 and 5)."""
    def pack(x):
        return [x[0], None, None, None, x[1], None, None, None]
    _sub_gemm("bq_cx_gemm", COMPLEX, pack(A), pack(B), pack(C), opA, opB, prec, slices, workspace, stream)
    return C


def rq_gemm(A, B, C, opA="N", opB="N", prec="fp64", slices=0, workspace=None, stream=None):
    """A, B, C: lists of 4 real tensors (units 1, i, j, k)."""
    def pack(x):
        return list(x) + [None] * 4
    _sub_gemm("bq_rq_gemm", REAL_QUAT, pack(A), pack(B), pack(C), opA, opB, prec, slices, workspace, stream)
    return C


def trace_enable(enable: bool = True, device: int = 0) -> None:
    check(lib().bq_trace_enable(handle(device), int(bool(enable))))


def trace_read(device: int = 0, cap: int = 4096) -> list[dict]:
    """Completed launch records since the last read (waits for them)."""
    recs = (BqTraceRecord * cap)()
    cnt = ctypes.c_int()
    out = []
    while True:
        check(lib().bq_trace_read(handle(device), recs, cap, ctypes.byref(cnt)))
        for r in recs[:cnt.value]:
            out.append({"kernel": KERNEL_NAMES.get(r.kernel, str(r.kernel)), "config": r.config,
                        "m": r.m, "n": r.n, "k": r.k, "ms": r.ms, "flops": r.flops, "bytes": r.bytes})
        if cnt.value < cap:
            return out


class GroupedPlan:
    """Batched plan over (A, B, C) triples of (8, rows, cols) device tensors,
    or (A, B, C, opA, opB) for per-problem ops (else opA, opB apply to all).

    The tensors are referenced by the plan and must stay alive (this object
    keeps them) until close().  Workspace comes from torch unless given."""

    def __init__(self, problems, prec="fp64", slices=0, opA="N", opB="N", device=0):
        self._keep = []
        arr = (BqProblem * max(1, len(problems)))()
        for i, prob in enumerate(problems):
            A, B, C = prob[:3]
            oa, ob = (prob[3], prob[4]) if len(prob) == 5 else (opA, opB)
            arr[i].opA, arr[i].opB = OPS[oa], OPS[ob]
            arr[i].A, arr[i].B, arr[i].C = matrix(A), matrix(B), matrix(C)
            self._keep.append((A, B, C))
        self.device = device
        self._plan = ctypes.c_void_p()
        check(lib().bq_grouped_plan_create(handle(device), len(problems), arr, PRECS[prec], slices,
                                           ctypes.byref(self._plan)))
        self._ws = None

    def workspace_size(self) -> int:
        b = ctypes.c_size_t()
        check(lib().bq_grouped_plan_workspace_size(self._plan, ctypes.byref(b)))
        return b.value

    def workspace(self):
        import torch

        if self._ws is None:
            self._ws = torch.empty(max(1, self.workspace_size()), dtype=torch.uint8, device=f"cuda:{self.device}")
        return self._ws

    def autotune(self, workspace=None, stream=None):
        ws = self.workspace() if workspace is None else workspace
        check(lib().bq_grouped_plan_autotune(self._plan, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                             _stream(stream)))

    def launch(self, workspace=None, stream=None):
        ws = self.workspace() if workspace is None else workspace
        check(lib().bq_grouped_plan_launch(self._plan, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                           _stream(stream)))

    def info(self) -> dict:
        c, d, n = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(lib().bq_grouped_plan_info(self._plan, ctypes.byref(c), ctypes.byref(d), ctypes.byref(n)))
        return {"tile_config": c.value, "dynamic": d.value & 1, "per_product_launches": d.value >> 1 & 1,
                "work_items": n.value}

    def close(self):
        if self._plan:
            lib().bq_grouped_plan_destroy(self._plan)
            self._plan = ctypes.c_void_p()
        self._keep = []
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
