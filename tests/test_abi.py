"""C-ABI contract, host only: the library loads, exports every symbol the
header declares, and every argument error is caught before any HIP call."""
import ctypes
import os
import re

import pytest

from paper_2609_02081_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bq.h")

OK, INVALID, UNSUPPORTED, ALIAS, WORKSPACE, HIP, ARCH = range(7)


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bq_[a-z0-9_]+)\s*\(", src)))


def test_header_symbols_exported():
    lib = B.lib()
    names = declared_symbols()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    # and the binding declares a signature for each of them
    assert sorted(n for n, _, _ in B._SIGS) == names


def test_status_strings():
    lib = B.lib()
    for code, name in B.STATUS.items():
        assert lib.bq_status_string(code).decode() == name
    assert lib.bq_status_string(99).decode() == "BQ_ERR_UNKNOWN"


FAKE = 1 << 40  # host integers standing in for device addresses; never dereferenced


def mat(rows, cols, base, ld=None, mask=0xFF, stride=None):
    M = B.BqMatrix()
    ld = ld if ld is not None else max(1, cols)
    stride = stride if stride is not None else ((rows * ld + 31) // 32 * 32) * 8
    for c in range(8):
        M.comp[c] = (base + c * stride) if (mask >> c & 1) else None
    M.rows, M.cols, M.ld = rows, cols, ld
    return M


def check(A, Bm, C, opA=0, opB=0, prec=0, slices=0, ws=None, ws_bytes=0):
    return B.lib().bq_gemm_check(opA, opB, ctypes.byref(A), ctypes.byref(Bm), ctypes.byref(C), prec,
                                 slices, ws, ws_bytes)


def ws_need(m, n, k, ma=0xFF, mb=0xFF):
    return B.workspace_size(m, n, k, ma, mb)


def test_valid_call_passes():
    m, n, k = 40, 30, 20
    res, mn = ws_need(m, n, k)
    assert check(mat(m, k, FAKE), mat(k, n, 2 * FAKE), mat(m, n, 3 * FAKE), ws=4 * FAKE,
                 ws_bytes=res) == OK
    assert check(mat(m, k, FAKE), mat(k, n, 2 * FAKE), mat(m, n, 3 * FAKE), ws=4 * FAKE,
                 ws_bytes=mn) == OK   # streamed plan


def test_null_arguments():
    lib = B.lib()
    A, Bm, C = mat(4, 4, FAKE), mat(4, 4, 2 * FAKE), mat(4, 4, 3 * FAKE)
    assert lib.bq_gemm_check(0, 0, None, ctypes.byref(Bm), ctypes.byref(C), 0, 0, None, 0) == INVALID
    C.comp[5] = None
    assert check(A, Bm, C, ws=4 * FAKE, ws_bytes=1 << 30) == INVALID
    assert "output component 5" in B.last_error()
    assert lib.bq_gemm(None, 0, 0, ctypes.byref(A), ctypes.byref(Bm), ctypes.byref(C), 0, 0, None, 0,
                       None) == INVALID


def test_shapes_and_leading_dimensions():
    ws = (4 * FAKE, 1 << 30)
    assert check(mat(4, 5, FAKE), mat(6, 3, 2 * FAKE), mat(4, 3, 3 * FAKE), ws=ws[0], ws_bytes=ws[1]) == INVALID
    assert check(mat(4, 5, FAKE), mat(5, 3, 2 * FAKE), mat(4, 4, 3 * FAKE), ws=ws[0], ws_bytes=ws[1]) == INVALID
    assert check(mat(4, 5, FAKE, ld=4), mat(5, 3, 2 * FAKE), mat(4, 3, 3 * FAKE), ws=ws[0],
                 ws_bytes=ws[1]) == INVALID
    bad = mat(4, 5, FAKE)
    bad.rows = -1
    assert check(bad, mat(5, 3, 2 * FAKE), mat(4, 3, 3 * FAKE), ws=ws[0], ws_bytes=ws[1]) == INVALID
    mis = mat(4, 5, FAKE + 4)
    assert check(mis, mat(5, 3, 2 * FAKE), mat(4, 3, 3 * FAKE), ws=ws[0], ws_bytes=ws[1]) == INVALID


def test_ops_and_precisions():
    A, Bm, C = mat(4, 4, FAKE), mat(4, 4, 2 * FAKE), mat(4, 4, 3 * FAKE)
    for op in (1, 2, 3):
        assert check(A, Bm, C, opA=op, ws=4 * FAKE, ws_bytes=1 << 30) == OK
        assert check(A, Bm, C, opB=op, ws=4 * FAKE, ws_bytes=1 << 30) == OK
    # op T / H take the stored matrix transposed: op(A) 4 x 5 from A stored
    # 5 x 4, op(B) 5 x 3 from B stored 3 x 5
    ws = dict(ws=4 * FAKE, ws_bytes=1 << 30)
    At, Bt = mat(5, 4, FAKE), mat(3, 5, 2 * FAKE)
    Bn, C43 = mat(5, 3, 2 * FAKE), mat(4, 3, 3 * FAKE)
    for op in (1, 3):
        assert check(At, Bn, C43, opA=op, **ws) == OK
        assert check(mat(4, 5, FAKE), Bt, C43, opB=op, **ws) == OK
        assert check(At, Bt, C43, opA=op, opB=op, **ws) == OK
        assert check(At, Bn, C43, **ws) == INVALID          # N: A 5 x 4 does not chain with B 5 x 3
        assert check(At, Bn, mat(5, 3, 3 * FAKE), opA=op, **ws) == INVALID  # C must be 4 x 3
    assert check(A, Bm, C, opA=7) == INVALID
    assert check(A, Bm, C, prec=9) == INVALID
    assert check(A, Bm, C, slices=-1) == INVALID
    # split forms: slice counts above the digit type's maximum are rejected
    res_bf, _ = B.workspace_size(4, 4, 4, 0xFF, 0xFF, "split_bf16", 0)
    assert check(A, Bm, C, prec=1, ws=4 * FAKE, ws_bytes=res_bf) == OK
    assert check(A, Bm, C, prec=1, slices=9, ws=4 * FAKE, ws_bytes=1 << 30) == INVALID
    assert check(A, Bm, C, prec=2, slices=14, ws=4 * FAKE, ws_bytes=1 << 30) == INVALID
    assert check(A, Bm, C, prec=3, slices=10, ws=4 * FAKE, ws_bytes=1 << 30) == INVALID


def test_alias_detection():
    m = n = k = 16
    res, _ = ws_need(m, n, k)
    A = mat(m, k, FAKE)
    # C overlapping A
    assert check(A, mat(k, n, 2 * FAKE), mat(m, n, FAKE + 8 * 100), ws=4 * FAKE, ws_bytes=res) == ALIAS
    # C overlapping the workspace
    assert check(A, mat(k, n, 2 * FAKE), mat(m, n, 4 * FAKE + 64), ws=4 * FAKE, ws_bytes=res) == ALIAS
    # two components of C overlapping each other
    assert check(A, mat(k, n, 2 * FAKE), mat(m, n, 3 * FAKE, stride=64), ws=4 * FAKE,
                 ws_bytes=res) == ALIAS
    # the workspace overlapping a component of A or of B (the pre-combination
    # would overwrite an input before the GEMMs read it)
    Bm = mat(k, n, 2 * FAKE)
    C = mat(m, n, 3 * FAKE)
    assert check(A, Bm, C, ws=FAKE + 7 * 2048, ws_bytes=res) == ALIAS        # inside A's last component
    assert "workspace overlaps" in B.last_error()
    assert check(A, Bm, C, ws=2 * FAKE - res + 8, ws_bytes=res) == ALIAS     # its end reaches B's first
    assert check(A, Bm, C, ws=2 * FAKE - res, ws_bytes=res) == OK            # ends where B starts
    # only the part of the workspace the plan uses counts: a larger buffer
    # whose tail covers an input is fine when the resident plan ends before it
    assert check(A, Bm, C, ws=2 * FAKE - res - 4096, ws_bytes=res + 8192) == OK
    # the split form's digit buffers count too
    rs, _ = B.workspace_size(m, n, k, 0xFF, 0xFF, "split_int8_crt", 0)
    assert check(A, Bm, C, prec=4, ws=2 * FAKE - rs + 8, ws_bytes=rs) == ALIAS


def test_workspace_sizes_and_errors():
    m, n, k = 100, 60, 40
    res, mn = ws_need(m, n, k)
    up8 = lambda x: (x + 7) // 8 * 8      # combination buffers: rows padded to 64 bytes,
    slot = lambda r, c: max(r * up8(c), c * up8(r)) * 8   # in either orientation (op N or T)
    a1 = (slot(m, k) + 255) // 256 * 256
    b1 = (slot(k, n) + 255) // 256 * 256
    assert res == 4 * (2 * a1 + 2 * b1) and mn == 2 * a1 + 2 * b1
    rq_res, rq_min = ws_need(m, n, k, 0x0F, 0x0F)
    assert rq_res == 4 * (a1 + b1) and rq_min == a1 + b1
    assert ws_need(m, n, k, 0x11, 0x11) == (0, 0)
    assert ws_need(m, n, k, 0x01, 0x01) == (0, 0)
    assert ws_need(m, n, 0) == (0, 0)
    # split form: + digit buffers of one real product (rows padded to 128,
    # columns to 64, k to 64; 2-byte BF16 digits, S = 8 by default at k = 40)
    r_bf, m_bf = B.workspace_size(m, n, k, 0xFF, 0xFF, "split_bf16", 0)
    dig = lambda rows: (8 * rows * 64 * 2 + 255) // 256 * 256 + (rows * 4 + 255) // 256 * 256
    assert r_bf == res + dig(128) + dig(64) and m_bf == mn + dig(128) + dig(64)
    A, Bm, C = mat(m, k, FAKE), mat(k, n, 2 * FAKE), mat(m, n, 3 * FAKE)
    assert check(A, Bm, C, ws=4 * FAKE, ws_bytes=mn - 1) == WORKSPACE
    assert check(A, Bm, C, ws=None, ws_bytes=0) == WORKSPACE
    assert check(A, Bm, C, ws=None, ws_bytes=16) == INVALID


def test_plan_counts_match_paper():
    """24 full, 8 real quaternion (also purely imaginary quaternion), 3
    complex, 1 real (Sec. III A)."""
    assert B.plan_real_gemms(0xFF, 0xFF) == 24
    assert B.plan_real_gemms(0x0F, 0x0F) == 8
    assert B.plan_real_gemms(0xF0, 0xF0) == 8
    assert B.plan_real_gemms(0x11, 0x11) == 3
    assert B.plan_real_gemms(0x01, 0x01) == 1
    assert B.plan_real_gemms(0x00, 0xFF) == 0


@pytest.mark.parametrize("ma,mb,count", [
    (0x0F, 0xFF, 16),   # real quaternion x biquaternion: 16 (4 real-by-complex pairs, twice)
    (0xFF, 0x0F, 16),
    (0xF0, 0xFF, 16),   # purely imaginary-field biquaternion [0,0,0,0,1,1,1,1] x full
    (0x11, 0xFF, 12),   # complex scalar x biquaternion: 4 complex products, 3 GEMMs each
    (0x01, 0xFF, 8),    # real scalar field x biquaternion: 8 real products
    (0x33, 0x33, 12),   # units 1 and i with complex coefficients: 4 complex products (component-wise < bilinear 15)
])
def test_plan_counts_general_masks(ma, mb, count):
    """Active-component patterns beyond the four subalgebras (Sec. III A:
    absent components are skipped): the planner's min(bilinear,
    component-wise) real-GEMM count."""
    assert B.plan_real_gemms(ma, mb) == count


def test_degenerate_shapes_validate():
    assert check(mat(0, 5, FAKE), mat(5, 3, 2 * FAKE), mat(0, 3, 3 * FAKE)) == OK
    assert check(mat(4, 0, FAKE), mat(0, 3, 2 * FAKE), mat(4, 3, 3 * FAKE)) == OK


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert B.lib().bq_create(ctypes.byref(h), 0) != OK
    assert not h.value


@pytest.mark.parametrize("k", [1, 40, 1000, 16384, 70000, 133120])
def test_crt_workspace_uses_oracle_moduli(k):
    """CRT form: digits are one byte per modulus (rows and columns padded to
    256, k to 128), plus exponents and N residue planes of m rows of n bytes
    rounded up to 16 for each of three real products; N = 0 resolves to the fewest moduli that carry 53 bits for this k,
    the count the oracle (which checks the modulus product with exact
    integers) picks."""
    from oracle import ozaki2

    m, n = 100, 60
    res, mn = ws_need(m, n, k)
    N = ozaki2.default_moduli(k)
    al = lambda x: (x + 255) // 256 * 256
    kp = (k + 127) // 128 * 128
    ldr = (n + 15) // 16 * 16
    # three sets of exponents and residue planes: the real products of one
    # complex product
    extra = al(N * 256 * kp) + al(N * 256 * kp) + 3 * (al(256 * 4) + al(256 * 4) + al(N * m * ldr))
    assert B.workspace_size(m, n, k, 0xFF, 0xFF, "split_int8_crt", 0) == (res + extra, mn + extra)
    N2 = max(1, N - 3)
    extra2 = al(N2 * 256 * kp) * 2 + 3 * (al(256 * 4) * 2 + al(N2 * m * ldr))
    assert B.workspace_size(m, n, k, 0xFF, 0xFF, "split_int8_crt", N2) == (res + extra2, mn + extra2)


def test_crt_limits():
    from oracle import ozaki2

    ws = dict(ws=4 * FAKE, ws_bytes=1 << 40)
    crt = B.PRECS["split_int8_crt"]

    def chk(k, slices=0):
        return check(mat(8, k, FAKE), mat(k, 8, 2 * FAKE), mat(8, 8, 3 * FAKE), prec=crt, slices=slices, **ws)

    assert chk(133120) == OK
    assert chk(133121) == UNSUPPORTED          # int32 sums of 127^2 products would overflow
    assert chk(64, slices=21) == INVALID       # 20 moduli at most
    for k in (1, 64, 5000):
        # the smallest count that still carries one bit passes, one fewer fails
        n_min = next(N for N in range(1, 21) if ozaki2.bits_for(N, k) >= 1)
        assert chk(k, slices=n_min) == OK
        if n_min > 1:
            assert chk(k, slices=n_min - 1) == INVALID


@pytest.mark.parametrize("k", [1, 2, 40, 256, 257, 4096, 16384, 100000])
@pytest.mark.parametrize("kind", ["bf16", "fp8", "int8"])
def test_default_slices_follow_k(kind, k):
    """slices = 0 in a digit form resolves, from the call's k, to the fewest
    slices whose digits carry 48 + ceil(log2(k) / 2) significand bits (the
    oracle's restatement of the rule): the workspace of the default equals
    that of the explicit count."""
    from oracle import ozaki

    prec = {"bf16": "split_bf16", "fp8": "split_fp8", "int8": "split_int8"}[kind]
    S = ozaki.default_slices(kind, k)
    assert ozaki.carried_bits(kind, S) >= 48 + ((k - 1).bit_length() + 1) // 2 or S == ozaki.MAX_SLICES[kind]
    assert B.workspace_size(50, 30, k, 0xFF, 0xFF, prec, 0) == B.workspace_size(50, 30, k, 0xFF, 0xFF, prec, S)
    if S > 1:
        assert B.workspace_size(50, 30, k, 0xFF, 0xFF, prec, 0) != \
            B.workspace_size(50, 30, k, 0xFF, 0xFF, prec, S - 1)


def test_default_slices_at_the_benchmark_size():
    """At k = 16384 the defaults carry 55 to 59 bits: BF16 8, FP8 12, INT8 8."""
    from oracle import ozaki

    assert [ozaki.default_slices(t, 16384) for t in ("bf16", "fp8", "int8")] == [8, 12, 8]
    assert [ozaki.carried_bits(t, S) for t, S in (("bf16", 8), ("fp8", 12), ("int8", 8))] == [56, 59, 55]


def test_variant_entry_points_take_the_gemm_arguments():
    """bq_re_gemm, bq_cx_gemm and bq_rq_gemm share bq_gemm's argument
    pattern (ops, precision, slices, workspace); argument errors come back
    before any HIP call."""
    lib = B.lib()
    A, Bm, C = mat(4, 4, FAKE), mat(4, 4, 2 * FAKE), mat(4, 4, 3 * FAKE)
    for name in ("bq_re_gemm", "bq_cx_gemm", "bq_rq_gemm"):
        f = getattr(lib, name)
        assert f(None, 1, 3, ctypes.byref(A), ctypes.byref(Bm), ctypes.byref(C), 4, 0, None, 0, None) == INVALID
        assert "handle" in B.last_error()
        h = ctypes.c_void_p(1)   # never dereferenced: validation fails first
        assert f(h, 7, 0, ctypes.byref(A), ctypes.byref(Bm), ctypes.byref(C), 0, 0, None, 0, None) == INVALID
        assert f(h, 0, 0, ctypes.byref(A), ctypes.byref(Bm), ctypes.byref(C), 9, 0, None, 0, None) == INVALID
        assert f(h, 0, 0, None, ctypes.byref(Bm), ctypes.byref(C), 0, 0, None, 0, None) == INVALID


def test_planner_log():
    """BQ_LOG=1 prints one plan line per validated call on stderr."""
    import subprocess
    import sys

    prog = f"""
import ctypes, sys
sys.path.insert(0, {ROOT!r})
from paper_2609_02081_amd import _binding as B
def mat(rows, cols, base, mask=0xFF):
    M = B.BqMatrix()
    for c in range(8):
        M.comp[c] = (base + c * (1 << 20)) if (mask >> c & 1) else None
    M.rows, M.cols, M.ld = rows, cols, cols
    return M
A, Bm, C = mat(40, 20, 1 << 40), mat(20, 30, 2 << 40), mat(40, 30, 3 << 40)
res, mn = B.workspace_size(40, 30, 20)
rc1 = B.lib().bq_gemm_check(1, 0, ctypes.byref(mat(20, 40, 1 << 40)), ctypes.byref(Bm), ctypes.byref(C), 0, 0,
                            4 << 40, mn)
rc2 = B.lib().bq_gemm_check(0, 0, ctypes.byref(mat(40, 20, 1 << 40, 0x0F)), ctypes.byref(mat(20, 30, 2 << 40, 0x0F)),
                            ctypes.byref(C), 4, 0, 4 << 40, 1 << 30)
print(rc1, rc2)
"""
    env = dict(os.environ, BQ_LOG="1")
    r = subprocess.run([sys.executable, "-c", prog], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.split() == ["0", "0"]
    lines = [l for l in r.stderr.splitlines() if l.startswith("[bq] plan")]
    assert len(lines) == 2, r.stderr
    assert "m=40 n=30 k=20 op=TN" in lines[0] and "form=bilinear real_gemms=24" in lines[0]
    assert "prec=fp64" in lines[0] and "workspace=streamed" in lines[0]
    assert "maskA=0x0f" in lines[1] and "real_gemms=8" in lines[1] and "prec=split_int8_crt" in lines[1]
    assert "slices=15" in lines[1] and "workspace=resident" in lines[1]
    # off by default
    env.pop("BQ_LOG")
    r = subprocess.run([sys.executable, "-c", prog], env=env, capture_output=True, text=True, timeout=120)
    assert "[bq] plan" not in r.stderr


def test_size_limits():
    """Dimensions of 2^31 and more, or a matrix above 2^40 elements, are
    refused before any size arithmetic could overflow."""
    for m, n, k in ((1 << 31, 4, 4), (4, 4, 1 << 31), (1 << 21, 4, 1 << 20), (4, 1 << 30, 1 << 11)):
        res, mn = ctypes.c_size_t(), ctypes.c_size_t()
        assert B.lib().bq_gemm_workspace_size(m, n, k, 0xFF, 0xFF, 0, 0, ctypes.byref(res),
                                              ctypes.byref(mn)) == UNSUPPORTED
    assert B.lib().bq_gemm_workspace_size(1 << 20, 4, 1 << 20, 0xFF, 0xFF, 4, 0, None, None) == OK
    assert check(mat(1 << 21, 8, FAKE), mat(8, 1 << 20, 2 * FAKE), mat(1 << 21, 1 << 20, 3 * FAKE)) == UNSUPPORTED
