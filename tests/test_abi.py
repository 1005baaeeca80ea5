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
    assert check(A, Bm, C, prec=2, slices=15, ws=4 * FAKE, ws_bytes=1 << 30) == INVALID
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
    # columns to 64, k to 64; 2-byte BF16 digits, S = 7 by default)
    r_bf, m_bf = B.workspace_size(m, n, k, 0xFF, 0xFF, "split_bf16", 0)
    dig = lambda rows: (7 * rows * 64 * 2 + 255) // 256 * 256 + (rows * 4 + 255) // 256 * 256
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
