"""Diagonalization of Hermitian biquaternions on the GPU (bq_heev through the
C-ABI) against the oracle (numpy eigh of the isomorph).

Eigenvalues: max |w - w_ref| <= 1e-12 ||Z||_2 (backward-stable solvers on
both sides).  Eigenvectors are not unique (degenerate pairs, phases), so they
are checked for what is unique: the residual ||Z V - V diag(w)||_F <=
1e-12 ||Z||_2 sqrt(2n) and orthonormality max |V^H V - I| <= 1e-12, with Z
the oracle's isomorph.  Every structure path: full, block diagonal (two
solves, equal blocks, conjugate blocks), block anti-diagonal (pure j, pure
k) and the j + k anti-diagonal case through the singular value decomposition of
Z12, and a mixed case that takes the full problem.
"""
import numpy as np
import pytest

import oracle
from paper_2609_02081_amd import inputs

pytestmark = pytest.mark.gpu
TOL = 1e-12

CASES = {
    "full": 0xFF,
    "real_quaternion": 0x0F,
    "blocks": 0x33,        # c1, c2, c5, c6: Z = diag(Z11, Z22)
    "blocks_equal": 0x11,  # c1, c5: Z22 = Z11
    "blocks_conj": 0x03,   # c1, c2: Z22 = conj(Z11)
    "anti_j": 0x44,        # c3, c7: Hadamard transform with a = i
    "anti_k": 0x88,        # c4, c8: a = 1
    "anti_jk": 0xCC,       # j and k: SVD of Z12
    "anti_jk_3": 0x4C,     # c3, c4, c7: SVD of Z12
    "anti_jk_4": 0x86,     # c2, c3, c8: field unit present, full problem
}


@pytest.fixture(scope="module")
def bq():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_02081_amd as bq

    bq.lib()
    return bq


def solve(bq, A, mask, vectors=True):
    import torch

    w, V, info = bq.heev(torch.from_numpy(A).to("cuda"), mask=mask, vectors=vectors)
    torch.cuda.synchronize()
    return w.cpu().numpy(), (V.cpu().numpy() if V is not None else None), int(info.item())


def check(A, w, V):
    Z = oracle.iso(A)
    w_ref, _ = oracle.heev(A)
    scale = max(1.0, float(np.max(np.abs(w_ref))))
    assert np.max(np.abs(w - w_ref)) <= TOL * scale
    if V is not None:
        N = Z.shape[0]
        res = np.linalg.norm(Z @ V - V * w) / (scale * np.sqrt(N))
        assert res <= TOL, res
        assert np.max(np.abs(V.conj().T @ V - np.eye(N))) <= TOL


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("n", [1, 37, 200])
def test_structure_paths(bq, case, n):
    mask = CASES[case]
    A = inputs.hermitian_random(n, mask, seed=40 + n)
    print(f"heev {case} n={n}", flush=True)
    w, V, info = solve(bq, A, mask)
    assert info == 0
    check(A, w, V)
    w2, V2, info2 = solve(bq, A, mask, vectors=False)
    assert info2 == 0 and V2 is None
    check(A, w2, None)


def test_known_spectrum(bq):
    """Fock-like Hermitian input of the benchmark (U diag(lambda) U^H,
    lambda signed, 1e0..1e-8): eigenvalues recovered to 1e-12 absolute."""
    import torch

    p = inputs.hermitian_params(300, seed=51, kind="fock")
    A = inputs.hermitian_blocks(p, "cuda")
    w, V, info = bq.heev(A)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    assert np.max(np.abs(w.cpu().numpy() - np.sort(p["lam"]))) <= 1e-12
    check(A.cpu().numpy(), w.cpu().numpy(), V.cpu().numpy())


def test_n1024_full(bq):
    mask = CASES["full"]
    A = inputs.hermitian_random(1024, mask, seed=52)
    print("heev full n=1024", flush=True)
    w, V, info = solve(bq, A, mask)
    assert info == 0
    check(A, w, V)


def test_errors_leave_outputs_untouched(bq):
    import ctypes

    import torch

    from paper_2609_02081_amd import _binding as B

    A = torch.from_numpy(inputs.hermitian_random(16, inputs.FULL, seed=53)).to("cuda")
    w = torch.full((32,), 5.0, dtype=torch.float64, device="cuda")
    Am = B.matrix(A)
    h = B.handle(0)
    need = B.heev_workspace_size(16, inputs.FULL, False)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    L = B.lib()
    stream = B._stream(None)
    # workspace too small
    assert L.bq_heev(h, ctypes.byref(Am), ctypes.c_void_p(w.data_ptr()), None, 32, None,
                     ctypes.c_void_p(ws.data_ptr()), need - 1, stream) == 4
    # w inside the workspace
    assert L.bq_heev(h, ctypes.byref(Am), ctypes.c_void_p(ws.data_ptr()), None, 32, None,
                     ctypes.c_void_p(ws.data_ptr()), need, stream) == 3
    # V with ldv < 2n
    V = torch.empty((32, 32), dtype=torch.complex128, device="cuda")
    assert L.bq_heev(h, ctypes.byref(Am), ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(V.data_ptr()), 31,
                     None, ctypes.c_void_p(ws.data_ptr()), need, stream) == 1
    # not square
    Ar = B.matrix(A[:, :, :15])
    assert L.bq_heev(h, ctypes.byref(Ar), ctypes.c_void_p(w.data_ptr()), None, 32, None,
                     ctypes.c_void_p(ws.data_ptr()), need, stream) == 1
    torch.cuda.synchronize()
    assert torch.all(w == 5.0).item()


def test_empty(bq):
    import torch

    A = torch.empty((8, 0, 0), dtype=torch.float64, device="cuda")
    w, V, info = bq.heev(A)
    torch.cuda.synchronize()
    assert w.numel() == 0 and int(info.item()) == 0


@pytest.mark.parametrize("case", ["full", "anti_j", "blocks"])
def test_strided_input_and_output(bq, case):
    """A with ld > n (a column slice of a wider buffer) and V with ldv > 2n:
    the padding of V is left alone."""
    import ctypes

    import torch

    from paper_2609_02081_amd import _binding as B

    n, mask = 45, CASES[case]
    A = inputs.hermitian_random(n, mask, seed=55)
    buf = torch.zeros((8, n, n + 7), dtype=torch.float64, device="cuda")
    buf[:, :, :n] = torch.from_numpy(A).to("cuda")
    Am = B.matrix(buf[:, :, :n], mask)
    ldv = 2 * n + 5
    Vt = torch.full((2 * n, ldv), 9.0 + 0j, dtype=torch.complex128, device="cuda")  # column-major V, ldv
    w = torch.empty(2 * n, dtype=torch.float64, device="cuda")
    need = B.heev_workspace_size(n, mask, True)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    B.check(B.lib().bq_heev(B.handle(0), ctypes.byref(Am), ctypes.c_void_p(w.data_ptr()),
                            ctypes.c_void_p(Vt.data_ptr()), ldv, None, ctypes.c_void_p(ws.data_ptr()), need,
                            B._stream(None)))
    torch.cuda.synchronize()
    Vfull = Vt.cpu().numpy()
    assert np.all(Vfull[:, 2 * n:] == 9.0)
    check(A, w.cpu().numpy(), Vfull[:, :2 * n].T)


@pytest.mark.parametrize("n", [64, 300])
def test_jk_svd_matches_full_problem(bq, n, monkeypatch):
    """The SVD reduction (both rocSOLVER SVD routines) and the full 2n
    eigensolve of the same j + k input agree on the eigenvalues, and both
    pass the residual and orthonormality checks."""
    A = inputs.hermitian_random(n, 0xCC, seed=60 + n)
    w0, V0, i0 = solve(bq, A, 0xCC)
    assert i0 == 0
    check(A, w0, V0)
    monkeypatch.setenv("BQ_SVD", "gesvd")
    w1, V1, i1 = solve(bq, A, 0xCC)
    assert i1 == 0
    check(A, w1, V1)
    monkeypatch.delenv("BQ_SVD")
    monkeypatch.setenv("BQ_HEEV_JK", "full")
    w2, V2, i2 = solve(bq, A, 0xCC)
    assert i2 == 0
    scale = max(1.0, float(np.max(np.abs(w2))))
    assert np.max(np.abs(w0 - w2)) <= TOL * scale and np.max(np.abs(w1 - w2)) <= TOL * scale
