"""Oracle for matrix-valued biquaternion multiplication (FP64, CPU).

TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The HIP library never
imports, links or calls it, and it imports nothing from the HIP library.

Contents
--------
gemm(A, B)        C = A B by the plain element-wise definition of
                  eq. MatrixQMultiplication with the scalar product of
                  eq. QMultiplication (Sec. II A), in C (bq_oracle.c).
iso(M), iso_inv(Z)  The 2m x 2n complex isomorph of Sec. III
                  (eqs. biquat-repres, main-biquat-eqn, M+/M-, mapping-formulas).
transpose/conj/herm  Sign rules for T, *, dagger (Sec. III).
trace(M)          Tr = 2 (Tr M1 + i Tr M5) (Sec. III).

Arrays are numpy float64 of shape (8, rows, cols), component order
[M1..M8] = [E_R, E_I, F_R, F_I, G_I, -G_R, H_I, -H_R] (eq. biquat-repres);
unit coefficients 1:(M1 + i M5), i:(M2 + i M6), j:(M3 + i M7), k:(M4 + i M8).
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(_LIB_PATH)
        P8 = ctypes.c_void_p * 8
        lib.bqo_gemm.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                 P8, ctypes.c_int64, P8, ctypes.c_int64, P8, ctypes.c_int64]
        lib.bqo_gemm.restype = ctypes.c_int
        lib.bqo_num_threads.restype = ctypes.c_int
        lib.bqo_set_num_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def num_threads() -> int:
    return _load().bqo_num_threads()


def set_num_threads(t: int) -> None:
    _load().bqo_set_num_threads(int(t))


def _blocks(M):
    M = np.asarray(M)
    if M.dtype != np.float64 or M.ndim != 3 or M.shape[0] != 8:
        raise ValueError("expected float64 array of shape (8, rows, cols)")
    return M


def gemm(A, B) -> np.ndarray:
    """C = A B for A (8, m, k), B (8, k, n); returns C (8, m, n)."""
    A = _blocks(A)
    B = _blocks(B)
    if A.shape[2] != B.shape[1]:
        raise ValueError("inner dimensions differ")
    A = np.ascontiguousarray(A)
    B = np.ascontiguousarray(B)
    m, k = A.shape[1], A.shape[2]
    n = B.shape[2]
    C = np.empty((8, m, n), dtype=np.float64)
    if m == 0 or n == 0:
        return C
    if k == 0:
        C[...] = 0.0
        return C
    P8 = ctypes.c_void_p * 8
    pa = P8(*[A[c].ctypes.data for c in range(8)])
    pb = P8(*[B[c].ctypes.data for c in range(8)])
    pc = P8(*[C[c].ctypes.data for c in range(8)])
    rc = _load().bqo_gemm(m, n, k, pa, k, pb, n, pc, n)
    if rc != 0:
        raise RuntimeError("oracle gemm rejected its arguments")
    return C


# ---------------------------------------------------------------------------
# Complex isomorph (Sec. III).  E = M1 + i M2, F = M3 + i M4,
# G = -M6 + i M5, H = -M8 + i M7;  M+ = [[E, F], [-F*, E*]],
# M- = [[G, H], [H*, -G*]], and Z(M) = M+ + M-.
# ---------------------------------------------------------------------------
def _efgh(M):
    M = _blocks(M)
    E = M[0] + 1j * M[1]
    F = M[2] + 1j * M[3]
    G = -M[5] + 1j * M[4]
    H = -M[7] + 1j * M[6]
    return E, F, G, H


def iso(M) -> np.ndarray:
    """2m x 2n complex matrix isomorphic to the biquaternion M (8, m, n)."""
    E, F, G, H = _efgh(M)
    top = np.concatenate([E + G, F + H], axis=1)
    bot = np.concatenate([-F.conj() + H.conj(), E.conj() - G.conj()], axis=1)
    return np.concatenate([top, bot], axis=0)


def iso_inv(Z) -> np.ndarray:
    """Inverse map, eq. mapping-formulas: E=(A+D*)/2, F=(B-C*)/2,
    G=(A-D*)/2, H=(B+C*)/2 for Z = [[A, B], [C, D]]."""
    Z = np.asarray(Z)
    if Z.ndim != 2 or Z.shape[0] % 2 or Z.shape[1] % 2:
        raise ValueError("expected a 2m x 2n complex matrix")
    m, n = Z.shape[0] // 2, Z.shape[1] // 2
    a, b = Z[:m, :n], Z[:m, n:]
    c, d = Z[m:, :n], Z[m:, n:]
    E = (a + d.conj()) / 2
    F = (b - c.conj()) / 2
    G = (a - d.conj()) / 2
    H = (b + c.conj()) / 2
    return np.stack([E.real, E.imag, F.real, F.imag, G.imag, -G.real, H.imag, -H.real])


def heev(M):
    """Eigenvalues (ascending) and eigenvectors (columns) of the complex
    isomorph of a Hermitian biquaternion M (8, n, n): the diagonalization of
    the implementation section maps M to Z(M) (eq. mapping-formulas) and
    solves the complex Hermitian problem; numpy's Hermitian eigensolver is
    the library step."""
    return np.linalg.eigh(iso(M))


# ---------------------------------------------------------------------------
# T, *, dagger as a transposition plus per-component sign flips (Sec. III).
# ---------------------------------------------------------------------------
SIGN_T = (1, 1, -1, 1, 1, 1, -1, 1)
SIGN_CONJ = (1, -1, 1, -1, -1, 1, -1, 1)
SIGN_HERM = (1, -1, -1, -1, -1, 1, 1, 1)


def transpose(M) -> np.ndarray:
    M = _blocks(M)
    return np.stack([s * M[c].T for c, s in enumerate(SIGN_T)])


def conj(M) -> np.ndarray:
    M = _blocks(M)
    return np.stack([s * M[c] for c, s in enumerate(SIGN_CONJ)])


def herm(M) -> np.ndarray:
    M = _blocks(M)
    return np.stack([s * M[c].T for c, s in enumerate(SIGN_HERM)])


def trace(M) -> complex:
    """Tr = 2 (Tr M1 + i Tr M5) for a square biquaternion matrix."""
    M = _blocks(M)
    return complex(2.0 * (np.trace(M[0]) + 1j * np.trace(M[4])))


def rel_frobenius(C, C_ref) -> float:
    """||C - C_ref||_F / ||C_ref||_F over all 8 blocks jointly (absolute
    error when C_ref is zero)."""
    C = np.asarray(C, dtype=np.float64)
    C_ref = np.asarray(C_ref, dtype=np.float64)
    num = float(np.sqrt(np.sum((C - C_ref) ** 2)))
    den = float(np.sqrt(np.sum(C_ref ** 2)))
    return num / den if den > 0 else num
