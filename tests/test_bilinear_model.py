"""The paper's bilinear scheme restated in numpy, checked against the oracle.

This model is not the oracle and not the product: it pins the reading of
Sec. III A (eqs. bilinearH and cmplx-3-real-mult) that the HIP kernels
implement, and it gives per-step intermediates for debugging.  It counts the
real GEMMs it performs so the 24 / 8 / 3 / 1 counts of the paper are pinned.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2609_02081_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# Hadamard rows for products 5..8 (eq. bilinearH)
H4 = np.array([[1, 1, 1, 1], [1, 1, -1, -1], [1, -1, 1, -1], [1, -1, -1, 1]], dtype=np.float64)
# operand pairs of products 1..4: P1=M1N1, P2=M4N3, P3=M2N4, P4=M3N2
PAIRS = [(0, 0), (3, 2), (1, 3), (2, 1)]


class Counter:
    def __init__(self):
        self.n = 0

    def mm(self, x, y):
        self.n += 1
        return x @ y


def gauss(cnt, LR, LI, RR, RI):
    """eq. cmplx-3-real-mult: P = (T1 - T2) + i (T3 - T1 - T2); zero parts skipped."""
    def nz(x):
        return x is not None
    if nz(LI) and nz(RI):
        T1 = cnt.mm(LR, RR)
        T2 = cnt.mm(LI, RI)
        T3 = cnt.mm(LR + LI, RR + RI)
        return T1 - T2, T3 - T1 - T2
    if nz(LI):
        return cnt.mm(LR, RR), cnt.mm(LI, RR)
    if nz(RI):
        return cnt.mm(LR, RR), cnt.mm(LR, RI)
    return cnt.mm(LR, RR), None


def bilinear(A, B, cnt, real_only=False):
    """Q = M N by eq. bilinearH; A, B (8, ., .); returns C (8, m, n)."""
    def part(X, u, imag):
        return None if (real_only and imag) else X[u + 4 * imag]
    P = []
    for (u, v) in PAIRS:
        P.append(gauss(cnt, part(A, u, 0), part(A, u, 1), part(B, v, 0), part(B, v, 1)))
    for h in H4:
        LR = sum(h[u] * A[u] for u in range(4))
        RR = sum(h[u] * B[u] for u in range(4))
        LI = None if real_only else sum(h[u] * A[u + 4] for u in range(4))
        RI = None if real_only else sum(h[u] * B[u + 4] for u in range(4))
        P.append(gauss(cnt, LR, LI, RR, RI))
    m, n = A.shape[1], B.shape[2]
    z = np.zeros((m, n))
    Pr = [p[0] for p in P]
    Pi = [p[1] if p[1] is not None else z for p in P]
    coef = [2.0, -2.0, -2.0, -2.0]
    C = np.empty((8, m, n))
    for w in range(4):
        s = np.array([-1.0, 1.0, 1.0, 1.0])[w] * 0.25
        C[w] = coef[w] * Pr[w] + s * sum(H4[w][q] * Pr[4 + q] for q in range(4))
        C[w + 4] = coef[w] * Pi[w] + s * sum(H4[w][q] * Pi[4 + q] for q in range(4))
    return C


def test_bilinear_equals_oracle_random():
    A, B = inputs.pair(33, 17, 29, "normal", seed=101)
    cnt = Counter()
    C = bilinear(A, B, cnt)
    assert cnt.n == 24
    assert oracle.rel_frobenius(C, oracle.gemm(A, B)) < 1e-14


def test_bilinear_integer_bit_exact():
    A, B = inputs.pair(16, 48, 20, "int", seed=102, bound=1024)
    C = bilinear(A, B, Counter())
    assert np.array_equal(C, oracle.gemm(A, B))


def test_counts_match_paper():
    with open(os.path.join(GOLDEN, "gemm_counts.json")) as f:
        g = json.load(f)
    A, B = inputs.pair(8, 8, 8, "normal", seed=103)
    cnt = Counter()
    bilinear(A, B, cnt)
    assert cnt.n == g["bilinear_gauss_real"]
    A, B = inputs.pair(8, 8, 8, "normal", seed=104, mask_a=inputs.REAL_QUAT, mask_b=inputs.REAL_QUAT)
    cnt = Counter()
    C = bilinear(A, B, cnt, real_only=True)
    assert cnt.n == g["real_quaternion_bilinear"]
    assert oracle.rel_frobenius(C, oracle.gemm(A, B)) < 1e-14


@pytest.mark.parametrize("u,v", [(a, b) for a in range(8) for b in range(8)])
def test_unit_blocks_bit_exact(u, v):
    """Every unit pair (including the commuting i) through the bilinear path."""
    A = np.zeros((8, 4, 4)); A[u] = np.eye(4)
    B = np.zeros((8, 4, 4)); B[v] = np.eye(4)
    assert np.array_equal(bilinear(A, B, Counter()), oracle.gemm(A, B))
