"""The paper's bilinear scheme restated in numpy (test helper).

Not the oracle and not the product: it restates Sec. III A (eqs. bilinearH
and cmplx-3-real-mult) so tests can pin that reading against the oracle, and
it takes the real GEMM as a parameter (Counter.mm) so the split-precision
form can be modelled with the same structure.
"""
import numpy as np

# Hadamard rows for products 5..8 (eq. bilinearH)
H4 = np.array([[1, 1, 1, 1], [1, 1, -1, -1], [1, -1, 1, -1], [1, -1, -1, 1]], dtype=np.float64)
# operand pairs of products 1..4: P1=M1N1, P2=M4N3, P3=M2N4, P4=M3N2
PAIRS = [(0, 0), (3, 2), (1, 3), (2, 1)]


class Counter:
    """Counts real GEMMs; `gemm` replaces x @ y (e.g. a split-form product)."""

    def __init__(self, gemm=None):
        self.n = 0
        self.gemm = gemm

    def mm(self, x, y):
        self.n += 1
        return self.gemm(x, y) if self.gemm else x @ y


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


