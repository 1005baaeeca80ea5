"""Oracle for the CRT-based split form of the real product (Ozaki scheme II).

TEST INFRASTRUCTURE: used only by tests; shares no code with the HIP path.

The paper computes every real GEMM in FP64; this split form is an extension
(Ozaki, Uchino and Imamura's scheme II, integer-modular), read here as:

* left factor X (m x k): per row i the exponent e_i, the frexp exponent of
  max_j |x_ij| (so |x_ij| < 2^e_i); the integer matrix X'_ij =
  rint(x_ij 2^(b - e_i)), |X'| <= 2^b; right factor Y (k x n) likewise per
  column j with f_j: Y'_ij = rint(y_ij 2^(b - f_j));
* P = X' Y' is an exact integer matrix with |P| <= k 2^(2b); it is carried
  as residues modulo N pairwise coprime odd moduli p_1..p_N <= 255 (so every
  symmetric residue fits a signed byte), whose product M exceeds 2 max|P|,
  and recovered by the Chinese remainder theorem;
* T = diag(2^e) 2^(-2b) P diag(2^f), rounded to FP64.

This module computes P exactly with Python integers (small sizes only), so
its result is the correctly rounded T.  The GPU rebuilds the same integer P
exactly from its residues (carried modulo 2^128) and rounds it to FP64 once,
so a real product of the GPU's CRT form equals this one bit for bit.
"""
import math

import numpy as np

# Odd, pairwise coprime, largest first: 255 = 3*5*17, 253 = 11*23,
# 247 = 13*19, the rest primes above 160.
MODULI = (255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 211, 199, 197, 193, 191, 181, 179, 173, 167, 163)


def bits_for(n_moduli: int, k: int) -> int:
    """Largest b with prod(p_1..p_N) > 2 k 2^(2b) (0 if none)."""
    logm = sum(math.log2(p) for p in MODULI[:n_moduli])
    # one above the floating-point estimate, then down to the exact answer
    b = min(53, int(math.floor((logm - 1.0 - math.log2(max(k, 1))) / 2.0)) + 1)
    while b > 0 and math.prod(MODULI[:n_moduli]) <= 2 * max(k, 1) * (1 << (2 * b)):
        b -= 1
    return max(0, min(b, 53))


def default_moduli(k: int) -> int:
    """Fewest moduli that carry b = 53 bits for an inner dimension k."""
    for n in range(1, len(MODULI) + 1):
        if bits_for(n, k) >= 53:
            return n
    return len(MODULI)


def exponents(X, axis):
    mx = np.max(np.abs(X), axis=axis) if X.size else np.zeros(X.shape[1 - axis])
    _, e = np.frexp(mx)
    return np.where(mx > 0, e, 0).astype(np.int64)


def integers(X, b, axis):
    """X' = rint(X 2^(b - e)) as int64 with the exponents e along `axis`
    (axis=1: one per row, the left factor; axis=0: per column)."""
    X = np.asarray(X, dtype=np.float64)
    e = exponents(X, axis)
    ee = e[:, None] if axis == 1 else e[None, :]
    Q = np.rint(np.ldexp(X, b - ee))
    return Q.astype(np.int64), e


def exact_product(Xi, Yi):
    """X' Y' with Python integers (object arrays): exact."""
    return np.asarray(Xi, dtype=object).dot(np.asarray(Yi, dtype=object))


def product(X, Y, n_moduli=0):
    """Split-form real product X @ Y (Ozaki scheme II): n_moduli = 0 takes
    the fewest moduli that carry 53 bits for this inner dimension."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    k = X.shape[1]
    N = n_moduli or default_moduli(k)
    b = bits_for(N, k)
    Xi, e = integers(X, b, 1)
    Yi, f = integers(Y, b, 0)
    P = exact_product(Xi, Yi)
    out = np.empty(P.shape, dtype=np.float64)
    for i in range(P.shape[0]):
        for j in range(P.shape[1]):
            # exact integer to FP64 (correct rounding), then exact power-of-two scaling
            out[i, j] = math.ldexp(float(P[i, j]), int(e[i] + f[j]) - 2 * b)
    return out


def residues(Xi, p):
    """Symmetric residues of an integer array modulo an odd p: values in
    [-(p-1)/2, (p-1)/2]."""
    r = np.mod(np.asarray(Xi, dtype=np.int64), p)
    return np.where(r > (p - 1) // 2, r - p, r)


def crt(res, moduli):
    """The integer x with |x| < M/2 and x = res[i] (mod moduli[i]): the
    Chinese remainder sum of r_i M_i (M_i^-1 mod p_i) modulo M, M_i = M / p_i
    (Python integers, exact)."""
    M = math.prod(moduli)
    x = 0
    for r, p in zip(res, moduli):
        m_i = M // p
        x += int(r) * m_i * pow(m_i, -1, p)
    x %= M
    return x - M if x > M // 2 else x
