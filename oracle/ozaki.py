"""Oracle for the split-precision (Ozaki-style) real product.

TEST INFRASTRUCTURE: used only by tests; shares no code with the HIP path.

The paper computes every real GEMM in FP64; the split form is an extension
(error-free splitting of Ozaki, Ogita, Oishi and Rump, 2012), read here as:

* left factor X (m x k): per row i an exponent e_i, the frexp exponent of
  max_j |x_ij| plus a headroom h (so |x_ij| 2^-e_i < 2^-h); right factor
  Y (k x n): per column j an exponent f_j;  h = 1 for INT8 digits (beta 7:
  without it the leading digit could reach 2^7 = 128, one past a signed
  byte) and for FP8 E4M3 digits (beta 5: every digit is then an integer in
  [-16, 16], all of which E4M3's four significant bits hold exactly), h = 0
  for BF16 (beta 7), whose leading digit 2^7 is representable;
* digits of y = x 2^-e: q_1 = rint(2^b y), y_1 = y - q_1 2^-b, and
  q_s = rint(2^{bs} y_{s-1}), y_s = y_{s-1} - q_s 2^{-bs} for s = 2..S;
* T = diag(2^e) [ sum_{s + t <= S + 1} 2^{-b(s+t)} Q_s R_t ] diag(2^f).

Digit products are exact integers here (int64); the sum over s + t is taken
in FP64 level by level.  The result therefore differs from the GPU split
path only by FP64 summation order.
"""
import numpy as np

BETA = {"bf16": 7, "fp8": 5, "int8": 7}
HEAD = {"bf16": 0, "fp8": 1, "int8": 1}
MAX_SLICES = {"bf16": 8, "fp8": 13, "int8": 9}


def carried_bits(kind, S):
    """Significand bits S digits carry for a row's largest element: the
    scaled element lies in [2^(-1-h), 2^-h) and the remainder after S digits
    is at most 2^(-beta S - 1), so beta S - h bits."""
    return BETA[kind] * S - HEAD[kind]


def default_slices(kind, k):
    """The split form's default slice count for inner dimension k: the
    fewest slices carrying 48 + ceil(log2(k) / 2) bits (the truncation of a
    length-k dot product grows like sqrt(k)), at most MAX_SLICES."""
    lg = (int(k) - 1).bit_length() if k > 1 else 0   # ceil(log2 k)
    need = 48 + (lg + 1) // 2
    for S in range(1, MAX_SLICES[kind] + 1):
        if carried_bits(kind, S) >= need:
            return S
    return MAX_SLICES[kind]


def exponents(X, axis, head=0):
    """frexp exponent of the largest magnitude along `axis` (rows: axis=1),
    plus `head`; all-zero lines get 0 (their digits are zero)."""
    mx = np.max(np.abs(X), axis=axis)
    _, e = np.frexp(mx)
    return np.where(mx > 0, e + head, 0).astype(np.int64), mx > 0


def digits(X, beta, S, axis, head=0):
    """Digit slices Q[s] (int64) and exponents of X along `axis`
    (axis=1: one exponent per row, the left factor; axis=0: per column)."""
    X = np.asarray(X, dtype=np.float64)
    e, nz = exponents(X, axis, head)
    ee = e[:, None] if axis == 1 else e[None, :]
    y = np.ldexp(X, -ee)
    Q = []
    for s in range(1, S + 1):
        q = np.rint(np.ldexp(y, beta * s))
        y = y - np.ldexp(q, -beta * s)
        Q.append(q.astype(np.int64))
    return Q, e, y  # y: remainder (scaled)


def product(X, Y, kind="bf16", S=7):
    """Split-form real product X @ Y."""
    beta, head = BETA[kind], HEAD[kind]
    QX, ex, _ = digits(X, beta, S, axis=1, head=head)
    QY, ey, _ = digits(Y, beta, S, axis=0, head=head)
    acc = np.zeros((X.shape[0], Y.shape[1]), dtype=np.float64)
    for d in range(2, S + 2):
        lvl = np.zeros_like(acc, dtype=np.int64)
        for s in range(1, d):
            t = d - s
            if s <= S and t <= S:
                lvl += QX[s - 1] @ QY[t - 1]
        acc = acc + np.ldexp(lvl.astype(np.float64), -beta * d)
    return np.ldexp(np.ldexp(acc, ex[:, None]), ey[None, :])
