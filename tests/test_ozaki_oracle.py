"""Pins for the split-form oracle (oracle/ozaki.py): exact reconstruction,
digit bounds, exact integer products, and convergence to the FP64 product
at the rate one digit (beta bits) per slice predicts."""
import numpy as np
import pytest

from oracle import ozaki
from paper_2609_02081_amd import inputs

KINDS = [("bf16", 8), ("fp8", 13), ("int8", 9)]


@pytest.mark.parametrize("kind,S", KINDS)
@pytest.mark.parametrize("dist", ["uniform", "logspread", "normal"])
def test_reconstruction(kind, S, dist):
    """x = 2^e (sum_s q_s 2^-bs + rem) exactly, |rem| <= 2^(-bS-1); numpy's
    uniform draws are multiples of 2^-52, so S * beta >= 53 digits hold them
    with no remainder at all."""
    beta, head = ozaki.BETA[kind], ozaki.HEAD[kind]
    rng = np.random.default_rng(5)
    X = inputs.blocks(rng, 20, 33, dist)[0]
    for axis in (1, 0):
        Q, e, rem = ozaki.digits(X, beta, S, axis, head)
        ee = e[:, None] if axis == 1 else e[None, :]
        rec = sum(np.ldexp(Q[s].astype(np.float64), -beta * (s + 1)) for s in range(S))
        assert np.array_equal(np.ldexp(rec + rem, ee), X)
        assert np.max(np.abs(rem)) <= 2.0 ** (-beta * S - 1)
        if dist == "uniform":
            assert np.array_equal(np.ldexp(rec, ee), X)


@pytest.mark.parametrize("kind,S", [("bf16", 6), ("fp8", 11), ("int8", 7)])
def test_digit_bounds(kind, S):
    beta, head = ozaki.BETA[kind], ozaki.HEAD[kind]
    rng = np.random.default_rng(6)
    X = inputs.blocks(rng, 40, 50, "logspread")[0]
    # rows whose largest entry sits just below a power of two: the leading
    # digit reaches its bound 2^(beta - head)
    X[0] *= 0.5 / np.max(np.abs(X[0]))
    X[0, 3] = 1.0 - 2.0 ** -12
    X[1] *= 0.25 / np.max(np.abs(X[1]))
    X[1, 7] = -(0.5 - 2.0 ** -20)
    Q, e, rem = ozaki.digits(X, beta, S, 1, head)
    assert np.max(np.abs(Q[0])) == 2 ** (beta - head)
    for s in range(1, S):
        assert np.max(np.abs(Q[s])) <= 2 ** (beta - 1)
    assert np.max(np.abs(rem)) <= 2.0 ** (-beta * S - 1)
    # the digit types hold these integers exactly
    lim = {"bf16": 256, "fp8": 16, "int8": 127}[kind]
    assert max(np.max(np.abs(q)) for q in Q) <= lim


def test_fp8_digits_fit_e4m3():
    """FP8 digits (beta 5, one bit of headroom) are integers in [-16, 16],
    every one of which E4M3 (4 significant bits, exponent bias 7) holds
    exactly; without the headroom the leading digit could reach 32, and 17
    .. 31 are not E4M3 values."""
    e4m3_ints = set()
    for e in range(0, 9):                    # normal values 1.mmm x 2^e
        for mant in range(8):
            v = (8 + mant) * 2.0 ** (e - 3)
            if v == int(v):
                e4m3_ints.add(int(v))
    assert set(range(0, 17)) <= e4m3_ints | {0} and 17 not in e4m3_ints and 31 not in e4m3_ints
    X = np.array([[1.0 - 2.0 ** -12, 0.25, -0.7], [-0.75, 0.125, 0.5 - 2.0 ** -30]])
    Q, _, _ = ozaki.digits(X, ozaki.BETA["fp8"], 6, 1, ozaki.HEAD["fp8"])
    assert max(np.max(np.abs(q)) for q in Q) == 16
    assert all(abs(int(v)) in e4m3_ints | {0} for q in Q for v in q.ravel())
    Q0, _, _ = ozaki.digits(X, ozaki.BETA["fp8"], 2, 1, head=0)
    assert np.max(np.abs(Q0[0])) == 32


def test_int8_needs_headroom():
    """Without the headroom bit a leading INT8 digit of beta 7 can be 128,
    which a signed byte cannot hold; with it every digit fits."""
    X = np.array([[1.0 - 2.0 ** -12, 0.25], [-0.75, 0.125]])
    Q0, _, _ = ozaki.digits(X, 7, 3, 1, head=0)
    assert np.max(np.abs(Q0[0])) == 128
    Q1, _, _ = ozaki.digits(X, 7, 3, 1, head=ozaki.HEAD["int8"])
    assert max(np.max(np.abs(q)) for q in Q1) <= 127


@pytest.mark.parametrize("kind,S", [("bf16", 3), ("fp8", 5), ("int8", 3)])
def test_integer_products_exact(kind, S):
    """Integers of at most 10 bits need 2 (bf16, int8) or 3 (fp8) digits;
    with those pairs kept (S = 3 or 5: every pair of the needed digits has
    s + t <= S + 1) the split product is exact."""
    rng = np.random.default_rng(7)
    X = rng.integers(-512, 513, size=(30, 70)).astype(np.float64)
    Y = rng.integers(-512, 513, size=(70, 20)).astype(np.float64)
    ref = (X.astype(np.int64) @ Y.astype(np.int64)).astype(np.float64)
    assert np.array_equal(ozaki.product(X, Y, kind, S), ref)


@pytest.mark.parametrize("kind", ["bf16", "fp8", "int8"])
def test_convergence_rate(kind):
    """The error falls by about 2^-beta per added slice until FP64 rounding."""
    beta = ozaki.BETA[kind]
    rng = np.random.default_rng(8)
    X = rng.uniform(-1, 1, (48, 96))
    Y = rng.uniform(-1, 1, (96, 40))
    ref = X @ Y
    errs = []
    for S in range(2, 6):
        T = ozaki.product(X, Y, kind, S)
        errs.append(np.linalg.norm(T - ref) / np.linalg.norm(ref))
    for a, b in zip(errs, errs[1:]):
        assert b < a * 2.0 ** (-beta + 2), errs


@pytest.mark.parametrize("kind,S", KINDS)
def test_full_slices_match_fp64(kind, S):
    rng = np.random.default_rng(9)
    X = rng.standard_normal((40, 64))
    Y = rng.standard_normal((64, 30))
    ref = X @ Y
    T = ozaki.product(X, Y, kind, S)
    assert np.linalg.norm(T - ref) <= 1e-14 * np.linalg.norm(ref)


def test_zero_rows_and_columns():
    X = np.zeros((5, 7)); X[1] = np.arange(7) + 1.0
    Y = np.zeros((7, 4)); Y[:, 2] = 1.0
    assert np.array_equal(ozaki.product(X, Y, "bf16", 4), X @ Y)


def deepest_level_pair(kind, S):
    """A 1 x 2 times 2 x 1 product carried by one digit pair alone: the
    left row [0.75, x] puts x = 2^(h - beta S) in its last slice only, the
    right column [0, 2^-6] puts 2^-6 in its first slice, so the product
    x 2^-6 lives in level S + 1 (scale 2^-beta (S + 1)) and nowhere else."""
    beta, head = ozaki.BETA[kind], ozaki.HEAD[kind]
    X = np.array([[0.75, 2.0 ** (head - beta * S)]])
    Y = np.array([[0.0], [2.0 ** -6]])
    return X, Y


@pytest.mark.parametrize("kind,S", KINDS + [("bf16", 1), ("int8", 1)])
def test_deepest_level_is_kept(kind, S):
    X, Y = deepest_level_pair(kind, S)
    Qx, _, _ = ozaki.digits(X, ozaki.BETA[kind], S, axis=1, head=ozaki.HEAD[kind])
    col = [int(q[0, 1]) for q in Qx]
    assert col[:-1] == [0] * (S - 1) and col[-1] != 0
    T = ozaki.product(X, Y, kind, S)
    assert T[0, 0] == X[0, 1] * Y[1, 0] != 0.0

