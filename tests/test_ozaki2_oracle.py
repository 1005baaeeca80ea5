"""Pins for the CRT-based split-form oracle (oracle/ozaki2.py): the moduli,
the bit budget they carry, residue recovery by the Chinese remainder
theorem, exact integer products, the rounding bound of the scaled integers,
and agreement with FP64 at the default modulus count."""
import math

import numpy as np
import pytest

from oracle import ozaki2


def test_moduli_pairwise_coprime_odd_and_byte_sized():
    P = ozaki2.MODULI
    assert all(p % 2 == 1 and p <= 255 for p in P)
    assert all(math.gcd(a, b) == 1 for i, a in enumerate(P) for b in P[i + 1:])
    for p in P:   # symmetric residues fit a signed byte
        r = ozaki2.residues(np.arange(-3 * p, 3 * p), p)
        assert r.min() == -(p - 1) // 2 and r.max() == (p - 1) // 2 <= 127


@pytest.mark.parametrize("n,k", [(14, 16384), (16, 16384), (16, 100), (20, 1 << 17)])
def test_bit_budget(n, k):
    """prod(p) > 2 k 2^(2b) holds for the returned b and fails for b + 1
    (unless b is capped at 53)."""
    b = ozaki2.bits_for(n, k)
    M = math.prod(ozaki2.MODULI[:n])
    assert M > 2 * k * (1 << (2 * b))
    if b < 53:
        assert M <= 2 * k * (1 << (2 * (b + 1)))


def test_default_count_carries_53_bits():
    for k in (64, 1000, 8192, 16384, 100000):
        n = ozaki2.default_moduli(k)
        assert ozaki2.bits_for(n, k) == 53 and (n == 1 or ozaki2.bits_for(n - 1, k) < 53)


def test_crt_recovers_integers():
    rng = np.random.default_rng(3)
    mods = ozaki2.MODULI[:16]
    M = math.prod(mods)
    for _ in range(200):
        x = int(rng.integers(-(1 << 62), 1 << 62)) * int(rng.integers(1, 1 << 50)) % M
        x = x - M if x > M // 2 else x
        res = [int(ozaki2.residues(np.array([x % p]), p)[0]) for p in mods]
        assert ozaki2.crt(res, mods) == x


def test_integer_products_exact():
    rng = np.random.default_rng(4)
    X = rng.integers(-1000, 1001, size=(17, 40)).astype(np.float64)
    Y = rng.integers(-1000, 1001, size=(40, 13)).astype(np.float64)
    assert np.array_equal(ozaki2.product(X, Y), X @ Y)


@pytest.mark.parametrize("n_moduli", [5, 7, 9])
def test_rounding_bound(n_moduli):
    """|T - XY|_ij <= k 2^(e_i + f_j - b): each scaled integer is within half
    a unit of 2^(e - b); with few moduli (small b) this bound dominates the
    FP64 rounding of the reference."""
    rng = np.random.default_rng(5)
    X = rng.standard_normal((12, 30))
    Y = rng.standard_normal((30, 9))
    k = X.shape[1]
    b = ozaki2.bits_for(n_moduli, k)
    assert 5 < b < 40
    T = ozaki2.product(X, Y, n_moduli)
    e = ozaki2.exponents(X, 1)
    f = ozaki2.exponents(Y, 0)
    bound = k * np.ldexp(1.0, (e[:, None] + f[None, :] - b).astype(int))
    assert np.all(np.abs(T - X @ Y) <= bound)
    # and the error is not far below it either: the bits are really dropped
    assert np.max(np.abs(T - X @ Y) / bound) > 1e-3


def test_default_matches_fp64():
    rng = np.random.default_rng(6)
    X = rng.standard_normal((20, 64))
    Y = rng.standard_normal((64, 15))
    ref = X @ Y
    assert np.linalg.norm(ozaki2.product(X, Y) - ref) <= 1e-15 * np.linalg.norm(ref)


def test_convergence_with_moduli():
    rng = np.random.default_rng(7)
    X = rng.uniform(-1, 1, (16, 48))
    Y = rng.uniform(-1, 1, (48, 12))
    ref = X @ Y
    errs = [np.linalg.norm(ozaki2.product(X, Y, n) - ref) / np.linalg.norm(ref) for n in (6, 8, 10, 12)]
    for a, b in zip(errs, errs[1:]):
        assert b < a * 2.0 ** -6   # two more moduli: ~16 more bits of M, ~8 of b
