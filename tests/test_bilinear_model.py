"""The bilinear model (tests/bilinear_model.py) against the oracle: pins the
reading of Sec. III A that the HIP kernels implement, and the 24 / 8 real
GEMM counts."""
import json
import os

import numpy as np
import pytest

import oracle
from bilinear_model import Counter, bilinear
from paper_2609_02081_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


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
