"""Split-precision (Ozaki-style) path on the GPU, through the C-ABI.

* Integer inputs whose digits fit the kept slices: bit-exact with the oracle.
* Random inputs: equal to the CPU split model (tests/bilinear_model.py with
  oracle/ozaki.py as the real GEMM: the same digits and pairs, exact digit
  products) to 1e-14 relative, the two differing only in FP64 summation order.
* At the default slice counts: relative Frobenius error <= 1e-12 against the
  FP64 oracle (uniform and log-spread inputs, n = 256 and sampled n = 8192).
"""
import numpy as np
import pytest

import oracle
from bilinear_model import Counter, bilinear
from oracle import ozaki
from paper_2609_02081_amd import inputs

pytestmark = pytest.mark.gpu
TOL = 1e-12
PRECS = {"bf16": "split_bf16", "fp8": "split_fp8", "int8": "split_int8"}


@pytest.fixture(scope="module")
def bq():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_02081_amd as bq

    bq.lib()
    return bq


def run(bq, A, B, kind, S, **kw):
    import torch

    C = bq.bq_gemm(torch.from_numpy(A).to("cuda"), torch.from_numpy(B).to("cuda"), prec=PRECS[kind],
                   slices=S, **kw)
    torch.cuda.synchronize()
    return C.cpu().numpy()


@pytest.mark.parametrize("kind,S", [("bf16", 4), ("fp8", 6), ("int8", 4)])
def test_integer_bit_exact(bq, kind, S):
    A, B = inputs.pair(96, 80, 72, "int", seed=12, bound=64)
    print(f"split {kind} S={S} integer", flush=True)
    assert np.array_equal(run(bq, A, B, kind, S), oracle.gemm(A, B))


@pytest.mark.parametrize("kind,S", [("bf16", 1), ("bf16", 3), ("bf16", 6), ("bf16", 8), ("fp8", 1), ("fp8", 5),
                                    ("fp8", 9), ("fp8", 12), ("fp8", 13), ("int8", 1), ("int8", 4), ("int8", 7),
                                    ("int8", 9)])
def test_matches_cpu_split_model(bq, kind, S):
    """The slice GEMM of each digit type against the CPU split model, from
    one slice up to the most each type is built for (INT8 at 9 slices
    scales its last level by 2^-70); ragged shape."""
    A, B = inputs.pair(130, 100, 70, "uniform", seed=13)
    print(f"split {kind} S={S} vs model", flush=True)
    ref = bilinear(A, B, Counter(lambda x, y: ozaki.product(x, y, kind, S)))
    got = run(bq, A, B, kind, S)
    assert oracle.rel_frobenius(got, ref) <= 1e-14


@pytest.mark.parametrize("kind,S", [("bf16", 8), ("fp8", 13), ("int8", 9), ("int8", 1)])
def test_deepest_level_scale(bq, kind, S):
    """A real product carried by one digit pair alone, slice S of the left
    operand with slice 1 of the right (level S + 1, scale 2^-beta (S + 1):
    2^-63 for BF16, 2^-70 for FP8 at 13 and INT8 at 9 slices): the left row
    [0.75, 2^(h - beta S)], the right column [0, 2^-6].  The result is the
    exact product, so a level dropped or scaled wrong shows."""
    import torch

    beta, head = ozaki.BETA[kind], ozaki.HEAD[kind]
    A = np.zeros((8, 1, 2))
    A[0, 0] = [0.75, 2.0 ** (head - beta * S)]
    B = np.zeros((8, 2, 1))
    B[0, :, 0] = [0.0, 2.0 ** -6]
    C = bq.bq_gemm(torch.from_numpy(A).to("cuda"), torch.from_numpy(B).to("cuda"), prec=PRECS[kind], slices=S,
                   mask_a=0x01, mask_b=0x01)
    torch.cuda.synchronize()
    got = C.cpu().numpy()
    assert got[0, 0, 0] == A[0, 0, 1] * B[0, 1, 0], (got[0, 0, 0], A[0, 0, 1] * B[0, 1, 0])
    assert not np.any(got[1:])


@pytest.mark.parametrize("flush", ["1", "3"])
@pytest.mark.parametrize("kind,S", [("bf16", 8), ("fp8", 9), ("int8", 8), ("int8", 9)])
def test_level_flush_interval(bq, kind, S, flush, monkeypatch):
    """Level sums kept across k-steps and flushed every 1 or 3 k-steps (K =
    700: several flushes and a partial last interval) against the model."""
    monkeypatch.setenv("BQ_SLICE_FLUSH", flush)
    A, B = inputs.pair(40, 700, 36, "logspread", seed=16)
    print(f"split {kind} S={S} flush {flush} vs model", flush=True)
    ref = bilinear(A, B, Counter(lambda x, y: ozaki.product(x, y, kind, S)))
    assert oracle.rel_frobenius(run(bq, A, B, kind, S), ref) <= 1e-14


@pytest.mark.parametrize("kind", ["bf16", "fp8", "int8"])
@pytest.mark.parametrize("dist", ["uniform", "logspread"])
def test_default_slices_accuracy(bq, kind, dist):
    A, B = inputs.pair(256, 256, 256, dist, seed=4)
    err = oracle.rel_frobenius(run(bq, A, B, kind, 0), oracle.gemm(A, B))
    print(f"split {kind} default S, {dist}: rel err {err:.3e}", flush=True)
    assert err <= TOL


OP_FN = {"N": lambda M: M, "T": oracle.transpose, "C": oracle.conj, "H": oracle.herm}


@pytest.mark.parametrize("kind,S,opA,opB", [("bf16", 4, "T", "H"), ("int8", 4, "H", "T"), ("fp8", 6, "T", "N")])
def test_transposed_ops_integer_bit_exact(bq, kind, S, opA, opB):
    """op T / H in the split form: exponents per row of op(A) and per column
    of op(B) taken along the stored layout's other dimension."""
    rng = np.random.default_rng(17)
    m, k, n = 96, 80, 72
    A = inputs.blocks(rng, *((k, m) if opA in "TH" else (m, k)), "int", bound=64)
    B = inputs.blocks(rng, *((n, k) if opB in "TH" else (k, n)), "int", bound=64)
    print(f"split {kind} S={S} ops {opA}{opB} integer", flush=True)
    got = run(bq, A, B, kind, S, opA=opA, opB=opB)
    assert np.array_equal(got, oracle.gemm(OP_FN[opA](A), OP_FN[opB](B)))


@pytest.mark.parametrize("kind,S", [("bf16", 7), ("int8", 7), ("fp8", 10)])
def test_transposed_ops_match_cpu_split_model(bq, kind, S):
    rng = np.random.default_rng(18)
    m, k, n = 130, 100, 70
    A = inputs.blocks(rng, k, m, "logspread")   # stored for op H
    B = inputs.blocks(rng, n, k, "logspread")   # stored for op T
    print(f"split {kind} S={S} ops HT vs model", flush=True)
    ref = bilinear(oracle.herm(A), oracle.transpose(B), Counter(lambda x, y: ozaki.product(x, y, kind, S)))
    assert oracle.rel_frobenius(run(bq, A, B, kind, S, opA="H", opB="T"), ref) <= 1e-14


@pytest.mark.parametrize("kind", ["bf16", "int8"])
def test_conj_and_masks(bq, kind):
    A, B = inputs.pair(90, 70, 60, "normal", seed=14)
    got = run(bq, A, B, kind, 0, opA="C")
    assert oracle.rel_frobenius(got, oracle.gemm(oracle.conj(A), B)) <= TOL
    for name in ("real_quaternion", "complex", "real"):
        mask = inputs.MASKS[name]
        Am, Bm = inputs.pair(90, 70, 60, "normal", seed=15, mask_a=mask, mask_b=mask)
        got = run(bq, Am, Bm, kind, 0, mask_a=mask, mask_b=mask)
        assert oracle.rel_frobenius(got, oracle.gemm(Am, Bm)) <= TOL, name


def _sample(n, r, seed):
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(n - 1, size=r - 1, replace=False))
    return np.append(idx, n - 1)


@pytest.mark.parametrize("kind", ["bf16", "int8", "fp8"])
@pytest.mark.parametrize("dist", ["uniform", "logspread"])
def test_n8192_sampled(bq, kind, dist):
    import torch

    n, r = 8192, 48
    rng = np.random.default_rng(4)
    print(f"split n=8192 {kind} {dist}: inputs", flush=True)
    if dist == "uniform":
        A = inputs.device_uniform(n, n, 41, "cuda")
        B = inputs.device_uniform(n, n, 42, "cuda")
    else:
        A = torch.from_numpy(inputs.blocks(rng, n, n, "logspread")).to("cuda")
        B = torch.from_numpy(inputs.blocks(rng, n, n, "logspread")).to("cuda")
    C = bq.bq_gemm(A, B, prec=PRECS[kind])
    torch.cuda.synchronize()
    rows, cols = _sample(n, r, 51), _sample(n, r, 52)
    ri, ci = torch.as_tensor(rows, device="cuda"), torch.as_tensor(cols, device="cuda")
    As, Bs = A[:, ri, :].cpu().numpy(), B[:, :, ci].cpu().numpy()
    Cs = C[:, ri][:, :, ci].cpu().numpy()
    err = oracle.rel_frobenius(Cs, oracle.gemm(As, Bs))
    print(f"split n=8192 {kind} {dist}: sampled rel err {err:.3e}", flush=True)
    assert err <= TOL


@pytest.mark.parametrize("kind", ["bf16", "int8", "fp8"])
@pytest.mark.parametrize("dist", ["uniform", "logspread"])
def test_n16384_default_slices_sampled(bq, kind, dist):
    """The library's default slice count at the benchmark size (k = 16384:
    BF16 8, FP8 12, INT8 8 slices) against the FP64 oracle on 40 x 40
    sampled entries (the last row and column included), <= 1e-12."""
    import torch

    n, r = 16384, 40
    print(f"split n=16384 {kind} {dist}: inputs", flush=True)
    gen = inputs.device_uniform if dist == "uniform" else inputs.device_logspread
    A = gen(n, n, 61, "cuda")
    B = gen(n, n, 62, "cuda")
    C = bq.bq_gemm(A, B, prec=PRECS[kind], slices=0)
    torch.cuda.synchronize()
    rows, cols = _sample(n, r, 63), _sample(n, r, 64)
    ri, ci = torch.as_tensor(rows, device="cuda"), torch.as_tensor(cols, device="cuda")
    As, Bs = A[:, ri, :].cpu().numpy(), B[:, :, ci].cpu().numpy()
    Cs = C[:, ri][:, :, ci].cpu().numpy()
    del A, B, C
    torch.cuda.empty_cache()
    err = oracle.rel_frobenius(Cs, oracle.gemm(As, Bs))
    print(f"split n=16384 {kind} {dist}: default slices, sampled rel err {err:.3e}", flush=True)
    assert err <= TOL
