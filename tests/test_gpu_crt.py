"""CRT-based split form (Ozaki scheme II) on the GPU, through the C-ABI.

Each real product of this form is the correctly rounded value of the product
of the scaled integers (the residues are reduced exactly and P is rounded to
FP64 once), so:

* one real product (masks with only the real unit component): bit-exact with
  oracle/ozaki2.product, which forms P with Python integers;
* integer inputs: bit-exact with the FP64 oracle (nothing rounds);
* random biquaternions: equal to the CPU split model (the bilinear scheme
  with ozaki2.product as the real GEMM) to 1e-14 relative, the two differing
  only in the FP64 order of the pre- and post-combination sums;
* default moduli: relative Frobenius error <= 1e-12 against the FP64 oracle.
"""
import numpy as np
import pytest

import oracle
from bilinear_model import Counter, bilinear
from oracle import ozaki2
from paper_2609_02081_amd import inputs

pytestmark = pytest.mark.gpu
TOL = 1e-12
PREC = "split_int8_crt"
OP_FN = {"N": lambda M: M, "T": oracle.transpose, "C": oracle.conj, "H": oracle.herm}


@pytest.fixture(scope="module")
def bq():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_02081_amd as bq

    bq.lib()
    return bq


def run(bq, A, B, N=0, **kw):
    import torch

    C = bq.bq_gemm(torch.from_numpy(A).to("cuda"), torch.from_numpy(B).to("cuda"), prec=PREC, slices=N, **kw)
    torch.cuda.synchronize()
    return C.cpu().numpy()


@pytest.mark.parametrize("tile", ["128", "256"])
@pytest.mark.parametrize("dist", ["uniform", "logspread", "normal"])
@pytest.mark.parametrize("N", [0, 9, 20])
def test_real_product_bit_exact(bq, dist, N, tile, monkeypatch):
    """m, k, n = 300, 200, 70 with either residue-GEMM block: several row
    tiles with a ragged last one, ragged columns, k two 128-steps with a
    ragged tail: every element equal to the oracle's."""
    monkeypatch.setenv("BQ_CRT_TILE", tile)
    R = inputs.MASKS["real"]
    A, B = inputs.pair(300, 200, 70, dist, seed=60, mask_a=R, mask_b=R)
    print(f"crt real product {dist} N={N} tile {tile}", flush=True)
    got = run(bq, A, B, N, mask_a=R, mask_b=R)
    assert np.array_equal(got[0], ozaki2.product(A[0], B[0], N))
    assert not np.any(got[1:])


@pytest.mark.parametrize("N", [2, 4, 6])
def test_few_moduli_bit_exact(bq, N):
    """Few moduli carry few bits: the rounding of the inputs to b-bit
    integers dominates and must match the oracle exactly."""
    R = inputs.MASKS["real"]
    A, B = inputs.pair(40, 64, 33, "uniform", seed=61, mask_a=R, mask_b=R)
    assert ozaki2.bits_for(N, 64) >= 1
    got = run(bq, A, B, N, mask_a=R, mask_b=R)
    assert np.array_equal(got[0], ozaki2.product(A[0], B[0], N))


def test_integer_bit_exact(bq):
    A, B = inputs.pair(96, 80, 72, "int", seed=62, bound=64)
    print("crt integer", flush=True)
    assert np.array_equal(run(bq, A, B), oracle.gemm(A, B))


@pytest.mark.parametrize("tile", ["128", "256"])
@pytest.mark.parametrize("N", [0, 12])
def test_matches_cpu_split_model(bq, N, tile, monkeypatch):
    monkeypatch.setenv("BQ_CRT_TILE", tile)
    A, B = inputs.pair(70, 60, 50, "logspread", seed=63)
    print(f"crt N={N} vs model", flush=True)
    ref = bilinear(A, B, Counter(lambda x, y: ozaki2.product(x, y, N)))
    assert oracle.rel_frobenius(run(bq, A, B, N), ref) <= 1e-14


@pytest.mark.parametrize("dist", ["uniform", "logspread"])
def test_default_moduli_accuracy(bq, dist):
    A, B = inputs.pair(256, 256, 256, dist, seed=4)
    err = oracle.rel_frobenius(run(bq, A, B), oracle.gemm(A, B))
    print(f"crt default moduli, {dist}: rel err {err:.3e}", flush=True)
    assert err <= TOL


@pytest.mark.parametrize("opA,opB", [("T", "H"), ("H", "N"), ("N", "T"), ("C", "C")])
def test_ops_integer_bit_exact(bq, opA, opB):
    rng = np.random.default_rng(64)
    m, k, n = 96, 80, 72
    A = inputs.blocks(rng, *((k, m) if opA in "TH" else (m, k)), "int", bound=64)
    B = inputs.blocks(rng, *((n, k) if opB in "TH" else (k, n)), "int", bound=64)
    print(f"crt ops {opA}{opB} integer", flush=True)
    got = run(bq, A, B, opA=opA, opB=opB)
    assert np.array_equal(got, oracle.gemm(OP_FN[opA](A), OP_FN[opB](B)))


def test_ops_match_cpu_split_model(bq):
    rng = np.random.default_rng(65)
    m, k, n = 70, 60, 50
    A = inputs.blocks(rng, k, m, "logspread")   # stored for op H
    B = inputs.blocks(rng, n, k, "logspread")   # stored for op T
    ref = bilinear(oracle.herm(A), oracle.transpose(B), Counter(lambda x, y: ozaki2.product(x, y, 0)))
    assert oracle.rel_frobenius(run(bq, A, B, opA="H", opB="T"), ref) <= 1e-14


@pytest.mark.parametrize("mask", [0x0F, 0x11, 0x5A, 0x0E])
def test_masks(bq, mask):
    A, B = inputs.pair(90, 70, 60, "normal", seed=66, mask_a=mask, mask_b=mask)
    got = run(bq, A, B, mask_a=mask, mask_b=mask)
    assert oracle.rel_frobenius(got, oracle.gemm(A, B)) <= TOL


def test_zero_rows_columns_and_degenerate_shapes(bq):
    """A zero row of A and a zero column of B (no exponent) give zero rows
    and columns of the product; k = 1; k = 0 writes zeros."""
    R = inputs.MASKS["real"]
    A, B = inputs.pair(33, 65, 17, "uniform", seed=67, mask_a=R, mask_b=R)
    A[0, 5, :] = 0.0
    B[0, :, 3] = 0.0
    got = run(bq, A, B, mask_a=R, mask_b=R)
    assert np.array_equal(got[0], ozaki2.product(A[0], B[0]))
    assert not np.any(got[0][5, :]) and not np.any(got[0][:, 3])
    A1, B1 = inputs.pair(7, 1, 9, "uniform", seed=68)
    assert oracle.rel_frobenius(run(bq, A1, B1), oracle.gemm(A1, B1)) <= 1e-14
    A0, B0 = np.zeros((8, 5, 0)), np.zeros((8, 0, 6))
    assert not np.any(run(bq, A0, B0))


@pytest.mark.parametrize("tile", ["128", "256"])
def test_int32_sums_at_max_k(bq, tile, monkeypatch):
    """k = 133120, the largest k the form takes: every row of A and column of
    B equals 251/256, whose scaled integer 251 2^45 is 127 modulo 255, so the
    INT8 GEMM of that modulus sums k 127^2 = 2147092480 (just under 2^31).
    The product k (251/256)^2 is exact in FP64."""
    import torch

    monkeypatch.setenv("BQ_CRT_TILE", tile)
    k = 133120
    x = 251.0 / 256.0
    A = torch.zeros((8, 4, k), dtype=torch.float64, device="cuda")
    B = torch.zeros((8, k, 4), dtype=torch.float64, device="cuda")
    A[0].fill_(x)
    B[0].fill_(x)
    R = inputs.MASKS["real"]
    print("crt k=133120 worst-case int32 sums", flush=True)
    C = bq.bq_gemm(A, B, mask_a=R, mask_b=R, prec=PREC)
    torch.cuda.synchronize()
    assert torch.all(C[0] == k * x * x).item()
    assert ozaki2.residues(np.array([251 << 45]), 255)[0] == 127


def _sample(n, r, seed):
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(n - 1, size=r - 1, replace=False))
    return np.append(idx, n - 1)


@pytest.mark.parametrize("dist", ["uniform", "logspread"])
def test_n8192_sampled(bq, dist):
    """Default block choice (256 x 256 at this size)."""
    import torch

    n, r = 8192, 48
    rng = np.random.default_rng(4)
    print(f"crt n=8192 {dist}: inputs", flush=True)
    if dist == "uniform":
        A = inputs.device_uniform(n, n, 41, "cuda")
        B = inputs.device_uniform(n, n, 42, "cuda")
    else:
        A = torch.from_numpy(inputs.blocks(rng, n, n, "logspread")).to("cuda")
        B = torch.from_numpy(inputs.blocks(rng, n, n, "logspread")).to("cuda")
    C = bq.bq_gemm(A, B, prec=PREC)
    torch.cuda.synchronize()
    rows, cols = _sample(n, r, 51), _sample(n, r, 52)
    ri, ci = torch.as_tensor(rows, device="cuda"), torch.as_tensor(cols, device="cuda")
    As, Bs = A[:, ri, :].cpu().numpy(), B[:, :, ci].cpu().numpy()
    Cs = C[:, ri][:, :, ci].cpu().numpy()
    err = oracle.rel_frobenius(Cs, oracle.gemm(As, Bs))
    print(f"crt n=8192 {dist}: sampled rel err {err:.3e}", flush=True)
    assert err <= TOL


def test_real_product_n8192_sampled_bit_exact(bq):
    """At n = 8192 with the default 15 moduli (k = 8192), sampled elements of
    one real product equal the oracle's exactly."""
    import torch

    n, r = 8192, 6
    R = inputs.MASKS["real"]
    A = inputs.device_uniform(n, n, 43, "cuda")
    B = inputs.device_uniform(n, n, 44, "cuda")
    C = bq.bq_gemm(A, B, mask_a=R, mask_b=R, prec=PREC)
    torch.cuda.synchronize()
    rows, cols = _sample(n, r, 53), _sample(n, r, 54)
    ri, ci = torch.as_tensor(rows, device="cuda"), torch.as_tensor(cols, device="cuda")
    X = A[0][ri, :].cpu().numpy()
    Y = B[0][:, ci].cpu().numpy()
    # the exponents are per whole row of A and column of B: the sampled rows
    # and columns carry theirs, so the sampled product is the full product's
    want = ozaki2.product(X, Y, ozaki2.default_moduli(n))
    assert np.array_equal(C[0][ri][:, ci].cpu().numpy(), want)


@pytest.mark.parametrize("prec", ["split_int8_crt", "split_int8", "split_bf16", "split_fp8"])
@pytest.mark.parametrize("bad", [np.nan, np.inf])
def test_non_finite_propagation(bq, prec, bad):
    """A NaN or infinity in row 11 of A (component 7) and column 5 of B
    (component 2) makes row 11 and column 5 of every output component NaN,
    as in the FP64 path (there an infinity can also give +-inf); the rest
    stays finite and matches the oracle."""
    import torch

    A, B = inputs.pair(40, 40, 40, "uniform", seed=10)
    A[6, 11, 3] = bad
    B[1, 7, 5] = bad
    C = bq.bq_gemm(torch.from_numpy(A).to("cuda"), torch.from_numpy(B).to("cuda"), prec=prec)
    torch.cuda.synchronize()
    C = C.cpu().numpy()
    assert np.all(np.isnan(C[:, 11, :])) and np.all(np.isnan(C[:, :, 5]))
    rest = np.delete(np.delete(C, 11, axis=1), 5, axis=2)
    assert np.all(np.isfinite(rest))
    A2, B2 = A.copy(), B.copy()
    A2[6, 11, 3] = 0.0
    B2[1, 7, 5] = 0.0
    ref = np.delete(np.delete(oracle.gemm(A2, B2), 11, axis=1), 5, axis=2)
    assert oracle.rel_frobenius(rest, ref) <= TOL


def test_n24576_hermitian_sampled(bq):
    """n = 24576 in the CRT form (one FP64 block is 4.8 GB > 2^32 bytes, one
    residue plane 604 MB, the residue GEMM offsets run past 2^32): Fock-like
    A times density-like B against the oracle on sampled rows and columns
    that include the last ones."""
    import torch

    n = 24576
    print(f"crt n={n}: building Hermitian inputs on the device", flush=True)
    A, B = inputs.hermitian_pair(n, 3, "cuda")
    torch.cuda.empty_cache()  # the builder's temporaries, before the workspace
    C = bq.bq_gemm(A, B, prec=PREC)
    torch.cuda.synchronize()
    print(f"crt n={n}: product done", flush=True)
    r = 48
    rows, cols = _sample(n, r, 33), _sample(n, r, 34)
    ri, ci = torch.as_tensor(rows, device="cuda"), torch.as_tensor(cols, device="cuda")
    As = A[:, ri, :].cpu().numpy()
    Bs = B[:, :, ci].cpu().numpy()
    Cs = C[:, ri][:, :, ci].cpu().numpy()
    del A, B, C
    torch.cuda.empty_cache()
    err = oracle.rel_frobenius(Cs, oracle.gemm(As, Bs))
    print(f"crt n={n}: sampled rel err {err:.3e}", flush=True)
    assert err <= TOL
