"""Grouped CRT plans on the GPU: every stage of every problem of a batch in
one launch per complex product (exponents, residues, residue GEMMs,
reconstruction), through the C-ABI.

The grouped launches run the same arithmetic as a single call, so each
product must equal the single-call CRT result bit for bit (same modulus
count per problem, same exponents, exact residue GEMMs, the same
reconstruction), and lie within the tolerance of the oracle.  The batches
mix modulus counts (the default count depends on k: 14 moduli at k = 1, 15
up to k = 1024, 16 beyond), op pairs, component masks whose plans leave
output components structurally zero, and empty problems (k = 0, m = 0).
"""
import numpy as np
import pytest

import oracle
from paper_2609_02081_amd import inputs

pytestmark = pytest.mark.gpu
TOL = 1e-12
PREC = "split_int8_crt"


@pytest.fixture(scope="module")
def bq():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_02081_amd as bq

    bq.lib()
    return bq


OP_FN = {"N": lambda M: M, "T": oracle.transpose, "C": oracle.conj, "H": oracle.herm}


def _problem(rng, m, k, n, oa="N", ob="N", mask_a=0xFF, mask_b=0xFF):
    import torch

    a = inputs.blocks(rng, *((k, m) if oa in "TH" else (m, k)), mask=mask_a)
    b = inputs.blocks(rng, *((n, k) if ob in "TH" else (k, n)), mask=mask_b)
    A = torch.from_numpy(a).to("cuda")
    B = torch.from_numpy(b).to("cuda")
    As = [A[c] if mask_a >> c & 1 else None for c in range(8)]
    Bs = [B[c] if mask_b >> c & 1 else None for c in range(8)]
    C = torch.full((8, m, n), float("nan"), dtype=torch.float64, device="cuda")
    return {"A": As, "B": Bs, "C": C, "oa": oa, "ob": ob, "a": a, "b": b, "shape": (m, k, n),
            "masks": (mask_a, mask_b)}


def _check(bq, probs, slices=0, oracle_check=True):
    import torch

    plan = bq.GroupedPlan([(p["A"], p["B"], p["C"], p["oa"], p["ob"]) for p in probs], prec=PREC,
                          slices=slices)
    print(f"grouped CRT batch of {len(probs)}: {plan.info()}, workspace {plan.workspace_size() / 2**20:.1f} MiB",
          flush=True)
    plan.launch()
    torch.cuda.synchronize()
    for p in probs:
        got = p["C"].cpu().numpy()
        single = bq.bq_gemm(p["A"], p["B"], opA=p["oa"], opB=p["ob"], prec=PREC, slices=slices)
        torch.cuda.synchronize()
        assert np.array_equal(got, single.cpu().numpy(), equal_nan=True), (p["shape"], p["oa"], p["ob"], p["masks"])
        if oracle_check and got.size:
            ref = oracle.gemm(OP_FN[p["oa"]](p["a"]), OP_FN[p["ob"]](p["b"]))
            assert oracle.rel_frobenius(got, ref) <= TOL, (p["shape"], p["oa"], p["ob"], p["masks"])
    return plan


def test_mixed_batch_bit_identical_to_single_calls(bq):
    rng = np.random.default_rng(81)
    specs = [
        ((17, 1, 9), "N", "N", 0xFF, 0xFF),        # 14 moduli
        ((64, 64, 64), "T", "N", 0xFF, 0xFF),      # 15
        ((130, 70, 129), "N", "H", 0xFF, 0xFF),
        ((200, 1536, 90), "N", "N", 0xFF, 0xFF),   # 16
        ((1, 5, 1), "C", "C", 0xFF, 0xFF),
        ((96, 200, 33), "H", "T", 0xFF, 0xFF),
        ((65, 65, 65), "N", "N", 0x0F, 0x0F),      # real quaternion: c5..c8 structurally zero
        ((40, 90, 70), "N", "N", 0x11, 0x11),      # complex
        ((33, 47, 29), "N", "N", 0x01, 0x01),      # real
        ((50, 60, 70), "N", "N", 0xF0, 0xF0),      # imaginary parts only
        ((70, 40, 50), "T", "N", 0x0F, 0xFF),      # real quaternion x biquaternion
        ((5, 0, 7), "N", "N", 0xFF, 0xFF),         # k = 0: C = 0
        ((0, 10, 4), "N", "N", 0xFF, 0xFF),        # m = 0: nothing
        ((257, 300, 31), "N", "T", 0xFF, 0xFF),
    ]
    probs = [_problem(rng, *shape, oa, ob, ma, mb) for (shape, oa, ob, ma, mb) in specs]
    _check(bq, probs).close()


def test_explicit_modulus_count(bq):
    rng = np.random.default_rng(82)
    probs = [_problem(rng, 48, 100, 52), _problem(rng, 130, 257, 70, "H", "N"), _problem(rng, 3, 4, 5)]
    # 9 moduli carry fewer bits: compare with single calls only
    _check(bq, probs, slices=9, oracle_check=False).close()
    _check(bq, probs, slices=20).close()


def test_uneven_batch_of_48(bq):
    rng = np.random.default_rng(83)
    sizes = inputs.batch_sizes(48, 64, 768, seed=84)
    probs = [_problem(rng, s, s, s) for s in sizes]
    _check(bq, probs, oracle_check=False).close()
    # the oracle on the three smallest
    for p in sorted(probs, key=lambda p: p["shape"][0])[:3]:
        ref = oracle.gemm(p["a"], p["b"])
        assert oracle.rel_frobenius(p["C"].cpu().numpy(), ref) <= TOL


def test_replays_identical_with_eager_work_between(bq):
    import torch

    rng = np.random.default_rng(85)
    probs = [_problem(rng, 100, 130, 90), _problem(rng, 64, 1, 64), _problem(rng, 33, 200, 17, "T", "H"),
             _problem(rng, 20, 30, 40, mask_a=0x0F, mask_b=0x0F)]
    plan = _check(bq, probs, oracle_check=False)
    first = [p["C"].cpu().numpy().copy() for p in probs]
    x = torch.randn(512, 512, dtype=torch.float64, device="cuda")
    for rep in range(3):
        for p in probs:
            p["C"].fill_(float("nan"))
        y = (x @ x).sum()  # unrelated eager work between replays
        plan.launch()
        torch.cuda.synchronize()
        assert torch.isfinite(y)
        for p, f in zip(probs, first):
            assert np.array_equal(p["C"].cpu().numpy(), f, equal_nan=True), rep
    plan.close()


def test_non_finite_and_long_k(bq):
    """NaN and infinity in some rows of A and columns of B (their exponents
    carry the non-finite marker through the atomic-free exponent kernel, so
    the rows / columns they touch come out NaN as in a single call), and a
    long reduced dimension (k = 20000: column exponents over 20000 rows in
    one block, 313 k-steps per residue GEMM block) in the same batch as
    small products."""
    import torch

    rng = np.random.default_rng(86)
    p1 = _problem(rng, 40, 50, 30)
    p1["A"][0][3, 7] = float("nan")
    p1["A"][5][11, 0] = float("inf")
    p1["B"][2][9, 4] = float("-inf")
    p2 = _problem(rng, 24, 33, 18, "T", "H")
    p2["B"][7][1, 2] = float("nan")
    p3 = _problem(rng, 64, 20000, 48)
    p4 = _problem(rng, 70, 90, 60)
    probs = [p1, p2, p3, p4]
    for p in (p1, p2):  # the host copies follow the device edits
        p["a"] = np.stack([t.cpu().numpy() if t is not None else np.zeros_like(p["a"][0]) for t in p["A"]])
        p["b"] = np.stack([t.cpu().numpy() if t is not None else np.zeros_like(p["b"][0]) for t in p["B"]])
    plan = _check(bq, probs, oracle_check=False)
    plan.close()
    c1 = p1["C"].cpu().numpy()
    assert np.isnan(c1[:, 3, :]).any() and np.isnan(c1[:, :, 4]).any()
    assert np.isfinite(c1[:, [0, 1, 2], :][:, :, [0, 1, 2]]).all()
    for p in (p3, p4):
        ref = oracle.gemm(p["a"], p["b"])
        assert oracle.rel_frobenius(p["C"].cpu().numpy(), ref) <= TOL


def test_smallest_problem_with_fewest_products(bq):
    """Problems are recorded largest first; the last ones here have plans
    with fewer complex products than the first (real: one; complex: one;
    real quaternion: eight real products), so every round of the largest
    plan must still be launched."""
    rng = np.random.default_rng(87)
    probs = [_problem(rng, 96, 80, 72), _problem(rng, 40, 30, 20, mask_a=0x0F, mask_b=0x0F),
             _problem(rng, 12, 10, 9, mask_a=0x11, mask_b=0x11), _problem(rng, 8, 8, 8, mask_a=0x01, mask_b=0x01)]
    _check(bq, probs).close()
