"""Parity of the HIP path (through the C-ABI) with the CPU oracle.

Tolerance: relative Frobenius error over all eight blocks <= 1e-12 for
random FP64 inputs (the accuracy target stated for the FP64 path); bit
equality wherever every intermediate is an exactly representable integer
(integer inputs, unit blocks).
"""
import numpy as np
import pytest

import oracle
from paper_2609_02081_amd import inputs

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def bq():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_02081_amd as bq

    bq.lib()
    return bq


def dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def run(bq, A, B, **kw):
    import torch

    C = bq.bq_gemm(dev(A), dev(B), **kw)
    torch.cuda.synchronize()
    return C.cpu().numpy()


@pytest.mark.parametrize("m,k,n", [(256, 256, 256), (70, 50, 45), (1, 1, 1), (130, 257, 67),
                                   (200, 16, 300), (64, 1000, 33)])
def test_random_uniform(bq, m, k, n):
    A, B = inputs.pair(m, k, n, "uniform", seed=1)
    print(f"random uniform m={m} k={k} n={n}", flush=True)
    C = run(bq, A, B)
    assert oracle.rel_frobenius(C, oracle.gemm(A, B)) <= TOL


@pytest.mark.parametrize("m,k,n", [(64, 64, 64), (70, 50, 45), (129, 96, 130)])
def test_integer_bit_exact(bq, m, k, n):
    A, B = inputs.pair(m, k, n, "int", seed=7, bound=1024)
    print(f"integer m={m} k={k} n={n}", flush=True)
    assert np.array_equal(run(bq, A, B), oracle.gemm(A, B))


def test_unit_blocks_bit_exact(bq):
    n = 48
    for u in range(8):
        for v in range(8):
            A = np.zeros((8, n, n)); A[u] = np.eye(n)
            B = np.zeros((8, n, n)); B[v] = np.eye(n)
            assert np.array_equal(run(bq, A, B), oracle.gemm(A, B)), (u, v)


OP_FN = {"N": lambda M: M, "T": oracle.transpose, "C": oracle.conj, "H": oracle.herm}


def stored_pair(m, k, n, opA, opB, dist, seed, **kw):
    """Stored operands for op(A) (m x k) and op(B) (k x n): T and H store
    the transpose (A k x m, B n x k)."""
    rng = np.random.default_rng(seed)
    A = inputs.blocks(rng, *((k, m) if opA in "TH" else (m, k)), dist, **kw)
    B = inputs.blocks(rng, *((n, k) if opB in "TH" else (k, n)), dist, **kw)
    return A, B


@pytest.mark.parametrize("opA", ["N", "T", "C", "H"])
@pytest.mark.parametrize("opB", ["N", "T", "C", "H"])
def test_all_ops(bq, opA, opB):
    """Every op pair (Sec. III sign rules for T, * and dagger), the oracle
    applying its own op to the stored operands; ragged shape."""
    A, B = stored_pair(96, 80, 72, opA, opB, "normal", seed=3)
    print(f"ops {opA}{opB}", flush=True)
    ref = oracle.gemm(OP_FN[opA](A), OP_FN[opB](B))
    assert oracle.rel_frobenius(run(bq, A, B, opA=opA, opB=opB), ref) <= TOL


@pytest.mark.parametrize("opA,opB", [("T", "N"), ("N", "H"), ("H", "T")])
def test_transposed_ops_integer_bit_exact(bq, opA, opB):
    """Integer inputs through the transposed loads: bit-exact; odd stored
    leading dimensions and ragged edges (unaligned and checked load paths)."""
    A, B = stored_pair(130, 257, 67, opA, opB, "int", seed=9, bound=1024)
    print(f"integer ops {opA}{opB}", flush=True)
    assert np.array_equal(run(bq, A, B, opA=opA, opB=opB), oracle.gemm(OP_FN[opA](A), OP_FN[opB](B)))


def test_transpose_reverses_products(bq):
    """T(A B) = T(B) T(A) (Sec. III): op T on the stored B and A gives the
    oracle's transpose of the plain product."""
    A, B = inputs.pair(64, 48, 40, "uniform", seed=11)
    CT = run(bq, B, A, opA="T", opB="T")
    assert oracle.rel_frobenius(CT, oracle.transpose(oracle.gemm(A, B))) <= TOL


@pytest.mark.parametrize("opA,opB", [("T", "H"), ("H", "N")])
def test_transposed_ops_streamed_and_masks(bq, opA, opB):
    """Transposed operands through the streamed plan and a real-quaternion
    mask (8 GEMMs)."""
    A, B = stored_pair(150, 140, 130, opA, opB, "uniform", seed=12)
    ref = oracle.gemm(OP_FN[opA](A), OP_FN[opB](B))
    C1 = run(bq, A, B, opA=opA, opB=opB)
    C2 = run(bq, A, B, opA=opA, opB=opB, streamed=True)
    assert np.array_equal(C1, C2)
    assert oracle.rel_frobenius(C2, ref) <= TOL
    mask = inputs.MASKS["real_quaternion"]
    A, B = stored_pair(90, 70, 60, opA, opB, "normal", seed=13, mask=mask)
    got = run(bq, A, B, opA=opA, opB=opB, mask_a=mask, mask_b=mask)
    assert oracle.rel_frobenius(got, oracle.gemm(OP_FN[opA](A), OP_FN[opB](B))) <= TOL


@pytest.mark.parametrize("name", ["real_quaternion", "complex", "real"])
def test_subalgebra_masks(bq, name):
    mask = inputs.MASKS[name]
    A, B = inputs.pair(100, 90, 80, "normal", seed=4, mask_a=mask, mask_b=mask)
    C = run(bq, A, B, mask_a=mask, mask_b=mask)
    assert oracle.rel_frobenius(C, oracle.gemm(A, B)) <= TOL
    for c in set(range(8)) - _reach(mask):
        assert not np.any(C[c]), c


@pytest.mark.parametrize("ma,mb", [(0x0F, 0xFF), (0xFF, 0x0F), (0xF0, 0xFF), (0x11, 0xFF), (0x01, 0xFF),
                                   (0x33, 0x33), (0xF0, 0xF0), (0x22, 0x44)])
def test_general_masks(bq, ma, mb):
    """Active-component patterns beyond the four subalgebras (mixed real
    quaternion x biquaternion, the imaginary-field pattern [0,0,0,0,1,1,1,1],
    scalars times biquaternions, two-unit patterns): every output block
    against the oracle, structurally zero blocks exactly 0."""
    A, B = inputs.pair(70, 60, 50, "normal", seed=21, mask_a=ma, mask_b=mb)
    C = run(bq, A, B, mask_a=ma, mask_b=mb)
    ref = oracle.gemm(A, B)
    assert oracle.rel_frobenius(C, ref) <= TOL
    for c in range(8):
        if not np.any(ref[c]):
            assert not np.any(C[c]), c


def _reach(mask):
    if mask == inputs.REAL:
        return {0}
    if mask == inputs.COMPLEX:
        return {0, 4}
    if mask == inputs.REAL_QUAT:
        return {0, 1, 2, 3}
    return set(range(8))


def test_variant_entry_points(bq):
    import torch

    A, B = inputs.pair(77, 65, 59, "normal", seed=5)
    a, b = dev(A), dev(B)
    # real
    c = torch.empty((77, 59), dtype=torch.float64, device="cuda")
    bq.re_gemm(a[0], b[0], c)
    torch.cuda.synchronize()
    assert np.allclose(c.cpu().numpy(), A[0] @ B[0], rtol=0, atol=1e-12)
    # complex
    cr = torch.empty_like(c); ci = torch.empty_like(c)
    bq.cx_gemm((a[0], a[4]), (b[0], b[4]), (cr, ci))
    torch.cuda.synchronize()
    ref = (A[0] + 1j * A[4]) @ (B[0] + 1j * B[4])
    assert np.allclose(cr.cpu().numpy() + 1j * ci.cpu().numpy(), ref, rtol=0, atol=1e-12)
    # complex conjugate of A
    bq.cx_gemm((a[0], a[4]), (b[0], b[4]), (cr, ci), opA="C")
    torch.cuda.synchronize()
    ref = (A[0] - 1j * A[4]) @ (B[0] + 1j * B[4])
    assert np.allclose(cr.cpu().numpy() + 1j * ci.cpu().numpy(), ref, rtol=0, atol=1e-12)
    # real quaternion
    cq = [torch.empty_like(c) for _ in range(4)]
    bq.rq_gemm([a[i] for i in range(4)], [b[i] for i in range(4)], cq)
    torch.cuda.synchronize()
    Aq = A.copy(); Aq[4:] = 0
    Bq = B.copy(); Bq[4:] = 0
    ref = oracle.gemm(Aq, Bq)
    got = np.stack([x.cpu().numpy() for x in cq] + [np.zeros((77, 59))] * 4)
    assert oracle.rel_frobenius(got, ref) <= TOL


def test_variant_entry_points_ops_and_split(bq):
    """The subalgebra entry points take bq_gemm's arguments: op T / H on
    stored-transposed operands, and the split forms."""
    import torch

    rng = np.random.default_rng(55)
    m, k, n = 70, 61, 53
    At = inputs.blocks(rng, k, m, "normal")     # stored k x m: op T / H gives m x k
    Bt = inputs.blocks(rng, n, k, "normal")     # stored n x k
    a, b = dev(At), dev(Bt)
    # real: op(A) = A^T, op(B) = B^T
    c = torch.empty((m, n), dtype=torch.float64, device="cuda")
    bq.re_gemm(a[0], b[0], c, opA="T", opB="H")
    torch.cuda.synchronize()
    assert np.allclose(c.cpu().numpy(), At[0].T @ Bt[0].T, rtol=0, atol=1e-12)
    # real quaternion, dagger of A and transpose of B, against the oracle's sign rules
    Aq = At.copy(); Aq[4:] = 0
    Bq = Bt.copy(); Bq[4:] = 0
    cq = [torch.empty((m, n), dtype=torch.float64, device="cuda") for _ in range(4)]
    bq.rq_gemm([a[i] for i in range(4)], [b[i] for i in range(4)], cq, opA="H", opB="T")
    torch.cuda.synchronize()
    ref = oracle.gemm(oracle.herm(Aq), oracle.transpose(Bq))
    got = np.stack([x.cpu().numpy() for x in cq] + [np.zeros((m, n))] * 4)
    assert np.all(ref[4:] == 0)
    assert oracle.rel_frobenius(got, ref) <= TOL
    # complex in the CRT form and in BF16 digits
    A, B = inputs.pair(m, k, n, "uniform", seed=56)
    a, b = dev(A), dev(B)
    for prec in ("split_int8_crt", "split_bf16"):
        cr = torch.empty((m, n), dtype=torch.float64, device="cuda"); ci = torch.empty_like(cr)
        bq.cx_gemm((a[0], a[4]), (b[0], b[4]), (cr, ci), opA="C", prec=prec)
        torch.cuda.synchronize()
        refc = (A[0] - 1j * A[4]) @ (B[0] + 1j * B[4])
        gotc = cr.cpu().numpy() + 1j * ci.cpu().numpy()
        assert np.linalg.norm(gotc - refc) / np.linalg.norm(refc) <= TOL, prec


def test_side_stream(bq):
    """A call on a caller's stream (not torch's current one): the binding
    allocates the output and workspace on that stream, so the caching
    allocator reuses them only in its order; the result is the same."""
    import torch

    A, B = inputs.pair(300, 280, 260, "uniform", seed=57)
    a, b = dev(A), dev(B)
    ref = bq.bq_gemm(a, b)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    outs = []
    for _ in range(4):
        # each call's temporaries are freed when it returns; the next call on
        # the same stream may take the same memory, in stream order
        outs.append(bq.bq_gemm(a, b, stream=s))
        junk = torch.empty(1 << 22, dtype=torch.float64, device="cuda")   # other work on the current stream
        junk.fill_(float("nan"))
    s.synchronize()
    torch.cuda.synchronize()
    for c in outs:
        assert torch.equal(c, ref)


def test_streamed_equals_resident(bq):
    A, B = inputs.pair(150, 140, 130, "uniform", seed=6)
    C1 = run(bq, A, B)
    C2 = run(bq, A, B, streamed=True)
    assert np.array_equal(C1, C2)
    assert oracle.rel_frobenius(C2, oracle.gemm(A, B)) <= TOL


def test_guard_band_untouched(bq):
    """C with ld > n: the padding columns keep their sentinel values."""
    import torch

    m, k, n, ld = 90, 70, 50, 64
    A, B = inputs.pair(m, k, n, "uniform", seed=8)
    Cbuf = torch.full((8, m, ld), 12345.0, dtype=torch.float64, device="cuda")
    C = Cbuf[:, :, :n]
    bq.bq_gemm(dev(A), dev(B), C)
    torch.cuda.synchronize()
    out = Cbuf.cpu().numpy()
    assert np.all(out[:, :, n:] == 12345.0)
    assert oracle.rel_frobenius(out[:, :, :n], oracle.gemm(A, B)) <= TOL


def test_degenerate(bq):
    import torch

    A, B = inputs.pair(5, 0, 7, "uniform", seed=9)
    C = torch.full((8, 5, 7), 3.0, dtype=torch.float64, device="cuda")
    # k == 0: C = 0
    bq.bq_gemm(torch.empty((8, 5, 0), dtype=torch.float64, device="cuda"),
               torch.empty((8, 0, 7), dtype=torch.float64, device="cuda"), C)
    torch.cuda.synchronize()
    assert not torch.any(C).item()
    # m == 0: no-op
    out = bq.bq_gemm(torch.empty((8, 0, 4), dtype=torch.float64, device="cuda"),
                     torch.zeros((8, 4, 3), dtype=torch.float64, device="cuda"))
    assert out.shape == (8, 0, 3)


def test_nan_row_propagation(bq):
    A, B = inputs.pair(40, 40, 40, "uniform", seed=10)
    A[6, 11, 3] = np.nan
    C = run(bq, A, B)
    assert np.all(np.isnan(C[:, 11, :]))
    assert not np.any(np.isnan(np.delete(C, 11, axis=1)))


def test_error_leaves_c_untouched(bq):
    import torch

    A, B = inputs.pair(32, 32, 32, "uniform", seed=11)
    C = torch.full((8, 32, 32), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(bq.BqError) as e:   # workspace below the streamed minimum
        bq.bq_gemm(dev(A), dev(B), C, workspace=torch.empty(16, dtype=torch.uint8, device="cuda"))
    assert e.value.code == 4
    torch.cuda.synchronize()
    assert torch.all(C == 7.0).item()


def _sample(n, r, seed):
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(n - 1, size=r - 1, replace=False))
    return np.append(idx, n - 1)


@pytest.mark.parametrize("name", ["biquaternion", "real_quaternion", "complex", "real"])
def test_n4096_sampled(bq, name):
    """n = 4096, N(0,1) entries, each subalgebra; rows/cols sampled (the last
    row and column always included) and checked against the oracle."""
    import torch

    n, r = 4096, 96
    mask = inputs.MASKS[name]
    print(f"n=4096 {name}: drawing inputs", flush=True)
    A, B = inputs.pair(n, n, n, "normal", seed=2, mask_a=mask, mask_b=mask)
    C = bq.bq_gemm(dev(A), dev(B), mask_a=mask, mask_b=mask)
    torch.cuda.synchronize()
    rows, cols = _sample(n, r, 21), _sample(n, r, 22)
    Cs = C[:, torch.as_tensor(rows, device="cuda")][:, :, torch.as_tensor(cols, device="cuda")].cpu().numpy()
    ref = oracle.gemm(A[:, rows, :], B[:, :, cols])
    err = oracle.rel_frobenius(Cs, ref)
    print(f"n=4096 {name}: rel err {err:.3e}", flush=True)
    assert err <= TOL
    # the isomorph: Z(C) = Z(A) Z(B) on the sampled block
    ZA = oracle.iso(A[:, rows, :])
    ZB = oracle.iso(B[:, :, cols])
    assert oracle.rel_frobenius(Cs, oracle.iso_inv(ZA @ ZB)) <= TOL


@pytest.mark.parametrize("n,streamed", [(16384, False), (24576, False), (24576, True)])
def test_large_hermitian(bq, n, streamed):
    """n = 16384 and 24576 (the 2n x 2n complex isomorph has more than 2^31
    elements at 24576, and one block is 4.8 GB > 2^32 bytes), resident and
    streamed plans: Fock-like A times density-like B, checked on sampled rows
    and columns that always include the last ones (largest offsets), and for
    the resident plans on every entry of C at once by a Gaussian probe: for a
    biquaternion X (n x p) with N(0,1) entries, E ||(C - AB) X||^2 is
    proportional to ||C - AB||_F^2 with the same constant as E ||AB X||^2 to
    ||AB||_F^2, so rho = ||C X - A (B X)||_F / ||A (B X)||_F estimates the
    relative Frobenius error.  C X, B X and A (B X) are the oracle's
    products, taken in row slabs of the device matrices."""
    import torch

    print(f"n={n} streamed={streamed}: building Hermitian inputs on the device", flush=True)
    A, B = inputs.hermitian_pair(n, 3, "cuda")
    torch.cuda.empty_cache()  # the builder's temporaries, before the workspace
    C = bq.bq_gemm(A, B, streamed=streamed)
    torch.cuda.synchronize()
    print(f"n={n}: product done", flush=True)
    r = 64
    rows, cols = _sample(n, r, 31), _sample(n, r, 32)
    ri, ci = torch.as_tensor(rows, device="cuda"), torch.as_tensor(cols, device="cuda")
    As = A[:, ri, :].cpu().numpy()
    Bs = B[:, :, ci].cpu().numpy()
    Cs = C[:, ri][:, :, ci].cpu().numpy()
    err = oracle.rel_frobenius(Cs, oracle.gemm(As, Bs))
    print(f"n={n}: sampled rel err {err:.3e}", flush=True)
    assert err <= TOL
    if not streamed:
        p, slab = 4, 1024
        X = inputs.blocks(np.random.default_rng(61), n, p, "normal")

        def apply(M, Y):
            out = np.empty((8, n, Y.shape[2]))
            for r0 in range(0, n, slab):
                out[:, r0:r0 + slab] = oracle.gemm(M[:, r0:r0 + slab].cpu().numpy(), Y)
            return out

        CX = apply(C, X)
        ABX = apply(A, apply(B, X))
        rho = oracle.rel_frobenius(CX, ABX)
        print(f"n={n}: Gaussian-probe relative error estimate {rho:.3e}", flush=True)
        assert rho <= TOL
    del A, B, C
    torch.cuda.empty_cache()


@pytest.mark.parametrize("mask", [0xFF, 0x01])
@pytest.mark.parametrize("k", [1040, 1031, 1024])
def test_large_products_odd_and_ragged_k(bq, k, mask):
    """m = n = 2048 (1024 tiles) with k >= 1024 takes the two-deep pipeline
    (complex products: k-steps of 16, real ones: of 32): odd k-step counts
    (k = 1040: 65 or 33 steps), a ragged last k-step (1031) and an even
    count (1024), checked against the oracle on sampled rows and columns
    (the last ones included)."""
    import torch

    m = n = 2048
    rng = np.random.default_rng(70 + k)
    A = torch.from_numpy(inputs.blocks(rng, m, k, "uniform", mask=mask)).to("cuda")
    B = torch.from_numpy(inputs.blocks(rng, k, n, "uniform", mask=mask)).to("cuda")
    C = bq.bq_gemm(A, B, mask_a=mask, mask_b=mask)
    torch.cuda.synchronize()
    rows, cols = _sample(m, 40, 71), _sample(n, 40, 72)
    ri, ci = torch.as_tensor(rows, device="cuda"), torch.as_tensor(cols, device="cuda")
    got = C[:, ri][:, :, ci].cpu().numpy()
    ref = oracle.gemm(A[:, ri, :].cpu().numpy(), B[:, :, ci].cpu().numpy())
    assert oracle.rel_frobenius(got, ref) <= TOL


@pytest.mark.parametrize("mask", [0x01, 0x0F])
@pytest.mark.parametrize("m,k,n", [(2040, 1001, 2040), (4100, 96, 4100), (2048, 33, 2056)])
def test_real_products_in_large_blocks(bq, m, k, n, mask):
    """Real x real products of this size run in 128 x 128 blocks of 16 waves
    (k-steps of 32): ragged edge tiles in m and n, ragged and short k, real
    and real-quaternion masks, against the oracle on sampled rows and
    columns (the last ones included)."""
    import torch

    rng = np.random.default_rng(m + k + n + mask)
    A = torch.from_numpy(inputs.blocks(rng, m, k, "uniform", mask=mask)).to("cuda")
    B = torch.from_numpy(inputs.blocks(rng, k, n, "uniform", mask=mask)).to("cuda")
    C = bq.bq_gemm(A, B, mask_a=mask, mask_b=mask)
    torch.cuda.synchronize()
    rows, cols = _sample(m, 40, 73), _sample(n, 40, 74)
    ri, ci = torch.as_tensor(rows, device="cuda"), torch.as_tensor(cols, device="cuda")
    got = C[:, ri][:, :, ci].cpu().numpy()
    ref = oracle.gemm(A[:, ri, :].cpu().numpy(), B[:, :, ci].cpu().numpy())
    assert oracle.rel_frobenius(got, ref) <= TOL


@pytest.mark.parametrize("opB", ["N", "T"])
def test_leading_dimension_beyond_buffer_offsets(bq, opB):
    """Operand rows 4.5e6 doubles apart: a 64-row tile spans more than 2^31
    bytes, so the single call and the batched plan read such operands with
    pointer loads instead of buffer resources.  A is 3 x 40 (op N), B is
    40 x 5 (op N) or stored 5 x 40 with the same row pitch (op T); against
    the oracle on contiguous copies."""
    import torch

    L = 4_500_000
    rng = np.random.default_rng(80)
    a = inputs.blocks(rng, 3, 40, "uniform")
    Abig = torch.zeros((8, 3, L), dtype=torch.float64, device="cuda")
    Abig[:, :, :40] = torch.from_numpy(a).to("cuda")
    A = Abig[:, :, :40]
    if opB == "N":
        b = inputs.blocks(rng, 40, 5, "uniform")
        B = torch.from_numpy(b).to("cuda")
        ref = oracle.gemm(a, b)
    else:
        bs = inputs.blocks(rng, 5, 40, "uniform")
        Bbig = torch.zeros((8, 5, L), dtype=torch.float64, device="cuda")
        Bbig[:, :, :40] = torch.from_numpy(bs).to("cuda")
        B = Bbig[:, :, :40]
        ref = oracle.gemm(a, oracle.transpose(bs))
    print(f"ld {L}, op B {opB}: single call and batched plan", flush=True)
    C = bq.bq_gemm(A, B, opB=opB)
    torch.cuda.synchronize()
    assert oracle.rel_frobenius(C.cpu().numpy(), ref) <= TOL
    C2 = torch.full_like(C, float("nan"))
    plan = bq.GroupedPlan([(A, B, C2)], opB=opB)
    plan.launch()
    torch.cuda.synchronize()
    assert oracle.rel_frobenius(C2.cpu().numpy(), ref) <= TOL
    plan.close()
    del Abig
    torch.cuda.empty_cache()


@pytest.mark.parametrize("m,k,n", [(2050, 1030, 2060), (2047, 1041, 2049)])
def test_two_deep_with_edge_tiles(bq, m, k, n):
    """Complex products large enough for the two-deep pipeline (k >= 1024,
    at least 1024 tiles) on grids with edge tiles: interior tiles take the
    buffer-load steady state, edge tiles and the ragged last k-step the
    bounds-checked buffer loads; sampled rows and columns (the last ones
    included) against the oracle."""
    import torch

    rng = np.random.default_rng(m + n)
    A = torch.from_numpy(inputs.blocks(rng, m, k, "uniform")).to("cuda")
    B = torch.from_numpy(inputs.blocks(rng, k, n, "uniform")).to("cuda")
    print(f"two-deep with edge tiles {m}x{k}x{n}", flush=True)
    C = bq.bq_gemm(A, B)
    torch.cuda.synchronize()
    rows, cols = _sample(m, 40, 73), _sample(n, 40, 74)
    ri, ci = torch.as_tensor(rows, device="cuda"), torch.as_tensor(cols, device="cuda")
    got = C[:, ri][:, :, ci].cpu().numpy()
    ref = oracle.gemm(A[:, ri, :].cpu().numpy(), B[:, :, ci].cpu().numpy())
    assert oracle.rel_frobenius(got, ref) <= TOL


@pytest.mark.parametrize("env,value", [("BQ_TILE_ORDER", "0,4"), ("BQ_TILE_ORDER", "1,1"),
                                       ("BQ_TILE_ORDER", "1,16"), ("BQ_TILE_CONFIG", "3"),
                                       ("BQ_TILE_CONFIG", "11"), ("BQ_TILE_CONFIG", "6")])
def test_tuning_switches_same_products(bq, monkeypatch, env, value):
    """The tile order and tile configuration switches change only which
    kernel shape runs and how blocks map to tiles: a biquaternion product
    and a real product (one component each) of integer inputs equal the
    oracle's exactly under every setting (configuration 3 or 11 selects the
    real products' tile, a complex product ignores it, and 6 is not a
    single-call configuration: it is ignored)."""
    A, B = inputs.pair(330, 200, 270, "int", seed=12, bound=1024)
    R = inputs.MASKS["real"]
    Ar, Br = A * (np.arange(8) == 0)[:, None, None], B * (np.arange(8) == 0)[:, None, None]
    monkeypatch.setenv(env, value)
    print(f"{env}={value}", flush=True)
    assert np.array_equal(run(bq, A, B), oracle.gemm(A, B))
    assert np.array_equal(run(bq, Ar, Br, mask_a=R, mask_b=R), oracle.gemm(Ar, Br))
