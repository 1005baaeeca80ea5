"""bq_gemm_noalloc (workspace from the library's static device array; no
allocation) against bq_gemm on the same inputs, through the C-ABI.

Both run the same kernels on the same plan, so the results are equal bit for
bit; each is also within 1e-12 of the oracle.  Two calls in a row, the second
smaller (the array keeps the first call's contents), a product that takes
the streamed plan, a split form, and one too large for the array
(BQ_ERR_WORKSPACE, C untouched).
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


def _pair(m, k, n, seed, dist="uniform"):
    import torch

    A, B = inputs.pair(m, k, n, dist, seed=seed)
    return A, B, torch.from_numpy(A).to("cuda"), torch.from_numpy(B).to("cuda")


def _noalloc(bq, a, b, m, n, **kw):
    import torch

    C = torch.full((8, m, n), float("nan"), dtype=torch.float64, device="cuda")
    bq.bq_gemm_noalloc(a, b, C, **kw)
    torch.cuda.synchronize()
    return C.cpu().numpy()


def test_two_calls_second_smaller(bq):
    import torch

    for (m, k, n, seed) in ((300, 280, 260, 81), (100, 90, 80, 82)):
        print(f"noalloc fp64 {m}x{k}x{n}", flush=True)
        A, B, a, b = _pair(m, k, n, seed)
        got = _noalloc(bq, a, b, m, n)
        ref = bq.bq_gemm(a, b)
        torch.cuda.synchronize()
        assert np.array_equal(got, ref.cpu().numpy())
        assert oracle.rel_frobenius(got, oracle.gemm(A, B)) <= TOL


def test_streamed_plan_and_split_form(bq):
    import torch

    # resident workspace 16 n^2 x 8 B = 512 MB > 256 MiB; streamed 128 MB fits
    n = 2000
    print(f"noalloc fp64 n={n} (streamed plan)", flush=True)
    a = inputs.device_uniform(n, n, 83, "cuda")
    b = inputs.device_uniform(n, n, 84, "cuda")
    got = _noalloc(bq, a, b, n, n)
    ref = bq.bq_gemm(a, b, streamed=True)
    torch.cuda.synchronize()
    assert np.array_equal(got, ref.cpu().numpy())
    del a, b, ref
    # a split form on a smaller product afterwards
    print("noalloc split_int8_crt 200x150x100", flush=True)
    A, B, a, b = _pair(200, 150, 100, 85, "logspread")
    got = _noalloc(bq, a, b, 200, 100, prec="split_int8_crt")
    ref = bq.bq_gemm(a, b, prec="split_int8_crt")
    torch.cuda.synchronize()
    assert np.array_equal(got, ref.cpu().numpy())
    assert oracle.rel_frobenius(got, oracle.gemm(A, B)) <= TOL


def test_too_large_is_refused(bq):
    import torch

    # streamed workspace 4 n^2 x 8 B = 288 MB at n = 3000: above 256 MiB
    n = 3000
    print(f"noalloc n={n}: refused", flush=True)
    a = torch.zeros((8, n, n), dtype=torch.float64, device="cuda")
    C = torch.full((8, n, n), float("nan"), dtype=torch.float64, device="cuda")
    with pytest.raises(bq.BqError) as e:
        bq.bq_gemm_noalloc(a, a.clone(), C)
    assert e.value.code == 4 and "static workspace" in e.value.detail
    torch.cuda.synchronize()
    assert bool(torch.isnan(C).all())
