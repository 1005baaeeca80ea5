"""Graph capture of the single-call product (GPU, through the C-ABI).

* bq_gemm and bq_gemm_noalloc enqueue kernels only (no allocation, copy,
  memset or synchronization), so a caller can record them into a HIP graph:
  the graph is replayed several times with eager work and synchronizations
  in between, and every replay is checked against the eager result.
* Misuse: a batched plan's first launch copies its tables synchronously
  (through the legacy stream) before recording on its own stream; while
  another stream captures in global mode the runtime refuses that (the
  legacy stream would depend on a capturing stream), and the plan reports
  BQ_ERR_HIP (code 5).
"""
import numpy as np
import pytest

import oracle
from paper_2609_02081_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bq():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_02081_amd as bq

    bq.lib()
    return bq


def _operands(m, k, n, seed):
    import torch

    rng = np.random.default_rng(seed)
    A = torch.from_numpy(inputs.blocks(rng, m, k, "uniform")).to("cuda")
    B = torch.from_numpy(inputs.blocks(rng, k, n, "uniform")).to("cuda")
    return A, B


@pytest.mark.parametrize("entry", ["bq_gemm", "bq_gemm_noalloc"])
def test_captured_product_replays(bq, entry):
    import torch

    m, k, n = 200, 130, 150
    A, B = _operands(m, k, n, 90)
    eager = bq.bq_gemm(A, B)
    torch.cuda.synchronize()
    ref = eager.cpu().numpy()
    assert oracle.rel_frobenius(ref, oracle.gemm(A.cpu().numpy(), B.cpu().numpy())) <= 1e-12
    C = torch.empty_like(eager)
    ws = torch.empty(bq.workspace_size(m, n, k)[0], dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    print(f"capture {entry} {m}x{k}x{n}", flush=True)
    with torch.cuda.stream(s):
        g.capture_begin(capture_error_mode="thread_local")
        if entry == "bq_gemm":
            bq.bq_gemm(A, B, C, workspace=ws, stream=s)
        else:
            bq.bq_gemm_noalloc(A, B, C, stream=s)
        g.capture_end()
    torch.cuda.synchronize()
    for rep in range(3):
        C.fill_(float("nan"))
        (A * 2.0).sum().item()  # eager work and a synchronization between replays
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(C.cpu().numpy(), ref), rep
    del g


def test_plan_recording_during_global_capture_is_reported(bq):
    """A batched plan records its graph on its own stream at its first
    launch, after copying its tables to the device through the legacy
    stream; while another stream captures in global mode the runtime
    refuses that copy, and the plan reports BQ_ERR_HIP (code 5).  After the
    capture is ended the same plan launches and is correct.  The capture is
    begun and ended through the HIP runtime itself, so that torch's caching
    allocator never routes allocations to a capture pool that an invalidated
    capture would leave in place."""
    import ctypes

    import torch

    hip = ctypes.CDLL("libamdhip64.so")
    m, k, n = 64, 64, 64
    A, B = _operands(m, k, n, 91)
    C = torch.full((8, m, n), float("nan"), dtype=torch.float64, device="cuda")
    plan = bq.GroupedPlan([(A, B, C)])
    ws = plan.workspace()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    h = ctypes.c_void_p(s.cuda_stream)
    print("batched plan recorded during a global capture", flush=True)
    code = None
    assert hip.hipStreamBeginCapture(h, 0) == 0  # hipStreamCaptureModeGlobal
    try:
        plan.launch(workspace=ws, stream=s)
    except bq.BqError as e:
        code = e.code
        print(f"reported: {e}", flush=True)
    finally:
        graph = ctypes.c_void_p()
        rc = hip.hipStreamEndCapture(h, ctypes.byref(graph))
        if rc == 0 and graph.value:
            hip.hipGraphDestroy(graph)
        hip.hipGetLastError()  # the invalidated capture's error is not left for later calls
    torch.cuda.synchronize()
    assert code == 5
    plan.launch(workspace=ws)
    torch.cuda.synchronize()
    ref = oracle.gemm(A.cpu().numpy(), B.cpu().numpy())
    assert oracle.rel_frobenius(C.cpu().numpy(), ref) <= 1e-12
    plan.close()
