"""The entry point that allocates nothing (mm_winograd_noalloc), through the
C ABI (needs a GPU): two calls in a row, the second with a smaller product,
each checked against the existing entry point mm_winograd (same recursion
control) within the float32 tolerance, against the Two Temp schedule of
mm_gemm_ex bitwise (the same schedule and leaf kernel), and against the
oracle; no device memory is allocated by either call; a product whose
workspace exceeds the static scratch is refused with nothing enqueued."""
import ctypes

import numpy as np
import pytest

from paper_2309_00628_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_00628_amd import _lib as L
    return L


def rel_fro(got, ref):
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(np.asarray(got, np.float64) - ref) / np.linalg.norm(ref))


def run(L, fn, A, B, C, cutoff, levels, s):
    m, k = A.shape
    n = B.shape[1]
    st = fn(m, n, k, A.data_ptr(), B.data_ptr(), C.data_ptr(), cutoff, levels, L.MM_F32, s)
    assert st == 0, L.last_error()


def test_two_calls_match_the_allocating_entry_points(lib, oracle_built):
    from oracle import naive
    L = lib
    cl = L.load()
    s = torch.cuda.current_stream().cuda_stream
    # warm the library's code object on this device (its load places the
    # static scratch) before measuring free memory
    w = torch.ones((64, 64), device="cuda")
    cw = torch.empty((64, 64), device="cuda")
    run(L, cl.mm_winograd_noalloc, w, w, cw, 1, 1, s)
    for (m, n, k), lv, seed in (((1536, 1536, 1536), 2, 61), ((1000, 904, 776), 1, 62)):
        print(f"noalloc {m}x{n}x{k} L={lv}", flush=True)
        A_np, B_np = inputs.pair("uniform", m, n, k, seed, np.float32)
        A, B = torch.from_numpy(A_np).cuda(), torch.from_numpy(B_np).cuda()
        C0 = torch.full((m, n), float("nan"), device="cuda")
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info()
        run(L, cl.mm_winograd_noalloc, A, B, C0, 1, lv, s)
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        assert free1 == free0, (free0, free1)          # nothing allocated on the device
        C1 = torch.empty((m, n), device="cuda")
        run(L, cl.mm_winograd, A, B, C1, 1, lv, s)
        # the same schedule through the extended form (caller workspace)
        need = cl.mm_workspace_size(2, 0, m, n, k, 1, lv, L.MM_F32)
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device="cuda")
        C2 = torch.empty((m, n), device="cuda")
        Ac, Bc = A.clone(), B.clone()
        st = cl.mm_gemm_ex(2, 0, m, n, k, Ac.data_ptr(), k, Bc.data_ptr(), n, C2.data_ptr(), n, 1, lv,
                           L.MM_F32, ws.data_ptr(), ws.numel(), s)
        assert st == 0, L.last_error()
        torch.cuda.synchronize()
        got = C0.cpu().numpy()
        assert np.isfinite(got).all()
        assert torch.equal(C0, C2)
        assert rel_fro(got, C1.cpu().numpy()) < 1e-5
        rows = np.unique(np.r_[0, np.linspace(0, m - 1, 24).astype(np.int64), m - 1])
        ref = naive.gemm_rows(A_np, B_np, rows)
        assert rel_fro(got[rows], ref) < 1e-5


def test_oversized_product_is_refused(lib):
    L = lib
    cl = L.load()
    s = torch.cuda.current_stream().cuda_stream
    n = 6144                     # Two Temp workspace 2 (n/2)^2 floats = 72 MiB > 60 MiB
    A = torch.zeros((n, n), device="cuda")
    C = torch.full((n, n), 5.0, device="cuda")
    st = cl.mm_winograd_noalloc(n, n, n, A.data_ptr(), A.data_ptr(), C.data_ptr(), 1, 1, L.MM_F32, s)
    assert L.STATUS[st] == "MM_E_WORKSPACE"
    assert "scratch" in L.last_error()
    torch.cuda.synchronize()
    assert bool(torch.all(C == 5.0))             # nothing was enqueued
