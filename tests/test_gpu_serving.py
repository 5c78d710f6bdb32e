"""Serving loop on the GPU: mixed sizes and dtypes admitted under an HBM
budget with overlapping execution; every result is bitwise the same as the
same request run alone, and close to the oracle."""
import numpy as np
import pytest

from paper_2309_00628_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def test_results_same_alone_and_in_the_mix(gpu, oracle_built):
    from oracle import naive
    from paper_2309_00628_amd import serving
    trace = inputs.serving_trace(24, 5, qps=4000, bands=((0.6, 128, 700), (0.4, 700, 2100)))
    reqs = serving.make_requests(trace, gpu)
    budget = 2 << 30
    ex = serving.GpuExecutor(n_slots=4, arena_bytes=budget)
    srv = serving.Server(ex, budget, n_slots=4)
    done, wall = srv.run(reqs)
    torch.cuda.synchronize()
    assert len(done) == 24 and all(not r.error for r in done), [r.error for r in done]
    assert srv.peak_reserved <= budget
    assert srv.max_running > 1                       # requests overlapped on the device
    stats = serving.summarize(done, wall)
    print(stats, flush=True)
    # each request alone, on the default stream
    for r in sorted(done, key=lambda r: r.rid):
        p = ex.plan(r)
        C = torch.empty_like(r.C)
        p(r.A, r.B, C)
        torch.cuda.synchronize()
        assert torch.equal(C, r.C), (r.rid, r.n, r.dtype)
    # and against the oracle on a few rows of each
    for r in done[:8]:
        A = r.A.cpu().numpy()
        B = r.B.cpu().numpy()
        rows = np.arange(0, r.m, max(1, r.m // 8))
        ref = naive.gemm_rows(A, B, rows)
        got = r.C[torch.from_numpy(rows).to(gpu)].double().cpu().numpy()
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert err < 1e-5, (r.rid, r.n, r.dtype, err)


def test_device_memory_stays_within_the_budget(gpu):
    """A trace with n = 8192 requests (float32 and split-bfloat16, whose
    Winograd workspaces are the largest) under a budget that holds only a
    few of them at once: the caching allocator's reservation and the
    device's used memory grow by no more than the budget (plus the plans'
    small descriptor tables), however many requests have run."""
    from paper_2309_00628_amd import serving
    trace = inputs.serving_trace(24, 9, qps=2000, bands=((0.5, 256, 1024), (0.25, 1024, 4096),
                                                          (0.25, 8192, 8192)))
    assert sum(t["n"] == 8192 for t in trace) >= 3
    reqs = serving.make_requests(trace, gpu)
    torch.cuda.synchronize()
    budget = 6 << 30
    res0 = torch.cuda.memory_reserved(gpu)
    free0, _ = torch.cuda.mem_get_info(gpu)
    ex = serving.GpuExecutor(n_slots=4, arena_bytes=budget, keep_outputs=False)
    for _ in range(2):                       # the second run reuses plans and the arena
        srv = serving.Server(ex, budget, n_slots=4)
        done, _ = srv.run(reqs)
        torch.cuda.synchronize()
        assert len(done) == 24 and all(not r.error for r in done), [r.error for r in done]
        assert srv.peak_reserved <= budget and srv.reserved == 0
        assert ex.arena.used_bytes == 0
        grow = torch.cuda.memory_reserved(gpu) - res0
        assert grow <= budget, (grow, budget)
        free1, _ = torch.cuda.mem_get_info(gpu)
        assert free0 - free1 <= budget + (256 << 20), (free0 - free1, budget)
