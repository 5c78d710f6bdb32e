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
    ex = serving.GpuExecutor(n_slots=4)
    budget = 2 << 30
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
