"""Two recursion levels per pre- and post-addition pass (the EW2 passes of
the grouped Winograd schedule) against the level-by-level passes
(MM_PLAN_LEVEL_PASSES), through the C ABI (needs a GPU).

The two forms compute every sum and every U combination in the same order,
so their results must be bitwise equal: float32, float64 and split-bfloat16
leaves, two to four levels, accumulating plans, and an operand that is not
16-byte aligned (its passes take the one-element path).  Each case is also
checked against the oracle."""
import numpy as np
import pytest

from paper_2309_00628_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_00628_amd import api as a
    return a


def rel_fro(got, ref):
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(np.asarray(got, np.float64) - ref) / np.linalg.norm(ref))


def run(api, A, B, C, levels, dtype, **kw):
    m, k = A.shape
    n = B.shape[1]
    p = api.Plan("winograd", "grouped", m, n, k, cutoff=1, levels=levels, dtype=dtype, lda=A.stride(0),
                 ldb=B.stride(0), ldc=C.stride(0), **kw)
    ws = torch.empty(max(p.ws_bytes, 256), dtype=torch.uint8, device="cuda")
    p(A, B, C, ws, **({"beta": 1.5} if kw.get("accumulate") else {}))
    return p


CASES = [(512, 512, 512, 2, "f32"), (1024, 768, 512, 2, "f32"), (1024, 1024, 1024, 3, "f32"),
         (2048, 2048, 2048, 4, "f32"), (256, 256, 256, 2, "f64"), (1024, 1024, 1024, 2, "bf16x3")]


@pytest.mark.parametrize("m,n,k,levels,dtype", CASES)
def test_two_level_passes_bitwise_equal_to_level_passes(api, oracle_built, m, n, k, levels, dtype):
    from oracle import naive
    tdt = torch.float64 if dtype == "f64" else torch.float32
    A_np, B_np = inputs.pair("uniform", m, n, k, 70, np.float64 if dtype == "f64" else np.float32)
    A, B = torch.from_numpy(A_np).cuda(), torch.from_numpy(B_np).cuda()
    outs = []
    for lp in (False, True):
        C = torch.full((m, n), float("nan"), dtype=tdt, device="cuda")
        p = run(api, A, B, C, levels, dtype, level_passes=lp)
        kinds = [l.split()[1] for l in p.describe().splitlines() if l.startswith("LAUNCH")]
        assert ("EW2" in kinds) != lp, kinds
        outs.append(C)
    torch.cuda.synchronize()
    print(f"{m}x{n}x{k} L={levels} {dtype}", flush=True)
    assert torch.equal(outs[0], outs[1])
    rows = np.unique(np.r_[0, np.linspace(0, m - 1, 12).astype(np.int64), m - 1])
    err = rel_fro(outs[0][torch.from_numpy(rows).cuda()].cpu().numpy(), naive.gemm_rows(A_np, B_np, rows))
    # float32 beyond three levels: 1e-4, as for the other deep recursions
    assert err < (1e-12 if dtype == "f64" else 1e-5 if levels <= 3 else 1e-4), err


def test_accumulating_plan(api, oracle_built):
    from oracle import naive
    n = 1024
    A_np, B_np = inputs.pair("uniform", n, n, n, 71, np.float32)
    C0 = inputs.pair("uniform", n, n, n, 72, np.float32)[0]
    A, B = torch.from_numpy(A_np).cuda(), torch.from_numpy(B_np).cuda()
    outs = []
    for lp in (False, True):
        C = torch.from_numpy(C0).cuda()
        run(api, A, B, C, 3, "f32", accumulate=True, level_passes=lp)
        outs.append(C)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])
    rows = np.array([0, 300, n - 1])
    ref = naive.gemm_rows(A_np, B_np, rows) + 1.5 * C0[rows].astype(np.float64)
    assert rel_fro(outs[0][torch.from_numpy(rows).cuda()].cpu().numpy(), ref) < 1e-5


def test_unaligned_operand_takes_the_element_path(api, oracle_built):
    # A starts one float past a 16-byte boundary: the passes that read it run
    # element by element; the results are still those of the level passes
    from oracle import naive
    n = 512
    A_np, B_np = inputs.pair("uniform", n, n, n, 73, np.float32)
    buf = torch.empty(n * n + 1, device="cuda")
    A = buf[1:].view(n, n)
    A.copy_(torch.from_numpy(A_np))
    B = torch.from_numpy(B_np).cuda()
    outs = []
    for lp in (False, True):
        C = torch.full((n, n), float("nan"), device="cuda")
        run(api, A, B, C, 2, "f32", level_passes=lp)
        outs.append(C)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])
    rows = np.array([0, 1, 255, 256, n - 1])
    assert rel_fro(outs[0][torch.from_numpy(rows).cuda()].cpu().numpy(), naive.gemm_rows(A_np, B_np, rows)) < 1e-5
