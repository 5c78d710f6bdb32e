"""Parity of the split-bfloat16 dtype (MM_BF16X3_REFINED) with the oracle.

Float32 inputs, float32 outputs, every leaf product on bfloat16 MFMA with
the hi/lo/residual split.  Target: relative Frobenius error <= 1e-5 against
the float64 oracle, also on the wide-range inputs of the precision workload
(Gaussian rows scaled by 10^u, u ~ U[-3, 3]).  Small integers split exactly
(hi = x), so on them the product must be exact.
"""
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


@pytest.fixture(scope="module")
def naive(oracle_built):
    from oracle import naive
    return naive


def rel_fro(got, ref):
    ref = np.asarray(ref, dtype=np.float64)
    return np.linalg.norm(np.asarray(got, dtype=np.float64) - ref) / np.linalg.norm(ref)


def run(api, A, B, **kw):
    C = api.mm(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), dtype="bf16x3", **kw)
    torch.cuda.synchronize()
    return C.cpu().numpy()


@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (17, 33, 65), (128, 128, 128), (333, 517, 259),
                                   (64, 1000, 31), (1024, 768, 512)])
@pytest.mark.parametrize("kind", ["uniform", "gauss_rowscaled"])
def test_naive_bf16x3_shapes(api, naive, m, n, k, kind):
    A, B = inputs.pair(kind, m, n, k, 1, np.float32)
    err = rel_fro(run(api, A, B, algo="naive"), naive.gemm(A, B))
    print(f"bf16x3 naive {kind} {m}x{n}x{k}: {err:.3e}", flush=True)
    assert err < 1e-5


def test_bf16x3_integer_exact(api, naive):
    A, B = inputs.pair("int", 256, 256, 256, 2, np.float32)
    ref = naive.gemm(A, B)
    for algo, sched, lv in [("naive", "auto", 0), ("winograd", "grouped", 2), ("winograd", "two_temp", 1),
                            ("strassen", "dfs3", 1), ("strassen", "grouped", 2)]:
        got = run(api, A, B, algo=algo, sched=sched, cutoff=1, levels=lv)
        assert np.array_equal(got.astype(np.float64), ref), (algo, sched, lv)


@pytest.mark.parametrize("n,levels", [(1024, 1), (2048, 2), (1000, 2)])
def test_winograd_bf16x3_gauss_rowscaled(api, naive, n, levels):
    A, B = inputs.pair("gauss_rowscaled", n, n, n, 3, np.float32)
    ref = naive.gemm(A, B)
    for algo, sched in (("winograd", "grouped"), ("winograd", "two_temp"), ("strassen", "grouped")):
        err = rel_fro(run(api, A, B, algo=algo, sched=sched, cutoff=1, levels=levels), ref)
        print(f"bf16x3 {algo} {sched} n={n} L={levels}: {err:.3e}", flush=True)
        assert err < 1e-5


def test_precision_workload_8192_sampled(api, naive):
    # the precision workload at full size: n = 8192, two Winograd levels;
    # the oracle computes a sample of output rows exactly as in the full product
    n = 8192
    A, B = inputs.pair("gauss_rowscaled", n, n, n, 0, np.float32)
    rows = np.sort(inputs.rng(4).choice(n, size=24, replace=False))
    ref = naive.gemm_rows(A, B, rows)
    At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    C = api.mm(At, Bt, algo="winograd", sched="grouped", cutoff=1, levels=2, dtype="bf16x3")
    torch.cuda.synchronize()
    err = rel_fro(C[torch.from_numpy(rows).cuda()].cpu().numpy(), ref)
    print(f"bf16x3 winograd n=8192 L=2 sampled rows: {err:.3e}", flush=True)
    assert err < 1e-5


@pytest.mark.parametrize("algo,m,n,k,levels", [("naive", 1, 1, 1, 0), ("naive", 17, 33, 65, 0),
                                               ("naive", 333, 517, 259, 0), ("naive", 1024, 768, 520, 0),
                                               ("winograd", 512, 512, 512, 1), ("winograd", 1000, 777, 555, 2),
                                               ("winograd", 2048, 2048, 2048, 2), ("winograd", 384, 640, 256, 3)])
def test_split_pass_bitwise_equal_to_split_pass(api, naive, algo, m, n, k, levels):
    # operands split once by the split pass (MM_PLAN_SPLIT_PASS) must give
    # the same bits as the leaf kernel splitting every staged tile, for every
    # tile configuration of the split-operand kernel
    A, B = inputs.pair("gauss_rowscaled", m, n, k, 5, np.float32)
    At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    sched = "grouped" if levels else "auto"
    print(f"split pass {algo} {m}x{n}x{k} L={levels}", flush=True)
    ref = api.mm(At, Bt, algo=algo, sched=sched, cutoff=1, levels=levels, dtype="bf16x3")
    # every tile of the in-loader split kernel gives the same bits too
    for tile in (0, 1, 3, 4, 6, 8):
        C = torch.full((m, n), float("nan"), device="cuda")
        api.mm(At, Bt, algo=algo, sched=sched, cutoff=1, levels=levels, dtype="bf16x3", tile=tile, out=C)
        torch.cuda.synchronize()
        assert torch.equal(C, ref), ("in-loader", tile)
    for tile in (None, 0, 1, 3, 4, 5, 6):
        C = torch.full((m, n), float("nan"), device="cuda")
        api.mm(At, Bt, algo=algo, sched=sched, cutoff=1, levels=levels, dtype="bf16x3", tile=tile, out=C,
               split_pass=True)
        torch.cuda.synchronize()
        assert torch.equal(C, ref), tile
    rows = np.arange(0, m, max(1, m // 16))
    assert rel_fro(ref[torch.from_numpy(rows).cuda()].cpu().numpy(), naive.gemm_rows(A, B, rows)) < 1e-5


@pytest.mark.parametrize("k", [16, 32, 48, 64, 80, 96])
def test_ring_tile_short_k_bitwise(api, naive, k):
    # the 256x256 tile on a ring of three LDS stages peels its last three
    # stages (16 k each) and runs products of fewer than three stages, and
    # tiles at the matrix edge, through a one-buffer loop: every count of
    # stages around the peel gives the bits of the 128x128 tile
    for m, n in ((512, 512), (520, 300)):
        A, B = inputs.pair("gauss_rowscaled", m, n, k, 9, np.float32)
        At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        print(f"ring tile {m}x{n}x{k}", flush=True)
        ref = api.mm(At, Bt, algo="naive", dtype="bf16x3", tile=0)
        C = torch.full((m, n), float("nan"), device="cuda")
        api.mm(At, Bt, algo="naive", dtype="bf16x3", tile=6, out=C)
        torch.cuda.synchronize()
        assert torch.equal(C, ref)
        assert rel_fro(C.cpu().numpy(), naive.gemm(A, B)) < 1e-5
