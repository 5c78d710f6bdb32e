"""Operands whose leading dimension is 2^21 floats or more (needs a GPU).

The large-tile loops address a stage with 32-bit per-lane byte offsets from
the stage's first element (direct-to-LDS loads of the float32 GEMM, buffer
loads of the split-bfloat16 ring tile); those offsets fit only for leading
dimensions below 2^21, and larger ones take the loops with 64-bit addresses.
Both loops issue the same products in the same order, so the product of a
strided operand must have the same bits as the product of its compact copy.
Each case is also checked against the oracle on sampled rows.
"""
import numpy as np
import pytest

from paper_2309_00628_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

BIG = (1 << 21) + 64  # floats per row of the strided operand


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_00628_amd import api as a
    return a


def strided(x, ld):
    """A device copy of x whose rows are ld floats apart."""
    buf = torch.empty((x.shape[0], ld), dtype=torch.float32, device="cuda")
    v = buf[:, :x.shape[1]]
    v.copy_(torch.from_numpy(x))
    return v


def rel_fro(got, ref):
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(np.asarray(got, np.float64) - ref) / np.linalg.norm(ref))


# (algo, levels, dtype, tile, m, n, k, which operand is strided)
CASES = [("naive", 0, "bf16x3", 6, 512, 512, 256, "B"), ("naive", 0, "bf16x3", 6, 256, 512, 256, "A"),
         ("naive", 0, "bf16x3", 6, 512, 256, 32, "B"), ("naive", 0, "f32", 3, 512, 512, 256, "B"),
         ("naive", 0, "f32", 3, 256, 512, 256, "A"), ("winograd", 1, "f32", 3, 512, 512, 512, "B"),
         ("winograd", 1, "bf16x3", 6, 512, 512, 512, "A")]


@pytest.mark.parametrize("algo,levels,dtype,tile,m,n,k,which", CASES)
def test_large_leading_dimension_same_bits(api, oracle_built, algo, levels, dtype, tile, m, n, k, which):
    from oracle import naive
    A_np, B_np = inputs.pair("gauss_rowscaled" if dtype == "bf16x3" else "uniform", m, n, k, 90, np.float32)
    A, B = torch.from_numpy(A_np).cuda(), torch.from_numpy(B_np).cuda()
    sched = "grouped" if levels else "auto"
    kw = dict(algo=algo, sched=sched, cutoff=1, levels=levels, dtype=dtype, tile=tile)
    print(f"large ld {algo} L={levels} {dtype} tile {tile} {m}x{n}x{k} strided {which}", flush=True)
    ref = api.mm(A, B, **kw)
    As = strided(A_np, BIG) if which == "A" else A
    Bs = strided(B_np, BIG) if which == "B" else B
    assert (As.stride(0) if which == "A" else Bs.stride(0)) == BIG
    C = torch.full((m, n), float("nan"), device="cuda")
    api.mm(As, Bs, out=C, **kw)
    torch.cuda.synchronize()
    assert torch.equal(C, ref)
    rows = np.unique(np.r_[0, np.linspace(0, m - 1, 9).astype(np.int64), m - 1])
    err = rel_fro(C[torch.from_numpy(rows).cuda()].cpu().numpy(), naive.gemm_rows(A_np, B_np, rows))
    assert err < 1e-5, err
    del As, Bs
    torch.cuda.empty_cache()
