"""Tiles at a matrix edge on the large-tile loops (needs a GPU).

The float32 direct-to-LDS loop and the split-bfloat16 ring read the rows of
A past its valid rows and the columns of B past its valid columns as copies
of the last valid ones when no output is stored there; otherwise (padded
products whose outputs reach past an operand's valid extent) they take
bounds-checked loops.  Every tile shape must give the same bits, and the
oracle's values on sampled rows (first and last included).
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


def rel_fro(got, ref):
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(np.asarray(got, np.float64) - ref) / np.linalg.norm(ref))


# (algo, levels, m, n, k): plain products with edge tiles in m, n or both
# (k a multiple of 16 or not), and grouped Winograd plans padded virtually
CASES = [("naive", 0, 1000, 1000, 1024), ("naive", 0, 520, 300, 256), ("naive", 0, 777, 1000, 520),
         ("naive", 0, 300, 1040, 1000), ("winograd", 1, 1000, 1000, 1000), ("winograd", 2, 1000, 777, 555),
         ("winograd", 2, 1536, 1300, 1024)]


@pytest.mark.parametrize("dtype,tiles", [("f32", (0, 3, 1)), ("bf16x3", (0, 6, 1))])
@pytest.mark.parametrize("algo,levels,m,n,k", CASES)
def test_edge_tiles_same_bits_on_every_tile(api, oracle_built, dtype, tiles, algo, levels, m, n, k):
    from oracle import naive
    # (uniform entries: the wide-range rows of the precision workload give
    # split-bf16 Winograd L = 2 errors near 1e-5 at such shapes on every tile)
    A_np, B_np = inputs.pair("uniform", m, n, k, 95, np.float32)
    A, B = torch.from_numpy(A_np).cuda(), torch.from_numpy(B_np).cuda()
    sched = "grouped" if levels else "auto"
    print(f"edge tiles {dtype} {algo} L={levels} {m}x{n}x{k}", flush=True)
    outs = []
    for t in tiles:
        C = torch.full((m, n), float("nan"), device="cuda")
        api.mm(A, B, algo=algo, sched=sched, cutoff=1, levels=levels, dtype=dtype, tile=t, out=C)
        outs.append(C)
    torch.cuda.synchronize()
    for t, C in zip(tiles[1:], outs[1:]):
        assert torch.equal(C, outs[0]), t
    rows = np.unique(np.r_[0, np.linspace(0, m - 1, 12).astype(np.int64), m - 1])
    err = rel_fro(outs[0][torch.from_numpy(rows).cuda()].cpu().numpy(), naive.gemm_rows(A_np, B_np, rows))
    assert err < 1e-5, err


@pytest.mark.parametrize("dtype,tile", [("f32", 3), ("f32", 0), ("bf16x3", 6)])
@pytest.mark.parametrize("m,n,k", [(600, 520, 256), (1000, 777, 96)])
def test_unaligned_output_rows_same_bits(api, oracle_built, dtype, tile, m, n, k):
    # the epilogue stores interior waves with one buffer store per row (or
    # per element when C's rows are not 16-byte aligned): an output whose
    # leading dimension is odd must get the bits of a compact one, and
    # nothing outside it may be written
    A_np, B_np = inputs.pair("uniform", m, n, k, 96, np.float32)
    A, B = torch.from_numpy(A_np).cuda(), torch.from_numpy(B_np).cuda()
    print(f"unaligned C {dtype} tile {tile} {m}x{n}x{k}", flush=True)
    ref = torch.full((m, n), float("nan"), device="cuda")
    api.mm(A, B, algo="naive", dtype=dtype, tile=tile, out=ref)
    wide = torch.full((m, n + 3), 7.0, device="cuda")
    api.mm(A, B, algo="naive", dtype=dtype, tile=tile, out=wide[:, 1:n + 1])
    torch.cuda.synchronize()
    assert torch.equal(wide[:, 1:n + 1], ref)
    assert bool((wide[:, 0] == 7.0).all()) and bool((wide[:, n + 1:] == 7.0).all())
