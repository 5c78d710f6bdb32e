"""Parity at the full sizes of the speed target and the batched workload
(needs a GPU), through the C ABI.

* Square float32 n = 8192 (the size the Winograd-beats-plain target is set
  at): Strassen-Winograd with one and two levels, each with the autotuner's
  options for that level count, the plain MFMA GEMM and Strassen beside
  them, on uniform and on row-scaled Gaussian inputs.  The oracle computes
  a sample of rows that includes the first and the last row and the rows on
  either side of every quadrant boundary.
* The batched workload: problems with m, n, k log-uniform in [64, 2048],
  levels 0..2, run as one batched plan replayed from a hipGraph, bitwise
  equal to the same products run one at a time and close to the oracle.

Besides the relative Frobenius norm, every floating-point comparison here
bounds each element's error: a wrong tile or row cannot hide under a norm
taken over millions of correct elements.  Fast methods do not satisfy
componentwise bounds in |A||B| (their block sums mix rows of A and columns
of B), so the per-element scale is alpha_i beta_j, with alpha_i the largest
2-norm among the rows of A that the recursion adds into row i (the rows at
the same offset in each of the 2^L row blocks of the padded matrix) and
beta_j the same for the columns of B.  For L = 0 that is |a_i| |b_j| >= |c_ij|.
"""
import numpy as np
import pytest

from paper_2309_00628_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U32 = 2.0 ** -24   # float32 unit roundoff


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
    return float(np.linalg.norm(np.asarray(got, dtype=np.float64) - ref) / np.linalg.norm(ref))


def mixed_norms(X, idx, padded, L, axis):
    """For each index in ``idx``: the largest 2-norm among the rows (axis 0)
    or columns (axis 1) of X at the same offset in each of the 2^L blocks of
    a dimension padded to ``padded``."""
    X = np.asarray(X, dtype=np.float64)
    norms = np.linalg.norm(X, axis=1 - axis)
    blk = padded >> L
    out = np.empty(len(idx))
    for t, i in enumerate(idx):
        cand = [(i % blk) + q * blk for q in range(1 << L)]
        out[t] = max(norms[c] for c in cand if c < len(norms))
    return out


def elem_ratio(got, ref, A, B, rows, L, M, N):
    """max over the checked elements of |C - C*|_ij / (alpha_i beta_j), in
    units of the float32 unit roundoff."""
    alpha = mixed_norms(A, rows, M, L, 0)
    beta = mixed_norms(B, np.arange(B.shape[1]), N, L, 1)
    err = np.abs(np.asarray(got, np.float64) - ref)
    return float(np.max(err / np.outer(alpha, beta)) / U32)


# Per-element bound in units of u: 64 u for the plain product, doubled per
# level (every level adds block sums of up to four terms before and after
# the products).  With uniform inputs |c_ij| / (alpha_i beta_j) ~ 3/sqrt(n),
# so at n = 8192 the plain product's bound flags a relative error of about
# 1e-3 in a single element; each case prints its observed maximum.
def elem_bound(L):
    return 64.0 * 2 ** L


def boundary_rows(n, L=2, count=24, seed=31):
    rows = {0, n - 1}
    for q in range(1, 1 << L):
        b = q * n >> L
        rows |= {b - 1, b}
    rows |= set(inputs.rng(seed).choice(n, size=count, replace=False).tolist())
    return np.array(sorted(rows), dtype=np.int64)


@pytest.fixture(scope="module")
def big_inputs(naive):
    n = 8192
    out = {}
    rows = boundary_rows(n)
    for kind in ("uniform", "gauss_rowscaled"):
        A, B = inputs.pair(kind, n, n, n, 40, np.float32)
        out[kind] = (A, B, rows, naive.gemm_rows(A, B, rows))
    return out


@pytest.mark.parametrize("kind", ["uniform", "gauss_rowscaled"])
def test_fp32_8192_winograd_tuned_options(api, big_inputs, kind):
    from paper_2309_00628_amd import tuner
    n = 8192
    A, B, rows, ref = big_inputs[kind]
    At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    ridx = torch.from_numpy(rows).cuda()
    cases = [("naive", "auto", 0, {})]
    for lv in (1, 2):
        o = tuner.options_at(n, n, n, "f32", lv)
        opts = {} if o is None else dict(tile=o[0], overlap=o[1], leaf_u=o[2], trans_b=o[3])
        cases += [("winograd", "grouped", lv, opts), ("winograd", "grouped", lv, {}),
                  ("strassen", "grouped", lv, {})]
    for algo, sched, lv, opts in cases:
        print(f"fp32 {kind} n={n} {algo}/{sched} L={lv} {opts}", flush=True)
        C = api.mm(At, Bt, algo=algo, sched=sched, cutoff=1, levels=lv, **opts)
        torch.cuda.synchronize()
        got = C[ridx].cpu().numpy()
        err = rel_fro(got, ref)
        ratio = elem_ratio(got, ref, A, B, rows, lv, n, n)
        print(f"   rel err {err:.3e}, max element error {ratio:.2f} u (bound {elem_bound(lv):.0f} u)",
              flush=True)
        assert err < 1e-5, (algo, lv, opts, err)
        assert ratio < elem_bound(lv), (algo, lv, opts, ratio)
        del C


def test_elementwise_bound_catches_a_local_error(big_inputs):
    """The per-element check of the plain product flags a relative error of
    1e-3 in one element of magnitude |c_ij| ~ sqrt(n)/3, which the relative
    Frobenius norm over the sampled rows does not."""
    A, B, rows, ref = big_inputs["uniform"]
    bad = ref.copy()
    j = int(np.argmax(np.abs(ref[3]) > 0.5 * np.sqrt(8192) / 3))
    bad[3, j] *= 1.0 + 1e-3
    assert rel_fro(bad, ref) < 1e-5
    assert elem_ratio(bad, ref, A, B, rows, 0, 8192, 8192) > elem_bound(0)


def test_batched_workload_graph_replay(api, naive):
    """96 problems of the batched workload's distribution (m, n, k
    log-uniform in [64, 2048], multiples of 16), levels 0, 1, 2 in turn,
    as one batched plan captured in a hipGraph: three replays with other
    work between them, each bitwise equal to the problems run one at a
    time, and every problem within tolerance of the oracle."""
    shapes = inputs.batched_shapes(96, 23)
    g = torch.Generator(device="cuda")
    g.manual_seed(23)
    As, Bs, Cs = [], [], []
    for (m, n, k) in shapes:
        As.append(torch.rand((m, k), generator=g, device="cuda") * 2 - 1)
        Bs.append(torch.rand((k, n), generator=g, device="cuda") * 2 - 1)
        Cs.append(torch.empty((m, n), device="cuda"))
    levels = [i % 3 for i in range(len(shapes))]
    plan = api.BatchedPlan(As, Bs, Cs, cutoff=[1] * len(shapes), levels=levels, graph=True)
    singles = []
    for A, B, lv in zip(As, Bs, levels):
        singles.append(api.mm(A, B, algo="winograd", sched="grouped", cutoff=1, levels=lv))
    torch.cuda.synchronize()
    scratch = torch.empty(1 << 22, device="cuda")
    for rep in range(3):
        for C in Cs:
            C.fill_(float("nan"))
        plan()
        scratch.normal_()                   # other work between replays
        torch.cuda.synchronize()
        for i, (C, S) in enumerate(zip(Cs, singles)):
            assert torch.equal(C, S), (rep, i, shapes[i], levels[i])
    for i, ((m, n, k), lv) in enumerate(zip(shapes, levels)):
        A, B = As[i].cpu().numpy(), Bs[i].cpu().numpy()
        rows = np.unique(np.r_[0, np.linspace(0, m - 1, 16).astype(np.int64), m - 1])
        ref = naive.gemm_rows(A, B, rows)
        got = Cs[i][torch.from_numpy(rows).cuda()].cpu().numpy()
        err = rel_fro(got, ref)
        # the batched plan pads each dimension to a multiple of 2^L (times
        # the 16-byte vector width when the leaf is large enough)
        step = 1 << lv
        g16 = 4 if lv and min(m, n, k) // step >= 32 else 1
        M = -(-m // (step * g16)) * step * g16 if lv else m
        N = -(-n // (step * g16)) * step * g16 if lv else n
        ratio = elem_ratio(got, ref, A, B, rows, lv, M, N)
        assert err < 1e-5, (i, shapes[i], lv, err)
        assert ratio < elem_bound(lv), (i, shapes[i], lv, ratio)


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_fp32_3000_padded_to_3072(api, naive, levels):
    """n = 3000 zero-padded (virtually) to 3072 (MM_PLAN_PAD): within
    tolerance of the oracle on sampled rows, first and last included, and
    no element of the padding written."""
    n = 3000
    A, B = inputs.pair("uniform", n, n, n, 44, np.float32)
    rows = np.unique(np.r_[0, inputs.rng(45).choice(n, 30, replace=False), n - 1])
    ref = naive.gemm_rows(A, B, rows)
    At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    p = api.Plan("winograd", "grouped", n, n, n, cutoff=1, levels=levels, pad_to=1024, ldc=n + 16)
    assert p.info["M"] == 3072
    Cw = torch.full((n, n + 16), 7.0, device="cuda")
    C = Cw[:, :n]
    ws = torch.empty(max(p.ws_bytes, 256), dtype=torch.uint8, device="cuda")
    p(At, Bt, C, ws)
    torch.cuda.synchronize()
    got = C[torch.from_numpy(rows).cuda()].cpu().numpy()
    err = rel_fro(got, ref)
    print(f"n=3000 padded to 3072 L={levels}: rel err {err:.3e}", flush=True)
    assert err < 1e-5
    assert bool(torch.all(Cw[:, n:] == 7.0))
    assert elem_ratio(got, ref, A, B, rows, levels, 3072, 3072) < elem_bound(levels)
