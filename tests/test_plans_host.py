"""Host-side checks of libmm's planner (no GPU needed).

The library lists the launch sequence it would run (mm_describe); the
simulator in plan_sim executes that listing on integer numpy buffers.  Every
schedule must reproduce the oracle's product exactly, with no two operations
of one launch conflicting, and the plan facts (levels, padding, workspace,
launches) must follow the paper's formulas.
"""
import os

import numpy as np
import pytest

import plan_sim
from paper_2309_00628_amd import inputs

L = pytest.importorskip("paper_2309_00628_amd._lib")


@pytest.fixture(scope="module")
def lib():
    try:
        return L.load()
    except RuntimeError as e:
        pytest.skip(str(e))


@pytest.fixture(scope="module")
def naive(oracle_built):
    from oracle import naive
    return naive


ESZ = {"f64": 8, "f32": 4}


def simulate(algo, sched, m, n, k, cutoff, levels=-1, dtype="f64", seed=0, lo=-9, hi=9):
    text, info = L.describe(algo, sched, m, n, k, cutoff=cutoff, levels=levels, dtype=dtype)
    A = inputs.integers((m, k), seed, lo, hi, dtype=np.int64)
    B = inputs.integers((k, n), seed + 1, lo, hi, dtype=np.int64)
    ws = np.full(max(info["ws_bytes"] // ESZ[dtype], 1), 10**9, dtype=np.int64)  # poison
    C = np.full(m * n, -(10**9), dtype=np.int64)
    mem = plan_sim.run(text, {0: A.ravel().copy(), 1: B.ravel().copy(), 2: C, 3: ws})
    return A, B, mem.bufs[2].reshape(m, n), info, text


CASES = [
    # algo, sched, m, n, k, cutoff
    ("naive", "auto", 7, 5, 3, 1),
    ("winograd", "two_temp", 4, 4, 4, 1),
    ("winograd", "two_temp", 8, 8, 8, 2),
    ("winograd", "two_temp", 16, 32, 8, 2),
    ("winograd", "two_temp", 13, 7, 5, 1),      # padded (copies)
    ("winograd", "two_temp", 100, 60, 80, 8),
    ("winograd", "in_place", 4, 4, 4, 1),
    ("winograd", "in_place", 8, 8, 8, 2),
    ("winograd", "in_place", 32, 16, 16, 2),
    ("winograd", "in_place", 12, 12, 12, 1),    # padded to 16
    ("winograd", "grouped", 4, 4, 4, 1),
    ("winograd", "grouped", 8, 8, 8, 1),
    ("winograd", "grouped", 13, 7, 5, 1),       # virtual padding
    ("winograd", "grouped", 100, 60, 80, 8),
    ("winograd", "grouped", 200, 136, 72, 16),
    ("winograd", "grouped", 128, 128, 128, 16),
    ("strassen", "dfs3", 4, 4, 4, 1),
    ("strassen", "dfs3", 8, 8, 8, 1),
    ("strassen", "dfs3", 16, 8, 32, 2),
    ("strassen", "dfs3", 13, 7, 5, 1),
    ("strassen", "dfs3", 64, 64, 64, 4),
    ("strassen", "grouped", 4, 4, 4, 1),
    ("strassen", "grouped", 8, 8, 8, 1),
    ("strassen", "grouped", 13, 7, 5, 1),       # virtual padding
    ("strassen", "grouped", 100, 60, 80, 8),
    ("strassen", "grouped", 200, 136, 72, 16),
]


@pytest.mark.parametrize("algo,sched,m,n,k,cutoff", CASES)
def test_schedule_exact_on_integers(lib, algo, sched, m, n, k, cutoff):
    A, B, C, info, _ = simulate(algo, sched, m, n, k, cutoff)
    assert np.array_equal(C, A @ B)


def test_oracle_agrees_with_simulated_plan(lib, naive):
    A, B, C, _, _ = simulate("winograd", "grouped", 24, 40, 16, 2)
    assert np.array_equal(C.astype(np.float64), naive.gemm(A, B))


def test_zero_inner_dimension_gives_zeros(lib):
    for algo, sched in [("naive", "auto"), ("winograd", "grouped"), ("winograd", "two_temp"),
                        ("strassen", "dfs3")]:
        A, B, C, info, _ = simulate(algo, sched, 6, 5, 0, 1)
        assert np.array_equal(C, np.zeros((6, 5), dtype=np.int64))
        assert info["levels"] == 0


def test_levels_rule_matches_oracle(lib):
    from oracle import recursions
    for (m, n, k, cutoff, levels) in [(512, 512, 512, 64, -1), (512, 512, 512, 64, 2),
                                      (8, 8, 8, 1, -1), (8, 8, 8, 2, -1), (4096, 4096, 4096, 2048, -1),
                                      (64, 32, 128, 4, -1), (16, 16, 16, 12, -1)]:
        _, info = L.describe("winograd", "two_temp", m, n, k, cutoff=cutoff, levels=levels)
        assert info["levels"] == recursions.levels_planned(m, k, n, cutoff, levels)


def test_two_temp_workspace_formula(lib):
    # Section 3.3: two temporaries per level, (n/2^l)^2 elements each
    for n, cutoff, dtype in [(512, 64, "f64"), (256, 32, "f32"), (64, 8, "f64")]:
        _, info = L.describe("winograd", "two_temp", n, n, n, cutoff=cutoff, dtype=dtype)
        Lv = info["levels"]
        assert info["ws_bytes"] == sum(2 * (n >> l) ** 2 for l in range(1, Lv + 1)) * ESZ[dtype]


def test_in_place_needs_no_workspace(lib):
    _, info = L.describe("winograd", "in_place", 512, 512, 512, cutoff=64, dtype="f64")
    assert info["ws_bytes"] == 0 and info["levels"] == 3


def test_grouped_launch_count_and_leaves(lib):
    def count(text, what):
        return sum(l.startswith("LAUNCH " + what) for l in text.splitlines())
    for L_ in (1, 2, 3):
        text, info = L.describe("winograd", "grouped", 4096, 4096, 4096, cutoff=1, levels=L_)
        assert info["levels"] == L_
        # S/T passes, the leaf products (one launch, or two that each fill
        # whole rounds of workgroups), U passes: levels 0 and 1 (2 and 3, ...)
        # as one two-level pass each, an unpaired last level on its own
        g = count(text, "GEMM")
        assert count(text, "EW2") == 2 * (L_ // 2) and count(text, "EW ") == 2 * (L_ % 2) and g in (1, 2)
        assert info["launches"] == 2 * (L_ // 2) + 2 * (L_ % 2) + g
        assert info["leaves"] == 7 ** L_ and info["fused"] == 0
        # with MM_PLAN_OVERLAP: fork, the S/T passes (auxiliary stream), the
        # products of blocks of A and B, join, the other products, the U passes
        text, info = L.describe("winograd", "grouped", 4096, 4096, 4096, cutoff=1, levels=L_, overlap=True)
        g = count(text, "GEMM")
        assert "FORK" in text and "JOIN" in text and g >= 2
        assert info["launches"] == 2 * (L_ // 2) + 2 * (L_ % 2) + g + 2
        # with MM_PLAN_FUSE the last level's S/T pass is formed in the leaf loader
        text, info = L.describe("winograd", "grouped", 4096, 4096, 4096, cutoff=1, levels=L_, fuse=True)
        assert count(text, "EW") == 2 * L_ - 1 and info["fused"] == 1


def test_grouped_strassen_launches(lib):
    # Strassen breadth first: one pass per level forms the ten operand sums,
    # the 7^L leaves run grouped, one pass per level forms the C quadrants;
    # the options particular to Winograd's operands are ignored
    def count(text, what):
        return sum(l.startswith("LAUNCH " + what) for l in text.splitlines())
    for L_ in (1, 2, 3):
        for opts in ({}, {"overlap": True}, {"fuse": True}, {"leaf_u": True}):
            text, info = L.describe("strassen", "grouped", 4096, 4096, 4096, cutoff=1, levels=L_, **opts)
            g = count(text, "GEMM")
            assert count(text, "EW") == 2 * L_ and g in (1, 2) and "FORK" not in text
            assert info["launches"] == 2 * L_ + g and info["leaves"] == 7 ** L_
            assert info["fused"] == 0 and info["leaf_u"] == 0
    # the schedule AUTO resolves to for Strassen
    _, info = L.describe("strassen", "auto", 512, 512, 512, cutoff=64)
    _, info_g = L.describe("strassen", "grouped", 512, 512, 512, cutoff=64)
    assert info["sched"] == info_g["sched"]


def test_leaf_launches_fill_whole_rounds(lib):
    # seven 2048^3 leaves: four on 256x256 tiles (256 workgroups, one round)
    # and three on 128x128 tiles (768 workgroups, three rounds)
    text, _ = L.describe("winograd", "grouped", 4096, 4096, 4096, cutoff=1, levels=1)
    gl = [l.split() for l in text.splitlines() if l.startswith("LAUNCH GEMM")]
    assert [(int(w[2]), int(w[3]), int(w[4])) for w in gl] == [(4, 256, 3), (3, 768, 0)]
    # a forced tile keeps one launch
    text, _ = L.describe("winograd", "grouped", 4096, 4096, 4096, cutoff=1, levels=1, tile=0)
    assert sum(l.startswith("LAUNCH GEMM") for l in text.splitlines()) == 1


def test_grouped_overlap_window(lib):
    # one level: the S and T passes run on the auxiliary stream beside
    # P1 = A11 B11 and P2 = A12 B21, which read only blocks of A and B
    text, info = L.describe("winograd", "grouped", 512, 512, 512, cutoff=1, levels=1, overlap=True)
    lines = [l for l in text.splitlines() if l in ("FORK", "JOIN") or l.startswith("LAUNCH")]
    assert lines[0] == "FORK" and lines[1].endswith(" aux") and lines[1].startswith("LAUNCH EW")
    assert lines[2].startswith("LAUNCH GEMM 2 ") and lines[3] == "JOIN"
    assert lines[4].startswith("LAUNCH GEMM 5 ") and lines[5].startswith("LAUNCH EW")
    # with the fused loader at one level there is nothing left to overlap
    text, info = L.describe("winograd", "grouped", 512, 512, 512, cutoff=1, levels=1, fuse=True,
                            overlap=True)
    assert "FORK" not in text and " aux" not in text and info["launches"] == 2
    for lv in (1, 2, 3):
        text, info = L.describe("winograd", "grouped", 1024, 1024, 1024, cutoff=1, levels=lv, overlap=True)
        plain = [l for l in text.split("JOIN")[0].splitlines() if l.startswith("GEMM")]
        assert len(plain) == 2 ** lv        # products of plain blocks of A and B


@pytest.mark.parametrize("m,n,k,levels,fuse", [(64, 64, 64, 1, False), (96, 40, 56, 2, False),
                                               (200, 136, 72, 3, False), (1000, 777, 555, 2, True),
                                               (130, 70, 90, 2, False)])
def test_overlapped_plan_is_exact(lib, m, n, k, levels, fuse):
    A = inputs.integers((m, k), 25, dtype=np.int64)
    B = inputs.integers((k, n), 26, dtype=np.int64)
    text, info = L.describe("winograd", "grouped", m, n, k, cutoff=1, levels=levels, dtype="f32", fuse=fuse,
                            overlap=True)
    assert "FORK" in text
    ws = np.full(max(info["ws_bytes"] // 4, 1), 10**9, dtype=np.int64)
    C = np.full(m * n, -(10**9), dtype=np.int64)
    plan_sim.run(text, {0: A.ravel().copy(), 1: B.ravel().copy(), 2: C, 3: ws})
    assert np.array_equal(C.reshape(m, n), A @ B)


@pytest.mark.parametrize("m,n,k,cutoff,levels", [(16, 16, 16, 1, 1), (32, 64, 16, 1, 2), (64, 64, 64, 4, -1),
                                                 (96, 40, 56, 1, 1), (200, 136, 72, 16, -1)])
def test_fused_leaves_exact_and_equal_to_unfused(lib, m, n, k, cutoff, levels):
    A = inputs.integers((m, k), 21, dtype=np.int64)
    B = inputs.integers((k, n), 22, dtype=np.int64)
    outs = []
    for fuse in (True, False):
        text, info = L.describe("winograd", "grouped", m, n, k, cutoff=cutoff, levels=levels, dtype="f32",
                                fuse=fuse)
        ws = np.full(max(info["ws_bytes"] // 4, 1), 10**9, dtype=np.int64)
        C = np.full(m * n, -(10**9), dtype=np.int64)
        plan_sim.run(text, {0: A.ravel().copy(), 1: B.ravel().copy(), 2: C, 3: ws})
        outs.append((C.reshape(m, n), info))
    assert np.array_equal(outs[0][0], A @ B)
    assert np.array_equal(outs[1][0], A @ B)
    if outs[0][1]["fused"]:
        assert outs[0][1]["ws_bytes"] <= outs[1][1]["ws_bytes"]


def test_fusion_needs_aligned_unpadded_operands(lib):
    # 3000 = 8 * 375: one level splits into 1500 (a multiple of 4 floats) -> fused
    text, info = L.describe("winograd", "grouped", 3000, 3000, 3000, cutoff=1, levels=1, fuse=True)
    assert info["fused"] == 1
    # float64 leaves are not fused
    _, info = L.describe("winograd", "grouped", 512, 512, 512, cutoff=64, dtype="f64", fuse=True)
    assert info["fused"] == 0
    # with virtual padding only the blocks that lie wholly inside the matrix
    # are fused; the listing marks every fused operand with a nonzero kind
    text, info = L.describe("winograd", "grouped", 3000, 3000, 3000, cutoff=1, levels=3, fuse=True)
    kinds = [tuple(map(int, l.split()[4:6])) for l in text.splitlines() if l.startswith("GEMM")]
    assert any(k != (0, 0) for k in kinds)
    assert sum(k == (0, 0) for k in kinds) > 2 * 49     # padded blocks stay unfused


@pytest.mark.parametrize("m,n,k", [(40, 24, 56), (1000, 777, 555)])
def test_partially_fused_padded_plan_is_exact(lib, m, n, k):
    # unaligned leading dimensions and virtual padding: only the blocks that
    # meet the fused loader's preconditions may go to the fused launch
    A = inputs.integers((m, k), 23, dtype=np.int64)
    B = inputs.integers((k, n), 24, dtype=np.int64)
    text, info = L.describe("winograd", "grouped", m, n, k, cutoff=1, levels=2, dtype="f32", fuse=True)
    ws = np.full(max(info["ws_bytes"] // 4, 1), 10**9, dtype=np.int64)
    C = np.full(m * n, -(10**9), dtype=np.int64)
    plan_sim.run(text, {0: A.ravel().copy(), 1: B.ravel().copy(), 2: C, 3: ws})
    assert np.array_equal(C.reshape(m, n), A @ B)


def test_depth_first_leaf_count(lib):
    _, info = L.describe("winograd", "two_temp", 512, 512, 512, cutoff=64, dtype="f64")
    assert info["leaves"] == 343
    _, info = L.describe("strassen", "dfs3", 512, 512, 512, cutoff=64, dtype="f64")
    assert info["leaves"] == 343


def test_grouped_pads_virtually_to_vector_multiple(lib):
    # 3000 = 8 * 375: three levels need no padding for the recursion itself;
    # the grouped schedule still rounds to a multiple of 2^L * 4 floats so
    # that every quadrant starts on a 16-byte boundary (no copy is made).
    _, info = L.describe("winograd", "grouped", 3000, 3000, 3000, cutoff=1, levels=3)
    assert (info["M"], info["N"], info["K"]) == (3008, 3008, 3008)
    _, info = L.describe("winograd", "two_temp", 3000, 3000, 3000, cutoff=1, levels=3)
    assert (info["M"], info["N"], info["K"]) == (3000, 3000, 3000)


def test_plan_listing_follows_table2_order(lib):
    text, _ = L.describe("winograd", "two_temp", 4, 4, 4, cutoff=2)
    kinds = [l.split()[0] + (" " + l.split()[1] if l.startswith("EW") else "")
             for l in text.splitlines() if not l.startswith("LAUNCH")]
    # ops 1-2, 3, 4-5, 6, 7-8, 9, 10, 11, 12, 13-17 + 18, 19+20, 21+22
    assert kinds == ["EW 2", "EW 2", "GEMM", "EW 1", "EW 2", "GEMM", "EW 2", "EW 2", "GEMM",
                     "EW 2", "GEMM", "GEMM", "EW 6", "EW 2", "GEMM", "GEMM"]


@pytest.mark.parametrize("args,msg", [
    (("winograd", "in_place", 8, 16, 8, 1), "in-place"),
    (("winograd", "two_temp", 4096, 4096, 4096, 1), "levels"),
    (("strassen", "two_temp", 8, 8, 8, 1), "Strassen"),
])
def test_rejected_plans(lib, args, msg):
    algo, sched, m, n, k, cutoff = args
    with pytest.raises(L.MMError) as e:
        L.describe(algo, sched, m, n, k, cutoff=cutoff)
    assert msg in str(e.value)


def test_batched_plan_exact(lib):
    shapes = [(16, 32, 8), (40, 24, 56), (7, 9, 11), (64, 64, 64), (0, 5, 3), (6, 4, 0)]
    cut = [2, 4, 1, 8, 1, 1]
    lev = [-1, 2, 1, -1, 1, 1]
    mem = []
    addrs = []
    mats = []
    pos = 0
    esz = 4
    for i, (m, n, k) in enumerate(shapes):
        A = inputs.integers((m, k), 100 + i, dtype=np.int64)
        B = inputs.integers((k, n), 200 + i, dtype=np.int64)
        a, b, c = pos, pos + A.size + 8, pos + A.size + B.size + 16
        pos = c + m * n + 8
        addrs.append(((a + 1024) * esz, (b + 1024) * esz, (c + 1024) * esz))
        mats.append((A, B, a, b, c))
    flat = np.full(pos + 2048, -(10**9), dtype=np.int64)
    for A, B, a, b, c in mats:
        flat[1024 + a:1024 + a + A.size] = A.ravel()
        flat[1024 + b:1024 + b + B.size] = B.ravel()
    text, info = L.batched_describe(shapes, addrs, dtype="f32", cutoff=cut, levels=lev)
    ws = np.full(max(info["ws_bytes"] // esz, 1), 10**9, dtype=np.int64)
    plan_sim.run(text, {plan_sim.MB_ABS: flat, plan_sim.MB_WS: ws})
    for (m, n, k), (A, B, a, b, c) in zip(shapes, mats):
        got = flat[1024 + c:1024 + c + m * n].reshape(m, n)
        assert np.array_equal(got, A @ B), (m, n, k)


def test_leaf_u_plan_shape(lib):
    # MM_PLAN_LEAF_U: L S/T passes, one launch for the last level's products
    # and U combinations, L - 1 U passes; no product temporaries at the last
    # level
    for lv in (1, 2, 3):
        _, ref = L.describe("winograd", "grouped", 4096, 4096, 4096, cutoff=1, levels=lv)
        text, info = L.describe("winograd", "grouped", 4096, 4096, 4096, cutoff=1, levels=lv, leaf_u=True)
        assert info["leaf_u"] == 1 and info["launches"] == 2 * lv and info["leaves"] == 7 ** lv
        assert info["ws_bytes"] < ref["ws_bytes"]
        assert sum(l.startswith("WINO") for l in text.splitlines()) == 7 ** (lv - 1)
        assert "GEMM" not in text
    # other dtypes / schedules ignore the flag
    _, info = L.describe("winograd", "grouped", 512, 512, 512, cutoff=64, dtype="f64", leaf_u=True)
    assert info["leaf_u"] == 0
    _, info = L.describe("winograd", "two_temp", 512, 512, 512, cutoff=64, leaf_u=True)
    assert info["leaf_u"] == 0


def test_zero_temporary_last_level(lib):
    # MM_PLAN_LEAF_U with MM_PLAN_FUSE: the last level reads A and B blocks,
    # forms S/T in the loader and writes C: one launch and no workspace at one
    # level (the plan's workspace size still covers the unfused plan it runs
    # when A or B is not 16-byte aligned); at L levels the last level's S/T
    # temporaries and pass disappear
    text, info = L.describe("winograd", "grouped", 4096, 4096, 4096, cutoff=1, levels=1, leaf_u=True, fuse=True)
    assert info["launches"] == 1 and info["fused"] == 1 and info["leaf_u"] == 1
    assert [l.split()[1] for l in text.splitlines() if l.startswith("LAUNCH")] == ["WINO"]
    assert not any(tok.startswith(f"{plan_sim.MB_WS}:") for tok in text.split())
    for lv in (2, 3):
        text, info = L.describe("winograd", "grouped", 4096, 4096, 4096, cutoff=1, levels=lv, leaf_u=True,
                                fuse=True)
        assert info["launches"] == 2 * lv - 1 and info["fused"] == 1
        assert sum(l.startswith("LAUNCH EW") for l in text.splitlines()) == 2 * (lv - 1)
    # a last level with padding keeps the S/T pass
    _, info = L.describe("winograd", "grouped", 1000, 777, 555, cutoff=1, levels=2, leaf_u=True, fuse=True)
    assert info["fused"] == 0 and info["leaf_u"] == 1


@pytest.mark.parametrize("m,n,k,levels", [(16, 16, 16, 1), (64, 64, 64, 2), (96, 40, 56, 2), (256, 128, 192, 3),
                                          (1000, 777, 555, 2), (128, 64, 96, 1)])
def test_zero_temporary_plan_is_exact(lib, m, n, k, levels):
    A = inputs.integers((m, k), 29, dtype=np.int64)
    B = inputs.integers((k, n), 30, dtype=np.int64)
    text, info = L.describe("winograd", "grouped", m, n, k, cutoff=1, levels=levels, dtype="f32", leaf_u=True,
                            fuse=True)
    ws = np.full(max(info["ws_bytes"] // 4, 1), 10**9, dtype=np.int64)
    C = np.full(m * n, -(10**9), dtype=np.int64)
    plan_sim.run(text, {0: A.ravel().copy(), 1: B.ravel().copy(), 2: C, 3: ws})
    assert np.array_equal(C.reshape(m, n), A @ B)


@pytest.mark.parametrize("m,n,k,levels", [(16, 16, 16, 1), (64, 64, 64, 2), (96, 40, 56, 2), (200, 136, 72, 3),
                                          (1000, 777, 555, 2), (130, 70, 90, 1), (8, 300, 64, 1)])
def test_leaf_u_plan_is_exact(lib, m, n, k, levels):
    A = inputs.integers((m, k), 27, dtype=np.int64)
    B = inputs.integers((k, n), 28, dtype=np.int64)
    text, info = L.describe("winograd", "grouped", m, n, k, cutoff=1, levels=levels, dtype="f32", leaf_u=True)
    assert info["leaf_u"] == 1
    ws = np.full(max(info["ws_bytes"] // 4, 1), 10**9, dtype=np.int64)
    C = np.full(m * n, -(10**9), dtype=np.int64)
    plan_sim.run(text, {0: A.ravel().copy(), 1: B.ravel().copy(), 2: C, 3: ws})
    assert np.array_equal(C.reshape(m, n), A @ B)


@pytest.mark.parametrize("algo,m,n,k,levels", [("naive", 100, 60, 36, 0), ("naive", 33, 17, 9, 0),
                                               ("winograd", 64, 64, 64, 1), ("winograd", 96, 40, 56, 2),
                                               ("winograd", 130, 70, 90, 1), ("winograd", 72, 48, 40, 3)])
def test_split_bf16_plans_are_exact(lib, algo, m, n, k, levels):
    # refined split-bfloat16 leaves read operands split by a split pass (the
    # last level's S/T sums formed there too); the listing, simulated on
    # integers, gives the exact product and has no hazards
    A = inputs.integers((m, k), 29, dtype=np.int64)
    B = inputs.integers((k, n), 30, dtype=np.int64)
    text, info = L.describe(algo, "grouped" if levels else "auto", m, n, k, cutoff=1, levels=levels,
                            dtype="bf16x3", split_pass=True)
    assert "LAUNCH SPLIT" in text and " spl" in text
    assert sum(l.startswith("GEMM") for l in text.splitlines()) == 7 ** levels
    ws = np.full(max(info["ws_bytes"] // 4, 1), 10**9, dtype=np.int64)
    C = np.full(m * n, -(10**9), dtype=np.int64)
    plan_sim.run(text, {0: A.ravel().copy(), 1: B.ravel().copy(), 2: C, 3: ws})
    assert np.array_equal(C.reshape(m, n), A @ B)
    # by default the leaf kernel splits its tiles itself
    text, _ = L.describe(algo, "grouped" if levels else "auto", m, n, k, cutoff=1, levels=levels,
                         dtype="bf16x3")
    assert "SPLIT" not in text and " spl" not in text


ACC_CASES = [("naive", "auto", 40, 24, 56, -1, {}), ("naive", "auto", 17, 9, 0, -1, {}),
             ("winograd", "grouped", 64, 64, 64, 1, {}), ("winograd", "grouped", 96, 40, 56, 2, {}),
             ("winograd", "grouped", 130, 70, 90, 2, {"leaf_u": True}),
             ("winograd", "grouped", 64, 48, 32, 1, {"leaf_u": True}),
             ("winograd", "grouped", 96, 64, 64, 2, {"overlap": True}),
             ("winograd", "grouped", 64, 64, 64, 1, {"fuse": True}),
             ("winograd", "two_temp", 64, 32, 48, 2, {}), ("winograd", "in_place", 64, 32, 32, 2, {}),
             ("winograd", "two_temp", 50, 30, 40, 2, {}), ("strassen", "dfs3", 48, 40, 24, 2, {}),
             ("strassen", "grouped", 48, 40, 24, 2, {}), ("strassen", "grouped", 70, 50, 90, 1, {})]


@pytest.mark.parametrize("algo,sched,m,n,k,levels,opts", ACC_CASES)
@pytest.mark.parametrize("beta", [2, 0, -1])
def test_accumulating_plans_are_exact(lib, algo, sched, m, n, k, levels, opts, beta):
    # MM_PLAN_ACCUMULATE: C <- A B + beta C, exact on integers for every
    # schedule; with beta = 0 the old C is never read
    A = inputs.integers((m, k), 31, dtype=np.int64)
    B = inputs.integers((k, n), 32, dtype=np.int64)
    C0 = inputs.integers((m, n), 33, dtype=np.int64)
    text, info = L.describe(algo, sched, m, n, k, cutoff=1, levels=levels, dtype="f32", accumulate=True,
                            **opts)
    ws = np.full(max(info["ws_bytes"] // 4, 1), 10**9, dtype=np.int64)
    C = C0.ravel().copy() if beta else np.full(m * n, 10**12, dtype=np.int64)
    plan_sim.run(text, {0: A.ravel().copy(), 1: B.ravel().copy(), 2: C, 3: ws}, beta=beta)
    want = A @ B + (beta * C0 if beta else 0)
    assert np.array_equal(C.reshape(m, n), want)


PEEL_CASES = [("winograd", 13, 7, 5, 1, -1), ("winograd", 100, 60, 80, 8, -1), ("winograd", 200, 136, 72, 1, 2),
              ("winograd", 161, 130, 199, 1, 2), ("winograd", 64, 64, 70, 1, 1), ("winograd", 70, 64, 64, 1, 1),
              ("winograd", 64, 70, 64, 1, 1), ("strassen", 161, 130, 199, 1, 2), ("strassen", 29, 31, 37, 1, 2)]


@pytest.mark.parametrize("algo,m,n,k,cutoff,levels", PEEL_CASES)
def test_peeled_plans_are_exact(lib, algo, m, n, k, cutoff, levels):
    # MM_PLAN_PEEL: the recursion on the leading block, thin products for the
    # rest; exact on integers, no virtual padding
    A = inputs.integers((m, k), 41, dtype=np.int64)
    B = inputs.integers((k, n), 42, dtype=np.int64)
    text, info = L.describe(algo, "grouped", m, n, k, cutoff=cutoff, levels=levels, dtype="f32", peel=True)
    _, info0 = L.describe(algo, "grouped", m, n, k, cutoff=cutoff, levels=levels, dtype="f32")
    dims, dims0 = (info["M"], info["N"], info["K"]), (info0["M"], info0["N"], info0["K"])
    # peeled (no side beyond the matrix), or padded when a side of the leading
    # block would be empty (13 x 7 x 5 has three levels: 5 < 2^3)
    assert (dims[0] <= m and dims[1] <= n and dims[2] <= k) or dims == dims0
    ws = np.full(max(info["ws_bytes"] // 4, 1), 10**9, dtype=np.int64)
    C = np.full(m * n, -(10**9), dtype=np.int64)
    plan_sim.run(text, {0: A.ravel().copy(), 1: B.ravel().copy(), 2: C, 3: ws})
    assert np.array_equal(C.reshape(m, n), A @ B)
    assert info0["levels"] == info["levels"]


@pytest.mark.parametrize("beta", [3, 0])
def test_peeled_accumulating_plan(lib, beta):
    m, n, k = 150, 98, 123
    A = inputs.integers((m, k), 43, dtype=np.int64)
    B = inputs.integers((k, n), 44, dtype=np.int64)
    C0 = inputs.integers((m, n), 45, dtype=np.int64)
    text, info = L.describe("winograd", "grouped", m, n, k, cutoff=1, levels=2, dtype="f32", peel=True,
                            accumulate=True)
    ws = np.full(max(info["ws_bytes"] // 4, 1), 10**9, dtype=np.int64)
    C = C0.ravel().copy() if beta else np.full(m * n, 10**12, dtype=np.int64)
    plan_sim.run(text, {0: A.ravel().copy(), 1: B.ravel().copy(), 2: C, 3: ws}, beta=beta)
    assert np.array_equal(C.reshape(m, n), A @ B + (beta * C0 if beta else 0))


def test_peel_launch_structure(lib):
    # 3000 = 93 * 32 + 24 with L = 3 and groups of 4 float32 (16 bytes): the
    # recursion runs on 2976^3 and one more launch holds the three thin products
    text, info = L.describe("winograd", "grouped", 3000, 3000, 3000, cutoff=1, levels=3, peel=True)
    _, info0 = L.describe("winograd", "grouped", 3000, 3000, 3000, cutoff=1, levels=3)
    assert (info["M"], info["N"], info["K"]) == (2976, 2976, 2976)
    assert (info0["M"], info0["N"], info0["K"]) == (3008, 3008, 3008)
    # the peeled recursion is entirely valid, so levels 0 and 1 pair into
    # two-level passes (2 launches for both levels' S/T and U) while the
    # zero-padded one keeps a pass per level: one launch per level fewer,
    # one more for the thin products
    kinds = [l.split()[1] for l in text.splitlines() if l.startswith("LAUNCH")]
    kinds0 = [l.split()[1] for l in L.describe("winograd", "grouped", 3000, 3000, 3000, cutoff=1,
                                                levels=3)[0].splitlines() if l.startswith("LAUNCH")]
    assert kinds.count("EW2") == 2 and kinds.count("EW") == 2 and kinds0.count("EW") == 6
    assert info["launches"] == info0["launches"] - 2 + 1
    last = [l for l in text.splitlines() if l.startswith("LAUNCH")][-1].split()
    assert last[1] == "GEMM" and int(last[2]) == 3
    # nothing to peel: the same plan
    t1, _ = L.describe("winograd", "grouped", 4096, 4096, 4096, cutoff=1, levels=2, peel=True)
    t0, _ = L.describe("winograd", "grouped", 4096, 4096, 4096, cutoff=1, levels=2)
    assert t1 == t0


def test_plain_product_copies_unaligned_operands(lib):
    # a large plain product whose rows are not 16-byte multiples runs on
    # aligned copies (one copy launch, then the GEMM); exact on integers
    m, n, k = 513, 515, 517
    A = inputs.integers((m, k), 48, dtype=np.int64)
    B = inputs.integers((k, n), 49, dtype=np.int64)
    text, info = L.describe("naive", "auto", m, n, k, dtype="f32")
    kinds = [l.split()[1] for l in text.splitlines() if l.startswith("LAUNCH")]
    assert kinds == ["EW", "GEMM"] and info["ws_bytes"] > 0
    ws = np.full(info["ws_bytes"] // 4, 10**9, dtype=np.int64)
    C = np.full(m * n, -(10**9), dtype=np.int64)
    plan_sim.run(text, {0: A.ravel().copy(), 1: B.ravel().copy(), 2: C, 3: ws})
    assert np.array_equal(C.reshape(m, n), A @ B)
    # aligned, or small: one GEMM, no workspace
    for shape in ((512, 512, 512), (100, 101, 99)):
        text, info = L.describe("naive", "auto", *shape, dtype="f32")
        assert [l.split()[1] for l in text.splitlines() if l.startswith("LAUNCH")] == ["GEMM"]
        assert info["ws_bytes"] == 0


@pytest.mark.parametrize("m,n,k,levels", [(16, 16, 16, 1), (64, 64, 64, 2), (96, 40, 56, 2), (200, 136, 72, 3),
                                          (1000, 777, 555, 2), (130, 70, 90, 1), (8, 300, 64, 1)])
def test_transposed_b_plan_is_exact(lib, m, n, k, levels):
    # MM_PLAN_TRANS_B: the last level's T pass writes T1..T4 and B11, B21,
    # B22 transposed and the leaves read them as transposed B operands
    A = inputs.integers((m, k), 53, dtype=np.int64)
    B = inputs.integers((k, n), 54, dtype=np.int64)
    text, info = L.describe("winograd", "grouped", m, n, k, cutoff=1, levels=levels, dtype="f32", trans_b=True)
    ws = np.full(max(info["ws_bytes"] // 4, 1), 10**9, dtype=np.int64)
    C = np.full(m * n, -(10**9), dtype=np.int64)
    plan_sim.run(text, {0: A.ravel().copy(), 1: B.ravel().copy(), 2: C, 3: ws})
    assert np.array_equal(C.reshape(m, n), A @ B)


def test_transposed_b_plan_shape(lib):
    for lv in (1, 2):
        # (the transposing pass replaces a level's own T pass: compared with
        # the level-by-level passes)
        _, ref = L.describe("winograd", "grouped", 4096, 4096, 4096, cutoff=1, levels=lv, level_passes=True)
        text, info = L.describe("winograd", "grouped", 4096, 4096, 4096, cutoff=1, levels=lv, trans_b=True)
        launches = [l.split() for l in text.splitlines() if l.startswith("LAUNCH")]
        # the last level's S pass and transposing T pass are two launches
        assert info["launches"] == ref["launches"] + 1
        assert sum(w[1] == "TRANS" for w in launches) == 1
        assert all("bt" in w for w in launches if w[1] == "GEMM")
        # three more quarter blocks per last-level block (each with the 4 KiB
        # gap the planner leaves after temporaries of 1 MiB or more)
        q = (4096 >> lv) ** 2 * 4 + 4096
        assert info["ws_bytes"] == ref["ws_bytes"] + 3 * q * 7 ** (lv - 1)
    # other dtypes, algorithms and schedules ignore the flag
    for args in (("winograd", "grouped", 512, 512, 512, 64, "f64"), ("strassen", "grouped", 512, 512, 512, 64, "f32"),
                 ("winograd", "two_temp", 512, 512, 512, 64, "f32")):
        text, _ = L.describe(*args[:5], cutoff=args[5], dtype=args[6], trans_b=True)
        assert "TRANS" not in text


@pytest.mark.parametrize("m,n,k,levels", [(8, 8, 8, 2), (8, 8, 8, 3), (16, 16, 16, 3), (32, 32, 32, 3),
                                          (28, 30, 26, 3), (16, 16, 16, 1), (64, 64, 64, 3), (60, 62, 58, 3)])
def test_unrolled_base_case_plan_is_exact(lib, m, n, k, levels):
    # MM_PLAN_UNROLL_BASE: leaves of order 1, 2, 4 or 8 by the unrolled base case
    A = inputs.integers((m, k), 57, dtype=np.int64)
    B = inputs.integers((k, n), 58, dtype=np.int64)
    text, info = L.describe("winograd", "grouped", m, n, k, cutoff=1, levels=levels, dtype="f32",
                            unroll_base=True)
    assert "LAUNCH BASE" in text and "LAUNCH GEMM" not in text
    assert info["leaves"] == 7 ** levels
    ws = np.full(max(info["ws_bytes"] // 4, 1), 10**9, dtype=np.int64)
    C = np.full(m * n, -(10**9), dtype=np.int64)
    plan_sim.run(text, {0: A.ravel().copy(), 1: B.ravel().copy(), 2: C, 3: ws})
    assert np.array_equal(C.reshape(m, n), A @ B)


def test_unrolled_base_case_only_for_tiny_leaves(lib):
    text, _ = L.describe("winograd", "grouped", 512, 512, 512, cutoff=1, levels=2, unroll_base=True)
    assert "BASE" not in text and "LAUNCH GEMM" in text
    text, _ = L.describe("winograd", "grouped", 64, 64, 64, cutoff=1, levels=4, dtype="f64", unroll_base=True)
    assert [l.split()[4] for l in text.splitlines() if l.startswith("LAUNCH BASE")] == ["4"]
    text, _ = L.describe("winograd", "grouped", 64, 64, 64, cutoff=1, levels=3, dtype="f64", unroll_base=True)
    assert [l.split()[4] for l in text.splitlines() if l.startswith("LAUNCH BASE")] == ["8"]
    text, _ = L.describe("winograd", "grouped", 128, 128, 128, cutoff=1, levels=3, unroll_base=True)
    assert "BASE" not in text              # leaves of 16: MFMA tiles


def test_plan_flag_fields_are_disjoint():
    # the single-bit options, the tile field MM_PLAN_TILE (bits 8-15), the
    # k-split field MM_PLAN_SPLIT_K (bits 16-19) and the padding field
    # MM_PLAN_PAD (bits 24-27) of include/mm.h share no bit
    import re
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "mm.h")).read()
    bits = {name: int(v, 0) for name, v in re.findall(r"#define (MM_PLAN_[A-Z_]+) (0x[0-9a-fA-F]+|[0-9]+)u", hdr)}
    assert len(bits) >= 9
    fields = {"TILE": 0xff << 8, "SPLIT_K": 0xf << 16, "PAD": 0xf << 24}
    seen = 0
    for name, b in list(bits.items()) + list(fields.items()):
        assert b and seen & b == 0, name
        seen |= b
    for name, b in bits.items():
        assert getattr(L, name) == b, name
    assert L.plan_tile(7) == 8 << 8 and L.plan_split_k(8) == 8 << 16 and L.plan_pad(128) == 7 << 24


def test_tile_choice_and_unrolled_base_are_independent(lib):
    # forcing tile 0 (field value 1) leaves the MFMA leaves in place, and the
    # unrolled base cases leave the planner's tile choice alone
    text, _ = L.describe("winograd", "grouped", 16, 16, 16, cutoff=1, levels=2, tile=0)
    assert "BASE" not in text and "LAUNCH GEMM" in text
    for tile in (None, 3, 7):
        a, _ = L.describe("winograd", "grouped", 4096, 4096, 4096, cutoff=1, levels=1, tile=tile)
        b, _ = L.describe("winograd", "grouped", 4096, 4096, 4096, cutoff=1, levels=1, tile=tile,
                          unroll_base=True)
        assert a == b


@pytest.mark.parametrize("m,n,k,s", [(64, 48, 256, 2), (100, 60, 300, 4), (33, 17, 1000, 8), (64, 64, 64, 4)])
@pytest.mark.parametrize("acc", [False, True])
def test_split_k_plans_are_exact(lib, m, n, k, s, acc):
    # MM_PLAN_SPLIT_K: partial products over k ranges (multiples of 64) in one
    # grouped launch, then one ordered sum (with beta when accumulating)
    A = inputs.integers((m, k), 61, dtype=np.int64)
    B = inputs.integers((k, n), 62, dtype=np.int64)
    C0 = inputs.integers((m, n), 63, dtype=np.int64)
    text, info = L.describe("naive", "auto", m, n, k, dtype="f32", split_k=s, accumulate=acc)
    parts = -(-k // (-(-(-(-k // s)) // 64) * 64))
    launches = [l.split()[1] for l in text.splitlines() if l.startswith("LAUNCH")]
    assert launches == (["GEMM", "EW"] if parts > 1 else ["GEMM"])
    ws = np.full(max(info["ws_bytes"] // 4, 1), 10**9, dtype=np.int64)
    C = C0.ravel().copy()
    plan_sim.run(text, {0: A.ravel().copy(), 1: B.ravel().copy(), 2: C, 3: ws}, beta=3)
    assert np.array_equal(C.reshape(m, n), A @ B + (3 * C0 if acc else 0))


@pytest.mark.parametrize("m,n,k,levels", [(64, 48, 40, 2), (50, 70, 30, 1)])
def test_option_combinations_are_exact(lib, m, n, k, levels):
    # every combination of up to three grouped-schedule options gives the
    # exact product (accumulating ones A B + 2 C) and hazard-free launches
    import itertools
    A = inputs.integers((m, k), 67, dtype=np.int64)
    B = inputs.integers((k, n), 68, dtype=np.int64)
    C0 = inputs.integers((m, n), 69, dtype=np.int64)
    opts = ("overlap", "leaf_u", "fuse", "trans_b", "peel", "accumulate")
    for r in range(4):
        for combo in itertools.combinations(opts, r):
            text, info = L.describe("winograd", "grouped", m, n, k, cutoff=1, levels=levels, dtype="f32",
                                    **{o: True for o in combo})
            ws = np.full(max(info["ws_bytes"] // 4, 1), 10**9, dtype=np.int64)
            C = C0.ravel().copy()
            plan_sim.run(text, {0: A.ravel().copy(), 1: B.ravel().copy(), 2: C, 3: ws}, beta=2)
            want = A @ B + (2 * C0 if "accumulate" in combo else 0)
            assert np.array_equal(C.reshape(m, n), want), combo


def test_bench_tile_table_matches_the_library(lib):
    # bench.py names the kernel of a leaf launch from its tile configuration
    # (to find its measured traffic); the tile edges it assumes must give the
    # grid the library launches
    import math
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    m, n = 1000, 700
    for c, (bm, bn, bkc, wgm, wgn) in bench.GEMM_F32_TILES.items():
        text, _ = L.describe("naive", "auto", m, n, 256, tile=c)
        lau = [x for x in bench.plan_launches(type("P", (), {"describe": lambda self: text})(), 4)
               if x["kind"] == "GEMM"]
        assert len(lau) == 1 and lau[0]["cfg"] == c
        assert lau[0]["grid"] == math.ceil(m / bm) * math.ceil(n / bn), c
        assert bench.launch_kernel_name(lau[0]) == f"gemm_kernel<float, {bm}, {bn}, {bkc}, {wgm}, {wgn}, false>"
    for c, (bm, bn, bkc, wgm, wgn) in bench.WINO_TILES.items():
        text, _ = L.describe("winograd", "grouped", 2 * m, 2 * n, 512, cutoff=1, levels=1, leaf_u=True, tile=c)
        lau = [x for x in bench.plan_launches(type("P", (), {"describe": lambda self: text})(), 4)
               if x["kind"] == "WINO"]
        assert len(lau) == 1 and lau[0]["grid"] == math.ceil(m / bm) * math.ceil(n / bn), c


def _persistent_segments(text):
    """(kind, [(wait, target, signal, task_start, ntasks)]) per segment of a
    persistent batched listing, in queue order."""
    segs, cur = [], []
    for line in text.splitlines():
        if line.startswith("PDEP"):
            cur.append(tuple(map(int, line.split()[1:])))
        elif line.startswith("LAUNCH") and not line.startswith("LAUNCH PERSIST"):
            segs.append((line.split()[1], cur))
            cur = []
    assert not cur
    return segs


def _batch_fixture(shapes, seed0=100):
    mats, addrs = [], []
    pos, esz = 0, 4
    for i, (m, n, k) in enumerate(shapes):
        A = inputs.integers((m, k), seed0 + i, dtype=np.int64)
        B = inputs.integers((k, n), seed0 + 100 + i, dtype=np.int64)
        a, b, c = pos, pos + A.size + 8, pos + A.size + B.size + 16
        pos = c + m * n + 8
        addrs.append(((a + 1024) * esz, (b + 1024) * esz, (c + 1024) * esz))
        mats.append((A, B, a, b, c))
    flat = np.full(pos + 2048, -(10**9), dtype=np.int64)
    for A, B, a, b, c in mats:
        flat[1024 + a:1024 + a + A.size] = A.ravel()
        flat[1024 + b:1024 + b + B.size] = B.ravel()
    return mats, addrs, flat


def test_persistent_batched_plan_exact_and_drains(lib):
    """MM_PLAN_PERSISTENT: one launch; its queue, executed segment by
    segment, gives the exact product of every problem (integers); every
    task waits only on a counter that earlier segments alone signal, for
    exactly the number of tasks that signal it, so the workgroup holding
    the earliest unfinished task never waits on an unfinished one."""
    shapes = [(16, 32, 8), (40, 24, 56), (7, 9, 11), (64, 64, 64), (0, 5, 3), (6, 4, 0), (96, 80, 112),
              (33, 65, 17)]
    cut = [2, 4, 1, 8, 1, 1, 1, 1]
    lev = [-1, 2, 1, -1, 1, 1, 3, 0]
    mats, addrs, flat = _batch_fixture(shapes)
    text, info = L.batched_describe(shapes, addrs, dtype="f32", cutoff=cut, levels=lev, persistent=True)
    assert info["launches"] == 1
    _, ref_info = L.batched_describe(shapes, addrs, dtype="f32", cutoff=cut, levels=lev)
    assert info["ws_bytes"] == ref_info["ws_bytes"] and info["leaves"] == ref_info["leaves"]
    ws = np.full(max(info["ws_bytes"] // 4, 1), 10**9, dtype=np.int64)
    plan_sim.run(text, {plan_sim.MB_ABS: flat, plan_sim.MB_WS: ws})
    for (m, n, k), (A, B, a, b, c) in zip(shapes, mats):
        got = flat[1024 + c:1024 + c + m * n].reshape(m, n)
        assert np.array_equal(got, A @ B), (m, n, k)
    segs = _persistent_segments(text)
    signalers = {}                        # counter -> (segments, tasks)
    for si, (_, items) in enumerate(segs):
        start = 0
        for w, t, s, ts, nt in items:
            assert ts == start and nt > 0
            start += nt
            if s >= 0:
                segset, tot = signalers.get(s, (set(), 0))
                signalers[s] = (segset | {si}, tot + nt)
    for si, (_, items) in enumerate(segs):
        for w, t, s, ts, nt in items:
            if w < 0:
                continue
            segset, tot = signalers[w]
            assert max(segset) < si, (si, w)
            assert t == tot, (si, w, t, tot)
    waited = {w for _, items in segs for w, *_ in items if w >= 0}
    assert waited == set(signalers)       # every signalled counter is waited on


def test_batched_null_levels_follow_the_size_classes(lib):
    """mm_batched_levels with NULL levels: the tuned level count of each
    problem's size class (the table the library read, or the documented rule
    without one), capped by the cutoff and the shape; a batched plan built
    with NULL levels has exactly those leaves."""
    import math
    shapes = [(64, 64, 64), (2048, 2048, 2048), (4096, 4096, 4096), (8192, 8192, 8192), (100, 3000, 50),
              (1536, 256, 2048)]
    got = L.batched_levels(shapes)
    src = L.tuning_source()
    table = {}
    if src:
        for line in open(src):
            line = line.split("#")[0].split()
            if len(line) == 3 and line[0] == "f32":
                table[float(line[1])] = int(line[2])

    def expect(m, n, k):
        vol = m * n * k
        if table:
            c = math.floor(2 * math.log2(vol) / 3 + 0.5) / 2
            lv = min(table.items(), key=lambda e: abs(e[0] - c))[1]
        else:
            lv = 0
            while lv < 2 and vol >= (2048 * (2 << lv)) ** 3:
                lv += 1
        # capped by the shape (cutoff 1): halve while the smallest side > 1
        cap = 0
        while cap < lv and min(-(-m // (1 << cap)), -(-n // (1 << cap)), -(-k // (1 << cap))) > 1:
            cap += 1
        return cap
    assert got == [expect(*s) for s in shapes], (got, src)
    assert L.batched_levels(shapes, levels=[1] * 6) == [1] * 6
    assert L.batched_levels(shapes, cutoff=[4096] * 6, levels=[3] * 6) == [0, 0, 0, 1, 0, 0]
    addrs = [(4096 * (3 * i + 1), 4096 * (3 * i + 2), 4096 * (3 * i + 3)) for i in range(len(shapes))]
    _, info = L.batched_describe(shapes, [(a << 20, b << 20, c << 20) for a, b, c in addrs])
    assert info["leaves"] == sum(7 ** lv for lv in got)


@pytest.mark.parametrize("sched", ["grouped", "two_temp"])
def test_pad_to_a_multiple_is_exact(lib, sched):
    """MM_PLAN_PAD: n = 3000 needs no padding for up to three levels (the
    grouped schedule rounds to 2^L times the 16-byte vector width: 3008),
    and with the flag pads to 3072 (multiples of 2^7); the padded plans are
    exact on integers (simulated), for the virtual padding of the grouped
    schedule and the copies of the depth-first one."""
    _, info = L.describe("winograd", "two_temp", 3000, 3000, 3000, cutoff=1, levels=3)
    assert info["M"] == 3000 and info["leaf_rows"] == 375
    _, info = L.describe("winograd", "grouped", 3000, 3000, 3000, cutoff=1, levels=3)
    assert info["M"] == 3008 and info["leaf_rows"] == 376
    _, info = L.describe("winograd", "grouped", 3000, 3000, 3000, cutoff=1, levels=3, pad_to=128)
    assert info["M"] == info["N"] == info["K"] == 3072 and info["leaf_rows"] == 384
    _, info = L.describe("winograd", "grouped", 3000, 3000, 3000, cutoff=1, levels=0, pad_to=128)
    assert info["M"] == 3000                       # no levels: nothing to pad
    m, n, k = 40, 36, 44
    A = inputs.integers((m, k), 71, dtype=np.int64)
    B = inputs.integers((k, n), 72, dtype=np.int64)
    text, info = L.describe("winograd", sched, m, n, k, cutoff=1, levels=2, pad_to=32)
    assert info["M"] == info["N"] == info["K"] == 64
    ws = np.full(max(info["ws_bytes"] // 4, 1), 10**9, dtype=np.int64)
    C = np.full(m * n, -(10**9), dtype=np.int64)
    plan_sim.run(text, {0: A.ravel().copy(), 1: B.ravel().copy(), 2: C, 3: ws})
    assert np.array_equal(C.reshape(m, n), A @ B)


PAIR_CASES = [(64, 64, 64, 2, "f32", {}), (128, 96, 64, 2, "f32", {}), (64, 64, 64, 3, "f32", {}),
              (128, 64, 96, 2, "f32", {"overlap": True}), (128, 128, 128, 3, "f32", {"overlap": True}),
              (128, 128, 128, 4, "f32", {}), (64, 64, 64, 2, "f64", {}), (96, 64, 128, 2, "f32",
                                                                          {"unroll_base": False}),
              (64, 64, 64, 2, "f32", {"accumulate": True}), (256, 128, 192, 3, "f32", {"tile": 8})]


@pytest.mark.parametrize("m,n,k,levels,dtype,opts", PAIR_CASES)
def test_two_level_passes_are_exact(lib, m, n, k, levels, dtype, opts):
    """Levels 0 and 1 (and 2 and 3) of the grouped Winograd schedule share one
    S/T pass and one U pass (EW2); exact on integers, and the same values as
    the level-by-level passes (MM_PLAN_LEVEL_PASSES), which the listing then
    has instead."""
    A = inputs.integers((m, k), 61, dtype=np.int64)
    B = inputs.integers((k, n), 62, dtype=np.int64)
    C0 = inputs.integers((m, n), 63, dtype=np.int64)
    results = []
    for lp in (False, True):
        text, info = L.describe("winograd", "grouped", m, n, k, cutoff=1, levels=levels, dtype=dtype,
                                level_passes=lp, **opts)
        kinds = [l.split()[1] for l in text.splitlines() if l.startswith("LAUNCH")]
        pairs = levels // 2
        if lp:
            assert "EW2" not in kinds and kinds.count("EW") == 2 * levels
        else:
            # the U pair at the top of an accumulating plan stays two passes
            u_pairs = pairs - (1 if opts.get("accumulate") else 0)
            assert kinds.count("EW2") == pairs + u_pairs
        ws = np.full(max(info["ws_bytes"] // (8 if dtype == "f64" else 4), 1), 10**9, dtype=np.int64)
        C = C0.ravel().copy()
        plan_sim.run(text, {0: A.ravel().copy(), 1: B.ravel().copy(), 2: C, 3: ws}, beta=2)
        want = A @ B + (2 * C0 if opts.get("accumulate") else 0)
        assert np.array_equal(C.reshape(m, n), want)
        results.append(C)
    assert np.array_equal(results[0], results[1])


def test_two_level_passes_need_whole_blocks(lib):
    # zero-padded operands (3000 -> 3008 at three levels) and the options that
    # change a level's form keep one pass per level
    for args, opts in (((3000, 3000, 3000, 3), {}),
                       ((4096, 4096, 4096, 2), {"leaf_u": True}), ((4096, 4096, 4096, 2), {"trans_b": True}),
                       ((4096, 4096, 4096, 2), {"fuse": True}), ((4096, 4096, 4096, 2), {"level_passes": True})):
        m, n, k, lv = args
        text, _ = L.describe("winograd", "grouped", m, n, k, cutoff=1, levels=lv, **opts)
        assert "EW2" not in text, (args, opts)
    text, _ = L.describe("strassen", "grouped", 4096, 4096, 4096, cutoff=1, levels=2)
    assert "EW2" not in text


def gemm_launches(text):
    """(count, workgroups, tile) of every GEMM launch in a plan listing."""
    return [tuple(int(x) for x in l.split()[2:5]) for l in text.splitlines() if l.startswith("LAUNCH GEMM")]


def test_split_bf16_tile_choice(lib):
    # the planner's split-bfloat16 tiles: the 256x256 ring (6) from half a
    # round of its tiles up, the 128x128 ring (0) below, 64-row tiles for
    # small products
    for n, tile in ((1024, 8), (1536, 0), (2048, 0), (2560, 0), (3000, 6), (4096, 6), (8000, 6)):
        text, _ = L.describe("naive", "auto", n, n, n, cutoff=1, levels=0, dtype="bf16x3")
        assert [t for _, _, t in gemm_launches(text)] == [tile], (n, text)
    # leaves of two Winograd levels at n = 8192: 48 on the 256x256 ring (12
    # whole rounds) and one on the 128x128 ring; the model's tie between
    # 48 + 1 and 47 + 2 goes to more 256x256 tiles
    text, _ = L.describe("winograd", "grouped", 8192, 8192, 8192, cutoff=1, levels=2, dtype="bf16x3")
    assert gemm_launches(text) == [(48, 3072, 6), (1, 256, 0)]
    # float32 keeps its own split (4096, two levels: 45 + 4)
    text, _ = L.describe("winograd", "grouped", 4096, 4096, 4096, cutoff=1, levels=2, dtype="f32")
    assert gemm_launches(text) == [(45, 720, 3), (4, 256, 0)]
