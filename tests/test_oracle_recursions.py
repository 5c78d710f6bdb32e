"""Pins for the oracle's restatements of Strassen (Section 2.2), Winograd
(Section 2.3) and the memory schedules of Section 3.3 (Tables 2 and 3).

They are checked against exact brute force on integers (every 2x2 pair with
entries in {-1, 0, 1}, random integer blocks), the paper's printed operation
tables (golden fixtures), the closed-form operation counts, the cutoff rule of
Section 3.4, the two-temporary workspace formula, and liveness of the
in-place schedule.
"""
import itertools
import os

import numpy as np
import pytest

from paper_2309_00628_amd import inputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def R(oracle_built):
    from oracle import recursions
    return recursions


@pytest.fixture(scope="module")
def naive(oracle_built):
    from oracle import naive
    return naive


ALGOS = ["strassen", "winograd", "winograd_knuth", "two_temp", "in_place"]


def _brute(A, B):
    A = np.asarray(A, dtype=np.int64)
    B = np.asarray(B, dtype=np.int64)
    m, k = A.shape
    n = B.shape[1]
    C = np.zeros((m, n), dtype=np.int64)
    for i in range(m):
        for j in range(n):
            C[i, j] = sum(int(A[i, p]) * int(B[p, j]) for p in range(k))
    return C


def test_all_2x2_sign_matrices_exact(R):
    vals = (-1, 0, 1)
    mats = [np.array(v, dtype=np.int64).reshape(2, 2) for v in itertools.product(vals, repeat=4)]
    fns = [getattr(R, a) for a in ALGOS]
    for A in mats:
        for B in mats:
            ref = _brute(A, B)
            for f in fns:
                assert np.array_equal(f(A, B, cutoff=1), ref)


@pytest.mark.parametrize("n", [4, 8])
@pytest.mark.parametrize("cutoff", [1, 2, 4])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_integer_exact_small(R, n, cutoff, seed):
    A = inputs.integers((n, n), seed, dtype=np.int64)
    B = inputs.integers((n, n), seed + 50, dtype=np.int64)
    ref = _brute(A, B)
    for a in ALGOS:
        assert np.array_equal(getattr(R, a)(A, B, cutoff=cutoff), ref), a


@pytest.mark.parametrize("m,k,n,cutoff", [(8, 4, 16, 1), (16, 8, 4, 1), (4, 16, 8, 1),
                                          (12, 12, 12, 3), (24, 8, 8, 1)])
def test_integer_exact_rectangular(R, m, k, n, cutoff):
    A = inputs.integers((m, k), 3, dtype=np.int64)
    B = inputs.integers((k, n), 4, dtype=np.int64)
    ref = _brute(A, B)
    for a in ["strassen", "winograd", "winograd_knuth", "two_temp"]:
        assert np.array_equal(getattr(R, a)(A, B, cutoff=cutoff), ref), a
    if k == n and n <= m:
        assert np.array_equal(R.in_place(A, B, cutoff=cutoff), ref)


def test_integer_exact_512_cutoff_64(R):
    # the FP64 correctness configuration with integer entries: three levels
    A = inputs.integers((512, 512), 5, dtype=np.int64)
    B = inputs.integers((512, 512), 6, dtype=np.int64)
    ref = A @ B
    for a in ["winograd", "two_temp", "in_place", "strassen"]:
        assert np.array_equal(getattr(R, a)(A, B, cutoff=64), ref), a


def _read_table(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            num, label, dest = line.split()
            rows.append((label, dest))
    return rows


def test_two_temp_follows_table2(R):
    ctr = R.Counter()
    A = inputs.integers((8, 8), 7, dtype=np.int64)
    B = inputs.integers((8, 8), 8, dtype=np.int64)
    R.two_temp(A, B, cutoff=2, ctr=ctr)
    assert ctr.trace == _read_table("table2_two_temp.txt")


def test_in_place_follows_table3(R):
    ctr = R.Counter()
    A = inputs.integers((8, 8), 9, dtype=np.int64)
    B = inputs.integers((8, 8), 10, dtype=np.int64)
    R.in_place(A, B, cutoff=2, ctr=ctr)
    assert ctr.trace == _read_table("table3_in_place.txt")


def _op_counts():
    out = {}
    with open(os.path.join(GOLDEN, "op_counts.txt")) as f:
        for line in f:
            if line.startswith("#"):
                continue
            k, n, s, w = map(int, line.split())
            out[n] = (s, w)
    return out


@pytest.mark.parametrize("n", [2, 4, 8, 16, 32])
def test_operation_counts(R, n):
    s_ops, w_ops = _op_counts()[n]
    A = inputs.integers((n, n), 11, dtype=np.int64)
    B = inputs.integers((n, n), 12, dtype=np.int64)
    for a, want in [("strassen", s_ops), ("winograd", w_ops), ("winograd_knuth", w_ops),
                    ("two_temp", w_ops), ("in_place", w_ops)]:
        ctr = R.Counter()
        getattr(R, a)(A, B, cutoff=1, ctr=ctr)
        assert ctr.ops == want, (a, ctr.ops, want)
        assert ctr.mults == 7 ** int(np.log2(n))


def test_additions_per_level(R):
    # 2x2: Strassen 7 multiplications and 18 additions; Winograd 7 and 15
    A = np.array([[1, 2], [3, 4]], dtype=np.int64)
    B = np.array([[5, 6], [7, 8]], dtype=np.int64)
    for a, adds in [("strassen", 18), ("winograd", 15), ("winograd_knuth", 15),
                    ("two_temp", 15), ("in_place", 15)]:
        ctr = R.Counter()
        getattr(R, a)(A, B, cutoff=1, ctr=ctr)
        assert (ctr.mults, ctr.adds) == (7, adds), a


def test_cutoff_rule_of_section_3_4(R):
    # operations of the naive method vs one Winograd level over naive halves
    with open(os.path.join(GOLDEN, "cutoff.txt")) as f:
        want = int([l for l in f if not l.startswith("#")][0].split()[1])
    best = None
    for n in range(2, 42, 2):
        A = np.ones((n, n), dtype=np.int64)
        c0, c1 = R.Counter(), R.Counter()
        R.winograd(A, A, cutoff=1, levels=0, ctr=c0)
        R.winograd(A, A, cutoff=1, levels=1, ctr=c1)
        if c0.ops <= c1.ops:
            best = n
        else:
            assert n > want
    assert best == want
    # the inequality itself, mkn <= 4(mk + kn + mn), on rectangular shapes
    for (m, k, n) in [(8, 16, 32), (20, 10, 12), (40, 12, 10), (6, 60, 100)]:
        A = np.ones((m, k), dtype=np.int64)
        B = np.ones((k, n), dtype=np.int64)
        c0, c1 = R.Counter(), R.Counter()
        R.winograd(A, B, cutoff=1, levels=0, ctr=c0)
        R.winograd(A, B, cutoff=1, levels=1, ctr=c1)
        assert (c0.ops <= c1.ops) == (m * k * n <= 4 * (m * k + k * n + m * n))


@pytest.mark.parametrize("n,cutoff", [(8, 1), (16, 2), (64, 8), (128, 16)])
def test_two_temp_workspace_formula(R, n, cutoff):
    ctr = R.Counter()
    A = inputs.integers((n, n), 13, dtype=np.int64)
    B = inputs.integers((n, n), 14, dtype=np.int64)
    R.two_temp(A, B, cutoff=cutoff, ctr=ctr)
    L = R.levels_planned(n, n, n, cutoff)
    assert ctr.ws_peak == sum(2 * (n >> l) ** 2 for l in range(1, L + 1))
    assert ctr.ws_peak < 2 * n * n / 3


def test_two_temp_workspace_rectangular(R):
    m, k, n = 16, 8, 32
    ctr = R.Counter()
    R.two_temp(np.ones((m, k), np.int64), np.ones((k, n), np.int64), cutoff=4, levels=1, ctr=ctr)
    assert ctr.ws_peak == (m // 2) * max(k, n) // 2 + (k // 2) * (n // 2)


def test_in_place_needs_no_workspace_and_survives_clobbering(R):
    A = inputs.integers((64, 64), 15, dtype=np.int64)
    B = inputs.integers((64, 64), 16, dtype=np.int64)
    ctr = R.Counter()
    assert np.array_equal(R.in_place(A, B, cutoff=4, ctr=ctr, clobber_leaves=True), A @ B)
    assert ctr.ws_peak == 0


def test_in_place_rejects_shapes_whose_slots_do_not_fit(R):
    with pytest.raises(ValueError):
        R.in_place(np.ones((8, 8)), np.ones((8, 16)), cutoff=1)


def test_schedules_agree_bitwise_in_double(R, naive):
    # each element sees the same operations in the same order
    A = inputs.uniform((128, 128), 17)
    B = inputs.uniform((128, 128), 18)
    w = R.winograd(A, B, cutoff=16)
    assert np.array_equal(R.two_temp(A, B, cutoff=16), w)
    assert np.array_equal(R.in_place(A, B, cutoff=16), w)
    assert np.array_equal(R.winograd_knuth(A, B, cutoff=16), w)
    ref = naive.gemm(A, B)
    for C in (w, R.strassen(A, B, cutoff=16)):
        assert np.linalg.norm(C - ref) / np.linalg.norm(ref) < 1e-14


def test_odd_split_raises(R):
    with pytest.raises(ValueError):
        R.winograd(np.ones((6, 6)), np.ones((6, 6)), cutoff=1)
