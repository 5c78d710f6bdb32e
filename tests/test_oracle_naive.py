"""Pins for the oracle's naive method (Section 2.1, Algorithm 1).

Each check compares the C triple loop with something other than itself:
exact integer brute force in Python, closed forms, identity and permutation
matrices, a summation-order witness, and numpy as a library cross-check.
"""
import numpy as np
import pytest

from paper_2309_00628_amd import inputs


@pytest.fixture(scope="module")
def naive(oracle_built):
    from oracle import naive
    return naive


def test_identity_exact(naive):
    A = inputs.uniform((37, 53), 1)
    B = inputs.uniform((53, 29), 2)
    assert np.array_equal(naive.gemm(A, np.eye(53)), A)
    assert np.array_equal(naive.gemm(np.eye(53), B), B)


def test_permutation_exact(naive):
    A = inputs.uniform((40, 24), 3)
    g = inputs.rng(4)
    pr = g.permutation(40)
    pc = g.permutation(24)
    P = np.eye(40)[pr]            # P @ A reorders rows
    Q = np.eye(24)[:, pc]         # A @ Q reorders columns
    assert np.array_equal(naive.gemm(P, A), A[pr])
    assert np.array_equal(naive.gemm(A, Q), A[:, pc])


@pytest.mark.parametrize("m,k,n,seed", [(4, 4, 4, 0), (8, 8, 8, 1), (3, 5, 7, 2),
                                        (7, 1, 6, 3), (1, 9, 1, 4), (16, 12, 10, 5)])
def test_integer_brute_force_exact(naive, m, k, n, seed):
    A = inputs.integers((m, k), seed)
    B = inputs.integers((k, n), seed + 100)
    ref = naive.naive_py(A.astype(np.int64).tolist(), B.astype(np.int64).tolist())
    got = naive.gemm(A, B)
    assert got.tolist() == [[float(v) for v in row] for row in ref]


def test_closed_forms(naive):
    m, k, n = 13, 21, 17
    # all-ones: every entry is the inner dimension (catches a dropped term)
    assert np.all(naive.gemm(np.ones((m, k)), np.ones((k, n))) == k)
    # a_ip = i+1, b_pj = j+1: c_ij = (i+1)(j+1)k
    A = np.repeat(np.arange(1, m + 1, dtype=np.float64)[:, None], k, axis=1)
    B = np.repeat(np.arange(1, n + 1, dtype=np.float64)[None, :], k, axis=0)
    i, j = np.meshgrid(np.arange(1, m + 1), np.arange(1, n + 1), indexing="ij")
    assert np.array_equal(naive.gemm(A, B), (i * j * k).astype(np.float64))
    # a_ip = p, b_pj = 1: c_ij = k(k-1)/2 (catches a wrong inner index)
    A = np.repeat(np.arange(k, dtype=np.float64)[None, :], m, axis=0)
    assert np.all(naive.gemm(A, np.ones((k, n))) == k * (k - 1) / 2)
    # a_ip = 1, b_pj = p * (j+1): catches an operand read transposed
    B = np.arange(k, dtype=np.float64)[:, None] * np.arange(1, n + 1)[None, :]
    assert np.array_equal(naive.gemm(np.ones((m, k)), B),
                          np.repeat((k * (k - 1) / 2 * np.arange(1, n + 1))[None, :], m, axis=0))


def test_summation_order_is_increasing_p(naive):
    # ((0 + 1e16) + 1) - 1e16 == 0 in double; any other order gives 1 or 2.
    A = np.array([[1e16, 1.0, -1e16]])
    B = np.ones((3, 1))
    assert naive.gemm(A, B)[0, 0] == 0.0
    A = np.array([[1.0, 1e16, 1.0, -1e16]])
    B = np.ones((4, 1))
    assert naive.gemm(A, B)[0, 0] == 0.0


def test_no_fused_multiply_add(naive):
    # with one rounding per product and per sum, a*b - a*b is exactly zero;
    # a fused a*b + c would leave the rounding error of a*b behind.
    a = 1.0 + 2.0**-30
    A = np.array([[a, -a]])
    B = np.array([[a], [a]])
    assert naive.gemm(A, B)[0, 0] == 0.0


def test_numpy_cross_check(naive):
    A = inputs.uniform((64, 48), 7)
    B = inputs.uniform((48, 80), 8)
    ref = A @ B
    got = naive.gemm(A, B)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-13


def test_thread_count_does_not_change_bits(naive):
    A = inputs.uniform((96, 70), 9)
    B = inputs.uniform((70, 33), 10)
    assert np.array_equal(naive.gemm(A, B, threads=1), naive.gemm(A, B, threads=4))


def test_rows_sample_matches_full(naive):
    A = inputs.uniform((50, 40), 11, np.float32)
    B = inputs.uniform((40, 30), 12, np.float32)
    rows = [0, 7, 49, 13]
    assert np.array_equal(naive.gemm_rows(A, B, rows), naive.gemm(A, B)[rows])


def test_degenerate_sizes(naive):
    assert naive.gemm(np.zeros((3, 0)), np.zeros((0, 4))).tolist() == [[0.0] * 4] * 3
    assert naive.gemm(np.zeros((0, 5)), np.zeros((5, 4))).shape == (0, 4)
    assert naive.gemm(np.zeros((3, 5)), np.zeros((5, 0))).shape == (3, 0)


def test_float32_inputs_are_widened_exactly(naive):
    A = inputs.uniform((8, 8), 13, np.float32)
    B = inputs.uniform((8, 8), 14, np.float32)
    assert np.array_equal(naive.gemm(A, B), naive.gemm(A.astype(np.float64), B.astype(np.float64)))
