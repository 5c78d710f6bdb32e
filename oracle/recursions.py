"""Strassen and Strassen-Winograd recursions, restated from the paper in numpy.

Test infrastructure only.  Each function follows the paper's steps in the
paper's order and notation, on numpy arrays of int64 (exact) or float64:

* ``strassen``        Section 2.2: products P1..P7 and C11..C22, recursively
                      (Algorithm 2).
* ``winograd``        Section 2.3, the 22-operation block form: S1..S4,
                      T1..T4, P1..P7, U1..U7, C = [U1 U5; U6 U7].
* ``winograd_knuth``  Section 2.3, the u, v, w form.  Reading: the second
                      factor is labelled [A C; B D], so B11=A, B12=C, B21=B,
                      B22=D; it is evaluated with seven products (the
                      product aA is formed once and reused inside w).
* ``two_temp``        Section 3.3, Table 2: the 22 operations in the table's
                      order with two temporaries X and Y per level.
* ``in_place``        Section 3.3, Table 3: the 22 operations in the table's
                      order with every intermediate stored in quadrants of A,
                      B and C.  A and B are overwritten (the inputs are copied
                      first so the caller's arrays survive).

Stopping rule (Sections 2.2 and 3.4).  The recursion stops and the naive
method runs when the smallest dimension is <= ``cutoff`` (cutoff 1 is
Algorithm 2's 1x1 base case; 12 is the cutoff of Section 3.4), or when
``levels`` halvings have been done (levels < 0: no limit).  A level that must
split an odd dimension raises ValueError: this restatement does not pad.

Dimensions: A is m x k, B is k x n, C is m x n (the cutoff section's names).

Counting.  An optional ``Counter`` records scalar multiplications and
additions (a subtraction counts as an addition; an r x c block addition counts
r*c) and the peak number of temporary elements alive at once.
"""
import numpy as np

from . import naive as _naive


class Counter:
    def __init__(self):
        self.mults = 0
        self.adds = 0
        self.ws_now = 0
        self.ws_peak = 0
        self.leaves = 0
        self.trace = []          # (level, label, destination) of block steps

    @property
    def ops(self):
        return self.mults + self.adds

    def alloc(self, elems):
        self.ws_now += elems
        self.ws_peak = max(self.ws_peak, self.ws_now)

    def free(self, elems):
        self.ws_now -= elems


def _base(A, B, ctr):
    """The naive method at the bottom of a recursion (Sections 2.1 and 3.4)."""
    m, k = A.shape
    n = B.shape[1]
    if ctr is not None:
        ctr.mults += m * k * n
        ctr.adds += m * n * max(k - 1, 0)
        ctr.leaves += 1
    if np.issubdtype(A.dtype, np.integer):
        return A @ B                       # exact integer arithmetic
    return _naive.gemm(A, B).astype(A.dtype, copy=False)


def _add(X, Y, ctr, sign=+1):
    if ctr is not None:
        ctr.adds += X.size
    return X + Y if sign > 0 else X - Y


def _stop(m, k, n, cutoff, levels):
    return levels == 0 or min(m, k, n) <= max(int(cutoff), 1)


def _split(M):
    r, c = M.shape
    if r % 2 or c % 2:
        raise ValueError(f"cannot split a {r}x{c} block into quadrants")
    r //= 2
    c //= 2
    return M[:r, :c], M[:r, c:], M[r:, :c], M[r:, c:]


def _check(A, B):
    if A.ndim != 2 or B.ndim != 2 or A.shape[1] != B.shape[0]:
        raise ValueError(f"shape mismatch {A.shape} x {B.shape}")


# --------------------------------------------------------------------------
# Section 2.2: Strassen
# --------------------------------------------------------------------------
def strassen(A, B, cutoff=1, levels=-1, ctr=None):
    _check(A, B)
    m, k = A.shape
    n = B.shape[1]
    if _stop(m, k, n, cutoff, levels):
        return _base(A, B, ctr)
    A11, A12, A21, A22 = _split(A)
    B11, B12, B21, B22 = _split(B)
    nl = levels - 1 if levels > 0 else levels

    def rec(X, Y):
        return strassen(X, Y, cutoff, nl, ctr)

    P1 = rec(_add(A11, A22, ctr), _add(B11, B22, ctr))
    P2 = rec(_add(A21, A22, ctr), B11)
    P3 = rec(A11, _add(B12, B22, ctr, -1))
    P4 = rec(A22, _add(B21, B11, ctr, -1))          # -B11 + B21
    P5 = rec(_add(A11, A12, ctr), B22)
    P6 = rec(_add(A21, A11, ctr, -1), _add(B11, B12, ctr))   # -A11 + A21
    P7 = rec(_add(A12, A22, ctr, -1), _add(B21, B22, ctr))
    C11 = _add(_add(_add(P1, P4, ctr), P5, ctr, -1), P7, ctr)
    C12 = _add(P3, P5, ctr)
    C21 = _add(P2, P4, ctr)
    C22 = _add(_add(_add(P1, P3, ctr), P2, ctr, -1), P6, ctr)
    return np.block([[C11, C12], [C21, C22]])


# --------------------------------------------------------------------------
# Section 2.3: Strassen-Winograd, the 22-operation block form
# --------------------------------------------------------------------------
def winograd(A, B, cutoff=1, levels=-1, ctr=None):
    _check(A, B)
    m, k = A.shape
    n = B.shape[1]
    if _stop(m, k, n, cutoff, levels):
        return _base(A, B, ctr)
    A11, A12, A21, A22 = _split(A)
    B11, B12, B21, B22 = _split(B)
    nl = levels - 1 if levels > 0 else levels

    def rec(X, Y):
        return winograd(X, Y, cutoff, nl, ctr)

    # eight additions
    S1 = _add(A21, A22, ctr)
    S2 = _add(S1, A11, ctr, -1)
    S3 = _add(A11, A21, ctr, -1)
    T1 = _add(B12, B11, ctr, -1)
    T2 = _add(B22, T1, ctr, -1)
    T3 = _add(B22, B12, ctr, -1)
    S4 = _add(A12, S2, ctr, -1)
    T4 = _add(T2, B21, ctr, -1)
    # seven recursive products
    P1 = rec(A11, B11)
    P2 = rec(A12, B21)
    P3 = rec(S4, B22)
    P4 = rec(A22, T4)
    P5 = rec(S1, T1)
    P6 = rec(S2, T2)
    P7 = rec(S3, T3)
    # seven additions
    U1 = _add(P1, P2, ctr)
    U2 = _add(P1, P6, ctr)
    U3 = _add(U2, P7, ctr)
    U4 = _add(U2, P5, ctr)
    U5 = _add(U4, P3, ctr)
    U6 = _add(U3, P4, ctr, -1)
    U7 = _add(U3, P5, ctr)
    return np.block([[U1, U5], [U6, U7]])


# --------------------------------------------------------------------------
# Section 2.3: Strassen-Winograd, Knuth's u, v, w form
# --------------------------------------------------------------------------
def winograd_knuth(A, B, cutoff=1, levels=-1, ctr=None):
    _check(A, B)
    m, k = A.shape
    n = B.shape[1]
    if _stop(m, k, n, cutoff, levels):
        return _base(A, B, ctr)
    a, b, c, d = _split(A)
    # second factor labelled [A C; B D]
    A_, C_, B_, D_ = _split(B)
    nl = levels - 1 if levels > 0 else levels

    def rec(X, Y):
        return winograd_knuth(X, Y, cutoff, nl, ctr)

    cd = _add(c, d, ctr)                 # c + d
    cda = _add(cd, a, ctr, -1)           # c + d - a
    abcd = _add(b, cda, ctr, -1)         # a + b - c - d
    CA = _add(C_, A_, ctr, -1)           # C - A
    ADC = _add(D_, CA, ctr, -1)          # A + D - C
    BCAD = _add(B_, ADC, ctr, -1)        # B + C - A - D
    ca = _add(c, a, ctr, -1)             # c - a
    CD = _add(C_, D_, ctr, -1)           # C - D
    aA = rec(a, A_)
    bB = rec(b, B_)
    u = rec(ca, CD)
    v = rec(cd, CA)
    w = _add(aA, rec(cda, ADC), ctr)
    t12 = rec(abcd, D_)
    t21 = rec(d, BCAD)
    wu = _add(w, u, ctr)
    C11 = _add(aA, bB, ctr)
    C12 = _add(_add(w, v, ctr), t12, ctr)
    C21 = _add(wu, t21, ctr)
    C22 = _add(wu, v, ctr)
    return np.block([[C11, C12], [C21, C22]])


# --------------------------------------------------------------------------
# Section 3.3, Table 2: Two Temp Winograd
# --------------------------------------------------------------------------
def two_temp(A, B, cutoff=1, levels=-1, ctr=None):
    _check(A, B)
    C = np.empty((A.shape[0], B.shape[1]), dtype=np.result_type(A, B))
    _two_temp_into(A, B, C, cutoff, levels, ctr, 0)
    return C


def _two_temp_into(A, B, C, cutoff, levels, ctr, depth):
    m, k = A.shape
    n = B.shape[1]
    if _stop(m, k, n, cutoff, levels):
        C[...] = _base(A, B, ctr)
        return
    A11, A12, A21, A22 = _split(A)
    B11, B12, B21, B22 = _split(B)
    C11, C12, C21, C22 = _split(C)
    h_m, h_k, h_n = m // 2, k // 2, n // 2
    nl = levels - 1 if levels > 0 else levels
    # X holds an S block (m/2 x k/2) and later P1 (m/2 x n/2); Y holds T blocks.
    X = np.empty((h_m, max(h_k, h_n)), dtype=C.dtype)
    Y = np.empty((h_k, h_n), dtype=C.dtype)
    if ctr is not None:
        ctr.alloc(X.size + Y.size)
    XS = X[:, :h_k]
    XP = X[:, :h_n]

    def step(label, dest, value):
        if ctr is not None and depth == 0:
            ctr.trace.append((label, dest))
        return value

    def rec(Aop, Bop, out):
        _two_temp_into(Aop, Bop, out, cutoff, nl, ctr, depth + 1)

    XS[...] = step("S3", "X", _add(A11, A21, ctr, -1))           # 1
    Y[...] = step("T3", "Y", _add(B22, B12, ctr, -1))            # 2
    step("P7", "C21", None); rec(XS, Y, C21)                     # 3
    XS[...] = step("S1", "X", _add(A21, A22, ctr))               # 4
    Y[...] = step("T1", "Y", _add(B12, B11, ctr, -1))            # 5
    step("P5", "C22", None); rec(XS, Y, C22)                     # 6
    XS[...] = step("S2", "X", _add(XS, A11, ctr, -1))            # 7
    Y[...] = step("T2", "Y", _add(B22, Y, ctr, -1))              # 8
    step("P6", "C12", None); rec(XS, Y, C12)                     # 9
    XS[...] = step("S4", "X", _add(A12, XS, ctr, -1))            # 10
    step("P3", "C11", None); rec(XS, B22, C11)                   # 11
    step("P1", "X", None); rec(A11, B11, XP)                     # 12
    C12[...] = step("U2", "C12", _add(XP, C12, ctr))             # 13: P1 + P6
    C21[...] = step("U3", "C21", _add(C12, C21, ctr))            # 14: U2 + P7
    C12[...] = step("U4", "C12", _add(C12, C22, ctr))            # 15: U2 + P5
    C22[...] = step("U7", "C22", _add(C21, C22, ctr))            # 16: U3 + P5
    C12[...] = step("U5", "C12", _add(C12, C11, ctr))            # 17: U4 + P3
    Y[...] = step("T4", "Y", _add(Y, B21, ctr, -1))              # 18: T2 - B21
    step("P4", "C11", None); rec(A22, Y, C11)                    # 19
    C21[...] = step("U6", "C21", _add(C21, C11, ctr, -1))        # 20: U3 - P4
    step("P2", "C11", None); rec(A12, B21, C11)                  # 21
    C11[...] = step("U1", "C11", _add(XP, C11, ctr))             # 22: P1 + P2
    if ctr is not None:
        ctr.free(X.size + Y.size)


# --------------------------------------------------------------------------
# Section 3.3, Table 3: In-Place Winograd
# --------------------------------------------------------------------------
def in_place(A, B, cutoff=1, levels=-1, ctr=None, clobber_leaves=False):
    """Table 3 on copies of A and B (the schedule overwrites its inputs).

    Shapes must satisfy k == n <= m at every level (the slot sizes of Table 3
    only fit then).  ``clobber_leaves`` overwrites the operands of every base
    case after use, which proves that no operand is read after a recursive
    call has destroyed it.
    """
    _check(A, B)
    A = np.array(A, copy=True)
    B = np.array(B, copy=True)
    C = np.empty((A.shape[0], B.shape[1]), dtype=np.result_type(A, B))
    _in_place_into(A, B, C, cutoff, levels, ctr, 0, clobber_leaves)
    return C


def _in_place_into(A, B, C, cutoff, levels, ctr, depth, clobber):
    m, k = A.shape
    n = B.shape[1]
    if _stop(m, k, n, cutoff, levels):
        C[...] = _base(A, B, ctr)
        if clobber:
            junk = -7777 if np.issubdtype(A.dtype, np.integer) else np.nan
            A[...] = junk
            B[...] = junk
        return
    if not (k == n and n <= m):
        raise ValueError(f"in-place schedule needs k == n <= m, got m={m} k={k} n={n}")
    A11, A12, A21, A22 = _split(A)
    B11, B12, B21, B22 = _split(B)
    C11, C12, C21, C22 = _split(C)
    h_k, h_n = k // 2, n // 2
    nl = levels - 1 if levels > 0 else levels

    def corner(M, r, c):
        return M[:r, :c]

    def step(label, dest):
        if ctr is not None and depth == 0:
            ctr.trace.append((label, dest))

    def rec(Aop, Bop, out):
        _in_place_into(Aop, Bop, out, cutoff, nl, ctr, depth + 1, clobber)

    S3 = corner(C11, A11.shape[0], h_k)      # slots that hold smaller blocks
    T1 = corner(C22, h_k, h_n)
    S2 = corner(C12, A11.shape[0], h_k)
    T4 = corner(C22, h_k, h_n)
    step("S3", "C11"); S3[...] = _add(A11, A21, ctr, -1)         # 1
    step("S1", "A21"); A21[...] = _add(A21, A22, ctr)            # 2
    step("T1", "C22"); T1[...] = _add(B12, B11, ctr, -1)         # 3
    step("T3", "B12"); B12[...] = _add(B22, B12, ctr, -1)        # 4
    step("P7", "C21"); rec(S3, B12, C21)                         # 5
    step("S2", "C12"); S2[...] = _add(A21, A11, ctr, -1)         # 6
    step("P1", "C11"); rec(A11, B11, C11)                        # 7
    step("T2", "B11"); B11[...] = _add(B22, T1, ctr, -1)         # 8
    step("P5", "A11"); rec(A21, T1, corner(A11, C11.shape[0], h_n))   # 9
    step("T4", "C22"); T4[...] = _add(B11, B21, ctr, -1)         # 10
    step("P4", "A21"); rec(A22, T4, corner(A21, C11.shape[0], h_n))   # 11
    step("S4", "A22"); A22[...] = _add(A12, S2, ctr, -1)         # 12
    step("P6", "C22"); rec(S2, B11, C22)                         # 13
    P5 = corner(A11, C11.shape[0], h_n)
    P4 = corner(A21, C11.shape[0], h_n)
    step("U2", "C22"); C22[...] = _add(C11, C22, ctr)            # 14: P1 + P6
    step("P2", "C12"); rec(A12, B21, C12)                        # 15
    step("U1", "C11"); C11[...] = _add(C11, C12, ctr)            # 16: P1 + P2
    step("U4", "C12"); C12[...] = _add(C22, P5, ctr)             # 17: U2 + P5
    step("U3", "C22"); C22[...] = _add(C22, C21, ctr)            # 18: U2 + P7
    step("U6", "C21"); C21[...] = _add(C22, P4, ctr, -1)         # 19: U3 - P4
    step("U7", "C22"); C22[...] = _add(C22, P5, ctr)             # 20: U3 + P5
    P3 = corner(A12, C11.shape[0], h_n)
    step("P3", "A12"); rec(A22, B22, P3)                         # 21
    step("U5", "C12"); C12[...] = _add(C12, P3, ctr)             # 22: U4 + P3


def levels_planned(m, k, n, cutoff=1, levels=-1):
    """Number of halvings the stopping rule above performs (even sizes)."""
    L = 0
    while not _stop(m, k, n, cutoff, levels - L if levels >= 0 else -1):
        if m % 2 or k % 2 or n % 2:
            break
        m, k, n = m // 2, k // 2, n // 2
        L += 1
    return L
