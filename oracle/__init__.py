"""CPU oracle for C = A x B (the paper's naive method and its recursions).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import this
package.  The GPU library never imports, links or calls it, and it imports
nothing from the GPU library; the two share only the seeded input generators,
which live in a module of their own and contain none of the method's
arithmetic.

Contents
--------
``naive``       the plain definition c_ij = sum_p a_ip b_pj (Section 2.1,
                Algorithm 1): a C triple loop in double precision, plus a
                pure-Python loop for tiny exact (integer) cases.
``recursions``  Strassen (Section 2.2, Algorithm 2), Strassen-Winograd in the
                Knuth form and in the 22-operation form (Section 2.3), and the
                two memory schedules of Section 3.3 (Tables 2 and 3), each with
                the naive method below a cutoff (Section 3.4).
"""
from . import naive, recursions  # noqa: F401
