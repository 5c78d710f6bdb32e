"""Compile the oracle's C triple loop into ``oracle/_liboracle.so`` with gcc.

Test infrastructure only (see the package docstring).  ``-ffp-contract=off``
keeps every product and every sum separately rounded, in the order written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gemm_f64.c")
LIB = os.path.join(HERE, "_liboracle.so")


def build(verbose: bool = False) -> str:
    # a private temporary per process, renamed into place: processes that
    # build at the same time (parallel test workers) never see a partial file
    tmp = f"{LIB}.{os.getpid()}.tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-std=c11", SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
