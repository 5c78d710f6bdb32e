"""Strassen and Strassen-Winograd matrix multiplication on AMD MI355X.

The hot path (naive MFMA GEMM, Strassen, Winograd and the paper's memory
schedules) lives in ``libmm.so`` (HIP kernels behind the C ABI of
``include/mm.h``).  This package holds its Python binding (``api``, ``_lib``),
the build script, the autotuner, the batched plans and the serving loop.
Importing the package loads nothing; the library is loaded on first use and
a missing library raises.
"""

__all__ = ["mm", "Plan", "BatchedPlan", "MMError"]


def __getattr__(name):
    if name in ("mm", "Plan", "BatchedPlan", "get_plan", "workspace"):
        from . import api
        return getattr(api, name)
    if name == "MMError":
        from ._lib import MMError
        return MMError
    raise AttributeError(name)
