"""Seeded synthetic inputs shared by the GPU path's tests, the benchmark and
the oracle's checks.

This module draws random numbers and nothing else: it holds none of the
multiplication method's arithmetic.  Every generator is numpy's PCG64
(``numpy.random.default_rng(seed)``), so the same seed gives the same matrices
on every machine.

The paper times square orders 2^k with unstated entries; these recipes extend
that workload to GPU sizes:

* ``uniform``          i.i.d. U[-1, 1] entries (square or rectangular).
* ``integers``         i.i.d. integers in [lo, hi], for exact checks.
* ``gauss_rowscaled``  N(0, 1) entries, every row multiplied by 10^u with
                       u ~ U[-3, 3] drawn per row (for A and for B
                       independently): a wide dynamic range that stresses
                       split-precision products.
* ``batched_shapes``   (m, n, k) triples, each dimension log-uniform in
                       [lo, hi] and rounded to a multiple of ``mult``.
* ``serving_trace``    Poisson arrivals with a mix of square orders and dtypes.
"""
import numpy as np


def rng(seed):
    return np.random.default_rng(int(seed))


def uniform(shape, seed, dtype=np.float64, lo=-1.0, hi=1.0):
    g = rng(seed)
    return g.uniform(lo, hi, size=shape).astype(dtype)


def integers(shape, seed, lo=-9, hi=9, dtype=np.float64):
    g = rng(seed)
    return g.integers(lo, hi + 1, size=shape).astype(dtype)


def gauss_rowscaled(shape, seed, dtype=np.float32, decades=3.0):
    g = rng(seed)
    x = g.standard_normal(size=shape, dtype=np.float64)
    u = g.uniform(-decades, decades, size=(shape[0], 1))
    return (x * np.power(10.0, u)).astype(dtype)


def pair(kind, m, n, k, seed, dtype):
    """(A, B) with A m x k and B k x n, drawn from one of the recipes."""
    if kind == "uniform":
        return (uniform((m, k), 2 * seed, dtype), uniform((k, n), 2 * seed + 1, dtype))
    if kind == "int":
        return (integers((m, k), 2 * seed, dtype=dtype),
                integers((k, n), 2 * seed + 1, dtype=dtype))
    if kind == "gauss_rowscaled":
        return (gauss_rowscaled((m, k), 2 * seed, dtype),
                gauss_rowscaled((k, n), 2 * seed + 1, dtype))
    raise ValueError(kind)


def batched_shapes(count, seed, lo=64, hi=2048, mult=16):
    g = rng(seed)
    x = np.exp(g.uniform(np.log(lo), np.log(hi), size=(count, 3)))
    x = np.clip(np.rint(x / mult) * mult, lo, hi).astype(np.int64)
    return [tuple(int(v) for v in row) for row in x]     # (m, n, k)


def serving_trace(count, seed, qps, bands=((0.70, 256, 1024), (0.25, 1024, 4096),
                                           (0.05, 8192, 8192)),
                  dtypes=("f32", "bf16x3")):
    """Poisson arrival times (seconds), square orders and dtypes per request."""
    g = rng(seed)
    gaps = g.exponential(1.0 / float(qps), size=count)
    t = np.cumsum(gaps) - gaps[0]
    probs = np.array([b[0] for b in bands], dtype=np.float64)
    probs /= probs.sum()
    band = g.choice(len(bands), size=count, p=probs)
    sizes = []
    for b in band:
        _, lo, hi = bands[b]
        sizes.append(int(g.integers(lo, hi + 1)))
    dt = g.choice(len(dtypes), size=count)
    seeds = g.integers(0, 2**31 - 1, size=count)
    return [dict(t=float(t[i]), n=sizes[i], dtype=dtypes[dt[i]], seed=int(seeds[i]))
            for i in range(count)]
