"""The three-way bfloat16 split of the refined-bfloat16 leaves is exact.

For a float32 x the leaf loader forms hi = bf16(x), lo = bf16(x - hi) and
res = bf16(x - hi - lo) with float32 subtractions.  This pins, on the CPU and
independently of the GPU code, the two facts that make float32 arithmetic
sufficient there: both subtractions are exact (the float32 result equals the
float64 one), and for |x| >= 2^-110 res needs no rounding, so
x = hi + lo + res exactly (below that the residual is a bfloat16 subnormal
and is rounded).
Rounding to bfloat16 is written out as round-to-nearest-even on the bit
pattern (the top 16 bits of a float32).
"""
import numpy as np

from paper_2309_00628_amd import inputs


def bf16_rne(x):
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def test_bf16_rne_rounding():
    # ties go to even; 1 + 2^-8 is halfway between 1 and 1 + 2^-7
    assert bf16_rne(np.float32(1 + 2.0 ** -8)) == np.float32(1.0)
    assert bf16_rne(np.float32(1 + 3 * 2.0 ** -8)) == np.float32(1 + 2.0 ** -6)
    assert bf16_rne(np.float32(1 + 2.0 ** -8 + 2.0 ** -20)) == np.float32(1 + 2.0 ** -7)
    assert bf16_rne(np.float32(-3.0)) == np.float32(-3.0)


def test_three_way_split_is_exact():
    g = inputs.rng(77)
    mant = g.uniform(-2.0, 2.0, size=400_000)
    expo = g.integers(-120, 120, size=mant.size)
    x = (mant * np.exp2(expo)).astype(np.float32)
    x = np.concatenate([x, inputs.gauss_rowscaled((200, 500), 3).ravel(),
                        np.float32([0.0, 1.0, -1.0, 2.0 ** -126, 3.0e-39, 1.0e-45])]).astype(np.float32)
    hi = bf16_rne(x)
    d1 = x - hi                                  # float32 subtraction
    assert np.array_equal(d1.astype(np.float64), x.astype(np.float64) - hi.astype(np.float64))
    lo = bf16_rne(d1)
    d2 = d1 - lo
    assert np.array_equal(d2.astype(np.float64), d1.astype(np.float64) - lo.astype(np.float64))
    res = bf16_rne(d2)
    big = (np.abs(x) >= 2.0 ** -110) | (x == 0)
    assert big.sum() > 300_000 and (~big).sum() > 1000
    assert np.array_equal(res[big], d2[big])     # res is already a bfloat16 number
    total = hi.astype(np.float64) + lo.astype(np.float64) + res.astype(np.float64)
    assert np.array_equal(total[big], x[big].astype(np.float64))
    # below 2^-110 the residual is rounded, to within a bfloat16 subnormal step
    err = np.abs(total[~big] - x[~big].astype(np.float64))
    assert err.max() <= 2.0 ** -134
