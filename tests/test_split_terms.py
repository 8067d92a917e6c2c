"""The three-term BF16 split behind the split-BF16 Schur update, checked in
exact arithmetic on the host (no GPU): every finite FP32 value x away from the
bottom of the exponent range is x_1 + x_2 + x_3 exactly, with x_1 = bf16(x),
x_2 = bf16(x - x_1), x_3 = bf16(x - x_1 - x_2) (nearest, ties to even), with
|x_2| <= 2^-8 |x| (the first rounding error is at most half a BF16 unit of x's
binade) and |x_3| <= 2^-17 |x| (half a unit of x_2's); so of the nine cross
products x_i y_j the six with i + j <= 4 reproduce x y to within
|x_2 y_3| + |x_3 y_2| + |x_3 y_3| <= (2^-24 + 2^-34) |x y|, one unit of FP32
rounding.  BF16 x BF16 products and their sums of a few terms are exact in
FP64, so the checks below are exact.
"""
import numpy as np


def _bf16(x32):
    """FP32 -> BF16 value (as FP32), round to nearest, ties to even."""
    b = np.asarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def _split3(x32):
    t1 = _bf16(x32)
    r1 = (x32 - t1).astype(np.float32)  # exact in FP32
    t2 = _bf16(r1)
    t3 = _bf16((r1 - t2).astype(np.float32))
    return t1, t2, t3


def _samples(n, seed):
    rng = np.random.default_rng(seed)
    mant = rng.uniform(-1.0, 1.0, n)
    expo = rng.integers(-60, 60, n)
    x = np.ldexp(mant, expo).astype(np.float32)
    # ties and near-ties of the first rounding: low 16 bits 0x8000 and 0x7fff
    b = rng.integers(0, 2**31, 64, dtype=np.uint64).astype(np.uint32)
    t = np.concatenate([(b & 0xFFFF0000) | 0x8000, (b & 0xFFFF0000) | 0x7FFF]).astype(np.uint32)
    t = t.view(np.float32)
    t = t[np.isfinite(t) & (np.abs(t) > 1e-30) & (np.abs(t) < 1e30)]
    return np.concatenate([x, t, np.float32([1.0, -3.0, 2.0 ** -20, 1.0 + 2.0 ** -23])])


def test_three_terms_are_exact():
    x = _samples(20000, 1)
    t1, t2, t3 = _split3(x)
    s = t1.astype(np.float64) + t2.astype(np.float64) + t3.astype(np.float64)
    np.testing.assert_array_equal(s, x.astype(np.float64))
    ax = np.abs(x.astype(np.float64))
    assert np.all(np.abs(t2.astype(np.float64)) <= 2.0 ** -8 * ax)
    assert np.all(np.abs(t3.astype(np.float64)) <= 2.0 ** -17 * ax)
    # each term carries at most 8 significant bits: it is its own BF16 rounding
    for t in (t1, t2, t3):
        np.testing.assert_array_equal(_bf16(t), t)


def test_six_products_within_one_fp32_unit():
    x = _samples(20000, 2)
    y = _samples(20000, 3)[: x.size]
    x = x[: y.size]
    a = [t.astype(np.float64) for t in _split3(x)]
    b = [t.astype(np.float64) for t in _split3(y)]
    kept = sum(a[i] * b[j] for i in range(3) for j in range(3) if i + j <= 2)
    exact = x.astype(np.float64) * y.astype(np.float64)  # 24 x 24 bits: exact in FP64
    err = np.abs(kept - exact)
    assert np.all(err <= (2.0 ** -24 + 2.0 ** -34) * np.abs(exact)), err.max()
    # and the bound is nearly reached: the dropped terms are of FP32's rounding order
    assert np.max(err / np.abs(exact)) > 2.0 ** -26
    # the three dropped terms are what is missing, and the largest is not negligible
    dropped = a[1] * b[2] + a[2] * b[1] + a[2] * b[2]
    np.testing.assert_array_equal(kept + dropped, exact)
    assert np.max(np.abs(dropped) / np.maximum(np.abs(exact), 1e-300)) > 2.0 ** -40
