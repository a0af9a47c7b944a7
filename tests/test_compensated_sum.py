"""The FP32 compensated accumulation of the overlap kernel (CPU, IEEE float32
through numpy): Dekker's Fast2Sum applied to the two addends ordered by
magnitude yields the same exact rounding error as Knuth's branch-free
two-sum, so a running (hi, lo) pair updated either way is bitwise the same;
and hi + lo carries the exact sum of the terms up to the rounding of lo,
far below that of a plain FP32 sum."""
from fractions import Fraction

import numpy as np

f32 = np.float32


def knuth(hi, lo, p):
    s = f32(hi + p)
    bp = f32(s - hi)
    ap = f32(s - bp)
    return s, f32(lo + f32(f32(hi - ap) + f32(p - bp)))


def ordered_fast2sum(hi, lo, p):
    ge = abs(hi) >= abs(p)
    big, small = (hi, p) if ge else (p, hi)
    s = f32(big + small)
    return s, f32(lo + f32(small - f32(s - big)))


def _terms(rng, n):
    # mixed signs, magnitudes over ~24 binary orders, cancelling pairs mixed in
    t = (rng.standard_normal(n) * np.exp2(rng.uniform(-12, 12, n))).astype(np.float32)
    k = n // 4
    t[rng.choice(n, k, replace=False)] = -t[rng.choice(n, k, replace=False)]
    return t


def test_bitwise_identical_running_pairs():
    rng = np.random.default_rng(2303)
    for _ in range(20):
        a = (f32(0), f32(0))
        b = (f32(0), f32(0))
        for p in _terms(rng, 2000):
            a = knuth(*a, p)
            b = ordered_fast2sum(*b, p)
            assert a[0].tobytes() == b[0].tobytes() and a[1].tobytes() == b[1].tobytes()


def test_error_of_each_update_is_exact():
    rng = np.random.default_rng(12980)
    for hi, p in zip(_terms(rng, 5000), _terms(rng, 5000)):
        s, e = ordered_fast2sum(hi, f32(0), p)
        assert Fraction(float(s)) + Fraction(float(e)) == Fraction(float(hi)) + Fraction(float(p))


def test_compensated_sum_close_to_exact():
    rng = np.random.default_rng(7)
    t = _terms(rng, 20000)
    exact = sum(Fraction(float(x)) for x in t)
    hi, lo = f32(0), f32(0)
    plain = f32(0)
    for p in t:
        hi, lo = ordered_fast2sum(hi, lo, p)
        plain = f32(plain + p)
    scale = float(sum(abs(float(x)) for x in t))
    err_comp = abs(float(Fraction(float(hi)) + Fraction(float(lo)) - exact))
    err_plain = abs(float(Fraction(float(plain)) - exact))
    # the pair's error is that of the FP32 low word: ~2^-24 of its size (not of the sum of |terms|)
    assert err_comp <= 2.0 ** -40 * scale
    assert err_plain > 100 * err_comp
