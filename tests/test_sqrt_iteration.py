"""The FP64 square-root and reciprocal-square-root iterations of the sweep
kernels (hardware estimate, one Goldschmidt step, one Newton correction of
the root with an FMA residual; two Newton steps for the reciprocal root),
emulated on the CPU with exactly rounded fused multiply-adds.  The estimate
is modelled as 1/sqrt(x) with a relative error up to E (the hardware
estimate's measured error is below 2^-22); the pins are facts of the
iteration: the root is the correctly rounded one for E up to 2^-22 and
within 1 ulp for E up to 2^-14, the reciprocal root within 2 ulp,
sqrt(0) = 0 and a negative argument gives NaN."""
import math
import random
from fractions import Fraction

import pytest


def _fma(a, b, c):
    if any(math.isnan(v) for v in (a, b, c)):
        return math.nan
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def _estimate(x, err):
    if x < 0 or math.isnan(x):
        return math.nan
    return (1.0 / math.sqrt(x)) * (1.0 + err)


def _fsqrt(x, err):
    y = _estimate(x + 2.0 ** -1022, err)
    g, h = x * y, 0.5 * y
    r = _fma(-g, h, 0.5)
    g, h = _fma(g, r, g), _fma(h, r, h)
    d = _fma(-g, g, x)
    return _fma(d, h, g)


def _frsq(x, err):
    y = _estimate(x, err)
    for _ in range(2):
        y = _fma(0.5 * y, _fma(-x * y, y, 1.0), y)
    return y


@pytest.mark.parametrize("emax,root_ulp", [(2.0 ** -22, 0), (2.0 ** -14, 1)])
def test_root_rounding_and_reciprocal_within_two_ulp(emax, root_ulp):
    rnd = random.Random(7)
    for _ in range(3000):
        x = 10.0 ** rnd.uniform(-250, 250) * rnd.uniform(1.0, 10.0)
        err = rnd.uniform(-emax, emax)
        assert abs(_fsqrt(x, err) - math.sqrt(x)) <= root_ulp * math.ulp(math.sqrt(x))
        want = 1.0 / math.sqrt(x)
        assert abs(_frsq(x, err) - want) <= 2 * math.ulp(want)


def test_special_arguments():
    for err in (-2.0 ** -22, 0.0, 2.0 ** -22):
        assert _fsqrt(0.0, err) == 0.0
        assert math.isnan(_fsqrt(-1e-3, err))
        # perfect squares and the squares of wave speeds seen in the solver
        for v in (1.0, 4.0, 0.25, 1e-24, 2.5e7):
            assert _fsqrt(v, err) == math.sqrt(v)
