"""The FP64 flux multiplier max(sqrt(x), g) of the kernels (max(gamma, |v|) of §2), emulated
on the CPU step by step: a reciprocal-root estimate y of relative error up to 2^-20 (the
hardware estimate is far better), one Goldschmidt step of the coupled pair
(s, h) ~ (sqrt(x), 1/(2 sqrt(x))) started from (x y, y/2), then the correction
s + h (x - s^2). Every fused multiply-add is emulated exactly (a rational product and sum,
rounded once to float64). The result is within one ulp of the correctly rounded root over
the range of |v|^2 the method meets and far beyond it; x <= g^2 and NaN give g."""
import math
from fractions import Fraction

import numpy as np
import pytest


def fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def mul(a, b):
    return float(Fraction(a) * Fraction(b))


def max_sqrt(x, g, rel_err):
    if not (x > g * g):
        return g
    y = (1.0 / math.sqrt(x)) * (1.0 + rel_err)
    s = mul(x, y)
    h = mul(0.5, y)
    r = fma(-s, h, 0.5)
    s = fma(s, r, s)
    h = fma(h, r, h)
    d = fma(-s, s, x)
    return fma(d, h, s)


def correctly_rounded_sqrt(x):
    # math.sqrt is correctly rounded (IEEE 754); checked here against integer square roots
    s = math.sqrt(x)
    fx = Fraction(x)
    lo, hi = Fraction(np.nextafter(s, 0.0)), Fraction(np.nextafter(s, math.inf))
    fs = Fraction(s)
    assert abs(fs * fs - fx) <= abs(lo * lo - fx) and abs(fs * fs - fx) <= abs(hi * hi - fx)
    return s


@pytest.mark.parametrize("rel_err", [-2.0 ** -20, -1e-7, -2.0 ** -30, 0.0, 3e-9, 2.0 ** -20])
def test_max_sqrt_within_an_ulp(rel_err):
    rng = np.random.default_rng(abs(hash(rel_err)) % 2 ** 32)
    g = 0.09
    xs = np.concatenate([np.exp(rng.uniform(np.log(g * g), np.log(64.0), 300)),
                         np.exp(rng.uniform(np.log(64.0), np.log(1e30), 40)),
                         [g * g * (1 + 2 ** -52), 1.0, 2.0, 4.0, 0.25]])
    worst = 0.0
    for x in xs:
        x = float(x)
        got = max_sqrt(x, g, rel_err)
        ref = correctly_rounded_sqrt(x)
        ulps = abs(got - ref) / (np.nextafter(ref, math.inf) - ref)
        worst = max(worst, ulps)
    assert worst <= 1.0, worst


def test_max_sqrt_floor_and_nan():
    g = 0.09
    for x in (0.0, 1e-300, g * g, np.nextafter(g * g, 0.0)):
        assert max_sqrt(float(x), g, 0.0) == g
    assert max_sqrt(float("nan"), g, 0.0) == g
    # just above the floor the root is taken, and it is >= g
    x = float(np.nextafter(g * g, 1.0))
    assert max_sqrt(x, g, 0.0) >= g - 1e-17


def test_a_planted_mistake_is_caught():
    """Dropping the residual correction leaves the Goldschmidt step's error, several ulps
    with a 2^-20 estimate: the check above would catch it."""
    x, g = 2.345, 0.09
    y = (1.0 / math.sqrt(x)) * (1.0 + 2.0 ** -20)
    s, h = mul(x, y), mul(0.5, y)
    r = fma(-s, h, 0.5)
    s = fma(s, r, s)
    ref = math.sqrt(x)
    assert abs(s - ref) / (np.nextafter(ref, math.inf) - ref) > 1.0
