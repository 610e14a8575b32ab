"""Pins of the oracle's specified exponential, logarithm and cosine
(oracle/elementary.py) against what fixes them independently: the platform's
libm (itself within 1 ulp), exact decimal arithmetic, special values and
identities.  A dropped or wrong-signed polynomial term, a wrong reduction
constant or a wrong interval split moves some result by far more than the
2- and 3-ulp bars below (measured worst cases over 3e6 random arguments:
exp 1 ulp, cos 2 ulp, log 2 ulp, 3 ulp near 1)."""
import math
from decimal import Decimal, localcontext
from fractions import Fraction

import numpy as np
import pytest

from oracle import elementary as EL


def _ulps(got, ref):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    return np.abs(got - ref) / np.spacing(np.abs(ref))


def test_constants_are_the_rounded_rationals():
    for k, c in enumerate(EL.EXP_C):
        assert Fraction(c) * math.factorial(k) == pytest.approx(1.0, abs=2.3e-16)
    for k, c in enumerate(EL.LOG_C):
        assert abs(Fraction(c) * (2 * k + 1) - 1) <= Fraction(1, 2 ** 52)
    assert EL.LN2_HI + EL.LN2_LO == math.log(2.0)
    assert EL.PIO2_HI + EL.PIO2_LO == math.pi / 2
    # the high parts leave room for exact products with the reduction multiple
    assert float(Fraction(EL.LN2_HI) * 1100) == EL.LN2_HI * 1100
    assert Fraction(EL.LN2_HI).denominator <= 2 ** 33
    assert Fraction(EL.PIO2_HI).denominator <= 2 ** 32


def test_exp_against_libm_over_its_range():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.uniform(-708.0, 709.8, 200_000),
                        rng.uniform(-1.0, 1.0, 100_000),
                        rng.standard_normal(100_000) * 1e-8,
                        np.arange(-708, 710, dtype=np.float64) * math.log(2.0) / 1.0001])
    x = x[(x >= -708.0) & (x <= 709.78)]
    ref = np.exp(x)
    assert _ulps(EL.exp_spec(x), ref).max() <= 2.0
    # past log(DBL_MAX) = 709.7827... the result overflows as the platform's does
    with np.errstate(over="ignore"):
        assert EL.exp_spec(709.79) == math.inf == np.exp(709.79)


def test_exp_against_exact_decimal():
    rng = np.random.default_rng(1)
    xs = np.concatenate([rng.uniform(-700, 700, 300), rng.uniform(-0.5, 0.5, 300)])
    got = EL.exp_spec(xs)
    with localcontext() as ctx:
        ctx.prec = 40
        ref = np.array([float(Decimal(float(v)).exp()) for v in xs])
    assert _ulps(got, ref).max() <= 1.5


def test_exp_special_values():
    assert EL.exp_spec(0.0) == 1.0
    assert EL.exp_spec(-0.0) == 1.0
    assert math.isnan(EL.exp_spec(float("nan")))
    assert EL.exp_spec(710.0) == math.inf and EL.exp_spec(math.inf) == math.inf
    assert EL.exp_spec(-708.5) == 0.0 and EL.exp_spec(-math.inf) == 0.0
    # the smallest argument kept gives a normal number
    assert EL.exp_spec(-708.0) >= 2.2250738585072014e-308
    # e^x e^-x = 1 within the rounding of the two results
    for v in (0.25, 3.0, 40.0, 700.0):
        assert EL.exp_spec(v) * EL.exp_spec(-v) == pytest.approx(1.0, rel=5e-16)


def test_log_against_libm_and_exact_decimal():
    rng = np.random.default_rng(2)
    x = np.concatenate([np.exp(rng.uniform(-700, 700, 200_000)),
                        1.0 + rng.standard_normal(50_000) * 1e-6,
                        rng.uniform(0.5, 2.0, 50_000),
                        np.array([5e-324, 1e-310, 2.2250738585072014e-308, 1.7e308])])
    # large results within 2 ulp; results below 1 in magnitude (x near 1)
    # within 3: the quotient (m - 1)/(m + 1) carries its own rounding
    big = np.abs(np.log(x)) >= 1.0
    assert _ulps(EL.log_spec(x[big]), np.log(x[big])).max() <= 2.0
    assert _ulps(EL.log_spec(x), np.log(x)).max() <= 3.0
    xs = x[rng.integers(0, x.size, 400)]
    with localcontext() as ctx:
        ctx.prec = 40
        ref = np.array([float(Decimal(float(v)).ln()) for v in xs])
    ok = ref != 0.0
    assert _ulps(EL.log_spec(xs)[ok], ref[ok]).max() <= 3.0


def test_log_special_values_and_identities():
    assert EL.log_spec(1.0) == 0.0
    assert EL.log_spec(0.0) == -math.inf
    assert EL.log_spec(math.inf) == math.inf
    assert math.isnan(EL.log_spec(-1.0)) and math.isnan(EL.log_spec(float("nan")))
    for k in (-1074, -1022, -1, 1, 7, 1023):
        assert _ulps(EL.log_spec(2.0 ** k), k * math.log(2.0)) <= 1.0
    # log(1 + d) = d - d^2/2 + ... keeps its relative accuracy near 1
    for d in (1e-12, -1e-12, 3e-9):
        assert EL.log_spec(1.0 + d) == pytest.approx(math.log1p((1.0 + d) - 1.0), rel=7e-16)


def test_cos_on_the_quarter_period():
    rng = np.random.default_rng(3)
    half_pi = math.pi / 2
    z = np.concatenate([rng.uniform(0.0, half_pi, 200_000),
                        half_pi - np.exp(rng.uniform(-30, -1, 20_000)),
                        np.array([0.0, EL.PIO4, np.nextafter(EL.PIO4, 2.0), half_pi])])
    z = z[(z >= 0.0) & (z <= half_pi)]
    got = EL.cos_spec(z)
    ref = np.cos(z)
    # within 2 ulp while pi/2 - z >= 1e-8; closer to pi/2 the two-part
    # pi/2 (33 + 53 bits, last bit of P_lo worth 1.3e-26) bounds the
    # absolute error by 1e-26
    rel = half_pi - z >= 1e-8
    assert _ulps(got[rel], ref[rel]).max() <= 2.0
    assert np.all(np.abs(got - ref) <= 1e-26 + 2.0 * np.spacing(ref))
    assert EL.cos_spec(0.0) == 1.0
    # cos(pi/2 rounded) is the remainder pi/2 - fl(pi/2) ~ 6.1e-17
    assert EL.cos_spec(half_pi) == pytest.approx(6.123233995736766e-17, rel=1e-9)


def test_functions_keep_array_shapes():
    x = np.linspace(-3.0, 3.0, 12).reshape(3, 4)
    assert EL.exp_spec(x).shape == (3, 4)
    assert np.array_equal(EL.exp_spec(x).ravel(), EL.exp_spec(x.ravel()))
    assert isinstance(EL.exp_spec(1.0), float) and isinstance(EL.log_spec(2.0), float)
