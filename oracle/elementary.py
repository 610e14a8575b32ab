"""FP64 exponential, logarithm and cosine defined as fixed sequences of IEEE
operations.  TEST INFRASTRUCTURE ONLY (same rule as sparsink_oracle.py: only
tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg use it).

The keep decision of eq. (pois) compares a uniform draw with p*_ij, and for
UOT p*_ij (eq. (pij-uot)) holds an exponential, logarithms of the masses and,
with the Wasserstein-Fisher-Rao cost, a cosine.  Library routines of two
platforms may differ in the last bit, which could move an entry across the
keep boundary.  These functions fix every operation instead: each product and
sum is a separately rounded IEEE FP64 operation (NumPy has no fused
multiply-add), in the order written here, so any implementation of the same
sequence returns the same bits.  The device side implements the same
definitions independently.

Methods (Cody & Waite, "Software Manual for the Elementary Functions",
Prentice-Hall 1980, additive argument reduction with a constant split in two
parts; Muller, "Elementary Functions: Algorithms and Implementation"):

* exp_spec(x): k = rint(x log2 e); r = (x - k L_hi) - k L_lo with
  L_hi + L_lo = ln 2 (L_hi has 33 significant bits, so k L_hi is exact);
  p = Taylor polynomial of e^r of degree 13 by Horner's rule; result
  p 2^k.  NaN stays NaN, x > 709.8 gives +inf, x < -708 gives 0 (no
  subnormal results).
* log_spec(x): x = m 2^e with m in [sqrt(1/2), sqrt(2)); z = (m-1)/(m+1);
  log m = 2 atanh z = 2 z sum_{k<=11} z^(2k) / (2k+1) by Horner's rule in
  z^2; result e L_hi + (e L_lo + log m).  0 gives -inf, +inf gives +inf,
  negative or NaN gives NaN.
* cos_spec(z), 0 <= z <= pi/2: the Taylor series of cos in t = z^2 to
  degree 10 for z <= pi/4, else sin(y) with y = (P_hi - z) + P_lo
  (P_hi + P_lo = pi/2, P_hi with 33 significant bits) and the Taylor
  series of sin y / y in y^2 to degree 10.  Relative error within 2 ulp
  while pi/2 - z >= 1e-8; nearer pi/2 the absolute error is below 1e-26
  (the last bit of P_lo).

Coefficients are the correctly rounded values of the exact rationals 1/k!,
1/(2k+1), (-1)^k/(2k)! and (-1)^k/(2k+1)!; L_lo and P_lo are the correctly
rounded remainders of ln 2 and pi/2 (60-digit decimal values) after the high
parts.
"""
from __future__ import annotations

import math
from decimal import Decimal
from fractions import Fraction

import numpy as np

# exact rationals of 60-digit decimal expansions (Decimal -> Fraction is exact)
_LN2 = Fraction(Decimal("0.693147180559945309417232121458176568075500134360255254120680"))
_PIO2 = Fraction(Decimal("1.57079632679489661923132169163975144209858469968755291048747"))

LOG2E = float(1 / _LN2)
LN2_HI = float.fromhex("0x1.62e42feep-1")
LN2_LO = float(_LN2 - Fraction(LN2_HI))
PIO2_HI = float.fromhex("0x1.921fb544p+0")
PIO2_LO = float(_PIO2 - Fraction(PIO2_HI))
PIO4 = float(_PIO2 / 2)
SQRT_HALF = math.sqrt(0.5)  # correctly rounded (IEEE square root)

EXP_C = [float(Fraction(1, math.factorial(k))) for k in range(14)]
LOG_C = [float(Fraction(1, 2 * k + 1)) for k in range(12)]
COS_C = [float(Fraction((-1) ** k, math.factorial(2 * k))) for k in range(11)]
SIN_C = [float(Fraction((-1) ** k, math.factorial(2 * k + 1))) for k in range(11)]

EXP_HI = 709.8
EXP_LO = -708.0


def _horner(coef, t):
    """c[K] t^K + ... + c[0] evaluated as ((c[K] t + c[K-1]) t + ...) + c[0],
    every product and sum rounded separately."""
    p = np.full_like(t, coef[-1])
    for c in coef[-2::-1]:
        p = p * t + c
    return p


_CH = 16384  # elements per chunk: the temporaries stay in cache


def _exp_chunk(x, out, k, r, p, ki):
    """exp_spec of a chunk with every x in [EXP_LO, EXP_HI], in place."""
    np.multiply(x, LOG2E, out=k)
    np.rint(k, out=k)
    np.multiply(k, LN2_HI, out=r)
    np.subtract(x, r, out=r)
    np.multiply(k, LN2_LO, out=p)
    np.subtract(r, p, out=r)
    p.fill(EXP_C[-1])
    for c in EXP_C[-2::-1]:
        np.multiply(p, r, out=p)
        np.add(p, c, out=p)
    ki[:] = k
    np.ldexp(p, ki, out=out)


def exp_spec(x):
    """e^x per the definition in the module docstring (arrays or scalars)."""
    x = np.asarray(x, dtype=np.float64)
    scalar = x.ndim == 0
    xf = np.ascontiguousarray(x).reshape(-1)
    inner = (xf >= EXP_LO) & (xf <= EXP_HI)
    xi = np.where(inner, xf, 0.0)
    out = np.empty_like(xi)
    k, r, p = np.empty(_CH), np.empty(_CH), np.empty(_CH)
    ki = np.empty(_CH, np.int32)
    with np.errstate(over="ignore"):  # x in (log DBL_MAX, 709.8]: +inf
        for s in range(0, xi.size, _CH):
            n = min(_CH, xi.size - s)
            _exp_chunk(xi[s:s + n], out[s:s + n], k[:n], r[:n], p[:n], ki[:n])
    out = np.where(inner, out, np.where(xf > EXP_HI, np.inf, 0.0))
    out = np.where(np.isnan(xf), np.nan, out).reshape(x.shape)
    return float(out) if scalar else out


def log_spec(x):
    """log x per the definition in the module docstring."""
    x = np.asarray(x, dtype=np.float64)
    scalar = x.ndim == 0
    x = np.atleast_1d(x)
    ok = (x > 0.0) & np.isfinite(x)
    xi = np.where(ok, x, 1.0)
    m, e = np.frexp(xi)               # m in [1/2, 1), exact
    low = m < SQRT_HALF
    m = np.where(low, m * 2.0, m)     # exact
    e = np.where(low, e - 1, e).astype(np.float64)
    z = (m - 1.0) / (m + 1.0)
    t = z * _horner(LOG_C, z * z)
    lm = t + t
    res = e * LN2_HI + (e * LN2_LO + lm)
    out = np.where(ok, res, np.where(x == 0.0, -np.inf, np.where(x == np.inf, np.inf, np.nan)))
    return float(out[0]) if scalar else out


def cos_spec(z):
    """cos z for 0 <= z <= pi/2 per the definition in the module docstring."""
    z = np.asarray(z, dtype=np.float64)
    scalar = z.ndim == 0
    z = np.atleast_1d(z)
    near = z <= PIO4
    c = _horner(COS_C, z * z)
    y = (PIO2_HI - z) + PIO2_LO
    s = y * _horner(SIN_C, y * y)
    out = np.where(near, c, s)
    return float(out[0]) if scalar else out
