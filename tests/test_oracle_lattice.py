"""Pins for the FP16 lattice and the inverse-CDF thresholds (Sec. 3.1, eq:g-fp-error).

* Cell boundaries: NumPy's float64 -> float16 cast (an independent RN
  implementation) must send mu_k - eps to v_k and mu_k + eps to v_{k+1}.
* Threshold values: recomputed with a different method (Python ``decimal``,
  the positive series erf(x) = 2/sqrt(pi) e^{-x^2} sum 2^n x^{2n+1}/(2n+1)!!,
  with pi from Machin's formula), independent of mpmath.
* Structure: non-decreasing, T_J = 2^63 - 1 at the documented cut.
"""
import decimal
import math

import numpy as np
import pytest

from oracle import lattice

D = decimal.Decimal


def _pi(ctx):
    def atan_inv(x):
        x = D(x)
        total = term = D(1) / x
        x2 = x * x
        n = 1
        while True:
            term = term / x2
            delta = term / (2 * n + 1)
            if delta < D(10) ** (-(ctx.prec + 5)):
                break
            total += -delta if n % 2 else delta
            n += 1
        return total
    return 16 * atan_inv(5) - 4 * atan_inv(239)


def _erf_decimal(x_float, prec=80):
    with decimal.localcontext() as ctx:
        ctx.prec = prec
        x = D(x_float) / D(2).sqrt()
        x2 = x * x
        term = x
        total = x
        n = 0
        while True:
            n += 1
            term = term * 2 * x2 / (2 * n + 1)
            total += term
            if term < total * D(10) ** (-prec):
                break
        return 2 / _pi(ctx).sqrt() * (-x2).exp() * total


def test_table_shape_and_cut():
    t = lattice.thresholds_f16()
    assert len(t) == 18571                      # J = 18570
    assert t[-1] == (1 << 63) - 1 and t[-2] < (1 << 63) - 1
    assert all(a <= b for a, b in zip(t, t[1:]))
    assert float(lattice.f16_midpoint(18570)) == 9.08203125


@pytest.mark.parametrize("k", [0, 1, 2, 3, 1023, 1024, 1025, 15360, 15361, 18569, 18570]
                         + list(np.random.default_rng(5).integers(0, 18571, 40)))
def test_thresholds_against_decimal_series(k):
    k = int(k)
    mu = float(lattice.f16_midpoint(k))
    e = _erf_decimal(mu)
    expect = int((e * D(1 << 63)).to_integral_value(rounding=decimal.ROUND_FLOOR))
    expect = min(expect, (1 << 63) - 1)
    assert lattice.thresholds_f16()[k] == expect


def test_cell_boundaries_against_numpy_rounding():
    k = np.arange(0, 18571)
    mu = lattice.f16_midpoint(k)
    below = np.nextafter(mu, 0.0)
    above = np.nextafter(mu, np.inf)
    assert np.array_equal(below.astype(np.float16).view(np.uint16), k.astype(np.uint16))
    assert np.array_equal(above.astype(np.float16).view(np.uint16), (k + 1).astype(np.uint16))


def test_cell_index_definition():
    t = lattice.thresholds_f16_array()
    u = np.array([0, t[0] - 1, t[0], t[1], t[1] + 1, (1 << 63) - 2, (1 << 63) - 1], dtype=np.uint64)
    assert lattice.cell_index(u).tolist() == [0, 0, 1, 2, 2, 18570, 18571]


def test_probabilities_sum_to_one_and_match_thresholds():
    import mpmath
    p = lattice.cell_probabilities_f16()
    with mpmath.workdps(60):
        assert abs(sum(p) - 1) < mpmath.mpf(10) ** -40
    t = lattice.thresholds_f16()
    # threshold gaps reproduce the cell probabilities to within 2^-63 each
    for k in (0, 1, 500, 14000, 15360, 16384, 18000):
        gap = (t[k] - (t[k - 1] if k else 0)) / 2.0 ** 63
        assert abs(gap - float(p[k])) <= 2.0 ** -62
