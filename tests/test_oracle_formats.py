"""Pins for Table 1 (Sec. 3.2) and the variance alpha_Y (Sec. 3.2.3).

The 18 printed counts must be reproduced exactly, and the 6 printed
probabilities to their one printed digit; the counts are also re-derived by
brute-force enumeration of every bit pattern for the 8- and 16-bit formats."""
import os

import numpy as np
import pytest

from oracle import formats, lattice

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1.txt")


def _rows():
    out = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        out[f[0]] = ([int(x) for x in f[1:4]], f[4], f[5])
    return out


@pytest.mark.parametrize("fmt", ["e4m3", "e5m2", "fp16", "bf16", "tf32", "fp32"])
def test_table1_counts(fmt):
    counts, _, _ = _rows()[fmt]
    assert [formats.count_within(fmt, s) for s in (0, 1, 2)] == counts


def _decode(fmt, bits):
    x_bits, y_bits, _ = formats.FORMATS[fmt]
    b = formats.bias(x_bits)
    e = (bits >> y_bits) & ((1 << x_bits) - 1)
    m = bits & ((1 << y_bits) - 1)
    sub = e == 0
    val = np.where(sub, m * 2.0 ** (1 - b - y_bits), (1 + m / 2.0 ** y_bits) * 2.0 ** (e - b))
    s = (bits >> (x_bits + y_bits)) & 1
    return np.where(s == 1, -val, val), e


@pytest.mark.parametrize("fmt", ["e4m3", "e5m2", "fp16"])
def test_table1_counts_bruteforce(fmt):
    x_bits, y_bits, vmax = formats.FORMATS[fmt]
    bits = np.arange(1 << (1 + x_bits + y_bits))
    val, e = _decode(fmt, bits)
    finite = np.abs(val) <= vmax
    if fmt != "e4m3":
        finite &= e != (1 << x_bits) - 1
    vals = np.unique(val[finite])               # +0 and -0 collapse to one value
    for s, expect in zip((0, 1, 2), _rows()[fmt][0]):
        assert int((np.abs(vals) < 2.0 ** s).sum()) == expect


@pytest.mark.parametrize("fmt", ["e4m3", "e5m2", "fp16"])
def test_table1_probabilities(fmt):
    _, p_nn, p_uf = _rows()[fmt]
    assert formats.one_significant_digit(formats.p_not_normalized(fmt)) == pytest.approx(float(p_nn))
    assert formats.one_significant_digit(formats.p_underflow(fmt)) == pytest.approx(float(p_uf))


@pytest.mark.parametrize("fmt", ["bf16", "tf32", "fp32"])
def test_table1_wide_exponent_bounds(fmt):
    assert formats.p_not_normalized(fmt) < 2e-12
    assert formats.p_underflow(fmt) < 2e-12


@pytest.mark.parametrize("fmt", list(formats.FORMATS))
def test_table1_overflow(fmt):
    assert formats.p_overflow(fmt) < 1e-12


def test_underflow_is_rn_to_zero_for_fp16():
    # RN sends |g| <= 2^-25 (half the smallest subnormal) to zero: the first
    # threshold of the FP16 sampler is the same event.
    t0 = lattice.thresholds_f16()[0] / 2.0 ** 63
    assert t0 == pytest.approx(formats.p_underflow("fp16"), rel=1e-12)


def test_variance_fp16():
    p = lattice.cell_probabilities_f16()
    vals = [float(lattice.f16_value(k)) for k in range(len(p))]
    alpha = float(formats.variance_from_cells(vals, p))
    # the lattice variance is within 1e-6 of 1 and below it (binade edges
    # round down more often than up); the value is stated in the design notes
    assert abs(alpha - 1.0) < 1e-6
    assert alpha < 1.0
    assert alpha == pytest.approx(0.99999995572, abs=2e-11)
