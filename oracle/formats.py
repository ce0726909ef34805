"""Table 1: Gaussian values represented in eXmY formats.  ORACLE (test only).

Sec. 3.2 studies three properties of g_eXmY, the round-to-nearest image of
g ~ N(0,1) in a format with X exponent and Y mantissa bits:
  * overflow, not-normalized and underflow probabilities (Table 1, top);
  * the number of representable values within 2^s sigma, s = 0, 1, 2
    (Table 1, bottom);
  * the variance alpha_Y = E[g_eXmY^2] (Sec. 3.2.3).

Readings (the printed formulas and the printed table disagree; the table wins):
  * counts: the printed entries are the number of finite values v, zero and
    subnormals included, with |v| < 2^s.  They are counted here binade by
    binade.
  * underflow: RN maps g to zero exactly when |g| <= half the smallest
    subnormal, 2^(-bias-Y); p_uf = erf(2^(-bias-Y) / sqrt 2).
  * not-normalized: the printed values equal erf(2^(-bias) / sqrt 2), the
    Sec. 3.2.1 expression evaluated at 2^(-bias).
  * overflow: p_of = erfc(max / sqrt 2) with max the largest finite value.
"""
import math

import mpmath

# (name, X exponent bits, Y mantissa bits, largest finite value)
FORMATS = {
    "e4m3": (4, 3, 448.0),          # OCP FP8 E4M3FN (no infinities)
    "e5m2": (5, 2, 57344.0),
    "fp16": (5, 10, 65504.0),
    "bf16": (8, 7, 3.3895313892515355e38),
    "tf32": (8, 10, 3.4011621342146535e38),
    "fp32": (8, 23, 3.4028234663852886e38),
}


def bias(x_bits):
    return 2 ** (x_bits - 1) - 1


def count_within(fmt, s):
    """#{finite v in format : |v| < 2^s}, counted binade by binade."""
    x_bits, y_bits, _ = FORMATS[fmt]
    b = bias(x_bits)
    positive = 2 ** y_bits - 1                   # subnormals m * 2^(1-b-Y), m = 1..2^Y-1
    e = 1 - b                                    # normal binades [2^e, 2^(e+1))
    while e + 1 <= s:
        positive += 2 ** y_bits
        e += 1
    return 2 * positive + 1                      # both signs, plus zero


def p_underflow(fmt):
    x_bits, y_bits, _ = FORMATS[fmt]
    with mpmath.workdps(40):
        return float(mpmath.erf(mpmath.mpf(2) ** (-bias(x_bits) - y_bits) / mpmath.sqrt(2)))


def p_not_normalized(fmt):
    x_bits, _, _ = FORMATS[fmt]
    with mpmath.workdps(40):
        return float(mpmath.erf(mpmath.mpf(2) ** (-bias(x_bits)) / mpmath.sqrt(2)))


def p_overflow(fmt):
    _, _, vmax = FORMATS[fmt]
    with mpmath.workdps(40):
        return float(mpmath.erfc(mpmath.mpf(vmax) / mpmath.sqrt(2)))


def one_significant_digit(p):
    """Round p to one significant digit, as Table 1 prints it."""
    if p == 0:
        return 0.0
    e = math.floor(math.log10(abs(p)))
    return round(p / 10 ** e) * 10 ** e


def variance_from_cells(values, probabilities):
    """alpha = sum_v v^2 P(RN(g) = v) for magnitudes ``values`` whose
    probabilities already include both signs."""
    with mpmath.workdps(60):
        return sum(mpmath.mpf(float(v)) ** 2 * p for v, p in zip(values, probabilities))
