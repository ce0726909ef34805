"""FP16 value lattice and the exact law of RN16(g), g ~ N(0,1).  ORACLE (test only).

Sec. 3.1 (eq:g-fp-error, eq:RN-range): a Gaussian value represented in a
floating-point format is the round-to-nearest image of the exact draw.  The
non-negative finite FP16 values, in increasing order, are exactly the bit
patterns 0x0000, 0x0001, ..., 0x7BFF.  Under round-to-nearest the magnitude
|g| is rounded to v_k exactly when |g| lies in the cell [mu_{k-1}, mu_k), where
mu_k = (v_k + v_{k+1}) / 2 is the midpoint to the next value (mu_{-1} := 0;
ties have probability zero).  Hence
    P(|RN16(g)| <= v_k) = P(|g| < mu_k) = erf(mu_k / sqrt 2) = 2 Phi(mu_k) - 1.

Inverse-CDF reading used by this build (the paper leaves the sampler open):
a uniform 63-bit integer u in [0, 2^63) selects magnitude v_k with
    k = #{ j : T_j <= u },   T_j = floor(2^63 * erf(mu_j / sqrt 2)),
which reproduces the cell probabilities to within 2^-63 each.  The table is
cut at index J, the first j with T_j = 2^63 - 1 (J = 18570, mu_J ~ 9.08); the
mass beyond it is below 2^-63.  Thresholds are evaluated with mpmath at 60
significant digits, far more than the 19 digits a 63-bit floor needs.
"""
import functools

import mpmath
import numpy as np

TWO63 = 1 << 63
F16_MAX_FINITE_BITS = 0x7BFF


def f16_value(bits):
    """Exact value (Python float) of FP16 bit pattern(s)."""
    b = np.asarray(bits, dtype=np.uint16)
    return b.view(np.float16).astype(np.float64)


def f16_midpoint(k):
    """mu_k = (v_k + v_{k+1}) / 2 for a non-negative FP16 bit index k (exact in FP64)."""
    k = np.asarray(k, dtype=np.int64)
    return 0.5 * (f16_value(k) + f16_value(k + 1))


@functools.lru_cache(maxsize=None)
def thresholds_f16():
    """Threshold table T_0..T_J as a tuple of Python ints (see module doc)."""
    with mpmath.workdps(60):
        out = []
        scale = mpmath.mpf(TWO63)
        root2 = mpmath.sqrt(2)
        k = 0
        while True:
            mu = mpmath.mpf(float(f16_midpoint(k)))  # exact: 12 significant bits
            t = int(mpmath.floor(scale * mpmath.erf(mu / root2)))
            out.append(t)
            if t >= TWO63 - 1:
                break
            k += 1
    return tuple(out)


def thresholds_f16_array():
    return np.array(thresholds_f16(), dtype=np.uint64)


def cell_index(u63):
    """k = #{j : T_j <= u} for uint64 array u (values < 2^63)."""
    t = thresholds_f16_array()
    return np.searchsorted(t, np.asarray(u63, dtype=np.uint64), side="right").astype(np.int64)


def cell_probabilities_f16():
    """Exact probability (mpmath, 60 digits) that |RN16(g)| = v_k, k = 0..J+1."""
    with mpmath.workdps(60):
        root2 = mpmath.sqrt(2)
        cdf = [mpmath.mpf(0)]
        for k in range(len(thresholds_f16())):
            mu = mpmath.mpf(float(f16_midpoint(k)))
            cdf.append(mpmath.erf(mu / root2))
        cdf.append(mpmath.mpf(1))
        return [cdf[i + 1] - cdf[i] for i in range(len(cdf) - 1)]
