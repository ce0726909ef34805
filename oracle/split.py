"""FP32 -> FP16 hi + 2^-11 * FP16 lo split of A.  ORACLE (test only).

Sec. 4.1, eq:shgemm-1 and eq:shgemm-2:
    A_hi = toF16(A),    A_lo = toF16((A - toF32(A_hi)) * 2^11)
with round-to-nearest-even conversions.  A - toF32(A_hi) and the scaling by
2^11 are exact in FP32, so the only new rounding is that of A_lo; Sec. 4.3
(eq:split-matrix-ineq) bounds the remainder A_Delta = A - A_hi - 2^-11 A_lo by
u16^2 |A| with u16 = 2^-11 (for A_hi, A_lo in the normal range).

Where |a| >= 65520 the FP16 image of a overflows to +-inf (the exponent-range
limit of Sec. 4.2); :func:`range_violation` reports it.
"""
import numpy as np

SPLIT_SCALE = np.float32(2048.0)


def split_f16(a):
    """Return (hi, lo) as float16 arrays for a float32 array ``a``."""
    a = np.asarray(a, dtype=np.float32)
    with np.errstate(over="ignore", invalid="ignore"):
        hi = a.astype(np.float16)
        lo = ((a - hi.astype(np.float32)) * SPLIT_SCALE).astype(np.float16)
    return hi, lo


def split_remainder(a):
    """A_Delta = a - hi - 2^-11 lo, evaluated exactly in FP64."""
    hi, lo = split_f16(a)
    return (np.asarray(a, np.float64) - hi.astype(np.float64)
            - lo.astype(np.float64) * 2.0 ** -11)


def range_violation(a):
    """True where toF16(a) overflows (finite |a| >= 65520, or a = +-inf)."""
    a = np.asarray(a, dtype=np.float32)
    return np.abs(a.astype(np.float64)) >= 65520.0
