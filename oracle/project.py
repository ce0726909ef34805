"""The random projection Y = A Omega and its error metrics.  ORACLE (test only).

eq:rp-vec (Sec. 2.2): Y = A Omega with A in R^{m x n}, Omega in R^{n x r}.
The reference value is the FP64 product of the FP32 / FP16 inputs converted
exactly to FP64, as Sec. 4.4.1 does for C_F64; the accuracy metric is the
relative Frobenius error ||Y - Y_F64||_F / ||Y_F64||_F of the same section.
"""
from fractions import Fraction

import numpy as np

from . import split as _split


def project_f64(a, omega):
    """Y_F64 = float64(A) @ float64(Omega)."""
    return np.asarray(a, np.float64) @ np.asarray(omega, np.float64)


def project_rows_f64(a_rows, omega):
    """The rows of Y_F64 belonging to a sample of A's rows."""
    return project_f64(a_rows, omega)


def rel_frobenius(y, y_ref):
    y = np.asarray(y, np.float64)
    y_ref = np.asarray(y_ref, np.float64)
    return float(np.linalg.norm(y - y_ref) / np.linalg.norm(y_ref))


def split_product_f64(a, omega16):
    """A_hi Omega + 2^-11 A_lo Omega in exact-ish FP64 (eq:shgemm-3 without
    matrix-unit rounding): the value the split method converges to when
    the only error left is the split remainder A_Delta."""
    hi, lo = _split.split_f16(a)
    om = np.asarray(omega16, np.float64)
    return hi.astype(np.float64) @ om + (lo.astype(np.float64) @ om) * 2.0 ** -11


def project_exact(a, omega):
    """Exact rational product (list of lists of Fraction) for tiny inputs."""
    a = np.asarray(a)
    omega = np.asarray(omega)
    m, n = a.shape
    n2, r = omega.shape
    assert n == n2
    fa = [[Fraction(float(a[i, k])) for k in range(n)] for i in range(m)]
    fo = [[Fraction(float(omega[k, j])) for j in range(r)] for k in range(n)]
    return [[sum((fa[i][k] * fo[k][j] for k in range(n)), Fraction(0))
             for j in range(r)] for i in range(m)]


def abs_product(a, omega):
    """|A| |Omega| (elementwise absolute values), the scale of the error bounds
    of Sec. 4.3 (eq:tc-err-bound and the SHGEMM bound that follows it)."""
    return np.abs(np.asarray(a, np.float64)) @ np.abs(np.asarray(omega, np.float64))


def gamma(n, u):
    """gamma_n(u) = n u / (1 - n u), the classical bound for an n-term
    floating-point dot product with unit roundoff u."""
    return n * u / (1.0 - n * u)
