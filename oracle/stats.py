"""Norm-preservation statistics of the projection.  ORACLE (test only).

Theorem sgt-fp (Sec. 3.2.3): for a Gaussian matrix with entry variance alpha,
E||S G T||_F^2 = alpha ||S||_F^2 ||T||_F^2.  With S = a row x of A and T = I_r
this is the Johnson-Lindenstrauss statement E||x Omega||^2 = alpha r ||x||^2.
The per-row ratio rho_i = ||Y_i||^2 / (alpha r ||A_i||^2) therefore has mean 1;
for orthonormal rows of A, rotation invariance makes the rho_i independent
chi^2_r / r variables (up to the lattice's departure from a true Gaussian).
"""
import numpy as np


def row_ratios(a, y, alpha, r):
    a = np.asarray(a, np.float64)
    y = np.asarray(y, np.float64)
    return (y * y).sum(axis=1) / (alpha * r * (a * a).sum(axis=1))
