"""Randomized SVD (Algorithm 1, Sec. 2.2) with the power scheme (Sec. 2.1).  ORACLE (test only).

Algorithm 1 in the paper's order, in FP64 with LAPACK factorizations:
    Y <- A Omega;  Q, R <- QR(Y);  B <- Q^T A;
    U', Sigma_1, V <- tSVD(B, rank p);  U <- Q U'
The power scheme replaces A by (A A^T)^q A (Sec. 2.1).  Applied literally it
squares the condition number of Y at every step, so it is run in the
re-orthonormalised form (reading of the paper's unstabilised formula):
    repeat q times:  Q <- QR(Y);  W <- QR(A^T Q);  Y <- A W
which spans the same subspace as (A A^T)^q A Omega in exact arithmetic.

QR is Householder QR (numpy.linalg.qr) with R's diagonal made positive, so
that Q is the unique thin QR factor of a full-rank Y; SVD is LAPACK's.  The
library uses different algorithms (CholeskyQR2, one-sided Jacobi), so
agreement is a real check and not a re-run of the same code.
"""
import numpy as np


def qr_pos(y):
    """Thin QR of y with diag(R) > 0.  Returns (Q, R)."""
    q, r = np.linalg.qr(np.asarray(y, np.float64), mode="reduced")
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d[None, :], r * d[:, None]


def range_finder(a, omega, power_iters=0):
    """Q with orthonormal columns spanning (A A^T)^q A Omega."""
    a = np.asarray(a, np.float64)
    y = a @ np.asarray(omega, np.float64)
    for _ in range(power_iters):
        q, _ = qr_pos(y)
        w, _ = qr_pos(a.T @ q)
        y = a @ w
    q, _ = qr_pos(y)
    return q


def rsvd(a, omega, k, power_iters=0):
    """Rank-k randomized SVD.  Returns (U m x k, S k, Vt k x n)."""
    a = np.asarray(a, np.float64)
    q = range_finder(a, omega, power_iters)
    b = q.T @ a
    ub, s, vt = np.linalg.svd(b, full_matrices=False)
    return q @ ub[:, :k], s[:k], vt[:k]


def residual_qqta(a, q):
    """||A - Q Q^T A||_F, the error measure of Sec. 3.3 and eq:qqta-acc."""
    a = np.asarray(a, np.float64)
    return float(np.linalg.norm(a - q @ (q.T @ a)))


def halko_bound(sigma_tail_fro, p, s):
    """Right-hand side of eq:qqta-acc: sqrt(1 + p/(s-1)) ||Sigma_2||_F."""
    return float(np.sqrt(1.0 + p / (s - 1.0)) * sigma_tail_fro)
