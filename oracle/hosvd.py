"""Random-projection HOSVD (Algorithm 2, Sec. 5.2).  ORACLE (test only).

For a tensor X of shape I_1 x ... x I_N stored in C order:
  for each mode i: W <- X_(i) Omega_(i);  Q_i <- QR(W)
  g <- X x_1 Q_1^T x_2 Q_2^T ... x_N Q_N^T
Readings: the unfolding X_(i) has rows indexed by i_i and columns by the
C-order linear index of the remaining modes (the paper leaves the column order
open); the mode product follows Kolda-Bader, (X x_n M)_{..j..} =
sum_{i_n} x_{..i_n..} M_{j, i_n}, so "x_i Q_i^T" contracts mode i of X with
the row index of Q_i; the approximation is X ~ g x_1 Q_1 ... x_N Q_N.
Per-mode ranks J_i are allowed (the paper writes a single target rank).
"""
import numpy as np

from .rsvd import qr_pos


def unfold(x, mode):
    """X_(mode): I_mode x prod(other dims), other modes in C order."""
    x = np.asarray(x)
    return np.moveaxis(x, mode, 0).reshape(x.shape[mode], -1)


def mode_product(x, m, mode):
    """X x_mode M for M of shape J x I_mode (Kolda-Bader)."""
    x = np.asarray(x, np.float64)
    y = np.tensordot(np.asarray(m, np.float64), x, axes=([1], [mode]))  # J x (others)
    return np.moveaxis(y, 0, mode)


def rp_hosvd(x, omegas):
    """Algorithm 2.  ``omegas[i]`` is prod(other dims) x J_i.
    Returns (core, [Q_1, ..., Q_N])."""
    x = np.asarray(x, np.float64)
    qs = []
    for i in range(x.ndim):
        w = unfold(x, i) @ np.asarray(omegas[i], np.float64)
        q, _ = qr_pos(w)
        qs.append(q)
    g = x
    for i, q in enumerate(qs):
        g = mode_product(g, q.T, i)
    return g, qs


def reconstruct(core, qs):
    x = np.asarray(core, np.float64)
    for i, q in enumerate(qs):
        x = mode_product(x, q, i)
    return x
