"""The Gaussian random matrix Omega (n x r, row i = contraction index).  ORACLE (test only).

Sec. 3 argues that the Gaussian matrix of a random projection tolerates a
short mantissa; Sec. 4 stores it in FP16 and rounds with RN (Sec. 3.1,
eq:RN-range; Sec. 3.3 and Sec. 4.4.1 draw in FP32 and round).  This module
defines the exact Omega that the library must reproduce bit for bit.

Random source (this build's reading; the paper does not fix one):
  element (i, j) of stream ``stream_id`` under ``seed`` takes word w = j mod 4
  of the Philox4x64-10 block with counter (i, floor(j/4), stream_id, 0) and
  key (seed, 0).  Its low bit is the sign, its upper 63 bits the uniform u.

FP16  |Omega| = v_k with k = #{T_j <= u}  (lattice.py), sign from the low bit,
      and zero is always +0.  This is an exact sample of RN16(g), g ~ N(0,1).
FP32  the same cell k, and a position inside it from the upper 32 bits f of
      word w of the block with counter (i, floor(j/4), stream_id, 1):
          |Omega| = RN32( mu_{k-1} + (mu_k - mu_{k-1}) * (f + 1/2) * 2^-32 )
      with mu_{-1} = 0.  The product is exact in FP64 (at most 35 significant
      bits), the sum is one FP64 round-to-nearest and the result one RN to
      FP32, so the value is fixed bit for bit.  Its RN16 image equals the FP16
      sample except at ties.
"""
import numpy as np

from . import lattice, philox


def _words(seed, stream_id, n, r, c3, rows=None):
    i = (np.arange(n, dtype=np.uint64) if rows is None
         else np.asarray(rows, dtype=np.uint64))[:, None]
    n = i.shape[0]
    jb = (np.arange(r, dtype=np.uint64) >> np.uint64(2))[None, :]
    x0, x1, x2, x3 = philox.philox4x64_10(i, jb, np.uint64(stream_id), np.uint64(c3),
                                          np.uint64(seed), np.uint64(0))
    stack = np.stack([x0, x1, x2, x3], axis=0)           # 4 x n x r
    w = (np.arange(r) & 3)[None, None, :]
    return np.take_along_axis(stack, np.broadcast_to(w, (1, n, r)), axis=0)[0]


def _cell_and_sign(seed, stream_id, n, r, rows=None):
    x = _words(seed, stream_id, n, r, 0, rows)
    sign = (x & np.uint64(1)).astype(np.uint16)
    k = lattice.cell_index(x >> np.uint64(1))
    return k, sign


def omega_f16_bits(seed, stream_id, n, r, rows=None):
    """FP16 bit patterns (uint16, n x r) of Omega; with ``rows`` given, only
    those rows (any indices, n ignored)."""
    k, sign = _cell_and_sign(seed, stream_id, n, r, rows)
    bits = k.astype(np.uint16) | (sign << np.uint16(15))
    return np.where(k == 0, np.uint16(0), bits).astype(np.uint16)


def omega_f16(seed, stream_id, n, r):
    return omega_f16_bits(seed, stream_id, n, r).view(np.float16)


def omega_f32(seed, stream_id, n, r):
    """FP32 Omega (float32, n x r)."""
    k, sign = _cell_and_sign(seed, stream_id, n, r)
    f = (_words(seed, stream_id, n, r, 1) >> np.uint64(32)).astype(np.float64)
    upper = lattice.f16_midpoint(k)
    lower = np.where(k == 0, 0.0, lattice.f16_midpoint(np.maximum(k - 1, 0)))
    mag = lower + (upper - lower) * ((f + 0.5) * 2.0 ** -32)
    mag32 = mag.astype(np.float32)
    return np.where(sign == 1, -mag32, mag32).astype(np.float32)
