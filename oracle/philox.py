"""Philox4x64-10, the counter-based generator of Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3" (SC'11).  ORACLE (test only).

The paper only says that the Gaussian matrix is generated in FP32 and rounded
to the low-precision format (Sec. 3.3, Sec. 4.4.1); it does not fix a random
source.  This build fixes one that both the CPU oracle and the GPU library can
reproduce bit for bit: Philox4x64 with 10 rounds.

One block maps a 256-bit counter (x0, x1, x2, x3) and a 128-bit key (k0, k1)
to four 64-bit words.  Each round multiplies x0 and x2 by two fixed odd
constants, keeping the full 128-bit products, and mixes the halves with the
other two words and the key:
    (x0, x1, x2, x3) <- (hi(M1*x2) ^ x1 ^ k0,  lo(M1*x2),
                         hi(M0*x0) ^ x3 ^ k1,  lo(M0*x0))
and the key is bumped by two Weyl constants between rounds.

This implementation is vectorised NumPy on uint64 arrays; the 64x64->128
product is formed from four 32x32->64 partial products.  It is pinned in the
tests against ``numpy.random.Philox`` (an independent implementation of the
same generator that ships with NumPy).
"""
import numpy as np

PHILOX_M0 = np.uint64(0xD2E7470EE14C6C93)
PHILOX_M1 = np.uint64(0xCA5A826395121157)
PHILOX_W0 = np.uint64(0x9E3779B97F4A7C15)
PHILOX_W1 = np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a, m):
    """Full 128-bit product of uint64 array ``a`` and uint64 scalar ``m``.

    Returns (hi, lo) as uint64 arrays."""
    a = np.asarray(a, dtype=np.uint64)
    a_lo, a_hi = a & _LO32, a >> _S32
    m_lo, m_hi = m & _LO32, m >> _S32
    ll = a_lo * m_lo
    lh = a_lo * m_hi
    hl = a_hi * m_lo
    hh = a_hi * m_hi
    mid = (ll >> _S32) + (lh & _LO32) + (hl & _LO32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    with np.errstate(over="ignore"):
        lo = a * m
    return hi, lo


def philox4x64_10(c0, c1, c2, c3, k0, k1):
    """Apply ten Philox4x64 rounds to counters (c0..c3) under key (k0, k1).

    All arguments broadcast; returns four uint64 arrays (x0, x1, x2, x3)."""
    c0, c1, c2, c3 = np.broadcast_arrays(*(np.asarray(c, dtype=np.uint64)
                                            for c in (c0, c1, c2, c3)))
    x0, x1, x2, x3 = (c.copy() for c in (c0, c1, c2, c3))
    k0 = np.uint64(k0)
    k1 = np.uint64(k1)
    with np.errstate(over="ignore"):
        for rnd in range(10):
            if rnd > 0:
                k0 = np.uint64(k0 + PHILOX_W0)
                k1 = np.uint64(k1 + PHILOX_W1)
            hi0, lo0 = _mulhilo(x0, PHILOX_M0)
            hi1, lo1 = _mulhilo(x2, PHILOX_M1)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return x0, x1, x2, x3
