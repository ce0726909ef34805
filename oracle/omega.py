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


# --------------------------------------------------------------------------- e4m3
# OCP FP8 E4M3FN: sign, 4 exponent bits (bias 7), 3 mantissa bits, no
# infinities; the code with all exponent and mantissa bits set is NaN, so the
# largest finite value is 1.75 * 2^8 = 448.  Normal values (e >= 1)
# (1 + m/8) 2^(e-7); subnormal values (e = 0) (m/8) 2^-6.

def e4m3_decode(codes):
    """Value of e4m3fn codes (uint8 array) as float64 (NaN for the NaN codes)."""
    c = np.asarray(codes, dtype=np.uint8).astype(np.int64)
    sign = np.where(c & 0x80, -1.0, 1.0)
    e = (c >> 3) & 0xF
    m = c & 0x7
    mag = np.where(e == 0, m / 8.0 * 2.0 ** -6, (1.0 + m / 8.0) * 2.0 ** (e - 7))
    mag = np.where((e == 15) & (m == 7), np.nan, mag)
    return sign * mag


def e4m3_encode_rne(x):
    """Round float64 values to e4m3fn (round to nearest, ties to an even
    mantissa), saturating at +-448; returns uint8 codes.  From the format's
    definition: the quantum is 2^(e-3) for |x| in [2^e, 2^(e+1)), e >= -6,
    and 2^-9 below 2^-6."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    e = np.maximum(e, -6.0)
    q = 2.0 ** (e - 3)
    t = a / q                                    # exact: division by a power of two
    r = np.floor(t)
    frac = t - r
    up = (frac > 0.5) | ((frac == 0.5) & (np.fmod(r, 2) == 1))
    v = np.minimum((r + up) * q, 448.0)          # may carry into the next binade: still exact
    # encode v (a representable magnitude)
    ve = np.floor(np.log2(np.where(v > 0, v, 1.0)))
    normal = v >= 2.0 ** -6
    exp_field = np.where(normal, ve + 7, 0).astype(np.int64)
    man = np.where(normal, v / 2.0 ** ve * 8 - 8, v / 2.0 ** -9).astype(np.int64)
    code = (exp_field << 3) | man
    code = np.where(v == 0, 0, code)
    return (code | np.where(np.signbit(x) & (v > 0), 0x80, 0)).astype(np.uint8)


def omega_e4m3(seed, stream_id, n, r):
    """The e4m3 Omega with a power-of-two scale per column:
        s_j = 2^floor(log2(448 / max_i |Omega32[i, j]|)),
        Omega8[i, j] = sat448(RNE_e4m3(Omega32[i, j] * s_j)),
    so that Y[:, j] = (A Omega8[:, j]) / s_j.  Returns (codes uint8 n x r,
    scale float64 r, value float64 n x r = Omega8 / s_j).  The quotient
    448 / max is one FP64 division; its exponent is taken exactly (frexp)."""
    w32 = omega_f32(seed, stream_id, n, r).astype(np.float64)
    cmax = np.abs(w32).max(axis=0) if n > 0 else np.zeros(r)
    mant, ex = np.frexp(448.0 / np.where(cmax > 0, cmax, 1.0))
    scale = np.where(cmax > 0, np.ldexp(1.0, ex - 1), 1.0)
    codes = e4m3_encode_rne(w32 * scale[None, :])
    return codes, scale, e4m3_decode(codes) / scale[None, :]


# ---------------------------------------------------------------- sparse Omega
# Sec. 2.2, eq:sp-rand: Omega_ij = sqrt(s) * (+1 with probability 1/(2s),
# 0 with probability 1 - 1/s, -1 with probability 1/(2s)), for s = 1 and 3
# (Achlioptas) and s = sqrt(n) (very sparse, Li et al.).  Sec. 3.4 drops the
# sqrt(s) factor (only the range of A Omega is used), so the entries are
# -1, 0 and +1.  This build's reading of the sampling: the whole 64-bit word x
# of element (i, j) (the same word as above) against T = floor(2^64 / (2s)):
# +1 if x < T, -1 if T <= x < 2T, 0 otherwise.

SPARSE_KINDS = ("sparse1", "sparse3", "vsparse")


def sparse_threshold(kind, n):
    """T = floor(2^64 / (2s)) in exact integer arithmetic; for s = sqrt(n),
    floor(2^63 / sqrt(n)) = isqrt(floor(2^126 / n))."""
    import math
    if kind == "sparse1":
        return 1 << 63
    if kind == "sparse3":
        return (1 << 64) // 6
    if kind == "vsparse":
        return math.isqrt((1 << 126) // max(int(n), 1))
    raise ValueError(kind)


def omega_sparse(seed, stream_id, n, r, kind):
    """Float64 n x r matrix of entries in {-1, 0, +1}."""
    t = sparse_threshold(kind, n)
    x = _words(seed, stream_id, n, r, 0)
    out = np.zeros(x.shape, dtype=np.float64)
    if t >= (1 << 64):
        raise ValueError("threshold out of range")
    tt = np.uint64(t)
    plus = x < tt
    minus = (~plus) & ((x - tt) < tt)
    out[plus] = 1.0
    out[minus] = -1.0
    return out


def omega_sparse_f16_bits(seed, stream_id, n, r, kind):
    """The same matrix as FP16 bit patterns (0x3C00, 0xBC00, 0)."""
    v = omega_sparse(seed, stream_id, n, r, kind)
    bits = np.zeros(v.shape, dtype=np.uint16)
    bits[v > 0] = 0x3C00
    bits[v < 0] = 0xBC00
    return bits
