"""Pins for the Gaussian matrix Omega (Sec. 3; Sec. 4.2 stores it in FP16).

* FP16 magnitudes follow the exact law of RN16(g): a chi-square test of the
  sampled binade frequencies against the exact cell probabilities, and a
  two-sample comparison against NumPy's own Gaussian rounded by NumPy's FP16
  cast (independent sampler, independent rounding).
* Mean 0 (Sec. 3.2.3) and variance alpha_FP16 within sampling error.
* FP32 Omega lies inside the FP16 cell it shares with the FP16 sample, and
  rounds back to it except on exact cell midpoints (ties).
"""
import numpy as np
import pytest
from scipy import stats

from oracle import lattice, omega

ALPHA16 = 0.99999995572


def _binade(bits):
    return ((bits.astype(np.int64) & 0x7FFF) >> 10).ravel()


def test_zero_is_positive_and_values_finite():
    b = omega.omega_f16_bits(3, 0, 4096, 64)
    v = b.view(np.float16).astype(np.float64)
    assert np.all(np.isfinite(v))
    assert not np.any(b == 0x8000)
    assert np.abs(v).max() < 9.09


def test_streams_and_seeds_differ():
    a = omega.omega_f16_bits(1, 0, 64, 64)
    assert not np.array_equal(a, omega.omega_f16_bits(1, 1, 64, 64))
    assert not np.array_equal(a, omega.omega_f16_bits(2, 0, 64, 64))
    # a sub-block is the same sample as the corresponding block of a larger one
    assert np.array_equal(a[:17, :9], omega.omega_f16_bits(1, 0, 17, 9))


def test_f16_law_chi_square():
    bits = omega.omega_f16_bits(11, 0, 4096, 512)     # 2M samples
    p = lattice.cell_probabilities_f16()
    kk = np.arange(len(p))
    pb = np.zeros(32)
    np.add.at(pb, kk >> 10, np.array([float(x) for x in p]))
    obs = np.bincount(_binade(bits), minlength=32)
    exp = pb * bits.size
    keep = exp > 20
    chi2 = ((obs[keep] - exp[keep]) ** 2 / exp[keep]).sum()
    assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-4


def test_f16_law_against_numpy_rounded_gaussian():
    bits = omega.omega_f16_bits(12, 0, 2048, 512)
    ref = np.random.default_rng(12).standard_normal(bits.size).astype(np.float16).view(np.uint16)
    a = np.bincount(_binade(bits), minlength=32)
    b = np.bincount(_binade(ref), minlength=32)
    keep = (a + b) > 40
    table = np.stack([a[keep], b[keep]])
    assert stats.chi2_contingency(table)[1] > 1e-4
    # and the signs are fair
    s = (bits >> 15).astype(np.int64)
    nz = (bits & 0x7FFF) != 0
    assert abs(s[nz].mean() - 0.5) < 4 * 0.5 / np.sqrt(nz.sum())


def test_mean_and_variance():
    v = omega.omega_f16(21, 0, 4096, 512).astype(np.float64).ravel()
    n = v.size
    assert abs(v.mean()) < 4 / np.sqrt(n)
    assert abs(v.var() - ALPHA16) < 4 * np.sqrt(2.0 / n)


def test_f32_in_cell_and_rounds_back():
    b16 = omega.omega_f16_bits(5, 2, 1024, 256)
    w = omega.omega_f32(5, 2, 1024, 256)
    k = (b16 & 0x7FFF).astype(np.int64)
    mag = np.abs(w.astype(np.float64))
    lower = np.where(k == 0, 0.0, lattice.f16_midpoint(np.maximum(k - 1, 0)))
    upper = lattice.f16_midpoint(k)
    assert np.all(mag >= lower) and np.all(mag <= upper)
    nz = k > 0
    assert np.all(np.signbit(w[nz]) == (b16[nz] >> 15).astype(bool))
    back = np.abs(w).astype(np.float16).view(np.uint16)
    tie = (mag == lower) | (mag == upper)
    assert np.array_equal(back[~tie], k[~tie].astype(np.uint16))
    assert tie.mean() < 1e-3


def test_row_subset_equals_full():
    full = omega.omega_f16_bits(8, 1, 300, 21)
    rows = [0, 5, 299, 17]
    assert np.array_equal(omega.omega_f16_bits(8, 1, 0, 21, rows=rows), full[rows])


def test_e4m3_encode_is_nearest_by_brute_force():
    """RNE to e4m3fn against a brute-force search over every finite code:
    the nearest value, ties to the even mantissa; beyond 448 saturation."""
    codes = np.arange(256, dtype=np.uint8)
    vals = omega.e4m3_decode(codes)
    finite = np.isfinite(vals) & ~((codes & 0x80).astype(bool) & (vals == 0))   # one zero
    fv, fc = vals[finite], codes[finite]
    assert np.sum(finite) == 253 and fv.max() == 448.0
    rng = np.random.default_rng(8)
    x = np.concatenate([rng.standard_normal(3000) * 50, rng.uniform(-2 ** -5, 2 ** -5, 2000),
                        (fv[:, None] + np.array([0.0])[None, :]).ravel(),
                        (fv[1:] + fv[:-1]) / 2])                  # every value and every midpoint
    x = x[np.abs(x) <= 448]
    got = omega.e4m3_decode(omega.e4m3_encode_rne(x))
    d = np.abs(fv[None, :] - x[:, None])
    best = d.min(axis=1)
    for xi, gi, bi, row in zip(x, got, best, d):
        cand = fc[np.isclose(row, bi, rtol=0, atol=0)]
        if cand.size == 1:
            assert gi == omega.e4m3_decode(cand)[0] or (gi == 0 and xi == 0), xi
        else:                                                      # a tie: the even mantissa
            even = cand[(cand & 1) == 0]
            assert gi == omega.e4m3_decode(even)[0], xi
    assert omega.e4m3_decode(omega.e4m3_encode_rne(np.array([460.0, -1e4])))[0] == 448.0


def test_e4m3_omega_scale_and_exactness():
    codes, scale, val = omega.omega_e4m3(3, 1, 3000, 40)
    w32 = omega.omega_f32(3, 1, 3000, 40).astype(np.float64)
    cmax = np.abs(w32).max(axis=0)
    # the scale is the largest power of two that keeps the column within 448
    assert np.all(cmax * scale <= 448.0) and np.all(cmax * scale * 2 > 448.0)
    assert np.all(np.log2(scale) == np.round(np.log2(scale)))
    # Omega8 / s_j is exact in FP16 (so the FP16 kernels take it unchanged)
    assert np.array_equal(val.astype(np.float16).astype(np.float64), val)
    # relative quantisation error of e4m3 (3 mantissa bits): at most 2^-4 for normals
    big = np.abs(w32 * scale) >= 2.0 ** -6
    assert np.all(np.abs(val - w32)[big] <= 2.0 ** -4 * np.abs(w32)[big])
