"""Pins for the hi/lo split (Sec. 4.1 eq:shgemm-1/2; bounds of Sec. 4.3,
eq:split-matrix-ineq)."""
import numpy as np

from oracle import split


def _values(rng, n=200000):
    e = rng.uniform(-13.0, 15.0, n)
    return (rng.choice([-1.0, 1.0], n) * 2.0 ** e * rng.uniform(1, 2, n)).astype(np.float32)


def test_hi_is_nearest_fp16():
    a = _values(np.random.default_rng(0))
    hi, _ = split.split_f16(a)
    h = hi.view(np.uint16).astype(np.int64)
    nb = [((h + d) & 0xFFFF).astype(np.uint16).view(np.float16).astype(np.float64) for d in (-1, 1)]
    err = np.abs(a.astype(np.float64) - hi.astype(np.float64))
    for v in nb:
        ok = np.isfinite(v)
        assert np.all(err[ok] <= np.abs(a.astype(np.float64) - v)[ok])


def test_split_bounds():
    a = _values(np.random.default_rng(1))
    hi, lo = split.split_f16(a)
    a64 = np.abs(a.astype(np.float64))
    u16 = 2.0 ** -11
    assert np.all(np.abs(hi.astype(np.float64)) <= (1 + u16) * a64)
    assert np.all(np.abs(lo.astype(np.float64)) * u16 <= u16 * a64 * (1 + u16))
    rem = np.abs(split.split_remainder(a))
    assert np.all(rem <= u16 * u16 * a64)


def test_split_recovers_fp16_representable_exactly():
    a = np.random.default_rng(2).standard_normal(1000).astype(np.float16).astype(np.float32)
    hi, lo = split.split_f16(a)
    assert np.array_equal(hi.astype(np.float32), a)
    assert np.all(lo == 0)


def test_remainder_mean_bits():
    # Sec. 4.3 quotes an expected loss of about 0.25 bit: |A_Delta| is on
    # average well below its bound u16^2 |a|.
    a = _values(np.random.default_rng(3))
    a = a[np.abs(a) > 2.0 ** -3]
    r = np.abs(split.split_remainder(a)) / np.abs(a.astype(np.float64))
    assert r.mean() < 0.5 * 2.0 ** -22


def test_range_flag():
    a = np.array([65519.0, 65520.0, -65520.0, 1e30, np.inf, 1.0], np.float32)
    assert split.range_violation(a).tolist() == [False, True, True, True, True, False]
    hi, _ = split.split_f16(a)
    assert np.isfinite(hi[0]) and np.isinf(hi[1]) and np.isinf(hi[2])
