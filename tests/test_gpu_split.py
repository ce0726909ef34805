"""The in-register split (Sec. 4.1) is bit-exact with NumPy's RNE casts,
including FP16 subnormal hi parts, exact ties and overflow."""
import numpy as np
import pytest

from gpu_helpers import announce, bits16, dev, rp
from oracle import split

pytestmark = pytest.mark.gpu


def _cases():
    rng = np.random.default_rng(0)
    e = rng.uniform(-30.0, 17.0, 200000)
    x = (rng.choice([-1.0, 1.0], e.size) * 2.0 ** e).astype(np.float32)
    specials = np.array([0.0, -0.0, 1.0, 2.0 ** -24, 2.0 ** -25, 3 * 2.0 ** -26, 2.0 ** -14,
                         65504.0, 65519.0, 65520.0, -65520.0, 1e-30, np.nan, np.inf, -np.inf,
                         1.0 + 2.0 ** -11, 1.0 + 3 * 2.0 ** -12, 2049.0, 2051.0], np.float32)
    ties = (np.float16(rng.standard_normal(4096)).astype(np.float32)
            + np.float32(2.0 ** -12)).astype(np.float32)
    return np.concatenate([x, specials, ties])


def test_split_bits_exact():
    x = _cases()
    announce(f"split dump count={x.size}")
    hi, lo = rp().rp_split_f16(dev(x))
    ref_hi, ref_lo = split.split_f16(x)
    gh, gl = bits16(hi), bits16(lo)
    rh, rl = ref_hi.view(np.uint16), ref_lo.view(np.uint16)
    nan_h = np.isnan(ref_hi)
    assert np.array_equal(gh[~nan_h], rh[~nan_h])
    assert np.all(np.isnan(hi.cpu().numpy().view(np.float16)[nan_h]))
    nan_l = np.isnan(ref_lo)
    assert np.array_equal(gl[~nan_l], rl[~nan_l])
