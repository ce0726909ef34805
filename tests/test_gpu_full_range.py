"""The full-exponent-range variant of the split projection (the role the
paper gives SHGEMM-TF32 in Sec. 4.2, without a TF32 matrix core): an
automatic power-of-two pre-scale per row of A (RP_A_SCALE_AUTO_ROW), on
inputs whose magnitudes leave the FP16 range, against the FP64 oracle on the
same A and the same Omega."""
import numpy as np
import pytest

import synth
from gpu_helpers import announce, dev, host, rp
from oracle import omega, project, rsvd as orsvd

pytestmark = pytest.mark.gpu

U32, U16 = 2.0 ** -24, 2.0 ** -11


def _rows_far_outside_fp16(m, n, seed):
    """Rows at magnitudes 2^-100 .. 2^100, entries spread over 2^+-10 within a
    row, plus an all-zero row."""
    rng = np.random.default_rng(seed)
    row_mag = 2.0 ** rng.uniform(-100, 100, m)
    a = rng.standard_normal((m, n)) * 2.0 ** rng.uniform(-10, 10, (m, n)) * row_mag[:, None]
    a[m // 2] = 0.0
    return a.astype(np.float32)


@pytest.mark.parametrize("m,n,r", [(300, 1000, 70), (129, 4096, 200), (64, 37, 5)])
def test_project_auto_row_scale_elementwise_bound(m, n, r):
    """Every Y within the split product's elementwise bound
    (gamma_{n+2}(2^-24) + 2^-22) |A| |Omega|; the same A without the
    pre-scale overflows FP16 and reports RP_ERR_RANGE."""
    announce(f"auto row pre-scale m={m} n={n} r={r}")
    a = _rows_far_outside_fp16(m, n, 5 + m)
    da = dev(a)
    y = host(rp().rp_project(da, r, seed=8, stream_id=2, a_scale_exp=rp().RP_A_SCALE_AUTO_ROW)).astype(np.float64)
    assert rp().rp_get_device_status(clear=True) == rp().RP_OK
    om = omega.omega_f16(8, 2, n, r)
    ref = project.project_f64(a, om)
    bound = (project.gamma(n + 2, U32) + U16 * U16) * project.abs_product(a, om)
    assert np.all(np.abs(y - ref) <= bound), float(np.max(np.abs(y - ref) / np.maximum(bound, 1e-300)))
    assert np.all(y[m // 2] == 0.0)
    rp().rp_project(da, r, seed=8, stream_id=2)
    assert rp().rp_get_device_status(clear=True) == rp().RP_ERR_RANGE


def test_auto_row_scale_rejected_where_not_taken():
    a = dev(np.ones((8, 64), np.float32))
    with pytest.raises(rp().RpError):
        rp().rp_project_grouped([(a, 4, 0, 0, rp().RP_A_SCALE_AUTO_ROW)])


def test_rsvd_auto_row_scale_cauchy_outside_fp16():
    """RSVD of an A_Cauchy-form matrix whose entries reach 10^6 (gamma =
    10^-6, x, y ~ U(-10^-3, 10^-3)): with the automatic pre-scale the
    singular values match the FP64 oracle's RSVD on the same Omega; the plain
    split reports RP_ERR_RANGE (the failure Sec. 5.1.1 expects of
    SHGEMM-FP16 on such inputs)."""
    n, k, s = 1024, 48, 10
    announce(f"rsvd auto row pre-scale, Cauchy gamma=1e-6 n={n} k={k}")
    a = synth.np_cauchy(n, np.random.default_rng(31), gamma=1e-6)
    assert np.abs(a).max() > 65504.0
    da = dev(a)
    _, sv, _ = rp().rsvd(da, k, s, 0, 17, "f16", "split_f16", a_scale_exp=rp().RP_A_SCALE_AUTO_ROW)
    assert rp().rp_get_device_status(clear=True) == rp().RP_OK
    _, sv_o, _ = orsvd.rsvd(a.astype(np.float64), omega.omega_f16(17, 0, n, k + s), k, 0)
    sv = host(sv)
    print(f"max |sigma - sigma_oracle| / sigma_1 = {np.abs(sv - sv_o).max() / sv_o[0]:.3e}")
    assert np.abs(sv - sv_o).max() <= 1e-5 * sv_o[0]
    rp().rsvd(da, k, s, 0, 17, "f16", "split_f16")
    assert rp().rp_get_device_status(clear=True) == rp().RP_ERR_RANGE
