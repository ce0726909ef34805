"""Boundary features of the C ABI against the oracle: the caller pre-scale
2^s of A (Sec. 4.2: FP16 limits the exponent range of the split), a caller
Omega with entries outside the single-accumulator range, a caller e4m3 Omega
with its column scales (Table 1's FP8 format), the range flag on the 16-byte
and contraction-split kernels, and rsvd with a caller-owned workspace."""
import numpy as np
import pytest

from gpu_helpers import announce, dev, host, rp
from oracle import omega, project

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
U16 = 2.0 ** -11


def _bound(a, om):
    n = a.shape[1]
    return (project.gamma(n + 2, U32) + U16 * U16) * project.abs_product(a, om)


def test_a_scale_exp_brings_large_a_into_range():
    """|a| up to ~5e6 overflows FP16; with s = -8 the split takes 2^-8 A
    (< 2e4) and Y comes back scaled by 2^8: within the elementwise bound, no
    RP_ERR_RANGE."""
    announce("a_scale_exp -8 on |a| ~ 1e6")
    m = rp()
    rng = np.random.default_rng(31)
    a = (rng.standard_normal((300, 1000)) * 1e6).astype(np.float32)
    om = omega.omega_f16(8, 0, 1000, 64)
    ref = project.project_f64(a, om)
    m.rp_get_device_status(clear=True)
    m.rp_project(dev(a), 64, seed=8)
    assert m.rp_get_device_status(clear=True) == m.RP_ERR_RANGE
    y = host(m.rp_project(dev(a), 64, seed=8, a_scale_exp=-8)).astype(np.float64)
    assert m.rp_get_device_status(clear=True) == m.RP_OK
    assert np.all(np.abs(y - ref) <= _bound(a, om))
    # the packed entry point and the grouped one take the same scale
    pk = m.rp_omega_pack(1000, 64, seed=8)
    y2 = host(m.rp_project_packed(dev(a), 64, pk, a_scale_exp=-8))
    assert np.array_equal(y2, y.astype(np.float32))
    (y3,) = m.rp_project_grouped([(dev(a), 64, 8, 0, -8)])
    assert np.array_equal(host(y3), y.astype(np.float32))
    assert m.rp_get_device_status(clear=True) == m.RP_OK


def test_a_scale_exp_keeps_tiny_a_precise():
    """|a| ~ 1e-9 lies below the FP16 normal range: hi would be subnormal.
    With s = +30 the split works at full precision and Y meets the bound."""
    announce("a_scale_exp +30 on |a| ~ 1e-9")
    rng = np.random.default_rng(32)
    a = (rng.standard_normal((128, 512)) * 1e-9).astype(np.float32)
    om = omega.omega_f16(9, 0, 512, 40)
    y = host(rp().rp_project(dev(a), 40, seed=9, a_scale_exp=30)).astype(np.float64)
    assert np.all(np.abs(y - project.project_f64(a, om)) <= _bound(a, om))


def test_a_scale_exp_rejected_outside_range():
    import torch
    with pytest.raises(rp().RpError) as e:
        rp().rp_project(torch.ones((4, 8), device="cuda"), 4, a_scale_exp=65)
    assert e.value.status == rp().RP_ERR_INVALID_ARG


def test_caller_omega_with_large_entry():
    """A 16-byte aligned A (the single-accumulator kernel's path) with a caller
    Omega holding 40.0 and -1000.0: rp_project routes the call to the
    two-accumulator kernel and Y meets the bound; packing that Omega for
    rp_project_packed records RP_ERR_OMEGA_RANGE."""
    announce("caller Omega with |omega| >= 32")
    m = rp()
    rng = np.random.default_rng(33)
    a = rng.standard_normal((256, 512)).astype(np.float32)
    om = omega.omega_f16(10, 0, 512, 48)
    om[7, 3] = 40.0
    om[300, 47] = -1000.0
    omt = dev(om.astype(np.float16).view(np.int16))
    m.rp_get_device_status(clear=True)
    y = host(m.rp_project(dev(a), 48, omega=omt)).astype(np.float64)
    assert m.rp_get_device_status(clear=True) == m.RP_OK
    assert np.all(np.abs(y - project.project_f64(a, om)) <= _bound(a, om))
    m.rp_omega_pack(512, 48, omega=omt)
    assert m.rp_get_device_status(clear=True) == m.RP_ERR_OMEGA_RANGE
    # an Omega inside the range packs without a report
    m.rp_omega_pack(512, 48, omega=dev(omega.omega_f16(10, 0, 512, 48).view(np.int16)))
    assert m.rp_get_device_status(clear=True) == m.RP_OK


@pytest.mark.parametrize("algo", ["split_f16", "f32"])
def test_caller_e4m3_omega_with_col_scale(algo):
    """The e4m3 codes and column scales of rp_omega_generate_e4m3, given back
    by the caller, give the same Y as the generated e4m3 Omega, bit for bit;
    the codes and scales equal the oracle's."""
    announce(f"caller e4m3 Omega {algo}")
    m = rp()
    rng = np.random.default_rng(34)
    n, r = 900, 70
    a = dev(rng.standard_normal((200, n)).astype(np.float32))
    codes, scale = m.rp_omega_generate_e4m3(n, r, seed=19)
    oc, osc, _ = omega.omega_e4m3(19, 0, n, r)
    assert np.array_equal(host(codes), oc) and np.array_equal(host(scale), osc.astype(np.float32))
    y1 = host(m.rp_project(a, r, seed=19, omega_type="e4m3", algo=algo))
    y2 = host(m.rp_project(a, r, omega=codes, col_scale=scale, omega_type="e4m3", algo=algo))
    assert np.array_equal(y1, y2)
    assert m.rp_get_device_status(clear=True) == m.RP_OK


def test_caller_e4m3_bad_scale_reported():
    import torch
    m = rp()
    codes, scale = m.rp_omega_generate_e4m3(64, 16, seed=2)
    bad = scale.clone()
    bad[5] = 3.0                                   # not a power of two
    m.rp_get_device_status(clear=True)
    m.rp_omega_pack(64, 16, omega=codes, col_scale=bad, omega_type="e4m3")
    assert m.rp_get_device_status(clear=True) == m.RP_ERR_OMEGA_RANGE
    with pytest.raises(m.RpError):
        m.rp_project(torch.ones((4, 64), device="cuda"), 16, omega=codes, omega_type="e4m3")   # no col_scale


@pytest.mark.parametrize("shape", [(70, 96, 20), (256, 16384, 256)])
def test_range_flag_on_fast_kernels(shape):
    """The range flag and NaN confinement on a 16-byte aligned A (the
    single-accumulator kernel) and on a shape whose contraction is split
    across workgroups (partial sums added by the last workgroup)."""
    mm, n, r = shape
    announce(f"range flag fast kernel {shape}")
    m = rp()
    m.rp_get_device_status(clear=True)
    a = np.full((mm, n), 0.5, np.float32)
    a[3, 4] = 65519.0
    y = host(m.rp_project(dev(a), r))
    assert np.all(np.isfinite(y))
    assert m.rp_get_device_status(clear=True) == m.RP_OK
    a[mm - 7, n - 5] = 65520.0
    m.rp_project(dev(a), r)
    assert m.rp_get_device_status(clear=True) == m.RP_ERR_RANGE
    a = np.full((mm, n), 0.5, np.float32)
    a[5, n // 2 + 3] = np.nan
    y = host(m.rp_project(dev(a), r))
    assert np.all(np.isnan(y[5])) and np.all(np.isfinite(np.delete(y, 5, axis=0)))
    assert m.rp_get_device_status(clear=True) == m.RP_ERR_RANGE


def test_rsvd_caller_workspace_matches_context_workspace():
    """rsvd with a caller workspace of rsvd_workspace_size() bytes gives the
    same bits as with the context workspace; a short or misaligned
    workspace is rejected before anything runs."""
    import torch
    announce("rsvd caller workspace")
    m = rp()
    rng = np.random.default_rng(35)
    a = dev(rng.standard_normal((700, 500)).astype(np.float32))
    k, s, q = 20, 12, 1
    need = m.rsvd_workspace_size(700, 500, k, s, q)
    assert need > 0
    u1, s1, v1 = m.rsvd(a, k, s, q, seed=3)
    work = torch.empty(need, dtype=torch.uint8, device="cuda")
    u2, s2, v2 = m.rsvd(a, k, s, q, seed=3, work=work)
    assert np.array_equal(host(s1), host(s2))
    assert np.array_equal(host(u1), host(u2)) and np.array_equal(host(v1), host(v2))
    with pytest.raises(m.RpError) as e:
        m.rsvd(a, k, s, q, seed=3, work=work[: need - 256])
    assert e.value.status == m.RP_ERR_INVALID_ARG
    with pytest.raises(m.RpError) as e:
        m.rsvd(a, k, s, q, seed=3, work=work[16:])
    assert e.value.status == m.RP_ERR_INVALID_ARG


def test_rsvd_a_scale_exp():
    """A = 1e6 x (planted rank 8): without the pre-scale the split overflows;
    with s = -12 the singular values match the planted ones."""
    import synth
    announce("rsvd a_scale_exp")
    m = rp()
    sig = np.array([8.0, 6.0, 5.0, 3.0, 2.0, 1.5, 1.0, 0.5]) * 1e6
    a = synth.np_planted(600, 400, sig, np.random.default_rng(36)).astype(np.float32)
    m.rp_get_device_status(clear=True)
    _, sv, _ = m.rsvd(dev(a), 8, 8, 0, seed=4, a_scale_exp=-12)
    assert m.rp_get_device_status(clear=True) == m.RP_OK
    assert np.allclose(host(sv), sig, rtol=2e-5)
