"""Sparse random matrices (Sec. 2.2 eq:sp-rand, without the sqrt(s) factor as
Sec. 3.4 allows) in the mixed-precision projection: the generated Omega bit
for bit against the oracle, the split projection within its elementwise
bound, and an RSVD and an RP-HOSVD on sparse Omega against the FP64 oracle on
the same Omega."""
import numpy as np
import pytest

import synth
from gpu_helpers import announce, bits16, dev, host, rp
from oracle import hosvd as ohosvd, omega, project, rsvd as orsvd

pytestmark = pytest.mark.gpu

U32, U16 = 2.0 ** -24, 2.0 ** -11


@pytest.mark.parametrize("kind", omega.SPARSE_KINDS)
@pytest.mark.parametrize("n,r", [(1000, 77), (37, 5), (4096, 256)])
def test_sparse_omega_bits_exact(kind, n, r):
    announce(f"sparse omega {kind} n={n} r={r}")
    got = bits16(rp().rp_omega_generate(n, r, 21, 3, kind))
    assert np.array_equal(got, omega.omega_sparse_f16_bits(21, 3, n, r, kind))


@pytest.mark.parametrize("kind", omega.SPARSE_KINDS)
@pytest.mark.parametrize("algo", ["split_f16", "f32"])
def test_sparse_projection_elementwise_bound(kind, algo):
    """Y = A Omega with the generated (packed) sparse Omega: the split path
    within (gamma_{n+2}(2^-24) + 2^-22) |A| |Omega|, the FP32 path within
    gamma_n(2^-24) |A| |Omega| (eq:g-fp-error)."""
    m, n, r = 700, 2052, 150
    announce(f"sparse projection {kind} {algo}")
    a = np.random.default_rng(4).standard_normal((m, n)).astype(np.float32)
    y = host(rp().rp_project(dev(a), r, seed=9, stream_id=1, omega_type=kind, algo=algo)).astype(np.float64)
    assert rp().rp_get_device_status(clear=True) == rp().RP_OK
    om = omega.omega_sparse(9, 1, n, r, kind)
    ref = project.project_f64(a, om)
    g = project.gamma(n + 2, U32) + U16 * U16 if algo == "split_f16" else project.gamma(n, U32)
    assert np.all(np.abs(y - ref) <= g * project.abs_product(a, om))


def test_rsvd_sparse3_matches_oracle():
    """RSVD with the Achlioptas Omega (s = 3) of a planted rank-k matrix: the
    singular values of the FP64 oracle on the same Omega, and the planted
    spectrum."""
    m, n, k, s = 1500, 1200, 24, 16
    announce(f"rsvd sparse3 {m}x{n} k={k}")
    rng = np.random.default_rng(6)
    sig = 10.0 ** (-3.0 * np.arange(k) / (k - 1))
    a = synth.np_planted(m, n, sig, rng)
    _, sv, _ = rp().rsvd(dev(a), k, s, 0, 14, "sparse3", "split_f16")
    assert rp().rp_get_device_status(clear=True) == rp().RP_OK
    _, sv_o, _ = orsvd.rsvd(a.astype(np.float64), omega.omega_sparse(14, 0, n, k + s, "sparse3"), k, 0)
    sv = host(sv)
    assert np.abs(sv - sv_o).max() <= 1e-5 * sv_o[0]
    assert np.abs(sv - sig).max() <= 1e-5 * sig[0]


def test_hosvd_very_sparse_matches_oracle():
    """RP-HOSVD with the very sparse Omega_i (s = sqrt(rows of Omega_i)) of
    a planted Tucker tensor: factors and core as the FP64 oracle's on the
    same Omega_i."""
    dims, core_dims = (48, 40, 64), (5, 4, 6)
    ranks = (9, 8, 10)
    announce(f"hosvd vsparse dims={dims}")
    x = synth.np_tucker(dims, core_dims, np.random.default_rng(8), noise_std=0.0)
    g, facs = rp().rp_hosvd(dev(x), ranks, 31, "vsparse", "split_f16")
    assert rp().rp_get_device_status(clear=True) == rp().RP_OK
    oms = [omega.omega_sparse(31, i, x.size // x.shape[i], ranks[i], "vsparse") for i in range(3)]
    g_o, qs_o = ohosvd.rp_hosvd(x.astype(np.float64), oms)
    rec = ohosvd.reconstruct(host(g).astype(np.float64), [host(f).astype(np.float64) for f in facs])
    rec_o = ohosvd.reconstruct(g_o, qs_o)
    assert np.linalg.norm(rec - rec_o) <= 5e-5 * np.linalg.norm(rec_o)
    assert np.linalg.norm(rec - x) <= 5e-5 * np.linalg.norm(x)
