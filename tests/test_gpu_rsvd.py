"""Randomized SVD (Algorithm 1 with the power scheme) on the GPU against the
FP64 oracle on the same inputs and the same Omega.

Singular values are unique, so they are compared directly; singular vectors
only up to sign (and rotation inside clusters), so U and V are compared as
projectors onto their span and through the reconstruction U S V^T."""
import numpy as np
import pytest

import synth
from gpu_helpers import announce, dev, host, rp
from oracle import omega, rsvd as orsvd

pytestmark = pytest.mark.gpu


def _run(a, k, s, q, seed, omega_type, algo):
    u, sv, vt = rp().rsvd(dev(a), k, s, q, seed, omega_type, algo)
    st = rp().rp_get_device_status(clear=True)
    return host(u).astype(np.float64), host(sv), host(vt).astype(np.float64), st


def _oracle(a, k, s, q, seed, omega_type):
    n = a.shape[1]
    om = omega.omega_f32(seed, 0, n, k + s) if omega_type == "f32" else omega.omega_f16(seed, 0, n, k + s)
    return orsvd.rsvd(a.astype(np.float64), om, k, q)


def _check(a, k, s, q, seed, omega_type, algo, sv_rtol, proj_tol):
    u, sv, vt, st = _run(a, k, s, q, seed, omega_type, algo)
    assert st == rp().RP_OK
    uo, so, vto = _oracle(a, k, s, q, seed, omega_type)
    assert np.all(np.diff(sv) <= 0)
    np.testing.assert_allclose(sv, so, rtol=sv_rtol, atol=sv_rtol * so[0])
    # orthonormal columns
    assert np.abs(u.T @ u - np.eye(k)).max() < 1e-4
    assert np.abs(vt @ vt.T - np.eye(k)).max() < 1e-4
    # same subspaces (projectors), same reconstruction error
    assert np.linalg.norm(u @ u.T - uo @ uo.T) < proj_tol
    rec = np.linalg.norm(a - (u * sv) @ vt)
    rec_o = np.linalg.norm(a - (uo * so) @ vto)
    assert rec <= rec_o * (1 + 1e-3) + 1e-5 * np.linalg.norm(a)


@pytest.mark.parametrize("omega_type,algo", [("f32", "f32"), ("f16", "split_f16"), ("f16", "f32")])
def test_rsvd_c1_shape(omega_type, algo):
    """1024 x 1024, sigma_i = 0.9^i, k = 32, s = 32, q = 0 (the all-FP32 RSVD
    workload, plus the FP16-Omega variants)."""
    announce(f"rsvd 1024 {omega_type} {algo}")
    a = synth.np_planted(1024, 1024, synth.sigma_geometric(1024, 0.9), np.random.default_rng(101))
    _check(a, 32, 32, 0, 201, omega_type, algo, 2e-5, 1e-3)


def test_rsvd_power_iteration_ragged():
    announce("rsvd power iteration 700 x 530")
    rng = np.random.default_rng(5)
    sig = 1.0 / np.arange(1, 501) ** 0.7
    a = synth.np_planted(700, 530, sig, rng)
    _check(a, 37, 13, 1, 9, "f16", "split_f16", 5e-5, 5e-3)


def test_rsvd_planted_rank_recovered():
    announce("rsvd planted rank 20")
    rng = np.random.default_rng(6)
    sig = np.linspace(10.0, 1.0, 20)
    a = synth.np_planted(900, 800, sig, rng)
    u, sv, vt, st = _run(a, 20, 12, 0, 3, "f16", "split_f16")
    assert st == rp().RP_OK
    np.testing.assert_allclose(sv, sig, rtol=1e-5)
    assert np.linalg.norm(a - (u * sv) @ vt) <= 2e-6 * np.linalg.norm(a)


def test_rsvd_zero_matrix_reports_breakdown():
    a = np.zeros((200, 150), np.float32)
    u, sv, vt, st = _run(a, 5, 5, 0, 1, "f16", "split_f16")
    assert st == rp().RP_ERR_NOT_SPD


@pytest.mark.parametrize("bad", [np.nan, 1e30])
def test_rsvd_nonfinite_input_reports_and_stays_in_bounds(bad):
    """An element that is NaN or beyond the FP16 range reaches the small SVD
    as NaN.  The ranking of its columns must stay a permutation, so that no
    gather indexes past the factors; the call reports the condition (split
    path: RP_ERR_RANGE; FP32 path: the Cholesky breakdown of the NaN Gram)."""
    announce(f"rsvd non-finite input {bad}")
    rng = np.random.default_rng(91)
    a = rng.standard_normal((300, 256)).astype(np.float32)
    a[17, 33] = bad
    _, _, _, st = _run(a, 8, 8, 1, 3, "f16", "split_f16")
    assert st == rp().RP_ERR_RANGE
    _, _, _, st = _run(a, 8, 8, 1, 3, "f32", "f32")
    if bad != bad:
        assert st == rp().RP_ERR_NOT_SPD


def test_rsvd_invalid_arguments():
    import torch
    a = torch.ones((50, 40), device="cuda")
    with pytest.raises(rp().RpError):
        rp().rsvd(a, 30, 20)          # k + s > min(m, n)


def _golden_sigma64():
    """FP64 oracle singular values of the 32768^2 workload and the SHA-256 of
    the A they were computed from (tests/golden/make_rsvd_sigma64.py)."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rsvd_32768_sigma64.txt")
    sha, vals = None, []
    with open(path) as f:
        for line in f:
            if line.startswith("# a_sha256:"):
                sha = line.split(":", 1)[1].strip()
            elif line.strip() and not line.startswith("#"):
                vals.append(float(line))
    return np.array(vals), sha


def test_rsvd_full_size_vs_fp64_oracle():
    """The 32768^2 workload (planted rank 512 + N(0, 1e-8) noise; k = 512,
    p = 640, one power step, FP16 Omega from seed 203) against the FP64
    oracle's singular values of the same A with the same Omega (stored by
    tests/golden/make_rsvd_sigma64.py, which calls only the oracle on the A
    drawn by synth).  Bound: the FP32 products A^T Q and Q^T A contract over
    m = 32768 rows, so each sigma_i moves by at most about gamma_m(2^-24) ||A||_2
    per product (Weyl); two such products give 2 gamma_m(2^-24) sigma_1."""
    import hashlib
    import torch
    from oracle import project
    announce("rsvd 32768^2 k=512 q=1 vs the FP64 oracle's sigma")
    sig64, sha = _golden_sigma64()
    a, _ = synth.torch_rsvd_workload("cuda")
    assert hashlib.sha256(a.cpu().numpy().tobytes()).hexdigest() == sha, "A differs from the oracle's input"
    _, sv, _ = rp().rsvd(a, 512, 128, 1, 203, "f16", "split_f16")
    assert rp().rp_get_device_status(clear=True) == rp().RP_OK
    sv = host(sv)
    del a
    torch.cuda.empty_cache()
    tol = 2.0 * project.gamma(32768, 2.0 ** -24) * sig64[0]
    err = np.abs(sv - sig64)
    print(f"max |sigma - sigma64| {err.max():.3e} (bound {tol:.3e}), max relative {(err / sig64).max():.3e}")
    assert err.max() <= tol


def test_rsvd_taller_than_65535_row_tiles():
    """m = 4,200,000 rows (65,625 tiles of 64, past one grid dimension's
    limit for the tall products: CholeskyQR2's Q = Y R^-1, U = Q U_r), n = 64,
    planted rank 6: the planted singular values recovered and U orthonormal
    (properties that hold at any size).  B = Q^T A sums m = 4.2M products in
    FP32, whose rounding grows like sqrt(m) u32 (u32 = 2^-24) for a sum of
    independent roundings; by Weyl's inequality |sigma_i - sigma_i(B exact)|
    <= ||dB||_2, so the bound is 4 sqrt(m) u32 sigma_1 (4.9e-4 sigma_1)."""
    import torch
    m, n, k, s = 4_200_000, 64, 6, 10
    announce(f"rsvd tall m={m} n={n} k={k}")
    sig = 10.0 ** (-np.arange(k) / 2.0)
    a = synth.torch_planted(m, n, sig, 9, "cuda")
    u, sv, vt = rp().rsvd(a, k, s, 0, 3, "f16", "split_f16")
    assert rp().rp_get_device_status(clear=True) == rp().RP_OK
    assert np.abs(host(sv) - sig).max() <= 4.0 * np.sqrt(m) * 2.0 ** -24 * sig[0]
    ud = u.double()
    gram = (ud.T @ ud).cpu().numpy()
    assert np.abs(gram - np.eye(k)).max() < 1e-4
    del a, u
    torch.cuda.empty_cache()
