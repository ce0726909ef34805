"""Pins for the randomized-SVD oracle (Algorithm 1, power scheme of Sec. 2.1):
exact recovery of planted low rank, the Eckart-Young lower bound (Theorem
eym), and the Halko et al. mean bound eq:qqta-acc averaged over ten seeds
(Sec. 5.1.1 also uses ten matrices).  Values for the 1024 x 1024, 0.9^i
workload: ||A||_F = 2.064742, ||Sigma_2||_F = 0.070897 (rank 32)."""
import numpy as np
import pytest

import synth
from oracle import omega, rsvd


def test_planted_rank_recovered_exactly():
    rng = np.random.default_rng(0)
    sig = np.array([5.0, 3.0, 2.0, 1.0, 0.5, 0.25])
    a = synth.np_planted(300, 200, sig, rng).astype(np.float64)
    om = omega.omega_f32(1, 0, 200, 16)
    u, s, vt = rsvd.rsvd(a, om, 6)
    assert np.allclose(s, sig, rtol=1e-6)
    assert np.linalg.norm(a - (u * s) @ vt) <= 1e-5 * np.linalg.norm(a)
    assert np.allclose(u.T @ u, np.eye(6), atol=1e-10)


def test_qr_pos_unique_factor():
    y = np.random.default_rng(1).standard_normal((50, 8))
    q, r = rsvd.qr_pos(y)
    assert np.all(np.diag(r) > 0)
    assert np.allclose(q @ r, y)
    # unique thin QR: Cholesky of the Gram matrix gives the same R
    assert np.allclose(np.linalg.cholesky(y.T @ y).T, r)


@pytest.mark.slow
def test_c1_eckart_young_and_halko():
    n, k, s = 1024, 32, 32
    sig = synth.sigma_geometric(n, 0.9)
    tail = float(np.sqrt((sig[k:] ** 2).sum()))
    assert tail == pytest.approx(0.070897, abs=5e-7)
    assert float(np.sqrt((sig ** 2).sum())) == pytest.approx(2.064742, abs=5e-7)
    resid = []
    for seed in range(10):
        a = synth.np_planted(n, n, sig, np.random.default_rng(100 + seed)).astype(np.float64)
        om = omega.omega_f32(200 + seed, 0, n, k + s)
        u, sv, vt = rsvd.rsvd(a, om, k)
        assert np.linalg.norm(a - (u * sv) @ vt) >= tail * (1 - 1e-6)
        q = rsvd.range_finder(a, om)
        resid.append(rsvd.residual_qqta(a, q))
    assert np.mean(resid) <= rsvd.halko_bound(tail, k, s)


def test_halko_bound_c1_value():
    # eq:qqta-acc at the 1024^2 workload: p = 32, s = 32, ||Sigma_2||_F = 0.070897
    sig = synth.sigma_geometric(1024, 0.9)
    tail = float(np.sqrt((sig[32:] ** 2).sum()))
    assert rsvd.halko_bound(tail, 32, 32) == pytest.approx(0.101068, abs=2e-6)


@pytest.mark.parametrize("p,s", [(8, 5), (32, 32)])
def test_halko_factor_is_gaussian_pinv_mean(p, s):
    """eq:qqta-acc comes from eq:sgg: the excess over ||Sigma_2||_F^2 is
    ||Sigma_2||_F^2 E||G_1^+||_F^2 with G_1 a p x (p + s) Gaussian matrix.
    A Monte Carlo mean of ||G_1^+||_F^2 must match (bound / tail)^2 - 1, which
    pins the p/(s-1) term and the square root independently of the formula."""
    rng = np.random.default_rng(5)
    n = 20000 if p < 16 else 4000
    vals = np.array([np.sum(np.linalg.pinv(rng.standard_normal((p, p + s))) ** 2) for _ in range(n)])
    mc, se = vals.mean(), vals.std() / np.sqrt(n)
    factor = (rsvd.halko_bound(1.0, p, s)) ** 2 - 1.0
    assert abs(mc - factor) <= 4 * se


def test_power_iteration_sharpens():
    rng = np.random.default_rng(3)
    sig = 1.0 / np.arange(1, 201) ** 0.5
    a = synth.np_planted(300, 300, sig, rng).astype(np.float64)
    om = omega.omega_f32(3, 0, 300, 20)
    r0 = rsvd.residual_qqta(a, rsvd.range_finder(a, om, 0))
    r2 = rsvd.residual_qqta(a, rsvd.range_finder(a, om, 2))
    best = float(np.sqrt((sig[20:] ** 2).sum()))
    assert best <= r2 < r0
