"""The accuracy-suite inputs (Sec. 3.3 Type 1 / Type 2, Sec. 5.1.1 A_linear,
A_exp, A_Poly, A_Cauchy) have the structure the paper prescribes: checked
against their definitions by properties computed independently (singular
values of the formed matrix, closed-form tails, element formulas)."""
import numpy as np

import synth


def test_sv_sequences_closed_forms():
    n, p, s_p = 512, 64, 1e-3
    lin = synth.sv_linear(n, p, s_p)
    assert lin[0] == 1.0 and np.allclose(lin[p:], s_p, rtol=1e-12, atol=0) and np.all(np.diff(lin) <= 0)
    # the Eckart-Young tail of the rank-p approximation: s_p sqrt(n - p)
    assert np.isclose(np.sqrt(np.sum(lin[p:] ** 2)), s_p * np.sqrt(n - p), rtol=1e-12)
    ex = synth.sv_exp(n, p, s_p)
    assert np.isclose(ex[p], s_p, rtol=1e-12) and ex[0] == 1.0
    # geometric tail sum with ratio q = 2^(-2 alpha_e): (s_p^2 - q^n) / (1 - q)
    q = 2.0 ** (-2.0 * np.log2(1.0 / s_p) / p)
    assert np.isclose(np.sum(ex[p:] ** 2), (s_p ** 2 - q ** n) / (1.0 - q), rtol=1e-10)
    poly = synth.sv_poly(n, 20, 3.0, 1e6)
    assert poly.size == n and np.all(poly[:20] == 1e6) and poly[20] == 2.0 ** -3 and poly[-1] == (n - 19) ** -3.0


def test_prescribed_spectrum_matrix():
    import torch
    s = synth.sv_exp(128, 16, 1e-3)
    a = synth.torch_sv_matrix(128, s, 7, "cpu").double().numpy()
    sv = np.linalg.svd(a, compute_uv=False)
    assert np.allclose(sv, s, rtol=0, atol=1e-6)    # FP32 storage of the formed product


def test_type1_and_cauchy():
    rng = np.random.default_rng(3)
    a = synth.np_type1(200, 20, 1e-4, rng).astype(np.float64)
    assert np.allclose(a, a.T, atol=1e-6)
    ev = np.sort(np.linalg.eigvalsh(a))[::-1]
    assert np.all(ev[:20] > 1.0) and np.all(ev[20:] < 1e-3)   # identity block plus a small PSD term
    c = synth.np_cauchy(300, np.random.default_rng(4)).astype(np.float64)
    assert c.min() > 1.0 / 3e-3 * 0.999 and c.max() <= 1.0 / 1e-3 * 1.0001
    # A_ij (|x_i - y_j| + gamma) == 1 with the same draws
    rng = np.random.default_rng(4)
    x, y = rng.uniform(-1e-3, 1e-3, 300), rng.uniform(-1e-3, 1e-3, 300)
    assert np.allclose(c * (np.abs(x[:, None] - y[None, :]) + 1e-3), 1.0, rtol=1e-6)
