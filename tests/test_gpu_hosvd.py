"""Random-projection HOSVD (Algorithm 2) on the GPU against the FP64 oracle on
the same tensor and the same Omega_i (stream i), bit-identical on both sides.

CholeskyQR2 returns the orthonormal factor whose R has a positive diagonal,
as the oracle's normalised Householder QR does, so the factors Q_i are
compared directly; the core and the reconstruction follow.  Tolerances come
from the FP32 storage of X, W_i and the factors (relative 2^-24 per element,
amplified by the condition number of W_i for the trailing columns)."""
import numpy as np
import pytest

import synth
from gpu_helpers import announce, dev, host, rp
from oracle import hosvd as ohosvd, omega

pytestmark = pytest.mark.gpu


def _oracle(x, ranks, seed, omega_type):
    gen = omega.omega_f32 if omega_type == "f32" else omega.omega_f16
    oms = [gen(seed, i, x.size // x.shape[i], ranks[i]) for i in range(x.ndim)]
    return ohosvd.rp_hosvd(x.astype(np.float64), oms)


def _gpu(x, ranks, seed, omega_type, algo):
    core, facs = rp().rp_hosvd(dev(x), ranks, seed, omega_type, algo)
    st = rp().rp_get_device_status(clear=True)
    return host(core).astype(np.float64), [host(f).astype(np.float64) for f in facs], st


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("dims,core_dims,ranks,noise,omega_type,algo", [
    ((64, 96, 128), (8, 6, 10), (8, 6, 10), 0.0, "f16", "split_f16"),      # grouped + transposed last mode
    ((64, 96, 128), (8, 6, 10), (12, 10, 14), 1e-3, "f16", "split_f16"),   # oversampled, noisy
    ((40, 36, 64), (5, 6, 7), (5, 6, 7), 0.0, "f32", "f32"),                # FP32 baseline
    ((40, 36, 64), (5, 6, 7), (5, 6, 7), 0.0, "f16", "f32"),
    ((33, 70, 45), (4, 5, 6), (4, 5, 6), 0.0, "f16", "split_f16"),         # ragged: two permuted modes
    ((16, 12, 64, 10), (3, 4, 5, 3), (3, 4, 5, 3), 0.0, "f16", "split_f16"),  # 4-way
    ((300, 20), (6, 6), (6, 6), 0.0, "f16", "split_f16"),                   # 2-way (a matrix)
])
def test_hosvd_matches_oracle(dims, core_dims, ranks, noise, omega_type, algo):
    announce(f"hosvd dims={dims} ranks={ranks} noise={noise} {omega_type}/{algo}")
    rng = np.random.default_rng(41)
    x = synth.np_tucker(dims, core_dims, rng, noise_std=noise)
    g, qs, st = _gpu(x, ranks, 7, omega_type, algo)
    assert st == rp().RP_OK
    g_o, qs_o = _oracle(x, ranks, 7, omega_type)
    for i, (q, q_o) in enumerate(zip(qs, qs_o)):
        assert q.shape == (dims[i], ranks[i])
        assert np.abs(q.T @ q - np.eye(ranks[i])).max() < 1e-5
        # Q_i = W_i R^-1 column by column (Gram-Schmidt order): the first
        # core_dims[i] columns span signal and are well determined; with noise
        # the trailing ones are normalised residuals of size ~noise and rotate
        # with the rounding of W_i, so only the leading block is compared then
        lead = ranks[i] if noise == 0.0 else core_dims[i]
        assert _rel(q[:, :lead], q_o[:, :lead]) < 2e-4, (i, _rel(q[:, :lead], q_o[:, :lead]))
    rec = ohosvd.reconstruct(g, qs)
    rec_o = ohosvd.reconstruct(g_o, qs_o)
    assert _rel(rec, rec_o) < (5e-5 if noise == 0.0 else 1e-3)
    err, err_o = _rel(rec, x.astype(np.float64)), _rel(rec_o, x.astype(np.float64))
    if noise == 0.0:
        assert err < 5e-5 and err_o < 5e-5        # exact recovery of a planted Tucker tensor
        assert _rel(g, g_o) < 1e-4
    else:
        assert abs(err - err_o) < 1e-3 * err_o


@pytest.mark.parametrize("dims,ranks", [
    ((64, 96, 128), (12, 10, 14)),     # grouped modes 1, 2; mode 3 transposed with a contraction split
    ((300, 20), (6, 7)),               # 2-way: mode 2 transposed, no split
    ((33, 70, 45), (4, 5, 6)),         # ragged: modes 2, 3 copied mode-first
    ((16, 12, 64, 12), (3, 4, 5, 6)),  # 4-way: modes 1, 2 in place, mode 3 copied, mode 4 transposed
])
def test_hosvd_project_elementwise_bound(dims, ranks):
    """Algorithm 2 line 2 for every mode (rp_hosvd_project): W_i within the
    split product's elementwise bound (gamma_{n+2}(2^-24) + 2^-22)
    |X_(i)| |Omega_i| of the FP64 oracle on the same X and Omega_i, whichever
    route the mode takes (in place, transposed, or copied)."""
    from oracle import project
    announce(f"hosvd_project dims={dims} ranks={ranks}")
    rng = np.random.default_rng(17)
    x = (rng.standard_normal(dims) * np.exp(rng.uniform(-3, 3, dims))).astype(np.float32)
    ws = rp().rp_hosvd_project(dev(x), ranks, 33, "f16", "split_f16")
    assert rp().rp_get_device_status(clear=True) == rp().RP_OK
    x64 = x.astype(np.float64)
    for i in range(len(dims)):
        a = ohosvd.unfold(x64, i)
        om = omega.omega_f16(33, i, a.shape[1], ranks[i]).astype(np.float64)
        ref = a @ om
        bound = (project.gamma(a.shape[1] + 2, 2.0 ** -24) + 2.0 ** -22) * (np.abs(a) @ np.abs(om))
        w = host(ws[i]).astype(np.float64)
        assert np.all(np.abs(w - ref) <= bound), (i, float(np.max(np.abs(w - ref) / bound)))


def test_hosvd_invalid_arguments():
    announce("hosvd invalid args")
    x = dev(np.ones((8, 8, 8), np.float32))
    with pytest.raises(rp().RpError):
        rp().rp_hosvd(x, (9, 2, 2))               # rank above the mode size
    with pytest.raises(rp().RpError):
        rp().rp_hosvd(x, (0, 2, 2))


def _tucker_512(gen):
    """The 512^3 workload: Tucker core 64^3 ~ U(-1, 1) times three Haar
    512 x 64 factors (FP64 on the GPU)."""
    import torch
    n, c = 512, 64
    core = torch.rand((c, c, c), device="cuda", generator=gen, dtype=torch.float64) * 2 - 1
    us = [synth.torch_haar(n, c, gen, "cuda") for _ in range(3)]
    return torch.einsum("abc,ia,jb,kc->ijk", core, us[0], us[1], us[2])


def test_hosvd_full_size_noiseless():
    """512^3 noiseless Tucker tensor with J = 64 (exact rank): the split path
    recovers it to rounding level, within twice the FP32 baseline path's error
    (same Omega widened exactly, FP32 products)."""
    import torch
    announce("hosvd 512^3 J=64 noiseless")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(104)
    x32 = _tucker_512(gen).float().contiguous()

    def run(algo):
        g, facs = rp().rp_hosvd(x32, (64, 64, 64), 204, "f16", algo)
        assert rp().rp_get_device_status(clear=True) == rp().RP_OK
        fd = [f.double() for f in facs]
        for q in fd:
            assert (q.T @ q - torch.eye(64, device="cuda", dtype=torch.float64)).abs().max().item() < 1e-5
        rec = torch.einsum("abc,ia,jb,kc->ijk", g.double(), fd[0], fd[1], fd[2])
        xd = x32.double()
        return ((rec - xd).norm() / xd.norm()).item()

    e_split, e_f32 = run("split_f16"), run("f32")
    print(f"noiseless J=64: rel. reconstruction error split {e_split:.3e}, f32 {e_f32:.3e}")
    assert e_split <= 2.0 * e_f32 + 1e-6 and e_split < 1e-2


def test_hosvd_full_size_vs_oracle():
    """The 512^3 workload with N(0, 1e-6) noise and J = 80, against the FP64
    oracle on the same X (copied back) and the same Omega_i (the oracle's own
    generator).

    * W_i = X_(i) Omega_i (the three 512 x 262144 unfoldings, rp_project):
      every element within the split path's bound (gamma_{n+2}(2^-24) +
      2^-22) (|X_(i)| |Omega_i|).
    * Factors: the thin QR factor with positive diag(R) is unique, and to
      first order ||dQ||_F <= sqrt(2) ||dW||_F / sigma_min(W) (perturbation
      of the QR factorisation); rp_hosvd runs the same split arithmetic
      with another summation order (modes 1 and 2: another contraction
      split; mode 3: X streamed in place through the transposed kernel, the
      same hi/lo split of every element against the same FP16 Omega_3), so
      its dW is taken as at most 4x the measured one.
    * Core: ||dg||_F <= (sum_i ||dQ_i||_2) ||X||_F to first order.
    * Reconstruction: eq:qqta-acc with k = 64 and oversampling J - k = 16
      bounds E||(I - Q_i Q_i^T) X_(i)||_F^2 by (1 + 64/15) times the tail
      energy of X_(i), itself at most ||E||_F^2 (X_(i) - E_(i) has rank 64);
      summed over the three modes, ||X - g x Q||_F <= sqrt(3 (1 + 64/15))
      ||E||_F in the mean.  One draw is allowed 5% above the mean.  The
      library's error must match the oracle's to 0.1%."""
    import torch
    from oracle import project
    announce("hosvd 512^3 J=80 noisy vs the FP64 oracle")
    n, j = 512, 80
    gen = torch.Generator(device="cuda")
    gen.manual_seed(104)
    xs = _tucker_512(gen)
    noise = torch.randn((n, n, n), device="cuda", generator=gen, dtype=torch.float64) * 1e-3
    frac = (noise.norm() / (xs + noise).norm()).item()
    x32 = (xs + noise).float().contiguous()
    del xs, noise
    x64 = host(x32).astype(np.float64)
    oms = [omega.omega_f16(204, i, n * n, j) for i in range(3)]
    # the three unfoldings as the library streams them (mode 3 through a
    # mode-first copy, made here by torch)
    unf = [(x32, rp().desc_from_tensor(x32, rows=n, cols=n * n, s_row=n * n, k_inner=n * n)),
           (x32, rp().desc_from_tensor(x32, rows=n, cols=n * n, s_row=n, k_inner=n, s_k_outer=n * n)),
           (x32.permute(2, 0, 1).contiguous(), None)]
    dw, smin = [], []
    for i, (t, d) in enumerate(unf):
        a = ohosvd.unfold(x64, i)
        w64 = a @ oms[i].astype(np.float64)
        w = host(rp().rp_project(t if d is not None else t.reshape(n, n * n), j, seed=204, stream_id=i,
                                 desc=d)).astype(np.float64)
        bound = (project.gamma(n * n + 2, 2.0 ** -24) + 2.0 ** -22) * (np.abs(a) @ np.abs(oms[i].astype(np.float64)))
        assert np.all(np.abs(w - w64) <= bound), i
        dw.append(np.linalg.norm(w - w64))
        smin.append(np.linalg.svd(w64, compute_uv=False)[-1])
        del a
    del unf
    assert rp().rp_get_device_status(clear=True) == rp().RP_OK
    g, facs = rp().rp_hosvd(x32, (j, j, j), 204, "f16", "split_f16")
    assert rp().rp_get_device_status(clear=True) == rp().RP_OK
    g, qs = host(g).astype(np.float64), [host(f).astype(np.float64) for f in facs]
    g_o, qs_o = ohosvd.rp_hosvd(x64, oms)
    tol_q = []
    for i in range(3):
        tol = 4.0 * np.sqrt(2.0) * dw[i] / smin[i] + 1e-5
        dq = np.linalg.norm(qs[i] - qs_o[i])
        print(f"mode {i}: ||dW||_F {dw[i]:.3e}, sigma_min(W) {smin[i]:.3e}, ||dQ||_F {dq:.3e} (tol {tol:.3e})")
        assert dq <= tol, i
        tol_q.append(tol)
    xn = np.linalg.norm(x64)
    dg = np.linalg.norm(g - g_o)
    print(f"core: ||dg||_F {dg:.3e} (tol {(sum(tol_q) + 1e-5) * xn:.3e})")
    assert dg <= (sum(tol_q) + 1e-5) * xn
    e = _rel(ohosvd.reconstruct(g, qs), x64)
    e_o = _rel(ohosvd.reconstruct(g_o, qs_o), x64)
    cap = 1.05 * np.sqrt(3.0 * (1.0 + 64.0 / 15.0)) * frac
    print(f"reconstruction error: library {e:.5e}, oracle {e_o:.5e}, eq:qqta-acc bound {cap:.5e} "
          f"(noise fraction {frac:.4e})")
    assert abs(e - e_o) <= 1e-3 * e_o
    assert e_o <= cap and e <= cap


def test_hosvd_e4m3_omega():
    """RP-HOSVD with the e4m3 Omega_i (column-scaled FP8 values, exact in
    FP16): same oracle comparison as the FP16 case."""
    dims, core_dims = (48, 64, 40), (6, 5, 4)
    announce(f"hosvd e4m3 dims={dims}")
    rng = np.random.default_rng(17)
    x = synth.np_tucker(dims, core_dims, rng)
    g, qs, st = _gpu(x, core_dims, 23, "e4m3", "split_f16")
    assert st == rp().RP_OK
    oms = [omega.omega_e4m3(23, i, x.size // x.shape[i], core_dims[i])[2] for i in range(x.ndim)]
    g_o, qs_o = ohosvd.rp_hosvd(x.astype(np.float64), oms)
    for i, (q, q_o) in enumerate(zip(qs, qs_o)):
        assert _rel(q, q_o) < 2e-4, i
    assert _rel(ohosvd.reconstruct(g, qs), x.astype(np.float64)) < 5e-5


def test_hosvd_omega_cache_repeat():
    """Repeated calls reuse the context's cached Omega_i: the same seed gives
    the same bits as the first (generating) call, and another seed (another
    cache key) gives the other Omega's result, still matching the oracle."""
    dims, core_dims = (40, 48, 36), (5, 6, 4)
    announce(f"hosvd Omega cache {dims}")
    x = synth.np_tucker(dims, core_dims, np.random.default_rng(8), noise_std=1e-3)
    ranks = (8, 9, 7)
    g1, q1, st1 = _gpu(x, ranks, 91, "f16", "split_f16")
    g2, q2, st2 = _gpu(x, ranks, 91, "f16", "split_f16")
    assert st1 == st2 == rp().RP_OK
    assert np.array_equal(g1, g2) and all(np.array_equal(a, b) for a, b in zip(q1, q2))
    g3, q3, st3 = _gpu(x, ranks, 92, "f16", "split_f16")
    assert st3 == rp().RP_OK and not np.array_equal(g1, g3)
    g_o, qs_o = _oracle(x, ranks, 92, "f16")
    rec, rec_o = ohosvd.reconstruct(g3, q3), ohosvd.reconstruct(g_o, qs_o)
    assert _rel(rec, rec_o) < 1e-3


def test_hosvd_more_than_65535_column_tiles():
    """4 x 2048 x 2048 with J = (4, 8, 8): the first mode's unfolding has
    4,194,304 columns (65,536 tiles of 64), past one grid dimension's limit.
    Properties that hold at any size (the oracle's Omega of 4.2M rows takes
    minutes on the host): orthonormal factors and exact recovery of the
    planted Tucker tensor of rank (2, 3, 3)."""
    dims, core_dims, ranks = (4, 2048, 2048), (2, 3, 3), (4, 8, 8)
    announce(f"hosvd dims={dims} ranks={ranks} (P > 65535 * 64)")
    x = synth.np_tucker(dims, core_dims, np.random.default_rng(71), noise_std=0.0)
    g, qs, st = _gpu(x, ranks, 12, "f16", "split_f16")
    assert st == rp().RP_OK
    for i in range(3):
        assert np.abs(qs[i].T @ qs[i] - np.eye(ranks[i])).max() < 1e-5, i
    rec = ohosvd.reconstruct(g, qs)
    assert _rel(rec, x.astype(np.float64)) < 5e-5
