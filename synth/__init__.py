"""Seeded synthetic inputs for the random-projection workloads.

This module is shared by the library's tests and benchmark and by the CPU
oracle.  It draws inputs only (matrices with a prescribed spectrum, Tucker
tensors, problem lists); it contains none of the projection method's own
arithmetic (no Omega generation, no split, no projection, no QR/SVD of the
method).  Two back ends draw the same *distributions*:

* NumPy (``np_*``): small and medium inputs, deterministic from the seed on any
  host.
* torch (``torch_*``): the full-size inputs (up to 4 GiB of FP32), drawn on the
  GPU; deterministic from the seed on a given torch build.  The oracle gets the
  very same array by copying the input back to the host.

Workloads (the paper's experiments are synthetic throughout):
  planted spectrum  A = U diag(sigma) V^T with Haar-distributed U, V
                    (Sec. 3.3 type 2; Sec. 5.1.1 use slatms for the same role)
  accuracy suites   A_linear, A_exp, A_Poly (= Type 2), Type 1, A_Cauchy
                    (Sec. 3.3, Sec. 5.1.1)
  tucker            core x_1 U_1 x_2 U_2 x_3 U_3 + noise (Sec. 5.2, Alg. 3 role)
"""
import math

import numpy as np


# --------------------------------------------------------------------------- numpy
def np_haar(n, k, rng):
    """n x k matrix with orthonormal columns, Haar distributed: QR of a
    Gaussian matrix with the signs of R's diagonal moved into Q."""
    g = rng.standard_normal((n, k))
    q, r = np.linalg.qr(g, mode="reduced")
    return q * np.sign(np.diag(r))[None, :]


def np_planted(m, n, sigma, rng, noise_std=0.0):
    """FP32 A = U diag(sigma) V^T (+ N(0, noise_std^2) noise), formed in FP64."""
    sigma = np.asarray(sigma, np.float64)
    k = sigma.size
    u = np_haar(m, k, rng)
    v = np_haar(n, k, rng)
    a = (u * sigma[None, :]) @ v.T
    if noise_std:
        a = a + noise_std * rng.standard_normal((m, n))
    return a.astype(np.float32)


def sigma_geometric(count, ratio, first_index=1):
    """sigma_i = ratio^i for i = first_index .. first_index + count - 1."""
    i = np.arange(first_index, first_index + count, dtype=np.float64)
    return ratio ** i


def sigma_decade(count, decades, length):
    """sigma_i = 10^(-decades * i / length), i = 1 .. count."""
    i = np.arange(1, count + 1, dtype=np.float64)
    return 10.0 ** (-decades * i / length)


def np_gaussian(shape, rng, std=1.0):
    return (std * rng.standard_normal(shape)).astype(np.float32)


def np_uniform(shape, rng, lo=0.0, hi=1.0):
    return rng.uniform(lo, hi, size=shape).astype(np.float32)


def np_tucker(dims, core_dims, rng, noise_std=0.0):
    """X = G x_1 U_1 x_2 U_2 x_3 U_3 (+ noise), G ~ U(-1, 1), U_i Haar."""
    g = rng.uniform(-1.0, 1.0, size=core_dims)
    x = g
    for mode, (i_dim, j_dim) in enumerate(zip(dims, core_dims)):
        u = np_haar(i_dim, j_dim, rng)
        x = np.moveaxis(np.tensordot(u, x, axes=([1], [mode])), 0, mode)
    if noise_std:
        x = x + noise_std * rng.standard_normal(dims)
    return np.ascontiguousarray(x, dtype=np.float32)


# --------------------------------------------------------------------------- accuracy suites
# Singular-value sequences and matrices of the paper's accuracy experiments
# (Sec. 3.3: Type 1 / Type 2; Sec. 5.1.1: A_linear, A_exp, A_Poly, A_Cauchy).
# The paper forms the prescribed-spectrum matrices with LAPACK slatms; here
# they are U diag(s) V^T with Haar U, V (the same law for the spectrum).

def sv_linear(n, p, s_p):
    """s_i = max(1 - alpha_l i, s_p), alpha_l = (1 - s_p) / p, i = 0 .. n-1."""
    i = np.arange(n, dtype=np.float64)
    return np.maximum(1.0 - (1.0 - s_p) / p * i, s_p)


def sv_exp(n, p, s_p):
    """s_i = 2^(-alpha_e i), alpha_e = log2(1 / s_p) / p, i = 0 .. n-1."""
    i = np.arange(n, dtype=np.float64)
    return 2.0 ** (-(np.log2(1.0 / s_p) / p) * i)


def sv_poly(n, r, alpha, phi):
    """Type 2 spectrum: phi (r times), then 2^-alpha, 3^-alpha, ..., (n - r + 1)^-alpha."""
    tail = np.arange(2, n - r + 2, dtype=np.float64) ** (-alpha)
    return np.concatenate([np.full(r, float(phi)), tail])


def np_type1(n, r, xi, rng):
    """Type 1: A = diag(I_r, 0) + (xi / n) G G^T with G an n x n Gaussian
    matrix (the noise scale xi / eps with eps read as n), FP32."""
    g = rng.standard_normal((n, n))
    a = (xi / n) * (g @ g.T)
    a[np.arange(r), np.arange(r)] += 1.0
    return a.astype(np.float32)


def np_cauchy(n, rng, gamma=1e-3, width=1e-3):
    """A_ij = 1 / (|x_i - y_j| + gamma) with x, y ~ U(-width, width), FP32
    (the paper's A_Cauchy with its |x_i - y_i| read as |x_i - y_j|)."""
    x = rng.uniform(-width, width, n)
    y = rng.uniform(-width, width, n)
    return (1.0 / (np.abs(x[:, None] - y[None, :]) + gamma)).astype(np.float32)


def torch_sv_matrix(n, s, seed, device):
    """FP32 n x n matrix U diag(s) V^T with Haar U, V, drawn on ``device``."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    sig = torch.as_tensor(np.asarray(s, np.float64), device=device)
    u = torch_haar(n, n, gen, device)
    v = torch_haar(n, n, gen, device)
    return ((u * sig[None, :]) @ v.T).to(torch.float32)


def batched_problem_list(count, seed, lo=512, hi=8192, kmin=16, kmax=128):
    """Shapes of the batched-RSVD workload: m, n log-uniform in [lo, hi],
    planted rank k ~ U{kmin..kmax}, width r = k + max(10, ceil(k/4))."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        m = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        n = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        k = int(rng.integers(kmin, kmax + 1))
        out.append((m, n, k, k + max(10, -(-k // 4))))
    return out


# --------------------------------------------------------------------------- torch
def torch_haar(n, k, gen, device):
    import torch
    g = torch.randn(n, k, generator=gen, device=device, dtype=torch.float64)
    q, r = torch.linalg.qr(g, mode="reduced")
    return q * torch.sign(torch.diagonal(r))[None, :]


def torch_planted(m, n, sigma, seed, device, noise_std=0.0):
    """FP32 A = U diag(sigma) V^T (+ noise) drawn and formed on ``device``."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    sig = torch.as_tensor(np.asarray(sigma, np.float64), device=device)
    k = sig.numel()
    u = torch_haar(m, k, gen, device)
    v = torch_haar(n, k, gen, device)
    a = torch.empty(m, n, device=device, dtype=torch.float32)
    rows = max(1, (1 << 28) // max(n, 1))      # form A in row blocks of <= 2 GiB FP64
    us = u * sig[None, :]
    vt = v.t().contiguous()
    for r0 in range(0, m, rows):
        blk = us[r0:r0 + rows] @ vt
        if noise_std:
            blk += noise_std * torch.randn(blk.shape, generator=gen, device=device,
                                           dtype=torch.float64)
        a[r0:r0 + rows] = blk.to(torch.float32)
        del blk
    del u, v, us, vt
    return a


def torch_rsvd_workload(device, m=32768, n=32768, k=512, noise_std=1e-4, seed=103):
    """The full randomized-SVD workload: FP32 A = U diag(sigma) V^T + E with
    planted rank k, sigma_i = 10^(-(i-1)/(k-1)), Haar U, V and E ~ N(0,
    noise_std^2), formed in FP64 row blocks on ``device``.  Returns (A,
    sigma) with sigma the planted values (FP64)."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    sig = torch.tensor(10.0 ** (-np.arange(k) / (k - 1)), device=device, dtype=torch.float64)
    u = torch_haar(m, k, gen, device)
    v = torch_haar(n, k, gen, device)
    a = torch.empty((m, n), dtype=torch.float32, device=device)
    for r0 in range(0, m, 4096):
        blk = (u[r0:r0 + 4096] * sig) @ v.T
        blk += torch.randn(blk.shape, generator=gen, device=device, dtype=torch.float64) * noise_std
        a[r0:r0 + 4096] = blk.float()
        del blk
    del u, v
    return a, sig

