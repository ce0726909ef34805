"""Pins for the RP-HOSVD oracle (Algorithm 2): unfolding and mode products
against explicit index loops, and exact recovery of a planted Tucker tensor
when J_i is at least the planted rank."""
import itertools

import numpy as np

import synth
from oracle import hosvd, omega


def test_unfold_against_loops():
    x = np.arange(2 * 3 * 4, dtype=np.float64).reshape(2, 3, 4)
    dims = x.shape
    for mode in range(3):
        u = hosvd.unfold(x, mode)
        others = [d for d in range(3) if d != mode]
        for idx in itertools.product(*[range(d) for d in dims]):
            col = 0
            for d in others:
                col = col * dims[d] + idx[d]
            assert u[idx[mode], col] == x[idx]


def test_mode_product_against_loops():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 4, 5))
    m = rng.standard_normal((2, 4))
    y = hosvd.mode_product(x, m, 1)
    assert y.shape == (3, 2, 5)
    for i, j, k in itertools.product(range(3), range(2), range(5)):
        assert np.isclose(y[i, j, k], sum(x[i, t, k] * m[j, t] for t in range(4)))


def test_planted_tucker_recovered():
    rng = np.random.default_rng(1)
    dims, core = (24, 20, 16), (4, 5, 3)
    x = synth.np_tucker(dims, core, rng).astype(np.float64)
    ranks = (8, 8, 8)
    oms = [omega.omega_f32(7, i, int(np.prod(dims)) // dims[i], ranks[i]) for i in range(3)]
    g, qs = hosvd.rp_hosvd(x, oms)
    assert g.shape == ranks
    xr = hosvd.reconstruct(g, qs)
    assert np.linalg.norm(xr - x) <= 1e-6 * np.linalg.norm(x)   # FP32 input storage
