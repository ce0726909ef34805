"""Pins for the FP64 projection oracle (eq:rp-vec): exact rational products on
tiny inputs, exact special cases (identity rows, integer A times a {-1,0,1}
sparse Omega, Sec. 3.4), and the split product within the split remainder."""
import numpy as np
import pytest

from oracle import omega, project, split


@pytest.mark.parametrize("m,n,r", [(1, 1, 1), (3, 5, 2), (7, 16, 5), (16, 13, 16)])
def test_f64_against_exact_rationals(m, n, r):
    rng = np.random.default_rng(m * 100 + n)
    a = rng.standard_normal((m, n)).astype(np.float32)
    om = omega.omega_f16(9, 0, n, r)
    exact = project.project_exact(a, om)
    y = project.project_f64(a, om)
    bound = project.gamma(n, 2.0 ** -53) * project.abs_product(a, om)
    for i in range(m):
        for j in range(r):
            assert abs(y[i, j] - float(exact[i][j])) <= bound[i, j] + 1e-300


def test_identity_rows_return_omega():
    om = omega.omega_f16(4, 0, 40, 24)
    a = np.eye(40, dtype=np.float32)[[0, 5, 39]]
    y = project.project_f64(a, om)
    assert np.array_equal(y, om.astype(np.float64)[[0, 5, 39]])


def test_integer_times_sparse_sign_matrix_is_exact():
    rng = np.random.default_rng(8)
    a = rng.integers(-8, 9, (12, 300)).astype(np.float32)
    om = rng.choice([-1.0, 0.0, 1.0], size=(300, 7), p=[1 / 6, 2 / 3, 1 / 6]).astype(np.float16)
    y = project.project_f64(a, om)
    exact = a.astype(np.int64) @ om.astype(np.int64)
    assert np.array_equal(y, exact.astype(np.float64))


def test_split_product_within_remainder_bound():
    rng = np.random.default_rng(10)
    a = rng.standard_normal((20, 64)).astype(np.float32)
    om = omega.omega_f16(1, 0, 64, 8)
    ys = project.split_product_f64(a, om)
    exact = project.project_exact(a, om)
    bound = (2.0 ** -22 + project.gamma(128, 2.0 ** -53)) * project.abs_product(a, om)
    for i in range(20):
        for j in range(8):
            assert abs(ys[i, j] - float(exact[i][j])) <= bound[i, j]


def test_rel_frobenius():
    y = np.ones((3, 3))
    assert project.rel_frobenius(y, y) == 0.0
    assert project.rel_frobenius(2 * y, y) == pytest.approx(1.0)
