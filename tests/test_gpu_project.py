"""Parity of Y = A Omega (split-FP16 and FP32 paths) with the FP64 oracle.

Exact cases: identity / e_i rows return Omega bit for bit; an integer A with a
{-1, 0, 1} Omega (Sec. 3.4) gives the exact integer product.  Random cases:
elementwise error within the dot-product bound (n u32 + u16^2) |A||Omega| for
sizes spanning several tiles with ragged edges, and the acceptance criterion
rel-F err(split) <= 2 rel-F err(FP32 kernel) against the FP64 oracle on the
same FP16 Omega.  Layout cases: strided unfolding descriptors, caller-supplied
Omega, empty sizes, the FP16 range flag and NaN propagation."""
import numpy as np
import pytest

from gpu_helpers import announce, dev, host, rp
from oracle import omega, project

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
U16 = 2.0 ** -11


def _run(a, r, seed, algo, stream=0, omega_type="f16"):
    y = rp().rp_project(dev(a), r, seed=seed, stream_id=stream, algo=algo, omega_type=omega_type)
    return host(y)


@pytest.mark.parametrize("algo", ["split_f16", "f32"])
@pytest.mark.parametrize("n,r", [(64, 16), (100, 7), (1000, 300)])
def test_identity_rows_return_omega(algo, n, r):
    announce(f"identity algo={algo} n={n} r={r}")
    rows = np.unique(np.r_[0, n - 1, np.random.default_rng(n).integers(0, n, 50)])
    a = np.eye(n, dtype=np.float32)[rows]
    y = _run(a, r, 3, algo)
    ref = omega.omega_f16(3, 0, n, r).astype(np.float32)[rows]
    assert np.array_equal(y.view(np.uint32), ref.view(np.uint32))


def test_identity_f32_omega_exact():
    a = np.eye(130, dtype=np.float32)
    y = _run(a, 70, 9, "f32", omega_type="f32")
    assert np.array_equal(y.view(np.uint32), omega.omega_f32(9, 0, 130, 70).view(np.uint32))


@pytest.mark.parametrize("algo", ["split_f16", "f32"])
def test_integer_times_sign_matrix_exact(algo):
    announce(f"integer x sign algo={algo}")
    rng = np.random.default_rng(8)
    m, n, r = 200, 777, 40
    a = rng.integers(-8, 9, (m, n)).astype(np.float32)
    om = rng.choice([-1.0, 0.0, 1.0], size=(n, r), p=[1 / 6, 2 / 3, 1 / 6]).astype(np.float16)
    omt = dev(om.view(np.int16))
    y = rp().rp_project(dev(a), r, omega=omt if algo == "split_f16" else omt, algo=algo)
    exact = a.astype(np.int64) @ om.astype(np.int64)
    assert np.array_equal(host(y), exact.astype(np.float32))


SHAPES = [(1, 1, 1), (5, 3, 2), (64, 64, 16), (65, 65, 17), (130, 200, 256), (257, 1000, 300),
          (300, 4099, 64), (1000, 2048, 257)]


@pytest.mark.parametrize("m,n,r", SHAPES)
def test_random_elementwise_bound(m, n, r):
    announce(f"random elementwise m={m} n={n} r={r}")
    rng = np.random.default_rng(m + 7 * n + 13 * r)
    a = rng.standard_normal((m, n)).astype(np.float32)
    om16 = omega.omega_f16(11, 0, n, r)
    ref = project.project_f64(a, om16)
    scale = project.abs_product(a, om16)
    for algo in ("split_f16", "f32"):
        y = _run(a, r, 11, algo).astype(np.float64)
        bound = (project.gamma(n + 2, U32) + U16 * U16) * scale
        assert np.all(np.abs(y - ref) <= bound), algo


@pytest.mark.parametrize("dist", ["normal", "uniform"])
def test_split_error_within_twice_f32(dist):
    """The acceptance criterion at a size the oracle does in full (Sec. 4.4.1
    uses N(0,1) and U(0,1) inputs)."""
    announce(f"criterion dist={dist}")
    rng = np.random.default_rng(21)
    m, n, r = 2048, 4096, 256
    a = (rng.standard_normal((m, n)) if dist == "normal" else rng.uniform(0, 1, (m, n))).astype(np.float32)
    ref = project.project_f64(a, omega.omega_f16(5, 0, n, r))
    e_split = project.rel_frobenius(_run(a, r, 5, "split_f16"), ref)
    e_f32 = project.rel_frobenius(_run(a, r, 5, "f32"), ref)
    print(f"rel err split {e_split:.3e}  f32 {e_f32:.3e}")
    assert e_split <= 2.0 * e_f32
    assert e_split < 1e-6


def test_strided_unfolding_descriptor():
    """Mode-2 unfolding of a C-order I1 x I2 x I3 tensor: row i2, column
    (i1, i3): runs of I3 contiguous elements, I2*I3 apart."""
    announce("strided mode-2 unfolding")
    import torch
    from oracle import hosvd
    I1, I2, I3, r = 3, 50, 128, 24
    x = np.random.default_rng(2).standard_normal((I1, I2, I3)).astype(np.float32)
    xt = dev(x)
    d = rp().rp_desc(xt.data_ptr(), I2, I1 * I3, I3, I3, 1, I2 * I3)
    for algo in ("split_f16", "f32"):
        y = host(rp().rp_project(xt, r, seed=4, stream_id=1, desc=d, algo=algo))
        ref = project.project_f64(hosvd.unfold(x, 1), omega.omega_f16(4, 1, I1 * I3, r))
        assert project.rel_frobenius(y, ref) < 1e-6, algo


def test_supplied_omega_matches_generated():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((150, 333)).astype(np.float32)
    om = rp().rp_omega_generate(333, 50, 77, 0, "f16")
    for algo in ("split_f16", "f32"):
        y1 = host(rp().rp_project(dev(a), 50, seed=77, algo=algo))
        y2 = host(rp().rp_project(dev(a), 50, omega=om, algo=algo))
        assert np.array_equal(y1, y2), algo


def test_empty_sizes():
    import torch
    a = torch.zeros((4, 0), dtype=torch.float32, device="cuda")
    y = torch.full((4, 3), 5.0, device="cuda")
    rp().rp_project(a, 3, y=y)
    torch.cuda.synchronize()
    assert bool((y == 0).all())
    a = torch.zeros((0, 8), dtype=torch.float32, device="cuda")
    assert rp().rp_project(a, 3).shape == (0, 3)
    a = torch.ones((4, 8), dtype=torch.float32, device="cuda")
    assert rp().rp_project(a, 0).shape == (4, 0)


def test_range_flag_and_nan():
    """An element outside the FP16 range of the split (Sec. 4.2) sets
    RP_ERR_RANGE; so does a non-finite element (its split is non-finite too).
    NaN propagates to its own row only."""
    m = rp()
    m.rp_get_device_status(clear=True)
    a = np.ones((70, 90), np.float32)
    a[3, 4] = 65519.0                      # largest value whose RN16 is finite
    m.rp_project(dev(a), 20)
    assert m.rp_get_device_status(clear=True) == m.RP_OK
    a[33, 44] = 65520.0
    m.rp_project(dev(a), 20)
    assert m.rp_get_device_status(clear=True) == m.RP_ERR_RANGE
    a = np.ones((70, 90), np.float32)
    a[33, 44] = -1e30
    m.rp_project(dev(a), 20)
    assert m.rp_get_device_status(clear=True) == m.RP_ERR_RANGE
    a = np.ones((70, 90), np.float32)
    a[5, 6] = np.nan
    y = host(m.rp_project(dev(a), 20))
    assert np.all(np.isnan(y[5])) and np.all(np.isfinite(np.delete(y, 5, axis=0)))
    assert m.rp_get_device_status(clear=True) == m.RP_ERR_RANGE
    # the FP32 path has no FP16 range limit
    a = np.ones((70, 90), np.float32)
    a[33, 44] = 1e30
    y = host(m.rp_project(dev(a), 20, algo="f32"))
    assert np.all(np.isfinite(y))
    assert m.rp_get_device_status(clear=True) == m.RP_OK


def test_invalid_arguments():
    import torch
    m = rp()
    a = torch.ones((8, 8), device="cuda")
    with pytest.raises(m.RpError) as e:
        m.rp_project(a, 4, omega_type="f32", algo="split_f16")
    assert e.value.status == m.RP_ERR_INVALID_ARG
    d = m.rp_desc(a.data_ptr(), 8, 8, 8, 8, 2, 0)
    with pytest.raises(m.RpError) as e:
        m.rp_project(a, 4, desc=d)
    assert e.value.status == m.RP_ERR_UNSUPPORTED


def test_packed_entry_points_match_rp_project():
    rng = np.random.default_rng(4)
    a = dev(rng.standard_normal((300, 700)).astype(np.float32))
    for algo in ("split_f16", "f32"):
        pk = rp().rp_omega_pack(700, 90, seed=6, stream_id=2, algo=algo)
        assert pk.numel() == rp().rp_omega_packed_size(700, 90, algo)
        y1 = host(rp().rp_project_packed(a, 90, pk, algo=algo))
        y2 = host(rp().rp_project(a, 90, seed=6, stream_id=2, algo=algo))
        assert np.array_equal(y1, y2), algo


@pytest.mark.parametrize("algo", ["split_f16", "f32"])
def test_e4m3_omega_projection(algo):
    """Generated e4m3 Omega: the projection uses Omega8 / s_j (exact in FP16),
    within the elementwise bound of the product with those values."""
    announce(f"e4m3 projection {algo}")
    rng = np.random.default_rng(12)
    m, n, r = 300, 2000, 96
    a = rng.standard_normal((m, n)).astype(np.float32)
    _, _, val = omega.omega_e4m3(17, 0, n, r)
    y = host(rp().rp_project(dev(a), r, seed=17, omega_type="e4m3", algo=algo)).astype(np.float64)
    ref = a.astype(np.float64) @ val
    bound = (project.gamma(n + 2, U32) + U16 * U16) * project.abs_product(a, val)
    assert np.all(np.abs(y - ref) <= bound)


@pytest.mark.parametrize("m,n,r", [(70, 96, 200), (512, 16384, 256)])
def test_range_on_the_fast_path(m, n, r):
    """The wide fast kernel's folded split takes |a| < 32; a row block with a
    larger element is recomputed by the two-accumulator kernel, which keeps
    the whole FP16 range: 1000 and 65519 give the exact product within the
    elementwise bound and RP_OK; 65520, -1e30 and NaN give RP_ERR_RANGE, and
    NaN stays in its own row.  Shapes on the 16-byte path, the second with a
    contraction split (partial sums reduced by the last workgroup of a tile)."""
    announce(f"range on the fast path {m}x{n}x{r}")
    lib = rp()
    lib.rp_get_device_status(clear=True)
    rng = np.random.default_rng(23)
    om = omega.omega_f16(5, 0, n, r)
    for big in (31.5, 1000.0, 65519.0):
        a = rng.standard_normal((m, n)).astype(np.float32)
        a[m // 2, n // 3] = big
        y = host(lib.rp_project(dev(a), r, seed=5)).astype(np.float64)
        assert lib.rp_get_device_status(clear=True) == lib.RP_OK, big
        ref = project.project_f64(a, om)
        bound = (project.gamma(n + 2, U32) + U16 * U16) * project.abs_product(a, om)
        assert np.all(np.abs(y - ref) <= bound), big
    for bad in (65520.0, -1e30):
        a = np.ones((m, n), np.float32)
        a[m - 1, n - 1] = bad
        lib.rp_project(dev(a), r, seed=5)
        assert lib.rp_get_device_status(clear=True) == lib.RP_ERR_RANGE, bad
    a = np.ones((m, n), np.float32)
    a[5, 6] = np.nan
    y = host(lib.rp_project(dev(a), r, seed=5))
    assert np.all(np.isnan(y[5])) and np.all(np.isfinite(np.delete(y, 5, axis=0)))
    assert lib.rp_get_device_status(clear=True) == lib.RP_ERR_RANGE
