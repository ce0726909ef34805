"""rp_project_packed_noalloc: the projection with the library's static device
scratch in place of any allocation.  Called through the C ABI on two (and
three) calls in a row, the later ones smaller, and checked against
rp_project_packed on the same packed Omega (same kernels and contraction
split, so equal bit for bit) and against the FP64 oracle within the
elementwise bound of the split path (Sec. 4.3: FP32 accumulation error plus
the 2^-22 relative split residual)."""
import numpy as np
import pytest

from gpu_helpers import announce, dev, host, rp
from oracle import omega, project

pytestmark = pytest.mark.gpu


def _case(m, n, r, seed):
    import torch
    lib = rp()
    a = np.random.default_rng(seed).standard_normal((m, n)).astype(np.float32)
    ad = dev(a)
    pk = lib.rp_omega_pack(n, r, seed=seed, algo="split_f16")
    y_ref = lib.rp_project_packed(ad, r, pk)
    y = torch.full((m, r), float("nan"), dtype=torch.float32, device="cuda")
    lib.rp_project_packed_noalloc(ad, r, pk, y)
    torch.cuda.synchronize()
    return a, host(y), host(y_ref)


@pytest.mark.parametrize("shapes", [[(1000, 4096, 256), (300, 2048, 200), (200, 1100, 80)]])
def test_noalloc_matches_project_packed(shapes):
    lib = rp()
    lib.rp_get_device_status(clear=True)
    for i, (m, n, r) in enumerate(shapes):
        announce(f"noalloc call {i}: {m}x{n}x{r}")
        a, y, y_ref = _case(m, n, r, 40 + i)
        assert np.array_equal(y.view(np.uint32), y_ref.view(np.uint32)), f"call {i} differs from rp_project_packed"
        om = omega.omega_f16(40 + i, 0, n, r)
        ref = project.project_f64(a, om)
        bound = (project.gamma(n + 2, 2.0 ** -24) + 2.0 ** -22) * project.abs_product(a, om)
        assert np.all(np.abs(y.astype(np.float64) - ref) <= bound), f"call {i} outside the error bound"
    assert lib.rp_get_device_status() == lib.RP_OK


def test_noalloc_fp32_and_empty():
    import torch
    lib = rp()
    m, n, r = 130, 260, 40
    a = np.random.default_rng(9).standard_normal((m, n)).astype(np.float32)
    pk = lib.rp_omega_pack(n, r, seed=9, algo="f32")
    y_ref = host(lib.rp_project_packed(dev(a), r, pk, algo="f32"))
    y = torch.empty((m, r), dtype=torch.float32, device="cuda")
    lib.rp_project_packed_noalloc(dev(a), r, pk, y, algo="f32")
    assert np.array_equal(host(y).view(np.uint32), y_ref.view(np.uint32))
    # n == 0 writes zeros
    z = torch.full((5, 3), 7.0, device="cuda")
    lib.rp_project_packed_noalloc(torch.empty((5, 0), device="cuda"), 3, pk, z)
    assert np.all(host(z) == 0.0)
