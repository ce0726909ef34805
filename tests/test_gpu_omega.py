"""Omega on the GPU is bit-exact with the oracle (FP16 and FP32 storage), for
ragged widths, several streams and seeds, and sampled rows of the full-size
16384 x 256 and 262144 x 80 matrices."""
import numpy as np
import pytest

from gpu_helpers import announce, bits16, host, rp
from oracle import omega

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("seed,stream,n,r", [(0, 0, 1, 1), (1, 0, 37, 5), (7, 3, 300, 64),
                                              (12345, 1, 129, 258), ((1 << 64) - 1, 2, 64, 80)])
def test_f16_bits_exact(seed, stream, n, r):
    announce(f"omega f16 seed={seed} stream={stream} n={n} r={r}")
    got = bits16(rp().rp_omega_generate(n, r, seed, stream, "f16"))
    assert np.array_equal(got, omega.omega_f16_bits(seed, stream, n, r))


@pytest.mark.parametrize("seed,stream,n,r", [(0, 0, 3, 7), (5, 2, 257, 64), (99, 0, 64, 33)])
def test_f32_bits_exact(seed, stream, n, r):
    announce(f"omega f32 seed={seed} stream={stream} n={n} r={r}")
    got = host(rp().rp_omega_generate(n, r, seed, stream, "f32"))
    ref = omega.omega_f32(seed, stream, n, r)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("n,r,stream", [(16384, 256, 0), (262144, 80, 1)])
def test_full_size_sampled_rows(n, r, stream):
    announce(f"omega full n={n} r={r}")
    got = bits16(rp().rp_omega_generate(n, r, 202, stream, "f16"))
    rows = np.sort(np.random.default_rng(n).choice(n, 96, replace=False))
    rows = np.concatenate([[0, n - 1], rows])
    ref = omega.omega_f16_bits(202, stream, 0, r, rows=rows)
    assert np.array_equal(got[rows], ref)


def test_zero_sizes():
    import torch
    out = torch.full((2, 3), 7, dtype=torch.int16, device="cuda")
    rp().rp_omega_generate(0, 3, 1, 0, "f16", out=out)
    rp().rp_omega_generate(2, 0, 1, 0, "f16", out=out)
    torch.cuda.synchronize()
    assert bool((out == 7).all())


@pytest.mark.parametrize("n,r", [(3000, 40), (1, 1), (257, 130), (0, 5)])
def test_e4m3_codes_and_scales_bit_exact(n, r):
    announce(f"e4m3 omega n={n} r={r}")
    codes, scale = rp().rp_omega_generate_e4m3(n, r, seed=21, stream_id=4)
    c_o, s_o, _ = omega.omega_e4m3(21, 4, n, r)
    assert np.array_equal(host(scale).astype(np.float64), s_o)
    assert np.array_equal(host(codes), c_o)
