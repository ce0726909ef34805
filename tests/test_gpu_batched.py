"""Grouped projections and batched randomized SVD (the batching pattern for
many problems of different shapes) against the FP64 oracle on the same
inputs and the same Omega_j (stream j, bit-identical on both sides)."""
import math

import numpy as np
import pytest

import synth
from gpu_helpers import announce, dev, host, rp
from oracle import omega, project, rsvd as orsvd

pytestmark = pytest.mark.gpu

U32, U16 = 2.0 ** -24, 2.0 ** -11


def test_project_grouped_elementwise_bound():
    """Mixed widths (r <= 128 and r > 128), shapes off the 16-byte path (odd
    n) and an empty problem in one call; every Y within the elementwise bound
    of the split product (gamma_{n+2}(u32) + u16^2) |A| |Omega|."""
    shapes = [(300, 4096, 200), (1000, 2048, 64), (65, 777, 17), (512, 8192, 256), (128, 128, 130),
              (2000, 64, 40), (0, 64, 8)]
    announce(f"grouped projections {shapes}")
    rng = np.random.default_rng(3)
    mats = [rng.standard_normal((m, n)).astype(np.float32) for m, n, _ in shapes]
    probs = [(dev(a), r, 9, j) for j, (a, (_, _, r)) in enumerate(zip(mats, shapes))]
    ys = rp().rp_project_grouped(probs)
    assert rp().rp_get_device_status(clear=True) == rp().RP_OK
    for j, (a, (m, n, r)) in enumerate(zip(mats, shapes)):
        if m == 0:
            continue
        om = omega.omega_f16(9, j, n, r)
        ref = project.project_f64(a, om)
        bound = (project.gamma(n + 2, U32) + U16 * U16) * project.abs_product(a, om)
        y = host(ys[j]).astype(np.float64)
        assert np.all(np.abs(y - ref) <= bound), (j, m, n, r)


def test_project_grouped_general_matches_single():
    """Problems off the 16-byte path go out in grouped launches of the general
    kernel (odd and 2 mod 4 row lengths, an unaligned strided view, a caller
    pre-scale 2^s, both column widths): every Y bit-identical to the same
    problem's single call (same tile, same arithmetic) and, for s = 0, within
    the elementwise bound of the split product."""
    rng = np.random.default_rng(21)
    big = rng.standard_normal((700, 1301)).astype(np.float32)
    mats = [big[:, 3:1003], rng.standard_normal((513, 999)).astype(np.float32),
            rng.standard_normal((1500, 333)).astype(np.float32), rng.standard_normal((257, 2050)).astype(np.float32),
            rng.standard_normal((300, 512)).astype(np.float32)]
    rs, exps = [150, 64, 300, 17, 100], [0, 0, 0, 0, 5]
    announce(f"grouped general-kernel projections {[a.shape for a in mats]} r {rs} s {exps}")
    dbig = dev(big)
    dmats = [dbig[:, 3:1003]] + [dev(a) for a in mats[1:]]
    probs = [(a, r, 4, j, s) for j, (a, r, s) in enumerate(zip(dmats, rs, exps))]
    ys = rp().rp_project_grouped(probs)
    assert rp().rp_get_device_status(clear=True) == rp().RP_OK
    for j, (a, da, r, s) in enumerate(zip(mats, dmats, rs, exps)):
        one = host(rp().rp_project(da, r, seed=4, stream_id=j, a_scale_exp=s))
        y = host(ys[j])
        assert np.array_equal(y, one), j
        if s == 0:
            n = a.shape[1]
            om = omega.omega_f16(4, j, n, r)
            ref = project.project_f64(a.astype(np.float64), om)
            bound = (project.gamma(n + 2, U32) + U16 * U16) * project.abs_product(a, om)
            assert np.all(np.abs(y.astype(np.float64) - ref) <= bound), j


def _planted_batch(count, seed, lo, hi, kmin, kmax):
    """m, n log-uniform in [lo, hi], planted rank k, sigma_i =
    10^(-3 (i-1)/(k-1)), Haar factors, noiseless; p = k + max(10, ceil(k/4))."""
    rng = np.random.default_rng(seed)
    out = []
    for (m, n, k, p) in synth.batched_problem_list(count, seed, lo, hi, kmin, kmax):
        sig = 10.0 ** (-3.0 * np.arange(k) / (k - 1))
        out.append((synth.np_planted(m, n, sig, rng), k, p - k, sig))
    return out


@pytest.mark.parametrize("omega_type", ["f16", "f32"])
def test_rsvd_batched_matches_oracle(omega_type):
    batch = _planted_batch(10, 55, 64, 700, 4, 24)
    announce(f"rsvd_batched {omega_type} shapes {[a.shape for a, _, _, _ in batch]}")
    mats = [dev(a) for a, _, _, _ in batch]
    ks = [k for _, k, _, _ in batch]
    ss = [s for _, _, s, _ in batch]
    outs = rp().rsvd_batched(mats, ks, ss, 0, 13, omega_type)
    assert rp().rp_get_device_status(clear=True) == rp().RP_OK
    gen = omega.omega_f32 if omega_type == "f32" else omega.omega_f16
    first = []
    for j, ((a, k, s, sig), (u, sv, vt)) in enumerate(zip(batch, outs)):
        sv = host(sv)
        first.append(sv.copy())
        _, sv_o, _ = orsvd.rsvd(a.astype(np.float64), gen(13, j, a.shape[1], k + s), k, 0)
        assert np.abs(sv - sv_o).max() <= 1e-5 * sv_o[0], j
        assert np.abs(sv - sig).max() <= 1e-5 * sig[0], j        # exact recovery of the planted spectrum
        u, vt = host(u).astype(np.float64), host(vt).astype(np.float64)
        rec = (u * sv) @ vt
        assert np.linalg.norm(rec - a) <= 1e-5 * np.linalg.norm(a), j
    # a second call with the same tensors replays the captured graph: same bits
    again = rp().rsvd_batched(mats, ks, ss, 0, 13, omega_type, outputs=outs)
    for j, (u, sv, vt) in enumerate(again):
        assert np.array_equal(host(sv), first[j])
    # the graph reads A afresh: doubling every A doubles every singular value
    # (up to rounding: a power-of-two scaling is exact everywhere except in
    # the FP16 split of elements whose hi part is subnormal, so the change is
    # bounded against sigma_1, not against each sigma_i)
    for t in mats:
        t.mul_(2.0)
    rp().rsvd_batched(mats, ks, ss, 0, 13, omega_type, outputs=outs)
    for j, (u, sv, vt) in enumerate(outs):
        assert np.abs(host(sv) - 2.0 * first[j]).max() <= 1e-6 * 2.0 * first[j][0], j


@pytest.mark.parametrize("kind", ["sparse3", "vsparse"])
def test_rsvd_batched_sparse_omega_matches_oracle(kind):
    """Batched RSVD with a sparse Omega_j (one grouped generation launch in
    the graph): planted rank-k matrices plus N(0, 1e-6^2) noise (with Omega
    in {-1, 0, 1} and FP16-valued split parts the projection's sums are
    exact, so a noiseless rank-k A gives an exactly rank-k Y and a singular
    CholeskyQR2 Gram); the singular values of the FP64 oracle's RSVD on the
    same A and Omega_j."""
    rng = np.random.default_rng(56)
    batch = []
    for (m, n, k, p) in synth.batched_problem_list(8, 57, 64, 600, 4, 20):
        sig = 10.0 ** (-3.0 * np.arange(k) / (k - 1))
        batch.append((synth.np_planted(m, n, sig, rng, noise_std=1e-6), k, p - k))
    announce(f"rsvd_batched {kind} shapes {[a.shape for a, _, _ in batch]}")
    outs = rp().rsvd_batched([dev(a) for a, _, _ in batch], [k for _, k, _ in batch], [s for _, _, s in batch], 0,
                             19, kind)
    assert rp().rp_get_device_status(clear=True) == rp().RP_OK
    for j, ((a, k, s), (_, sv, _)) in enumerate(zip(batch, outs)):
        _, sv_o, _ = orsvd.rsvd(a.astype(np.float64), omega.omega_sparse(19, j, a.shape[1], k + s, kind), k, 0)
        assert np.abs(host(sv) - sv_o).max() <= 1e-5 * sv_o[0], j


def test_rsvd_batched_power_iteration_and_errors():
    batch = _planted_batch(4, 77, 80, 300, 5, 12)
    announce("rsvd_batched q=1")
    mats = [dev(a) for a, _, _, _ in batch]
    outs = rp().rsvd_batched(mats, [k for _, k, _, _ in batch], [s for _, _, s, _ in batch], 1, 3, "f16")
    assert rp().rp_get_device_status(clear=True) == rp().RP_OK
    for j, ((a, k, s, sig), (_, sv, _)) in enumerate(zip(batch, outs)):
        _, sv_o, _ = orsvd.rsvd(a.astype(np.float64), omega.omega_f16(3, j, a.shape[1], k + s), k, 1)
        assert np.abs(host(sv) - sv_o).max() <= 1e-5 * sv_o[0], j
    assert rp().rsvd_batched([], [], [], 0, 0, "f16") == []
    with pytest.raises(rp().RpError):
        rp().rsvd_batched([dev(np.ones((10, 10), np.float32))], [8], [8], 0, 0, "f16")   # p > min(m, n)


def test_rsvd_batched_full_size_planted():
    """256 problems, m, n log-uniform in [512, 8192], planted rank k in
    [16, 128] with sigma_i = 10^(-3 (i-1)/(k-1)), noiseless, FP16 Omega_j:
    every singular value recovered (a property that holds at any size)."""
    import torch
    shapes = synth.batched_problem_list(256, 105, 512, 8192, 16, 128)
    announce(f"rsvd_batched 256 problems, total A {sum(m * n for m, n, _, _ in shapes) * 4 / 1e9:.2f} GB")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(105)
    mats, sigs = [], []
    for m, n, k, p in shapes:
        sig = torch.tensor(10.0 ** (-3.0 * np.arange(k) / (k - 1)), device="cuda", dtype=torch.float64)
        u = synth.torch_haar(m, k, gen, "cuda")
        v = synth.torch_haar(n, k, gen, "cuda")
        mats.append(((u * sig) @ v.T).float().contiguous())
        sigs.append(sig.cpu().numpy())
    ks = [k for _, _, k, _ in shapes]
    ss = [p - k for _, _, k, p in shapes]
    outs = rp().rsvd_batched(mats, ks, ss, 0, 205, "f16")
    assert rp().rp_get_device_status(clear=True) == rp().RP_OK
    worst = max(float(np.abs(host(sv) - sig).max()) for (_, sv, _), sig in zip(outs, sigs))
    print(f"max |sigma - planted| over 256 problems: {worst:.3e}")
    assert worst <= 1e-5


def test_rsvd_batched_e4m3_omega():
    """The e4m3 Omega variant (power-of-two scale per column): same oracle
    comparison with the e4m3 values; the planted spectrum is still recovered
    exactly, and the error of a noisy problem is reported beside FP16's."""
    batch = _planted_batch(6, 91, 100, 600, 6, 20)
    announce("rsvd_batched e4m3")
    mats = [dev(a) for a, _, _, _ in batch]
    ks = [k for _, k, _, _ in batch]
    ss = [s for _, _, s, _ in batch]
    outs = rp().rsvd_batched(mats, ks, ss, 0, 31, "e4m3")
    assert rp().rp_get_device_status(clear=True) == rp().RP_OK
    for j, ((a, k, s, sig), (u, sv, vt)) in enumerate(zip(batch, outs)):
        _, _, val = omega.omega_e4m3(31, j, a.shape[1], k + s)
        _, sv_o, _ = orsvd.rsvd(a.astype(np.float64), val, k, 0)
        assert np.abs(host(sv) - sv_o).max() <= 1e-5 * sv_o[0], j
        assert np.abs(host(sv) - sig).max() <= 1e-5 * sig[0], j
    # noisy: rank-k approximation error with e4m3 vs FP16 Omega (both near the optimum)
    rng = np.random.default_rng(5)
    sig = 10.0 ** (-3.0 * np.arange(30) / 29)
    a = synth.np_planted(400, 500, sig, rng, noise_std=1e-4)
    errs = {}
    for ot in ("f16", "e4m3"):
        (u, sv, vt), = rp().rsvd_batched([dev(a)], [20], [10], 0, 2, ot)
        rec = (host(u).astype(np.float64) * host(sv)) @ host(vt).astype(np.float64)
        errs[ot] = np.linalg.norm(rec - a) / np.linalg.norm(a)
    opt = np.sqrt(np.sum(np.linalg.svd(a.astype(np.float64), compute_uv=False)[20:] ** 2)) / np.linalg.norm(a)
    print(f"rank-20 relative error: f16 {errs['f16']:.4e}  e4m3 {errs['e4m3']:.4e}  optimum {opt:.4e}")
    assert errs["e4m3"] <= 1.5 * errs["f16"] and errs["f16"] <= 3.0 * opt


def test_project_grouped_e4m3():
    """Grouped projections with the e4m3 Omega: every Y within the
    elementwise bound of the product with Omega8 / s_j (exact in FP16)."""
    shapes = [(256, 2048, 96), (100, 1000, 160), (513, 640, 33)]
    announce(f"grouped e4m3 {shapes}")
    rng = np.random.default_rng(4)
    mats = [rng.standard_normal((m, n)).astype(np.float32) for m, n, _ in shapes]
    ys = rp().rp_project_grouped([(dev(a), r, 6, j) for j, (a, (_, _, r)) in enumerate(zip(mats, shapes))], "e4m3")
    assert rp().rp_get_device_status(clear=True) == rp().RP_OK
    for j, (a, (m, n, r)) in enumerate(zip(mats, shapes)):
        _, _, val = omega.omega_e4m3(6, j, n, r)
        ref = a.astype(np.float64) @ val
        bound = (project.gamma(n + 2, U32) + U16 * U16) * project.abs_product(a, val)
        assert np.all(np.abs(host(ys[j]).astype(np.float64) - ref) <= bound), j


def test_rsvd_batched_wide_and_breakdown():
    """A set whose widest problem (p = 210) exceeds the one-workgroup
    Cholesky of the grouped stages takes the per-problem stages; the result
    is the same oracle comparison.  A zero matrix in a grouped set reports
    the Cholesky breakdown (RP_ERR_NOT_SPD) from the grouped kernel."""
    rng = np.random.default_rng(21)
    sig_a = 10.0 ** (-3.0 * np.arange(200) / 199)
    sig_b = 10.0 ** (-3.0 * np.arange(12) / 11)
    a = synth.np_planted(600, 500, sig_a, rng)
    b = synth.np_planted(300, 260, sig_b, rng)
    announce("rsvd_batched p=210 (per-problem stages)")
    outs = rp().rsvd_batched([dev(a), dev(b)], [200, 12], [10, 10], 0, 19, "f16")
    assert rp().rp_get_device_status(clear=True) == rp().RP_OK
    for j, (x, k, s) in enumerate(((a, 200, 10), (b, 12, 10))):
        _, sv_o, _ = orsvd.rsvd(x.astype(np.float64), omega.omega_f16(19, j, x.shape[1], k + s), k, 0)
        assert np.abs(host(outs[j][1]) - sv_o).max() <= 1e-5 * sv_o[0], j
    announce("rsvd_batched with a zero matrix (grouped stages)")
    rp().rsvd_batched([dev(b), dev(np.zeros((300, 260), np.float32))], [12, 12], [10, 10], 0, 19, "f16")
    assert rp().rp_get_device_status(clear=True) == rp().RP_ERR_NOT_SPD


def test_tuning_cache_persists(tmp_path, monkeypatch):
    """The autotuner's choice survives the context: saved, loaded into a
    fresh context (same plan, so bit-identical results), picked up through
    RPMI_TUNING_FILE and rewritten there after a new tuning; a file that does
    not parse is an error."""
    rng = np.random.default_rng(8)
    shapes = [(300, 256), (200, 128), (520, 384), (96, 64)]
    announce(f"tuning cache with rsvd_batched {shapes}")
    mats = [dev(rng.standard_normal(s).astype(np.float32)) for s in shapes]
    ks, ss = [8, 6, 10, 4], [8, 8, 8, 8]
    c1 = rp().Context(0)
    assert rp().rp_tuning_count(ctx=c1) == 0
    out1 = rp().rsvd_batched(mats, ks, ss, 0, 5, "f16", ctx=c1)
    n1 = rp().rp_tuning_count(ctx=c1)
    assert n1 >= 1
    path = tmp_path / "tune.txt"
    rp().rp_tuning_save(str(path), ctx=c1)
    assert len(path.read_text().split("\n")) - 1 == n1
    c2 = rp().Context(0)
    rp().rp_tuning_load(str(path), ctx=c2)
    assert rp().rp_tuning_count(ctx=c2) == n1
    out2 = rp().rsvd_batched(mats, ks, ss, 0, 5, "f16", ctx=c2)
    assert rp().rp_tuning_count(ctx=c2) == n1          # nothing new to tune
    for (u1, s1, v1), (u2, s2, v2) in zip(out1, out2):
        assert np.array_equal(host(s1), host(s2))
        assert np.array_equal(host(u1), host(u2))
    monkeypatch.setenv("RPMI_TUNING_FILE", str(path))
    c3 = rp().Context(0)
    assert rp().rp_tuning_count(ctx=c3) == n1
    rp().rsvd_batched(mats[:2], ks[:2], ss[:2], 0, 5, "f16", ctx=c3)   # a new signature
    assert rp().rp_tuning_count(ctx=c3) == n1 + 1
    assert len(path.read_text().split("\n")) - 1 == n1 + 1
    bad = tmp_path / "bad.txt"
    bad.write_text("not a tuning line\n")
    with pytest.raises(rp().RpError):
        rp().rp_tuning_load(str(bad), ctx=c2)
    with pytest.raises(rp().RpError):
        rp().rp_tuning_load(str(tmp_path / "missing.txt"), ctx=c2)
    for c in (c1, c2, c3):
        c.close()


@pytest.mark.parametrize("form", ["0", "1"])
def test_grouped_narrow_kernel_forms(form, monkeypatch):
    """Both kernel forms of the narrow (r <= 128) 16-byte-path problems
    (RPMI_GROUP_FORM fixes the one the autotuner would pick): grouped
    projections within the split product's elementwise bound, and a batched
    RSVD that recovers its planted spectra like the oracle."""
    monkeypatch.setenv("RPMI_GROUP_FORM", form)
    c = rp().Context(0)
    shapes = [(300, 4096, 100), (1000, 2048, 64), (64, 512, 8), (257, 1024, 128), (700, 2048, 200)]
    announce(f"grouped projections, narrow form {form}: {shapes}")
    rng = np.random.default_rng(12)
    mats = [rng.standard_normal((m, n)).astype(np.float32) for m, n, _ in shapes]
    ys = rp().rp_project_grouped([(dev(a), r, 6, j) for j, (a, (_, _, r)) in enumerate(zip(mats, shapes))], ctx=c)
    assert rp().rp_get_device_status(clear=True, ctx=c) == rp().RP_OK
    for j, (a, (m, n, r)) in enumerate(zip(mats, shapes)):
        om = omega.omega_f16(6, j, n, r)
        ref = project.project_f64(a, om)
        bound = (project.gamma(n + 2, U32) + U16 * U16) * project.abs_product(a, om)
        assert np.all(np.abs(host(ys[j]).astype(np.float64) - ref) <= bound), (form, j)
    batch = [b for b in _planted_batch(8, 66, 64, 600, 4, 20) if b[0].shape[1] % 4 == 0] or \
        _planted_batch(3, 67, 64, 64, 4, 8)
    outs = rp().rsvd_batched([dev(a) for a, _, _, _ in batch], [k for _, k, _, _ in batch],
                             [s for _, _, s, _ in batch], 0, 21, "f16", ctx=c)
    assert rp().rp_get_device_status(clear=True, ctx=c) == rp().RP_OK
    for j, ((a, k, s, sig), (_, sv, _)) in enumerate(zip(batch, outs)):
        _, sv_o, _ = orsvd.rsvd(a.astype(np.float64), omega.omega_f16(21, j, a.shape[1], k + s), k, 0)
        assert np.abs(host(sv) - sv_o).max() <= 1e-5 * sv_o[0], (form, j)
    c.close()


@pytest.mark.parametrize("graph_sweeps", ["0", "2"])
def test_batched_eager_jacobi_sweeps_match_graph(graph_sweeps, monkeypatch):
    """Jacobi sweeps beyond the first graph's run eagerly while a problem is
    open: with 0 or 2 sweeps in the graph (RPMI_BATCHED_GRAPH_SWEEPS) the
    same sweeps run in the same order as with the default count, so S, U and
    V^T are bit-identical, on the first call and on a replay.  Gaussian
    inputs of widths 20 to 48 need more sweeps than either count."""
    rng = np.random.default_rng(31)
    shapes = [(300, 200), (260, 180), (150, 120)]
    ks, ss = [40, 24, 12], [8, 8, 8]
    announce(f"eager Jacobi sweeps after {graph_sweeps} captured: rsvd_batched {shapes}")
    mats = [dev(rng.standard_normal(s).astype(np.float32)) for s in shapes]
    c1 = rp().Context(0)
    ref = rp().rsvd_batched(mats, ks, ss, 0, 9, "f16", ctx=c1)
    monkeypatch.setenv("RPMI_BATCHED_GRAPH_SWEEPS", graph_sweeps)
    c2 = rp().Context(0)
    for _ in range(2):   # capture, then replay
        out = rp().rsvd_batched(mats, ks, ss, 0, 9, "f16", ctx=c2)
        for (u1, s1, v1), (u2, s2, v2) in zip(ref, out):
            assert np.array_equal(host(s1), host(s2))
            assert np.array_equal(host(u1), host(u2))
            assert np.array_equal(host(v1), host(v2))
    assert rp().status_string(rp().rp_get_device_status(clear=True, ctx=c2)) == "RP_OK"
    for c in (c1, c2):
        c.close()
