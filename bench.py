"""Benchmark of the random projection Y = A Omega on one MI355X.

Workload (16384 x 16384 projection, r = 256): A is FP32 with singular values
sigma_i = 10^(-6 i / 16384) and Haar-distributed singular vectors (drawn on the
GPU from a fixed seed); Omega is 16384 x 256 FP16 from the counter-based
generator.  One step is the whole hot path on inputs resident in HBM: generate
Omega in fragment order, then the split-FP16 projection kernel.  The plain
FP32 kernel is timed the same way on the same A and the same FP16 Omega
(widened exactly), and both results are checked against the FP64 oracle on a
row sample in the CPU-baseline leg.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

M = N = 16384
R = 256
SEED_A = 102
SEED_OMEGA = 202
METRIC = "Y=AΩ TFLOP/s split-FP16 MFMA vs FP32 GEMM at equal error; RSVD wall s"
HBM_PEAK_GBS = 8000.0
ROOT = os.path.dirname(os.path.abspath(__file__))
# HBM traffic of the split kernel measured with rocprofv3 counters (FETCH_SIZE,
# WRITE_SIZE) and scaled by the same counters on a copy of known size; valid
# only while the kernel sources hash to the value recorded with it.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "project_split_f16_16384x16384x256_hbm_traffic.txt")
KERNEL_SOURCES = ("paper_2304_04612_amd/csrc/proj_common.h", "paper_2304_04612_amd/csrc/proj_lds.h",
                  "paper_2304_04612_amd/csrc/project_wide.hip", "paper_2304_04612_amd/csrc/rpmi_internal.h")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--cpu-rows", type=int, default=M)
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--no-rsvd", action="store_true", help="skip the 32768^2 randomized SVD")
    p.add_argument("--no-batched", action="store_true", help="skip the 256-problem batched RSVD")
    p.add_argument("--no-hosvd", action="store_true", help="skip the 512^3 RP-HOSVD")
    p.add_argument("--no-accuracy", action="store_true", help="skip the 4096^2 accuracy suites")
    p.add_argument("--a-cache", default=None,
                   help="file holding A (raw FP32, row-major); written on first use, read afterwards")
    return p.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """Counter-measured HBM bytes per launch of the split kernel, or None when
    no measurement exists for the current kernel sources."""
    try:
        fields = {}
        with open(TRAFFIC_FILE) as f:
            for line in f:
                key, sep, val = line.partition(":")
                if sep:
                    fields[key.strip()] = val.strip()
        if fields.get("kernel_source_sha256") != kernel_source_hash():
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    sys.path.insert(0, ROOT)
    import paper_2304_04612_amd as rp
    import synth

    torch.cuda.set_device(0)
    dev = "cuda:0"
    t = time.time()
    if args.a_cache and os.path.exists(args.a_cache) and os.path.getsize(args.a_cache) == 4 * M * N:
        a = torch.from_numpy(np.fromfile(args.a_cache, dtype=np.float32).reshape(M, N)).to(dev)
        log(f"A read from {args.a_cache} in {time.time() - t:.1f} s")
    else:
        sigma = synth.sigma_decade(N, 6.0, N)
        a = synth.torch_planted(M, N, sigma, SEED_A, dev)
        torch.cuda.synchronize()
        log(f"A generated in {time.time() - t:.1f} s")
        if args.a_cache:
            a.cpu().numpy().tofile(args.a_cache)

    # a copy of known size (A itself, 1 GiB read + 1 GiB written) for
    # calibrating the HBM byte counters of a profiled run; outside every timed region
    scratch = torch.empty_like(a)
    scratch.copy_(a)
    torch.cuda.synchronize()
    del scratch

    y = torch.empty((M, R), dtype=torch.float32, device=dev)
    y32 = torch.empty((M, R), dtype=torch.float32, device=dev)
    pk16 = torch.empty(rp.rp_omega_packed_size(N, R, "split_f16"), dtype=torch.uint8, device=dev)
    pk32 = torch.empty(rp.rp_omega_packed_size(N, R, "f32"), dtype=torch.uint8, device=dev)
    rp.rp_get_device_status(clear=True)

    def timed(algo, pk, out, steps, warmup):
        """Time `steps` whole steps; per-step events around the projection kernel."""
        for _ in range(warmup):
            rp.rp_omega_pack(N, R, seed=SEED_OMEGA, algo=algo, out=pk)
            rp.rp_project_packed(a, R, pk, algo=algo, y=out)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        t0 = time.perf_counter()
        for k in range(steps):
            rp.rp_omega_pack(N, R, seed=SEED_OMEGA, algo=algo, out=pk)
            ev[k][0].record()
            rp.rp_project_packed(a, R, pk, algo=algo, y=out)
            ev[k][1].record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kern = [s.elapsed_time(e) * 1e-3 for s, e in ev]
        return wall / steps, sum(kern) / len(kern), min(kern)

    step_s, kern_s, kern_min = timed("split_f16", pk16, y, args.steps, args.warmup)
    log(f"split-FP16: step {step_s * 1e3:.3f} ms, kernel avg {kern_s * 1e6:.1f} us")
    step32_s, kern32_s, _ = timed("f32", pk32, y32, max(3, args.steps // 2), 1)
    log(f"FP32: step {step32_s * 1e3:.3f} ms, kernel avg {kern32_s * 1e6:.1f} us")
    status = rp.rp_get_device_status(clear=True)

    flops = 2.0 * M * N * R
    alg_bytes = 4.0 * M * N + 2.0 * N * R + 4.0 * M * R
    value = flops / step_s / 1e12
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_s * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16",
        "dtype_note": "FP32 A split into FP16 hi + 2^-11 lo in registers; FP16 MFMA products, FP32 accumulation",
        "data": "synthetic",
        "config": {"workload": "projection Y=A*Omega, A 16384x16384 FP32 (sigma_i=10^(-6i/16384), "
                               "Haar U,V), Omega 16384x256 FP16 (Philox4x64 + exact FP16 inverse CDF)",
                   "m": M, "n": N, "r": R, "seed_A": SEED_A, "seed_omega": SEED_OMEGA},
        "roofline": {
            "kernel": "project_split_lds_single_kernel (256-column tile)",
            "bound": "hbm",
            "achieved": round(alg_bytes / kern_s / 1e9, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(alg_bytes / kern_s / 1e9 / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(),
            "kernel_avg_us": round(kern_s * 1e6, 2),
            "kernel_min_us": round(kern_min * 1e6, 2),
            "alg_bytes_per_launch": alg_bytes,
        },
        "fp32_gemm": {
            "value": round(flops / step32_s / 1e12, 2),
            "unit": "TFLOP/s",
            "ms_per_step": round(step32_s * 1e3, 4),
            "kernel_avg_us": round(kern32_s * 1e6, 2),
            "frac_of_fp32_peak": round(flops / kern32_s / 157.3e12, 4),
        },
        "speedup_vs_fp32_step": round(step32_s / step_s, 3),
        "speedup_vs_fp32_kernel": round(kern32_s / kern_s, 3),
        "device_status": rp.status_string(status),
    }

    if not args.no_cpu:
        out["cpu_baseline"], errs = cpu_leg(a, y, y32, args.cpu_rows)
        out.update(errs)
    del a, y, y32, pk16, pk32
    torch.cuda.empty_cache()
    if not args.no_rsvd:
        out["rsvd_c1"] = c1_leg(rp, synth, torch, dev)
        out["rsvd"] = rsvd_leg(rp, synth, torch, dev)
    if not args.no_batched:
        out["batched_rsvd"] = batched_leg(rp, synth, torch, dev)
    if not args.no_hosvd:
        out["rp_hosvd"] = hosvd_leg(rp, synth, torch, dev)
    if not args.no_accuracy:
        out["accuracy_suites"] = accuracy_leg(rp, synth, torch, dev)
    print(json.dumps(out), flush=True)


def accuracy_leg(rp, synth, torch, dev, seeds=(1, 2, 3)):
    """The accuracy experiment of the randomized SVD: 4096 x 4096 FP32
    A_linear and A_exp (s_p = 1e-3), A_Poly (r = 20, alpha = 3, phi = 1e6) and
    A_Cauchy (one step of orthogonal iteration), target rank 256, oversampling
    10: mean relative residual ||A - U S V^T||_F / ||A||_F over the seeds for
    the split-FP16 path and the FP32 path, beside the Eckart-Young optimum."""
    import numpy as np
    n, p, s_over = 4096, 256, 10
    res = {}
    for kind in ("linear", "exp", "poly", "cauchy"):
        acc = {"split_f16": [], "f32": [], "optimum": []}
        for seed in seeds:
            if kind == "cauchy":
                a = torch.from_numpy(synth.np_cauchy(n, np.random.default_rng(seed))).to(dev)
                sv_all = torch.linalg.svdvals(a.double())
                opt = float((sv_all[p:].norm() / sv_all.norm()).item())
            else:
                sv = {"linear": synth.sv_linear(n, p, 1e-3), "exp": synth.sv_exp(n, p, 1e-3),
                      "poly": synth.sv_poly(n, 20, 3.0, 1e6)}[kind]
                a = synth.torch_sv_matrix(n, sv, seed, dev)
                opt = float(np.sqrt(np.sum(sv[p:] ** 2) / np.sum(sv ** 2)))
            ad = a.double()
            for omega_type, algo in (("f16", "split_f16"), ("f32", "f32")):
                u, s, vt = rp.rsvd(a, p, s_over, 1 if kind == "cauchy" else 0, 100 + seed, omega_type, algo)
                rec = (u.double() * s[None, :]) @ vt.double()
                acc[algo].append(float(((ad - rec).norm() / ad.norm()).item()))
            acc["optimum"].append(opt)
        res[kind] = {k: float(np.mean(v)) for k, v in acc.items()}
        log(f"accuracy {kind}: {res[kind]}")
    return {"workload": "rsvd 4096^2 FP32, target rank 256, oversampling 10, seeds " + str(list(seeds)),
            "mean_rel_residual": res, "device_status": rp.status_string(rp.rp_get_device_status(clear=True))}


def hosvd_leg(rp, synth, torch, dev):
    """RP-HOSVD of a 512^3 FP32 tensor: Tucker core 64^3 ~ U(-1, 1), Haar
    factors, N(0, (1e-3)^2) noise, J = 80 per mode, FP16 Omega_i (stream i).
    Wall time of rp_hosvd (three split-FP16 projections of 512 x 262144
    unfoldings, all streaming X in place; CholeskyQR2; the core), and,
    separately, the projection stage (rp_hosvd_project) with its HBM bytes."""
    n, c, j = 512, 64, 80
    gen = torch.Generator(device=dev)
    gen.manual_seed(104)
    core = torch.rand((c, c, c), device=dev, generator=gen, dtype=torch.float64) * 2 - 1
    us = [synth.torch_haar(n, c, gen, dev) for _ in range(3)]
    x = torch.einsum("abc,ia,jb,kc->ijk", core, us[0], us[1], us[2])
    x += torch.randn(x.shape, device=dev, generator=gen, dtype=torch.float64) * 1e-3
    x32 = x.float().contiguous()
    del x
    walls = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g, facs = rp.rp_hosvd(x32, (j, j, j), 204, "f16", "split_f16")
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
    status = rp.rp_get_device_status(clear=True)
    rec = torch.einsum("abc,ia,jb,kc->ijk", g.double(), facs[0].double(), facs[1].double(), facs[2].double())
    err = float(((rec - x32.double()).norm() / x32.double().norm()).item())
    del rec
    # the projection stage alone (Algorithm 2 line 2, all three modes, as
    # rp_hosvd issues it: modes 1 and 2 grouped in place, mode 3 as X^T Omega_3
    # on the transposed split kernel; the packed Omega_i come from the cache)
    rp.rp_hosvd_project(x32, (j, j, j), 204, "f16", "split_f16")
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    reps = 10
    for _ in range(reps):
        rp.rp_hosvd_project(x32, (j, j, j), 204, "f16", "split_f16")
    e1.record()
    torch.cuda.synchronize()
    t_proj = e0.elapsed_time(e1) / reps * 1e-3
    st2 = rp.rp_get_device_status(clear=True)
    status = status if status != 0 else st2
    pbytes = 3 * (4.0 * n ** 3 + 2.0 * n * n * j + 4.0 * n * j)
    log(f"RP-HOSVD 512^3 J=80: wall {walls}, rel. reconstruction error {err:.4e}; "
        f"projection stage (3 modes) {t_proj * 1e6:.1f} us")
    return {"workload": "rp_hosvd 512^3 FP32, Tucker 64^3 + N(0,1e-3) noise, J=80, FP16 Omega",
            "wall_s": round(min(walls), 5), "rel_reconstruction_error": err,
            "projection_stage": {"us_per_call": round(t_proj * 1e6, 1), "alg_bytes": pbytes,
                                 "achieved_GBps": round(pbytes / t_proj / 1e9, 1),
                                 "hbm_frac": round(pbytes / t_proj / 8e12, 3),
                                 "note": "rp_hosvd_project: X read once per mode (3 x 512 MiB), FP16 Omega_i "
                                         "(cached) read, W_i written"},
            "device_status": rp.status_string(status)}


def load_sigma64():
    """(sigma, a_sha256) of the FP64 oracle's RSVD of the 32768^2 workload
    (tests/golden/rsvd_32768_sigma64.txt), or (None, None)."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "rsvd_32768_sigma64.txt")
    if not os.path.exists(path):
        return None, None
    sha, vals = None, []
    with open(path) as f:
        for line in f:
            if line.startswith("# a_sha256:"):
                sha = line.split(":", 1)[1].strip()
            elif line.strip() and not line.startswith("#"):
                vals.append(float(line))
    return np.array(vals), sha


def c1_leg(rp, synth, torch, dev):
    """The small RSVD: A 1024 x 1024 FP32 = U diag(0.9^i) V^T (Haar U, V), k = 32,
    oversampling 32, no power iteration; the all-FP32 path (FP32 Omega, FP32
    kernels) and the split-FP16 path.  Wall time per call (median of 20 after
    3 warm-up calls, inputs resident; the matrix is cache-resident, so this is
    a latency figure) and the singular-value error against the planted values
    (for scale: the first discarded singular value is 0.9^33 = 0.031)."""
    import numpy as np
    a = torch.from_numpy(synth.np_planted(1024, 1024, synth.sigma_geometric(1024, 0.9),
                                          np.random.default_rng(101))).to(dev)
    planted = torch.tensor(synth.sigma_geometric(1024, 0.9)[:32], device=dev)
    out = {"workload": "rsvd A 1024x1024 FP32 sigma_i=0.9^i, k=32, s=32, q=0"}
    for omega_type, algo in (("f32", "f32"), ("f16", "split_f16")):
        walls = []
        for rep in range(23):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, sv, _ = rp.rsvd(a, 32, 32, 0, 201, omega_type, algo)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t0)
        walls = sorted(walls[3:])
        out[algo] = {"wall_s_median": round(walls[len(walls) // 2], 6), "wall_s_min": round(walls[0], 6),
                     "max_abs_sigma_err_vs_planted": float((sv - planted).abs().max().item()),
                     "device_status": rp.status_string(rp.rp_get_device_status(clear=True))}
    log(f"C1 RSVD 1024^2: {out}")
    return out


def rsvd_leg(rp, synth, torch, dev):
    """Full randomized SVD: A 32768 x 32768 FP32 = U diag(sigma) V^T + noise,
    planted rank 512 with sigma_i = 10^(-(i-1)/511), noise N(0, (1e-4)^2);
    k = 512, oversampling 128 (Omega 32768 x 640 FP16), one power iteration,
    CholeskyQR2 in FP64.  Wall time of rsvd() (inputs resident); the
    singular-value error against the FP64 oracle's RSVD of the same A with the
    same Omega, and against the planted values (bounded by Weyl's inequality
    by ||E||_2 ~ 1e-4 * 2 sqrt(32768) = 0.036)."""
    import hashlib
    m = n = 32768
    k, s, q = 512, 128, 1
    t = time.time()
    a, sig = synth.torch_rsvd_workload(dev, m, n, k)
    torch.cuda.synchronize()
    log(f"RSVD A generated in {time.time() - t:.1f} s")
    walls = []
    for rep in range(2):                               # the first call also sizes the workspace
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        uu, sv, vt = rp.rsvd(a, k, s, q, 203, "f16", "split_f16")
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
    status = rp.rp_get_device_status(clear=True)
    err = float((sv - sig).abs().max().item())
    sig64, sha = load_sigma64()
    out = {"workload": "rsvd A 32768x32768 FP32 planted rank 512 (sigma_i=10^(-(i-1)/511)) + N(0,1e-4) noise; "
                       "k=512, p=640, Omega FP16, q=1, CholeskyQR2 FP64",
           "wall_s": round(min(walls), 4), "wall_s_first_call": round(walls[0], 4),
           "max_abs_sigma_err_vs_planted": err, "weyl_bound": 1e-4 * 2 * math.sqrt(m)}
    if sig64 is not None:
        d = sv.double().cpu().numpy() - sig64
        out["sigma_err_vs_fp64"] = {"max_abs": float(abs(d).max()), "max_rel": float((abs(d) / sig64).max()),
                                    "same_A_as_oracle": hashlib.sha256(a.cpu().numpy().tobytes()).hexdigest() == sha}
    out["device_status"] = rp.status_string(status)
    log(f"RSVD 32768^2 k=512: wall {walls}, max |sigma - planted| {err:.3e}, vs FP64 {out.get('sigma_err_vs_fp64')}")
    del a, uu, vt
    torch.cuda.empty_cache()
    return out


def batched_leg(rp, synth, torch, dev):
    """256 randomized SVDs: m, n log-uniform in [512, 8192], planted rank
    k in [16, 128] with sigma_i = 10^(-3(i-1)/(k-1)), noiseless, width
    p = k + max(10, ceil(k/4)), Omega_j FP16 (and e4m3) from stream j.  The
    first call tunes the grouped projection and captures the graph; the timed
    calls replay it."""
    import numpy as np
    shapes = synth.batched_problem_list(256, 105, 512, 8192, 16, 128)
    gen = torch.Generator(device=dev)
    gen.manual_seed(105)
    t = time.time()
    mats, sigs = [], []
    for m, n, k, p in shapes:
        sig = torch.tensor(10.0 ** (-3.0 * np.arange(k) / (k - 1)), device=dev, dtype=torch.float64)
        u = synth.torch_haar(m, k, gen, dev)
        v = synth.torch_haar(n, k, gen, dev)
        mats.append(((u * sig) @ v.T).float().contiguous())
        sigs.append(sig)
    torch.cuda.synchronize()
    log(f"batched A generated in {time.time() - t:.1f} s")
    ks = [k for _, _, k, _ in shapes]
    ss = [p - k for _, _, k, p in shapes]
    res = {"workload": "batched rsvd, 256 problems, m,n log-uniform [512,8192], planted rank 16-128, noiseless",
           "a_bytes": int(sum(4 * m * n for m, n, _, _ in shapes))}
    for ot in ("f16", "e4m3"):
        t0 = time.perf_counter()
        outs = rp.rsvd_batched(mats, ks, ss, 0, 205, ot)
        torch.cuda.synchronize()
        first = time.perf_counter() - t0
        walls = []
        for _ in range(3):
            t0 = time.perf_counter()
            rp.rsvd_batched(mats, ks, ss, 0, 205, ot, outputs=outs)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t0)
        err = max(float((sv - sg).abs().max().item()) for (_, sv, _), sg in zip(outs, sigs))
        res[ot] = {"wall_s_graph_replay": round(min(walls), 5), "wall_s_first_call": round(first, 4),
                   "max_abs_sigma_err_vs_planted": err,
                   "device_status": rp.status_string(rp.rp_get_device_status(clear=True))}
        log(f"batched {ot}: first {first:.3f} s, replay {min(walls) * 1e3:.2f} ms, sigma err {err:.2e}")
    return res


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_leg(a, y, y32, rows):
    """The FP64 oracle on a row sample, timed on the host cores; its result
    also gives the relative errors of both GPU kernels on that sample."""
    import numpy as np
    from threadpoolctl import threadpool_info
    from oracle import omega, project

    rng = np.random.default_rng(7)
    idx = np.arange(M) if rows >= M else np.sort(rng.choice(M, rows, replace=False))
    a_rows = a[idx].cpu().numpy()
    t0 = time.perf_counter()
    om = omega.omega_f16(SEED_OMEGA, 0, N, R)
    t1 = time.perf_counter()
    ref = project.project_rows_f64(a_rows, om)
    t2 = time.perf_counter()
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    e_split = project.rel_frobenius(y[idx].cpu().numpy(), ref)
    e_f32 = project.rel_frobenius(y32[idx].cpu().numpy(), ref)
    log(f"cpu oracle: omega {t1 - t0:.2f} s, product {t2 - t1:.2f} s; err split {e_split:.3e} f32 {e_f32:.3e}")
    flops = 2.0 * rows * N * R
    base = {
        "value": round(flops / (t2 - t0) / 1e12, 5),
        "unit": "TFLOP/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": f"{rows} of {M} rows of A x full Omega ({N}x{R}); time = oracle Omega generation "
                  f"({t1 - t0:.2f} s) + FP64 product ({t2 - t1:.2f} s)",
        "host_cpus": os.cpu_count(),
        "cpu_model": cpu_model(),
    }
    errs = {"relerr_split_vs_fp64": e_split, "relerr_fp32_vs_fp64": e_f32,
            "error_ratio_split_over_fp32": e_split / e_f32 if e_f32 > 0 else None,
            "error_sample_rows": rows}
    return base, errs


if __name__ == "__main__":
    main()
