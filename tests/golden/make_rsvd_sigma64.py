"""Writes rsvd_32768_sigma64.txt: the FP64 oracle's singular values for the
full randomized-SVD workload (Algorithm 1 with one step of the power scheme,
Sec. 2.1 and 2.2), against which the library's RSVD is compared.

    python tests/golden/make_rsvd_sigma64.py [out_path]

Needs a GPU only to draw the input: A is the 32768 x 32768 FP32 planted
matrix of synth.torch_rsvd_workload (seed 103, rank 512, sigma_i =
10^(-(i-1)/511), N(0, 1e-8) noise), copied to the host.  Everything else runs
in the CPU oracle in FP64: Omega = oracle.omega.omega_f16(203, 0, 32768, 640)
(the generator the library reproduces bit for bit), then
oracle.rsvd.rsvd(A, Omega, k=512, power_iters=1).  The file records a
fingerprint of A (its FP64 sum and the SHA-256 of its bytes) so that a test
can tell whether it drew the same A.
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

M = N = 32768
K, S, Q, SEED = 512, 128, 1, 203


def main():
    import torch
    import synth
    from oracle import omega, rsvd

    out = sys.argv[1] if len(sys.argv) > 1 else os.path.join(HERE, "rsvd_32768_sigma64.txt")
    t0 = time.time()
    a32, _ = synth.torch_rsvd_workload("cuda:0")
    a = a32.cpu().numpy()
    del a32
    sha = hashlib.sha256(a.tobytes()).hexdigest()
    a = a.astype(np.float64)
    asum = float(a.sum())
    print(f"A drawn and copied in {time.time() - t0:.1f} s; sum {asum!r}", flush=True)
    t0 = time.time()
    om = omega.omega_f16(SEED, 0, N, K + S)
    print(f"oracle Omega in {time.time() - t0:.1f} s", flush=True)
    t0 = time.time()
    _, s, _ = rsvd.rsvd(a, om, K, power_iters=Q)
    print(f"oracle RSVD in {time.time() - t0:.1f} s; sigma_1 {float(s[0])!r} sigma_512 {float(s[-1])!r}",
          flush=True)
    with open(out, "w") as f:
        f.write("# FP64 oracle singular values of the 32768^2 RSVD workload (k=512, p=640, q=1, FP16 Omega seed 203)\n")
        f.write("# written by tests/golden/make_rsvd_sigma64.py (oracle.rsvd.rsvd on synth.torch_rsvd_workload)\n")
        f.write(f"# a_sha256: {sha}\n")
        f.write(f"# a_sum_f64: {asum!r}\n")
        for v in s:
            f.write(f"{float(v)!r}\n")
    print(f"wrote {out}", flush=True)


if __name__ == "__main__":
    main()
