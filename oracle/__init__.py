"""CPU FP64 oracle for the mixed-precision random projection path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) imports, calls, links or executes anything in this package.
The only callers are ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py``.

Every function here is a plain, slow, obviously-correct restatement of what
the paper (Ootomo & Yokota, "Mixed-Precision Random Projection for RandNLA on
Tensor Cores", arXiv 2304.04612) defines, written in NumPy / mpmath / Python
integers, with no blocking, fusion or reordering beyond the definition.  It
shares no code, table or constant generator with the HIP path; the only code
both sides use is the seeded synthetic-input module ``synth``.

Modules
  philox    Philox4x64-10 counter-based generator (Salmon et al., SC'11)
  lattice   FP16 value lattice, round-to-nearest cells and their inverse-CDF
            thresholds for N(0,1)                        (Sec. 3.1, eq:g-fp-error)
  omega     the Gaussian random matrix in FP16 / FP32 / FP8-e4m3 (Sec. 3, Sec. 4.4.1)
  formats   Table 1 statistics and the variance of a rounded Gaussian (Sec. 3.2)
  split     the FP32 -> FP16 hi + 2^-11 lo split      (Sec. 4.1, eq:shgemm-1/2)
  project   Y = A Omega in FP64, error metrics, brute force (eq:rp-vec, Sec. 4.4.1)
  rsvd      Randomized SVD, Algorithm 1 (+ power scheme, Sec. 2.1)
  hosvd     Random-projection HOSVD, Algorithm 2
  stats     Johnson-Lindenstrauss norm statistics (Theorem sgt-fp)
"""
