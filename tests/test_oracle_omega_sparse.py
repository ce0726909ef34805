"""Pins of the oracle's sparse Omega (Sec. 2.2 eq:sp-rand without its sqrt(s)
factor, as Sec. 3.4 allows): the thresholds against their defining
inequalities, the entry frequencies against the eq:sp-rand probabilities,
and the word-to-entry rule against scalar brute force on the Philox words."""
import math

import numpy as np
import pytest

from oracle import omega, philox


def test_thresholds_satisfy_their_definition():
    # T = floor(2^64 / (2s)):  2s T <= 2^64 < 2s (T + 1)
    t1, t3 = omega.sparse_threshold("sparse1", 10), omega.sparse_threshold("sparse3", 10)
    assert 2 * t1 <= 1 << 64 < 2 * (t1 + 1)
    assert 6 * t3 <= 1 << 64 < 6 * (t3 + 1)
    # s = sqrt(n):  T <= 2^63 / sqrt(n) < T + 1, i.e. n T^2 <= 2^126 < n (T + 1)^2
    for n in (1, 2, 3, 37, 4096, 262144, 10 ** 9 + 7):
        t = omega.sparse_threshold("vsparse", n)
        assert n * t * t <= 1 << 126 < n * (t + 1) * (t + 1), n


@pytest.mark.parametrize("kind,n", [("sparse1", 2048), ("sparse3", 2048), ("vsparse", 4096)])
def test_entry_frequencies_match_eq_sp_rand(kind, n):
    """+1 and -1 each with probability 1/(2s), 0 with 1 - 1/s: counts over
    n x 256 entries within 6 standard deviations of the binomial means."""
    v = omega.omega_sparse(11, 2, n, 256, kind)
    assert set(np.unique(v)) <= {-1.0, 0.0, 1.0}
    s = {"sparse1": 1.0, "sparse3": 3.0, "vsparse": math.sqrt(n)}[kind]
    N = v.size
    for val, p in ((1.0, 1 / (2 * s)), (-1.0, 1 / (2 * s)), (0.0, 1 - 1 / s)):
        cnt = int(np.count_nonzero(v == val))
        mean, sd = N * p, math.sqrt(N * p * (1 - p))
        assert abs(cnt - mean) <= 6 * sd + 1e-9, (kind, val, cnt, mean)


def test_word_rule_by_brute_force():
    """Scalar Python-integer evaluation of the rule on the element's own
    Philox word (word j mod 4 of the block with counter (i, floor(j/4),
    stream, 0), key (seed, 0))."""
    seed, stream, n, r = 99, 5, 37, 13
    for kind in omega.SPARSE_KINDS:
        v = omega.omega_sparse(seed, stream, n, r, kind)
        t = omega.sparse_threshold(kind, n)
        for i in (0, 1, 17, 36):
            for j in (0, 3, 4, 11, 12):
                words = philox.philox4x64_10(np.uint64(i), np.uint64(j // 4), np.uint64(stream), np.uint64(0),
                                             np.uint64(seed), np.uint64(0))
                x = int(words[j % 4])
                want = 1.0 if x < t else (-1.0 if x < 2 * t else 0.0)
                assert v[i, j] == want, (kind, i, j)


def test_fp16_bits():
    v = omega.omega_sparse(4, 0, 64, 40, "sparse3")
    b = omega.omega_sparse_f16_bits(4, 0, 64, 40, "sparse3")
    assert np.array_equal(b.view(np.float16).astype(np.float64), v)
