"""Pin: the oracle's Philox4x64-10 against numpy.random.Philox, an independent
implementation of the same generator (Salmon et al., SC'11) shipped with NumPy.
NumPy advances its 256-bit counter before producing a block, so a block for
counter c is read from a generator whose counter is set to c - 1."""
import numpy as np
import pytest

from oracle import philox


def _numpy_block(ctr, key):
    c = list(ctr)
    # c - 1 with borrow over the four 64-bit words
    for w in range(4):
        if c[w] > 0:
            c[w] -= 1
            break
        c[w] = (1 << 64) - 1
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(c, dtype=np.uint64))
    return [int(v) for v in g.random_raw(4)]


@pytest.mark.parametrize("seed", [0, 1, 7, 12345, (1 << 64) - 1, 0x0123456789ABCDEF])
def test_philox_matches_numpy(seed):
    rng = np.random.default_rng(seed & 0xFFFF)
    ctrs = [(0, 0, 0, 0), (1, 0, 0, 0), (0, 1, 2, 0), ((1 << 64) - 1, 5, 3, 0)]
    ctrs += [tuple(int(x) for x in rng.integers(0, 1 << 63, size=4, dtype=np.uint64)) for _ in range(16)]
    for ctr in ctrs:
        got = philox.philox4x64_10(*[np.uint64(c) for c in ctr], np.uint64(seed), np.uint64(0))
        assert [int(x) for x in got] == _numpy_block(ctr, (seed, 0)), ctr


def test_philox_vectorised_equals_scalar():
    i = np.arange(37, dtype=np.uint64)[:, None]
    j = np.arange(5, dtype=np.uint64)[None, :]
    v = philox.philox4x64_10(i, j, np.uint64(3), np.uint64(1), np.uint64(99), np.uint64(0))
    for a in (0, 17, 36):
        for b in (0, 4):
            s = philox.philox4x64_10(np.uint64(a), np.uint64(b), np.uint64(3), np.uint64(1),
                                     np.uint64(99), np.uint64(0))
            assert [int(w[a, b]) for w in v] == [int(x) for x in s]


def test_key_word1_matters():
    a = philox.philox4x64_10(1, 2, 3, 4, 5, 0)
    b = philox.philox4x64_10(1, 2, 3, 4, 5, 1)
    assert [int(x) for x in a] == _numpy_block((1, 2, 3, 4), (5, 0))
    assert [int(x) for x in b] == _numpy_block((1, 2, 3, 4), (5, 1))
    assert a != b
