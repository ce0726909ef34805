"""The library's inverse-CDF threshold table (built on the host in IEEE
binary128 when a context is created) against the oracle's mpmath table, entry
by entry, and the guide table that brackets the search (Sec. 3.1,
eq:g-fp-error).  Both tables are built by exported host functions, so this
runs without a GPU.  The GPU tests sample Omega cells, so a one-unit
disagreement in a single threshold would only show here."""
import ctypes
import os

import numpy as np
import pytest

from oracle import lattice

GUIDE_LOG2 = 16          # buckets over the top 16 bits of the 63-bit uniform


@pytest.fixture(scope="module")
def L():
    import paper_2304_04612_amd as rp
    if not os.path.exists(rp.LIB_PATH):
        from paper_2304_04612_amd import build
        build.build()
    return rp.lib()


@pytest.fixture(scope="module")
def lib_table(L):
    cap = 20000
    buf = (ctypes.c_uint64 * cap)()
    n = L.rpmi_build_f16_thresholds(buf, cap)
    assert n > 0
    return np.frombuffer(buf, dtype=np.uint64, count=n).copy()


def test_thresholds_equal_oracle_entry_by_entry(lib_table):
    ref = lattice.thresholds_f16_array()
    assert lib_table.shape == ref.shape == (18571,)
    diff = np.nonzero(lib_table != ref)[0]
    assert diff.size == 0, f"{diff.size} entries differ, first at t = {diff[:5]}"


def test_too_small_capacity_is_reported(L):
    buf = (ctypes.c_uint64 * 100)()
    assert L.rpmi_build_f16_thresholds(buf, 100) == -1


def test_guide_brackets_every_cell(L, lib_table):
    n = lib_table.size
    nb = 1 << GUIDE_LOG2
    guide = (ctypes.c_uint32 * (nb + 1))()
    L.rpmi_build_guide(lib_table.ctypes.data_as(ctypes.c_void_p), n, guide, GUIDE_LOG2)
    g = np.frombuffer(guide, dtype=np.uint32).astype(np.int64)
    edges = (np.arange(nb + 1, dtype=np.uint64) << np.uint64(63 - GUIDE_LOG2))
    # guide[b] = #{t : T_t < b 2^(63-16)}
    assert np.array_equal(g, np.searchsorted(lib_table, edges, side="left"))
    # every u in bucket b has its cell k = #{t : T_t <= u} inside [guide[b], guide[b+1]]
    rng = np.random.default_rng(11)
    u = rng.integers(0, 1 << 63, size=200000, dtype=np.uint64)
    u = np.concatenate([u, lib_table, lib_table[lib_table > 0] - np.uint64(1)])
    k = np.searchsorted(lib_table, u, side="right")
    b = (u >> np.uint64(63 - GUIDE_LOG2)).astype(np.int64)
    assert np.all(g[b] <= k) and np.all(k <= g[b + 1])
