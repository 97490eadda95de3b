"""GPU tests of the baselines beside the GGArray: the mapped (memMap) array, grown
by mapping physical memory onto a reserved virtual range, and the static array's
per-element atomic insertion.  Contents against the oracle as multisets (their
insertion order across threads is not fixed)."""
import ctypes

import numpy as np
import pytest

import oracle
from oracle import Oracle
from paper_2209_00103_amd import workloads as wl
from tests.gpu_util import gg

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("elem", [4, 8])
def test_mapped_grows_without_copies_and_matches_oracle(elem):
    G = gg()
    m = G.MappedArray(elem, 1 << 26)
    o = Oracle(elem, 1, 1)
    try:
        rounds = [1 << 12] + [1 << (12 + r) for r in range(1, 10)]  # 2^12 .. 2^21 threads
        for r, n in enumerate(rounds):
            m.insert_gen(G.make_gen(G.GEN_ROUND_TAG, round=r, tag_shift=27), n)
            o.insert_gen(oracle.GEN_ROUND_TAG, n, round=r, tag_shift=27)
        m.rw(G.MUL3ADD1)
        o.rw(oracle.OP_MUL3ADD1)
        assert m.size() == o.size()
        got = np.sort(G.as_unsigned(m.data()))
        assert np.array_equal(got, np.sort(o.flatten()))
        assert m.maps() >= 2  # it grew in place more than once
    finally:
        m.close()
        o.close()


def test_mapped_buffer_rounds_and_limit():
    G = gg()
    m = G.MappedArray(4, 100000)
    o = Oracle(4, 1, 1)
    rng = np.random.default_rng(4)
    try:
        for n in (1000, 30000, 0, 50000):
            vals, flags = wl.random_round(rng, n, 0.5, 4)
            m.insert(G.to_device(vals), G.to_device(flags))
            o.insert(vals, flags)
        assert m.size() == o.size()
        assert np.array_equal(np.sort(G.as_unsigned(m.data())), np.sort(o.flatten()))
        vals, flags = wl.random_round(rng, 100000, 0.1, 4)
        with pytest.raises(G.GGAError) as e:  # worst case past the reserved range: refused up front
            m.insert(G.to_device(vals), G.to_device(flags))
        assert e.value.status == G.ERANGE
        assert m.size() == o.size()
    finally:
        m.close()
        o.close()


@pytest.mark.parametrize("elem", [4, 8])
def test_static_per_element_atomics_match_oracle_multiset(elem):
    """The per-element atomic strategy inserts the same elements as the scan (order
    across threads is free), and stops at the capacity with GGA_ERANGE."""
    G = gg()
    st = G.StaticArray(400000, elem)
    o = Oracle(elem, 1, 1)
    try:
        for r, n in enumerate([1 << 18, 12345, 0, 99999]):
            st.insert_gen_atomic(G.make_gen(G.GEN_BERNOULLI, seed=6, round=r), n)
            o.insert_gen(oracle.GEN_BERNOULLI, n, seed=6, round=r)
        assert st.size() == o.size() and st.last_error() == 0
        assert np.array_equal(np.sort(G.as_unsigned(st.data())), np.sort(o.flatten()))
        st.insert_gen_atomic(G.make_gen(G.GEN_ROUND_TAG, round=9, tag_shift=30), 300000)
        assert st.last_error() == G.ERANGE
        v = ctypes.c_uint64()
        assert G.lib().gga_static_size(st._h, ctypes.byref(v), G._stream(None)) == G.ERANGE
        assert v.value == 400000
    finally:
        st.close()
        o.close()
