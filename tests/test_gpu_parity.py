"""GPU parity: the HIP library, called through its C ABI, against the CPU oracle.

Integer work throughout, so every comparison is bit-exact: LFVector sizes, the
flattened contents, the prefix of sizes and the capacity held by allocated buckets.
Sizes span several tiles (4096 logical threads for 0/1 producers, 1024 for
multi-element producers) with ragged tails, several tiles per LFVector (look-back),
bucket boundaries inside a tile, empty rounds and empty LFVectors.
"""
import ctypes

import numpy as np
import pytest

import oracle
from oracle import Oracle
from paper_2209_00103_amd import workloads as wl
from tests.conftest import read_golden
from tests.gpu_util import assert_same, both, dev, gg, gpu_flat, gpu_sizes

pytestmark = pytest.mark.gpu

MiB = 1 << 20


@pytest.fixture
def pool():
    p = gg().Pool(512 * MiB)
    yield p
    p.close()


def test_hand_example(pool):
    g = {row[0]: [int(x) for x in row[1:]] for row in read_golden("tiny_insert_hand.txt")}
    G = gg()
    a = G.GGArray(pool, 4, 2, 1)
    a.insert(dev(np.array(g["values"], dtype=np.uint32)), dev(np.array(g["flags"], dtype=np.uint8)))
    assert gpu_sizes(a).tolist() == g["after_insert_sizes"]
    assert gpu_flat(a).tolist() == g["after_insert_flatten"]
    assert a.capacity() == g["after_insert_capacity"][0]
    a.shrink(1, 2)
    assert gpu_flat(a).tolist() == g["after_shrink_flatten"]
    assert a.capacity() == g["after_shrink_capacity"][0]
    a.rw(G.ADD1)
    assert gpu_flat(a).tolist() == g["after_rw_flatten"]
    a.close()
    assert pool.stats()["in_use"] == 0


CASES = [  # elem, V, F, n_threads, p
    (4, 1, 1024, 3 * 4096 + 17, 0.5),    # one LFVector, 4 tiles: look-back chain
    (4, 3, 64, 50000, 0.7),             # 5 tiles per LFVector, ragged chunks
    (4, 256, 1024, 1 << 18, 0.5),        # configuration 1 shape, one tile per LFVector
    (8, 7, 2, 20011, 0.9),              # small first bucket: many buckets per tile
    (4, 2, 1, 10000, 1.0),              # F = 1: buckets of 1, 2, 4 ... elements
    (8, 300, 16, 257, 0.5),             # fewer threads than LFVectors
    (4, 5, 8, 0, 0.5),                  # empty round
    (4, 1, 4096, 1 << 22, 0.3),          # 1024 tiles in one LFVector
    (4, 4097, 8, 300000, 0.6),          # prefix over several workgroups, last chunk of one LFVector
    (8, 70000, 1, 500000, 0.4),         # 69 chunks of the multi-workgroup prefix, many empty LFVectors
]


@pytest.mark.parametrize("elem,V,F,n,p", CASES)
def test_buffer_insert_rounds(pool, elem, V, F, n, p):
    print(f"case elem={elem} V={V} F={F} n={n} p={p}", flush=True)
    rng = np.random.default_rng(n + V)
    a, o = both(elem, V, F, pool)
    for r in range(3):
        vals, flags = wl.random_round(rng, n, p, elem)
        a.insert(dev(vals), dev(flags))
        o.insert(vals, flags)
        assert_same(a, o, f"round {r}")
    a.close()
    assert pool.stats()["in_use"] == 0


def test_insert_without_flags(pool):
    a, o = both(4, 9, 32, pool)
    rng = np.random.default_rng(1)
    for n in (1, 4095, 4096, 4097, 12345):
        vals, _ = wl.random_round(rng, n, 1.0, 4)
        a.insert(dev(vals))
        o.insert(vals)
    assert_same(a, o)
    a.close()


@pytest.mark.parametrize("elem", [4, 8])
def test_rounds_shrink_rw_interleaved(pool, elem):
    rng = np.random.default_rng(7 + elem)
    V, F = 11, 8
    a, o = both(elem, V, F, pool)
    G = gg()
    ops = ["ins", "ins", "shr", "rw0", "ins", "shr", "rw1", "ins", "rw2", "shr", "ins", "ins", "shr"]
    for i, op in enumerate(ops):
        if op == "ins":
            n = int(rng.integers(0, 60000))
            vals, flags = wl.random_round(rng, n, float(rng.random()), elem)
            a.insert(dev(vals), dev(flags))
            o.insert(vals, flags)
        elif op == "shr":
            num, den = [(1, 10), (1, 2), (3, 7), (1, 1)][i % 4]
            a.shrink(num, den)
            o.shrink(num, den)
        else:
            a.rw(int(op[2]))
            o.rw(int(op[2]))
        assert_same(a, o, f"op {i} {op}")
    a.close()
    assert pool.stats()["in_use"] == 0


@pytest.mark.parametrize("elem", [4, 8])
def test_insert_counts(pool, elem):
    rng = np.random.default_rng(11)
    a, o = both(elem, 13, 16, pool)
    for r in range(3):
        n = 5000 + 777 * r
        mc = [16, 5, 1][r]
        counts = rng.integers(0, mc + 1, size=n, dtype=np.uint8)
        counts[::97] = 255  # above max_count: clamped to it
        vals, _ = wl.random_round(rng, n * mc, 1.0, elem)
        a.insert_counts(dev(vals), dev(counts), mc)
        o.insert_counts(vals, counts, mc)
        assert_same(a, o, f"round {r}")
    a.close()


def test_gen_bernoulli_config1(pool):
    """Configuration 1 at full size: V=256, F=1024, 2^18 threads, 4 rounds, r/w +1, flatten."""
    G = gg()
    cfg = wl.CFG1
    a, o = both(4, cfg["V"], cfg["F"], pool)
    for r in range(cfg["rounds"]):
        a.insert_gen(G.make_gen(G.GEN_BERNOULLI, seed=42, round=r), cfg["n_threads"])
        o.insert_gen(oracle.GEN_BERNOULLI, cfg["n_threads"], seed=42, round=r)
    assert_same(a, o, "inserted")
    a.rw(G.ADD1)
    o.rw(oracle.OP_ADD1)
    assert_same(a, o, "rw")
    a.close()


def test_gen_matches_buffer_mode(pool):
    """The device generator and the numpy generator give the same array."""
    G = gg()
    a = G.GGArray(pool, 4, 17, 128)
    b = G.GGArray(pool, 4, 17, 128)
    for r in range(3):
        a.insert_gen(G.make_gen(G.GEN_BERNOULLI, seed=1, round=r), 70001)
        vals, flags = wl.bernoulli_round(1, r, 70001, 4)
        b.insert(dev(vals), dev(flags))
    np.testing.assert_array_equal(gpu_flat(a), gpu_flat(b))
    a.close()
    b.close()


def test_gen_round_tag_scaled_config2(pool):
    """Configuration 2 per-LFVector shape (each LFVector sees n_r/512 threads per round)
    with V=8: 12 rounds, shrink 1/10 after each, r/w 3x+1, flatten."""
    G = gg()
    V = 8
    a, o = both(4, V, 1024, pool)
    for r, n_r in enumerate(wl.cfg2_round_threads()):
        n = n_r // 512 * V
        a.insert_gen(G.make_gen(G.GEN_ROUND_TAG, round=r, tag_shift=27), n)
        o.insert_gen(oracle.GEN_ROUND_TAG, n, round=r, tag_shift=27)
        a.shrink(1, 10)
        o.shrink(1, 10)
        assert_same(a, o, f"round {r}")
    a.rw(G.MUL3ADD1)
    o.rw(oracle.OP_MUL3ADD1)
    assert_same(a, o, "rw")
    a.close()


@pytest.mark.parametrize("elem", [8, 4])
def test_gen_poisson_scaled_config3(pool, elem):
    """Configuration 3 shape at 1/1024 of the threads: Poisson(3) counts capped at 16,
    4 insert phases each followed by r/w +1."""
    G = gg()
    thr = wl.poisson_thresholds(3, 16)
    V, n = 64, 1 << 16
    a, o = both(elem, V, 1024, pool)
    for i in range(4):
        a.insert_gen(G.make_gen(G.GEN_POISSON, seed=1, round=i, max_count=16, thresholds=thr), n)
        o.insert_gen(oracle.GEN_POISSON, n, seed=1, round=i, max_count=16, thresholds=thr)
        a.rw(G.ADD1)
        o.rw(oracle.OP_ADD1)
        assert_same(a, o, f"phase {i}")
    a.close()


def test_flatten_too_small(pool):
    G = gg()
    a = G.GGArray(pool, 4, 3, 4)
    a.insert(dev(np.arange(100, dtype=np.uint32)))
    out = G.to_device(np.full(99, 7, dtype=np.uint32))
    a.flatten_into(out)
    assert a.last_error() == G.ERANGE
    assert (G.as_unsigned(out) == 7).all()
    a.close()


def test_static_and_semistatic_baselines():
    G = gg()
    rng = np.random.default_rng(5)
    st = G.StaticArray(200000, 4)
    ss = G.SemiStaticArray(4, 1000)
    o = Oracle(4, 1, 1)
    cap, resizes = 1000, 0  # host rule: before a round, double until size + n fits
    for r in range(4):
        vals, flags = wl.random_round(rng, 30000 + r, 0.6, 4)
        if o.size() + vals.size > cap:
            while cap < o.size() + vals.size:
                cap *= 2
            resizes += 1
        st.insert(dev(vals), dev(flags))
        ss.insert(dev(vals), dev(flags))
        o.insert(vals, flags)
    st.rw(G.MUL3ADD1)
    ss.rw(G.MUL3ADD1)
    o.rw(oracle.OP_MUL3ADD1)
    ref = np.sort(o.flatten())
    assert st.size() == ss.size() == o.size()
    np.testing.assert_array_equal(np.sort(G.as_unsigned(st.data())), ref)
    np.testing.assert_array_equal(np.sort(G.as_unsigned(ss.data())), ref)
    assert ss.resizes() == resizes
    # static overflow: elements past the capacity are dropped and reported
    small = G.StaticArray(100, 4)
    small.insert(dev(np.arange(150, dtype=np.uint32)))
    assert small.last_error() == G.ERANGE
    v = ctypes.c_uint64()  # size still reports the sticky error, and the clamped size
    assert G.lib().gga_static_size(small._h, ctypes.byref(v), None) == G.ERANGE
    assert v.value == 100
    for x in (st, ss, small):
        x.close()


def test_static_gen_matches_oracle_multiset():
    G = gg()
    st = G.StaticArray(1 << 20, 8)
    thr = wl.poisson_thresholds(3, 16)
    o = Oracle(8, 1, 1)
    for i in range(2):
        st.insert_gen(G.make_gen(G.GEN_POISSON, seed=3, round=i, max_count=16, thresholds=thr), 50000)
        o.insert_gen(oracle.GEN_POISSON, 50000, seed=3, round=i, max_count=16, thresholds=thr)
    np.testing.assert_array_equal(np.sort(G.as_unsigned(st.data())), np.sort(o.flatten()))
    st.close()


def test_determinism_repeat(pool):
    G = gg()
    outs = []
    for _ in range(3):
        a = G.GGArray(pool, 4, 5, 16)
        for r in range(4):
            a.insert_gen(G.make_gen(G.GEN_BERNOULLI, seed=9, round=r), 100003)
        a.shrink(1, 3)
        outs.append(gpu_flat(a))
        a.close()
    assert all(np.array_equal(outs[0], x) for x in outs[1:])


def test_pool_allocation_count_matches_oracle(pool):
    """One device allocation per bucket the oracle allocates (Alg. 2 winners);
    shrink returns exactly the buckets the oracle frees."""
    G = gg()
    a, o = both(4, 16, 64, pool)
    before = pool.stats()
    rng = np.random.default_rng(2)
    for r in range(5):
        vals, flags = wl.random_round(rng, 40000, 0.5, 4)
        a.insert(dev(vals), dev(flags))
        o.insert(vals, flags)
        a.shrink(1, 4)
        o.shrink(1, 4)
    after = pool.stats()
    assert after["allocs"] - before["allocs"] == o.alloc_count()
    assert after["frees"] - before["frees"] == o.free_count()
    assert_same(a, o)
    a.close()


def _round_prefixes(elem, V, F, rounds):
    """Oracle states (per-LFVector contents) after 0, 1, ... rounds."""
    o = Oracle(elem, V, F)
    states = []

    def snap():
        pre = o.prefix().astype(np.int64)
        flat = o.flatten()
        states.append([flat[pre[v]:pre[v + 1]].copy() for v in range(V)])

    snap()
    for vals, flags in rounds:
        o.insert(vals, flags)
        snap()
    return states


def _check_round_prefixes(a, states, V):
    pre = a.prefix().cpu().numpy().astype(np.int64)
    flat = gpu_flat(a)
    for v in range(V):
        seg = flat[pre[v]:pre[v + 1]]
        assert any(np.array_equal(seg, st[v]) for st in states), f"LFVector {v} is not a round prefix"


def test_pool_exhaustion_keeps_round_prefixes():
    G = gg()
    pool = G.Pool(4 * MiB)  # 2 MiB header + 2 MiB of buckets
    V, F = 4, 256
    rng = np.random.default_rng(4)
    # 24 rounds x 32000 kept elements x 4 B = 3 MB of live data > the 2 MiB region
    rounds = [wl.random_round(rng, 40000, 0.8, 4) for _ in range(24)]
    a = G.GGArray(pool, 4, V, F)
    for vals, flags in rounds:
        a.insert(dev(vals), dev(flags))
    assert a.last_error() == G.ENOMEM
    _check_round_prefixes(a, _round_prefixes(4, V, F, rounds), V)
    a.close()
    assert pool.stats()["in_use"] == 0
    pool.close()


@pytest.mark.parametrize("fault_at", [1, 2, 5, 9])
def test_fault_injection_keeps_round_prefixes(pool, fault_at):
    G = gg()
    V, F = 6, 32
    rng = np.random.default_rng(fault_at)
    rounds = [wl.random_round(rng, 9000, 0.7, 4) for _ in range(4)]
    a = G.GGArray(pool, 4, V, F)
    pool.set_fault(fault_at)
    for vals, flags in rounds:
        a.insert(dev(vals), dev(flags))
    pool.set_fault(0)
    assert a.last_error() == G.ENOMEM
    _check_round_prefixes(a, _round_prefixes(4, V, F, rounds), V)
    # a frozen LFVector stays as it was; shrink, r/w and flatten still work
    a.shrink(1, 2)
    a.rw(G.ADD1)
    a.flatten()
    a.close()
    assert pool.stats()["in_use"] == 0


def test_invalid_arguments_with_gpu(pool):
    G = gg()
    L = G.lib()
    a = G.GGArray(pool, 4, 4, 8)
    assert L.ggarray_shrink(a.handle if hasattr(a, "handle") else a._h, 3, 2, None) == G.EINVAL
    assert L.ggarray_rw(a._h, 7, None) == G.EINVAL
    assert L.ggarray_insert_counts(a._h, None, None, 17, 0, None) == G.EINVAL
    g = G.make_gen(G.GEN_POISSON, round=8, max_count=16)
    assert L.ggarray_insert_gen(a._h, g, 10, None) == G.EINVAL
    with pytest.raises(G.GGAError):
        G.GGArray(pool, 4, 4, 3)
    a.close()


@pytest.mark.parametrize("elem", [4, 8])
def test_insert_segments_and_snapshot_restore(pool, elem):
    """Segment append against the oracle (appending to non-empty LFVectors, empty
    segments, segments crossing many buckets), a flat snapshot (flatten + prefix)
    restored into an empty array, and invalid segments reported with ERANGE."""
    G = gg()
    rng = np.random.default_rng(17)
    V, F = 37, 8
    a, o = both(elem, V, F, pool)
    for r in range(2):
        vals, flags = wl.random_round(rng, 30000, 0.6, elem)
        a.insert(dev(vals), dev(flags))
        o.insert(vals, flags)
    lens = rng.integers(0, 3000, size=V)
    lens[::5] = 0
    prefix = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
    seg, _ = wl.random_round(rng, int(prefix[-1]), 1.0, elem)
    a.insert_segments(dev(seg), dev(prefix))
    assert o.insert_segments(seg, prefix) == oracle.OK
    assert_same(a, o, "segments appended")
    # restore: flatten + prefix of a, appended to an empty array of the same shape
    flat = gpu_flat(a)
    pre = a.prefix().cpu().numpy().astype(np.uint64)
    b, ob = both(elem, V, F, pool)
    b.insert_segments(dev(flat), dev(pre))
    assert ob.insert_segments(o.flatten(), o.prefix()) == oracle.OK
    assert_same(b, ob, "restored")
    assert np.array_equal(gpu_flat(b), gpu_flat(a)) and b.capacity() == a.capacity()
    # an invalid pair: that LFVector is unchanged, the others append, ERANGE is sticky
    c, oc = both(elem, 4, F, pool)
    bad = np.array([0, 5, 3, 9, 12], dtype=np.uint64)
    vals, _ = wl.random_round(rng, 12, 1.0, elem)
    c.insert_segments(dev(vals), dev(bad))
    assert oc.insert_segments(vals, bad) == oracle.ERANGE
    assert c.last_error() == G.ERANGE
    assert gpu_sizes(c).tolist() == oc.vector_sizes().tolist() == [5, 0, 6, 3]
    for x in (a, b, c):
        x.close()
