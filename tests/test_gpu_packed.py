"""GPU parity of the packed multi-element insertion (ggarray_insert_packed): each
thread inserts counts[g] elements taken in order from a packed buffer.  Against
the CPU oracle, bit-exact: several tiles per LFVector (tickets and look-back),
counts up to 255, F = 1 (runs over many buckets), ragged tails, empty tiles and
rounds, too few values (sticky GGA_ERANGE, nothing inserted); and the
configuration-3 producer given as a packed buffer equals the generated round."""
import numpy as np
import pytest
import torch

import oracle
from oracle import Oracle
from paper_2209_00103_amd import workloads as wl
from tests.gpu_util import assert_same, both, dev, gg

pytestmark = pytest.mark.gpu

MiB = 1 << 20
TILE = 1024


@pytest.fixture
def pool():
    p = gg().Pool(2048 * MiB)
    yield p
    p.close()


CASES = [  # elem, V, F, threads per LFVector, largest count
    (8, 1, 1024, 12 * TILE + 5, 16),
    (4, 1, 1, 3 * TILE + 100, 255),
    (8, 4, 1, 5 * TILE + 999, 7),
    (4, 13, 16, 777, 40),
    (8, 512, 1024, 3 * TILE + 1, 16),
    (4, 512, 1, 2 * TILE + 600, 3),
    (8, 300, 8, 1, 16),  # fewer threads than LFVectors would leave: chunk 1
]


@pytest.mark.parametrize("elem,V,F,chunk,mc", CASES)
def test_insert_packed_rounds(pool, elem, V, F, chunk, mc):
    print(f"case packed elem={elem} V={V} F={F} chunk={chunk} max={mc}", flush=True)
    rng = np.random.default_rng(V * 31 + chunk + mc)
    a, o = both(elem, V, F, pool)
    n = V * chunk
    for r in range(4):
        counts = rng.integers(0, mc + 1, size=n, dtype=np.uint8)
        if r == 1:
            counts[rng.random(n) < 0.7] = 0
        if r == 2:
            counts[:] = 0  # an empty round
        total = int(counts.sum(dtype=np.uint64))
        vals, _ = wl.random_round(rng, total + 3, 1.0, elem)
        a.insert_packed(dev(vals), dev(counts))
        assert o.insert_packed(vals, counts) == oracle.OK
        assert_same(a, o, f"round {r}")
    a.rw(gg().ADD1)
    o.rw(oracle.OP_ADD1)
    assert_same(a, o, "rw")
    a.close()
    assert pool.stats()["in_use"] == 0


def test_insert_packed_too_few_values(pool):
    G = gg()
    a, o = both(8, 5, 4, pool)
    rng = np.random.default_rng(9)
    counts = rng.integers(1, 9, size=40000, dtype=np.uint8)
    total = int(counts.sum(dtype=np.uint64))
    vals, _ = wl.random_round(rng, total, 1.0, 8)
    a.insert_packed(dev(vals), dev(counts), n_values=total - 1)
    assert a.last_error() == G.ERANGE
    assert a.size(check_error=False) == 0
    assert int(a.vector_sizes().sum()) == 0
    a.close()
    o.close()


def test_packed_poisson_equals_generated(pool):
    """The configuration-3 producer (Poisson(3) counts capped at 16, payloads
    K(seed, gid, 16 i + j)) given as counts plus packed payloads from the numpy
    generator gives the array the generated rounds give, and the oracle's."""
    G = gg()
    thr = wl.poisson_thresholds(3, 16)
    V, F, n = 64, 1024, 64 * (3 * TILE + 17)
    gen_arr = G.GGArray(pool, 8, V, F)
    pk_arr, o = both(8, V, F, pool)
    for i in range(3):
        c = wl.poisson_counts(5, i, n, thr)
        gid = np.repeat(np.arange(n, dtype=np.uint64), c.astype(np.int64))
        j = np.concatenate([np.arange(int(x), dtype=np.uint64) for x in c])
        vals = wl.poisson_payload(5, i, gid, j)
        gen_arr.insert_gen(G.make_gen(G.GEN_POISSON, seed=5, round=i, max_count=16, thresholds=thr), n)
        pk_arr.insert_packed(dev(vals), dev(c))
        assert o.insert_packed(vals, c) == oracle.OK
        gen_arr.rw(G.ADD1)
        pk_arr.rw(G.ADD1)
        o.rw(oracle.OP_ADD1)
        assert_same(pk_arr, o, f"phase {i}")
        assert torch.equal(gen_arr.flatten(), pk_arr.flatten())
    gen_arr.close()
    pk_arr.close()


@pytest.mark.parametrize("V", [65536, 512])
def test_packed_full_size_equals_generated(V):
    """Configuration 3 at full size (2^26 threads, Poisson(3) counts capped at 16,
    uint64, F = 1024) with V = 65536 (65536 tiles: the tile-total scan runs over
    several passes) and V = 512 (128 tiles per LFVector): two rounds given as
    host counts plus the generated round's payloads in thread order equal the
    generated rounds element by element (those are checked against the oracle
    at full size elsewhere), and an r/w between them sees the same array."""
    G = gg()
    thr = wl.poisson_thresholds(3, 16)
    n = 1 << 26
    pool = G.Pool(24 << 30)
    gen_arr = G.GGArray(pool, 8, V, 1024)
    pk_arr = G.GGArray(pool, 8, V, 1024)
    src = G.GGArray(pool, 8, V, 1024)  # produces each round's payloads in thread order
    for i in range(2):
        print(f"case packed full size V={V} round {i}", flush=True)
        g = G.make_gen(G.GEN_POISSON, seed=1, round=i, max_count=16, thresholds=thr)
        src.insert_gen(g, n)
        vals = src.flatten()
        src.shrink(1, 1)
        counts = torch.from_numpy(wl.poisson_counts(1, i, n, thr)).to("cuda")
        assert int(counts.sum()) == vals.numel()
        gen_arr.insert_gen(g, n)
        pk_arr.insert_packed(vals, counts)
        gen_arr.rw(G.ADD1)
        pk_arr.rw(G.ADD1)
        assert pk_arr.last_error() == 0 and gen_arr.last_error() == 0
        assert torch.equal(gen_arr.vector_sizes(), pk_arr.vector_sizes())
        assert torch.equal(gen_arr.flatten(), pk_arr.flatten())
        assert gen_arr.capacity() == pk_arr.capacity()
        del vals, counts
    for x in (gen_arr, pk_arr, src):
        x.close()
    pool.close()


def test_insert_packed_too_few_values_one_tile_per_lfvector(pool):
    """One tile per LFVector (the LFVectors grow while the tile totals are taken):
    a round whose counts ask for more values than given leaves every LFVector,
    its capacity and the pool exactly as the round before left them."""
    G = gg()
    V, chunk = 64, 700
    a, o = both(8, V, 16, pool)
    rng = np.random.default_rng(21)
    counts = rng.integers(0, 9, size=V * chunk, dtype=np.uint8)
    vals, _ = wl.random_round(rng, int(counts.sum(dtype=np.uint64)), 1.0, 8)
    a.insert_packed(dev(vals), dev(counts))
    assert o.insert_packed(vals, counts) == oracle.OK
    assert_same(a, o, "valid round")
    in_use = pool.stats()["in_use"]
    counts2 = rng.integers(1, 17, size=V * chunk, dtype=np.uint8)
    total2 = int(counts2.sum(dtype=np.uint64))
    vals2, _ = wl.random_round(rng, total2, 1.0, 8)
    a.insert_packed(dev(vals2), dev(counts2), n_values=total2 - 1)
    assert a.last_error() == G.ERANGE
    np.testing.assert_array_equal(a.vector_sizes().cpu().numpy().astype(np.uint64), o.vector_sizes())
    np.testing.assert_array_equal(G.as_unsigned(a.flatten()), o.flatten())
    assert a.capacity(check_error=False) == o.capacity()
    assert pool.stats()["in_use"] == in_use
    a.close()
    o.close()
