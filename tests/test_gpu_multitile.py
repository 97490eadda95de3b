"""GPU parity of the multi-element insertion when an LFVector's share of a round
spans several 1024-thread tiles: the per-LFVector tickets and the decoupled
look-back that chain the tiles of one LFVector (the block prefix sum of Sec. III-B
with one size update per LFVector and round, Alg. 1).  Seeded, deterministic
shapes; every comparison against the CPU oracle is bit-exact (sizes, contents,
prefix, capacity).  Also: the failure path of an expired bounded wait, forced from
the host with a tiny poll limit, leaves every LFVector it does not freeze exact."""
import numpy as np
import pytest
import torch

import oracle
from oracle import Oracle
from paper_2209_00103_amd import workloads as wl
from tests.gpu_util import assert_same, both, dev, gg, gpu_flat, gpu_sizes

pytestmark = pytest.mark.gpu

MiB = 1 << 20
TILE = 1024  # logical threads per tile of the multi-element kernel


@pytest.fixture
def pool():
    p = gg().Pool(2048 * MiB)
    yield p
    p.close()


# elem, V, F, threads per LFVector (chunk), max_count
COUNT_CASES = [
    (4, 1, 1, 9 * TILE + 333, 16),      # one LFVector, 10 tiles, F = 1: many buckets per tile
    (8, 1, 1024, 40 * TILE + 1, 3),     # 41 tiles, last tile of one thread
    (4, 4, 1024, 7 * TILE + 500, 16),   # 8 tiles per LFVector, ragged
    (8, 4, 1, 3 * TILE, 5),             # exact multiple of the tile
    (4, 512, 1024, 3 * TILE + 77, 16),  # 512 LFVectors of 4 tiles
    (8, 512, 1, 2 * TILE + 9, 2),       # 512 LFVectors, F = 1
]


@pytest.mark.parametrize("elem,V,F,chunk,mc", COUNT_CASES)
def test_insert_counts_multi_tile(pool, elem, V, F, chunk, mc):
    print(f"case counts elem={elem} V={V} F={F} chunk={chunk} max={mc}", flush=True)
    rng = np.random.default_rng(1000 + V * 7 + F + chunk)
    a, o = both(elem, V, F, pool)
    n = V * chunk
    for r in range(3):
        counts = rng.integers(0, mc + 1, size=n, dtype=np.uint8)
        if r == 1:
            counts[rng.random(n) < 0.6] = 0  # sparse round: many tiles count few elements
        if r == 2:
            counts[: n // 3] = 0  # whole tiles with nothing to insert
        vals, _ = wl.random_round(rng, n * mc, 1.0, elem)
        a.insert_counts(dev(vals), dev(counts), mc)
        o.insert_counts(vals, counts, mc)
        assert_same(a, o, f"round {r}")
        if r == 1:
            a.shrink(1, 3)
            o.shrink(1, 3)
            assert_same(a, o, "shrink")
    a.close()
    assert pool.stats()["in_use"] == 0


POISSON_CASES = [  # elem, V, F, threads per LFVector
    (8, 1, 1024, 12 * TILE + 5),
    (4, 4, 1, 5 * TILE + 999),
    (8, 4, 1024, 16 * TILE),
    (8, 512, 1024, 3 * TILE + 1),
    (4, 512, 1, 2 * TILE + 600),
]


@pytest.mark.parametrize("elem,V,F,chunk", POISSON_CASES)
def test_poisson_multi_tile(pool, elem, V, F, chunk):
    """The configuration-3 producer (Poisson(3) counts capped at 16, generated
    payloads) over several tiles per LFVector, with r/w +1 after each round."""
    print(f"case poisson elem={elem} V={V} F={F} chunk={chunk}", flush=True)
    G = gg()
    thr = wl.poisson_thresholds(3, 16)
    a, o = both(elem, V, F, pool)
    n = V * chunk
    for i in range(3):
        a.insert_gen(G.make_gen(G.GEN_POISSON, seed=7, round=i, max_count=16, thresholds=thr), n)
        o.insert_gen(oracle.GEN_POISSON, n, seed=7, round=i, max_count=16, thresholds=thr)
        a.rw(G.ADD1)
        o.rw(oracle.OP_ADD1)
        assert_same(a, o, f"phase {i}")
    a.close()
    assert pool.stats()["in_use"] == 0


@pytest.mark.parametrize("polls", [1, 64, 1024, 16384])
def test_expired_wait_freezes_only_its_lfvectors(pool, polls):
    """A small poll limit makes look-back and bucket waits give up early (the path a
    logic error would take); how many do depends on timing.  Whatever the outcome:
    the sticky status is GGA_EHIP exactly when some LFVector froze, every LFVector
    left unfrozen holds exactly the oracle's contents, and a frozen LFVector
    ignores later rounds.  Frozen LFVectors are told apart by a following round in
    which every thread inserts at least one element."""
    G = gg()
    elem, V, F, chunk, mc = 4, 64, 1, 8 * TILE + 17, 4
    n = V * chunk
    rng = np.random.default_rng(4242 + polls)
    a = G.GGArray(pool, elem, V, F)
    o = Oracle(elem, V, F, forms=oracle.FORM_LIST)
    a.set_spin_limit(polls)
    counts1 = rng.integers(0, mc + 1, size=n, dtype=np.uint8)
    vals1, _ = wl.random_round(rng, n * mc, 1.0, elem)
    a.insert_counts(dev(vals1), dev(counts1), mc)
    a.set_spin_limit(0)  # back to the default for the probe round
    err = a.last_error()
    counts2 = rng.integers(1, mc + 1, size=n, dtype=np.uint8)
    vals2, _ = wl.random_round(rng, n * mc, 1.0, elem)
    after1 = gpu_sizes(a)
    a.insert_counts(dev(vals2), dev(counts2), mc)
    after2 = gpu_sizes(a)
    o.insert_counts(vals1, counts1, mc)
    o.insert_counts(vals2, counts2, mc)
    frozen = after2 == after1
    print(f"polls {polls}: frozen LFVectors {int(frozen.sum())} of {V}, status {err}", flush=True)
    assert err == (G.EHIP if frozen.any() else 0)
    ref_sizes = o.vector_sizes()
    np.testing.assert_array_equal(after2[~frozen], ref_sizes[~frozen])
    pre = a.prefix().cpu().numpy()
    flat_t = torch.empty(max(int(pre[V]), 1), dtype=torch.int32, device="cuda")
    a.flatten_into(flat_t[: int(pre[V])])
    flat = G.as_unsigned(flat_t[: int(pre[V])])
    ref = o.flatten()
    rpre = o.prefix()
    for v in np.nonzero(~frozen)[0]:
        got = flat[int(pre[v]):int(pre[v + 1])]
        want = ref[int(rpre[v]):int(rpre[v + 1])]
        assert np.array_equal(got, want), f"LFVector {v} (not frozen) differs"
    o.close()
    a.close()
    assert pool.stats()["in_use"] == 0
