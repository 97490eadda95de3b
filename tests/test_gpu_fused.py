"""ggarray_insert_gen_shrink: an insertion round and a shrink in one call (one
launch where the round runs one wave per LFVector).  It must leave exactly what
ggarray_insert_gen followed by ggarray_shrink leaves: sizes, contents, prefix,
capacity and the pool's allocation and release counts, checked against the CPU
oracle running the two operations one after the other."""
import numpy as np
import pytest
import torch

import oracle
from oracle import Oracle
from tests.gpu_util import assert_same, gg, gpu_flat

pytestmark = pytest.mark.gpu
MiB = 1 << 20


@pytest.fixture
def pool():
    p = gg().Pool(512 * MiB)
    yield p
    p.close()


def _gen(G, kind, r):
    if kind == "round_tag":
        return G.make_gen(G.GEN_ROUND_TAG, round=r, tag_shift=20), dict(kind=oracle.GEN_ROUND_TAG, round=r, tag_shift=20)
    if kind == "keyed":
        return G.make_gen(G.GEN_KEYED, seed=7, round=r, tag=2), dict(kind=oracle.GEN_KEYED, seed=7, round=r, tag=2)
    return G.make_gen(G.GEN_BERNOULLI, seed=5, round=r), dict(kind=oracle.GEN_BERNOULLI, seed=5, round=r)


# (elem, V, F, rounds of (threads, num, den, payload)): fused launches (at most 8
# tiles per LFVector, or V >= 512), rounds too large to fuse (more than 8 tiles per
# LFVector with V < 512), Bernoulli rounds (never fused), empty rounds, rounds with
# fewer threads than LFVectors, pops larger than the round, full clears, F = 1.
CASES = [
    (4, 8, 64, [(100000, 1, 10, "round_tag"), (5, 1, 10, "keyed"), (0, 1, 3, "round_tag"),
                (400000, 3, 4, "keyed"), (7, 1, 1, "round_tag"), (90000, 1, 2, "bernoulli"),
                (65536, 0, 4, "keyed"), (30000, 9, 10, "round_tag")]),
    (8, 512, 16, [(131072, 1, 10, "round_tag"), (262144, 1, 10, "keyed"), (300, 1, 10, "round_tag"),
                  (1 << 20, 2, 3, "keyed"), (100, 1, 1, "keyed"), (4 << 20, 1, 10, "round_tag")]),
    (4, 700, 1024, [(1 << 21, 1, 10, "keyed"), (699, 1, 2, "round_tag"), (1 << 22, 1, 10, "round_tag")]),
    (4, 3, 1, [(20000, 1, 10, "round_tag"), (3, 1, 2, "keyed"), (50000, 2, 5, "keyed"), (1, 1, 1, "round_tag")]),
    (8, 1, 4096, [(4096 * 8, 1, 10, "round_tag"), (4096 * 8 + 1, 1, 10, "keyed"), (12345, 1, 1, "keyed")]),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_fused_rounds_equal_insert_then_shrink(pool, case):
    G = gg()
    elem, V, F, rounds = CASES[case]
    a, o = G.GGArray(pool, elem, V, F), Oracle(elem, V, F)
    before = pool.stats()
    try:
        for r, (n, num, den, kind) in enumerate(rounds):
            gen, og = _gen(G, kind, r)
            a.insert_gen_shrink(gen, n, num, den)
            o.insert_gen(og.pop("kind"), n, **og)
            o.shrink(num, den)
            assert_same(a, o, f"round {r} ({n} threads, shrink {num}/{den}, {kind})")
            st = pool.stats()
            assert st["allocs"] - before["allocs"] == o.alloc_count(), f"round {r}: allocations"
            assert st["frees"] - before["frees"] == o.free_count(), f"round {r}: releases"
    finally:
        a.close()
        o.close()
    assert pool.stats()["in_use"] == before["in_use"]


def test_fused_matches_separate_calls_on_the_gpu(pool):
    """The configuration-2 rounds (512 LFVectors, 2^17 .. 2^22 threads, shrink 1/10)
    through the fused call and through the two calls give identical arrays."""
    G = gg()
    a, b = G.GGArray(pool, 4, 512, 1024), G.GGArray(pool, 4, 512, 1024)
    for r, n in enumerate([1 << 17] + [1 << (16 + k) for k in range(1, 7)]):
        gen = G.make_gen(G.GEN_ROUND_TAG, round=r, tag_shift=27)
        a.insert_gen_shrink(gen, n, 1, 10)
        b.insert_gen(gen, n)
        b.shrink(1, 10)
    assert np.array_equal(gpu_flat(a), gpu_flat(b))
    assert np.array_equal(a.vector_sizes().cpu().numpy(), b.vector_sizes().cpu().numpy())
    assert a.capacity() == b.capacity()
    a.close()
    b.close()


def test_fused_rejects_bad_fractions(pool):
    G = gg()
    a = G.GGArray(pool, 4, 4, 16)
    gen = G.make_gen(G.GEN_ROUND_TAG, round=0, tag_shift=20)
    for num, den in ((1, 0), (3, 2)):
        with pytest.raises(G.GGAError):
            a.insert_gen_shrink(gen, 1000, num, den)
    assert a.size() == 0
    a.close()


def _frozen_candidates(elem, V, F, rounds):
    """Per LFVector, every state the fused rounds can leave it in when its growth
    fails in some round: the oracle's contents after the earlier rounds, cut by
    that round's shrink and every later one (a frozen LFVector takes no elements
    but is still shrunk), plus the state with no failure."""
    o = Oracle(elem, V, F)
    before = []
    for n, num, den, kind, r in rounds:
        pre = o.prefix().astype(np.int64)
        flat = o.flatten()
        before.append([flat[pre[v]:pre[v + 1]].copy() for v in range(V)])
        gen = {"kind": oracle.GEN_KEYED if kind == "keyed" else oracle.GEN_ROUND_TAG, "round": r}
        if kind == "keyed":
            gen.update(seed=7, tag=2)
        else:
            gen.update(tag_shift=20)
        o.insert_gen(gen.pop("kind"), n, **gen)
        o.shrink(num, den)
    pre = o.prefix().astype(np.int64)
    flat = o.flatten()
    cands = [[flat[pre[v]:pre[v + 1]].copy()] for v in range(V)]
    for fail, state in enumerate(before):
        for v in range(V):
            seg = state[v]
            for n, num, den, _, _ in rounds[fail:]:
                s = seg.size
                seg = seg[:s - (s // den) * num - ((s % den) * num) // den]
            cands[v].append(seg)
    o.close()
    return cands


@pytest.mark.parametrize("fault_at", [1, 3, 8, 20])
def test_fused_rounds_under_a_failed_allocation(pool, fault_at):
    """Allocation number fault_at fails: the array reports GGA_ENOMEM, every
    LFVector holds one of the states the two-call sequence can leave, and all its
    buckets go back to the pool when it is destroyed."""
    G = gg()
    V, F = 6, 32
    rounds = [(3000, 1, 10, "round_tag", 0), (9000, 1, 4, "keyed", 1), (20000, 1, 10, "round_tag", 2),
              (40000, 1, 3, "keyed", 3)]
    before = pool.stats()
    a = G.GGArray(pool, 4, V, F)
    pool.set_fault(fault_at)
    for n, num, den, kind, r in rounds:
        gen = _gen(G, kind, r)[0]
        a.insert_gen_shrink(gen, n, num, den)
    pool.set_fault(0)
    assert a.last_error() == G.ENOMEM
    cands = _frozen_candidates(4, V, F, rounds)
    pre = a.prefix().cpu().numpy().astype(np.int64)
    flat = gpu_flat(a)
    for v in range(V):
        seg = flat[pre[v]:pre[v + 1]]
        assert any(np.array_equal(seg, c) for c in cands[v]), f"LFVector {v}: not a state of the two calls"
    a.close()
    assert pool.stats()["in_use"] == before["in_use"]


def test_fused_step_as_a_graph(pool):
    """Fused rounds, r/w and flatten captured once and replayed after an eager clear:
    every replay equals the oracle."""
    G = gg()
    V, F = 512, 1024
    a, o = G.GGArray(pool, 4, V, F), Oracle(4, V, F)
    ns = [1 << 17, 1 << 17, 1 << 18, 1 << 19, 1 << 20]
    gens = [G.make_gen(G.GEN_ROUND_TAG, round=r, tag_shift=27) for r in range(len(ns))]
    out = torch.zeros(sum(ns), dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for gen, n in zip(gens, ns):
            a.insert_gen_shrink(gen, n, 1, 10)
        a.shrink(1, 1)
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for gen, n in zip(gens, ns):
            a.insert_gen_shrink(gen, n, 1, 10)
        a.rw(G.MUL3ADD1)
        a.flatten_into(out)
    for rep in range(3):
        a.shrink(1, 1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        o.shrink(1, 1)
        for r, n in enumerate(ns):
            o.insert_gen(oracle.GEN_ROUND_TAG, n, round=r, tag_shift=27)
            o.shrink(1, 10)
        o.rw(oracle.OP_MUL3ADD1)
        ref = o.flatten()
        assert np.array_equal(G.as_unsigned(out[:ref.size]), ref), f"replay {rep}"
        assert_same(a, o, f"replay {rep}")
    a.close()
    o.close()
