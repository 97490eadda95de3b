"""ggarray_insert_gen_rounds: several generated insertion rounds (Alg. 1 with
Alg. 2), each followed by the same shrink, against the oracle's rounds one by one
and against the library's own calls one by one on a twin array in a pool of its
own (sizes, contents, capacity, the pool's in-use bytes and allocation and
release counts), in one launch where the rounds allow it and round by round where
they do not; argument errors leave the array as it was; a captured graph of the
rounds replays them."""
import numpy as np
import pytest
import torch

import oracle
from oracle import Oracle
from tests.gpu_util import gg

pytestmark = pytest.mark.gpu
MiB = 1 << 20


def _pool_counts(p):
    st = p.stats()
    return st["in_use"], st["allocs"], st["frees"]


def _gens(G, kind, rounds, tag_shift, seed=3, tag=0):
    if kind == "round_tag":
        return [G.make_gen(G.GEN_ROUND_TAG, round=r, tag_shift=tag_shift) for r in rounds]
    return [G.make_gen(G.GEN_KEYED, seed=seed, round=r, tag_shift=tag_shift, tag=tag) for r in rounds]


def _oracle_rounds(o, kind, rounds, ns, tag_shift, num, den, seed=3, tag=0):
    for r, n in zip(rounds, ns):
        if kind == "round_tag":
            o.insert_gen(oracle.GEN_ROUND_TAG, n, round=r, tag_shift=tag_shift)
        else:
            o.insert_gen(oracle.GEN_KEYED, n, seed=seed, round=r, tag_shift=tag_shift, tag=tag)
        if num:
            o.shrink(num, den)


CASES = {
    # V >= 512: one launch whatever the round sizes (a round of 2^19 threads gives 1024 per LFVector)
    "one-launch-V512": dict(V=512, F=64, elem=4, kind="round_tag", tag_shift=27,
                            ns=[4099, 8192, 5000, 32845, 0, 65536, 1 << 19], num=1, den=10),
    "one-launch-keyed-u64": dict(V=600, F=16, elem=8, kind="keyed", tag_shift=24,
                                 ns=[1007, 20011, 60000, 7, 150001], num=1, den=3),
    # few LFVectors, at most 8 tiles of 4096 threads each: one launch
    "one-launch-V8": dict(V=8, F=64, elem=4, kind="round_tag", tag_shift=27,
                          ns=[20000, 100003, 262144, 5], num=1, den=10),
    "one-launch-no-shrink": dict(V=700, F=1, elem=4, kind="keyed", tag_shift=30,
                                 ns=[3000, 1, 99999, 4096], num=0, den=1),
    "one-launch-clear": dict(V=512, F=1024, elem=4, kind="round_tag", tag_shift=20,
                             ns=[70000, 3, 1 << 18], num=1, den=1),
    # a round of 16 tiles per LFVector on 8 LFVectors: round by round
    "round-by-round": dict(V=8, F=64, elem=4, kind="round_tag", tag_shift=27,
                           ns=[20000, 1 << 19, 777], num=1, den=10),
}


@pytest.mark.parametrize("clear", [False, True], ids=["", "clear-first"])
@pytest.mark.parametrize("case", list(CASES))
def test_rounds_equal_the_calls_one_by_one_and_the_oracle(case, clear):
    """With clear_first the launch starts with the clear of the array the pass
    before left full, so its rounds take kept buckets again; the twin array calls
    ggarray_shrink(1, 1) first."""
    c = CASES[case]
    G = gg()
    rounds = [5 + 2 * r for r in range(len(c["ns"]))]
    gens = _gens(G, c["kind"], rounds, c["tag_shift"])
    pa, pb = G.Pool(512 * MiB), G.Pool(512 * MiB)
    a = G.GGArray(pa, c["elem"], c["V"], c["F"])
    b = G.GGArray(pb, c["elem"], c["V"], c["F"])
    o = Oracle(c["elem"], c["V"], c["F"])
    try:
        for rep in range(2):  # the second pass starts from the first's state
            print(f"case {case} pass {rep}", flush=True)
            a.insert_gen_rounds(gens, c["ns"], c["num"], c["den"], clear_first=clear)
            if clear:
                b.shrink(1, 1)
                o.shrink(1, 1)
            for g, n in zip(gens, c["ns"]):
                if c["num"]:
                    b.insert_gen_shrink(g, n, c["num"], c["den"])
                else:
                    b.insert_gen(g, n)
            _oracle_rounds(o, c["kind"], rounds, c["ns"], c["tag_shift"], c["num"], c["den"])
            ref = o.flatten()
            for arr in (a, b):
                got = G.as_unsigned(arr.flatten())
                assert got.size == ref.size and np.array_equal(got, ref), f"{case} pass {rep}"
                np.testing.assert_array_equal(arr.vector_sizes().cpu().numpy().astype(np.uint64), o.vector_sizes())
                assert arr.capacity() == o.capacity()
            assert _pool_counts(pa) == _pool_counts(pb)
        assert a.last_error() == 0 and b.last_error() == 0
    finally:
        o.close()
        a.close()
        b.close()
        pa.close()
        pb.close()


def test_rounds_argument_errors_leave_the_array_unchanged():
    G = gg()
    p = G.Pool(64 * MiB)
    a = G.GGArray(p, 4, 512, 64)
    try:
        good = _gens(G, "round_tag", [1, 2, 3], 27)
        a.insert_gen_rounds(good, [5000, 6000, 7000], 1, 10)
        before = G.as_unsigned(a.flatten()).copy()
        bad_keyed = G.make_gen(G.GEN_KEYED, seed=1, round=4, tag_shift=0)  # tag_shift must be 1..47
        for gens, ns, num, den in [
            (good[:1] + [bad_keyed] + good[1:], [100, 100, 100, 100], 1, 10),  # invalid generator in the second round
            (good, [100, 100, 100], 2, 1),                                      # num > den
            (good, [100, 100, 100], 1, 0),                                      # den == 0
            (_gens(G, "round_tag", range(17), 27), [10] * 17, 1, 10),           # more than 16 rounds
            (good, [100, 1 << 42, 100], 1, 10),                                 # 2^33 threads per LFVector
        ]:
            with pytest.raises(G.GGAError):
                a.insert_gen_rounds(gens, ns, num, den)
            assert np.array_equal(G.as_unsigned(a.flatten()), before)
        with pytest.raises(ValueError):
            a.insert_gen_rounds(good, [1, 2], 1, 10)
        a.insert_gen_rounds([], [], 1, 10)  # no rounds: nothing to do
        assert np.array_equal(G.as_unsigned(a.flatten()), before) and a.last_error() == 0
    finally:
        a.close()
        p.close()


@pytest.mark.parametrize("clear", [False, True], ids=["", "clear-first"])
def test_rounds_in_a_captured_graph_replay(clear):
    """The one-launch rounds captured in a graph: every replay, with an eager
    flatten between replays, equals the oracle's rounds; without clear_first an
    eager clear follows each check, with it each replay clears the array the one
    before filled and takes its buckets again."""
    G = gg()
    p = G.Pool(256 * MiB)
    V, F = 512, 1024
    ns = [1 << 14, 3 << 14, 1 << 17, 99999]
    rounds = [0, 1, 2, 3]
    gens = _gens(G, "round_tag", rounds, 27)
    a = G.GGArray(p, 4, V, F)
    o = Oracle(4, V, F)
    s = torch.cuda.Stream()
    try:
        with torch.cuda.stream(s):
            a.insert_gen_rounds(gens, ns, 1, 10, stream=s)  # warm-up outside the capture
            a.shrink(1, 1, stream=s)
        s.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            a.insert_gen_rounds(gens, ns, 1, 10, clear_first=clear, stream=s)
        torch.cuda.synchronize()
        for rep in range(3):
            g.replay()
            torch.cuda.synchronize()
            _oracle_rounds(o, "round_tag", rounds, ns, 27, 1, 10)
            got, ref = G.as_unsigned(a.flatten()), o.flatten()
            assert got.size == ref.size and np.array_equal(got, ref), f"replay {rep}"
            if not clear:
                a.shrink(1, 1)
            o.shrink(1, 1)
        assert a.last_error() == 0
    finally:
        o.close()
        a.close()
        p.close()


@pytest.mark.parametrize("clear", [False, True], ids=["", "clear-first"])
@pytest.mark.parametrize("V,fault_at", [(6, 1), (6, 5), (6, 20), (512, 1), (512, 400), (512, 1200)])
def test_rounds_under_a_failed_allocation(V, fault_at, clear):
    """Allocation number fault_at fails inside the one launch (with clear_first,
    after the clear of a full array, where a kept bucket's reuse may be the attempt
    that fails): the array reports GGA_ENOMEM; every LFVector holds one of the
    states its own rounds can leave it in (the rounds before its failed one, then
    no more elements but every later shrink), whichever LFVector the failure hit;
    and all its buckets go back to the pool when it is destroyed."""
    from tests.gpu_util import gpu_flat
    from tests.test_gpu_fused import _frozen_candidates

    G = gg()
    F = 32
    ns = [3000, 9000, 20000, 40000]
    rounds = [(n, 1, 10, "round_tag", r) for r, n in enumerate(ns)]
    pool = G.Pool(256 * MiB)
    before = pool.stats()
    a = G.GGArray(pool, 4, V, F)
    gens = [G.make_gen(G.GEN_ROUND_TAG, round=r, tag_shift=20) for r in range(len(ns))]
    try:
        if clear:  # a full array first: the clear keeps its buckets for the rounds under the fault
            a.insert_gen_rounds(gens, ns, 1, 10)
        pool.set_fault(fault_at)
        a.insert_gen_rounds(gens, ns, 1, 10, clear_first=clear)
        pool.set_fault(0)
        assert a.last_error() == G.ENOMEM
        cands = _frozen_candidates(4, V, F, rounds)
        pre = a.prefix().cpu().numpy().astype(np.int64)
        flat = gpu_flat(a)
        for v in range(V):
            seg = flat[pre[v]:pre[v + 1]]
            assert any(np.array_equal(seg, c) for c in cands[v]), f"LFVector {v}: not a state of its rounds"
    finally:
        a.close()
    assert pool.stats()["in_use"] == before["in_use"]
    pool.close()
