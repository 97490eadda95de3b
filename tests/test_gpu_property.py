"""Property-based GPU parity: random shapes (V, F, element size), random rounds of
every producer kind (buffer with and without flags, Bernoulli, round-tag, keyed,
per-thread counts, Poisson), random shrinks, rounds fused with their shrink,
several rounds with their shrinks in one call, and r/w passes, drawn by Hypothesis;
after every operation the GPU array must equal the CPU oracle bit for bit."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from oracle import Oracle
from paper_2209_00103_amd import workloads as wl
from tests.gpu_util import assert_same, gg

pytestmark = pytest.mark.gpu
MiB = 1 << 20

OPS = st.one_of(
    st.tuples(st.just("buffer"), st.integers(0, 70000), st.floats(0.0, 1.0), st.booleans()),
    st.tuples(st.just("bernoulli"), st.integers(0, 70000), st.integers(0, 255)),
    st.tuples(st.just("round_tag"), st.integers(0, 70000), st.integers(0, 255)),
    st.tuples(st.just("keyed"), st.integers(0, 70000), st.integers(0, 255)),
    st.tuples(st.just("counts"), st.integers(0, 20000), st.integers(1, 16)),
    st.tuples(st.just("poisson"), st.integers(0, 20000), st.integers(0, 7)),
    st.tuples(st.just("shrink"), st.integers(0, 7), st.integers(1, 7)),
    st.tuples(st.just("rw"), st.integers(0, 2)),
    st.tuples(st.just("fused"), st.integers(0, 70000), st.booleans(), st.integers(0, 7), st.integers(1, 7)),
    st.tuples(st.just("rounds"), st.lists(st.integers(0, 70000), min_size=2, max_size=4), st.booleans(),
              st.integers(0, 7), st.integers(1, 7)),
)


@pytest.fixture(scope="module")
def pool():
    p = gg().Pool(1024 * MiB)
    yield p
    p.close()


@settings(max_examples=25, deadline=None, suppress_health_check=[HealthCheck.function_scoped_fixture])
@given(elem=st.sampled_from([4, 8]), V=st.sampled_from([1, 2, 5, 64, 300, 512, 1024]),
       F_log2=st.integers(0, 12), ops=st.lists(OPS, min_size=1, max_size=6), seed=st.integers(0, 2 ** 31))
def test_random_operation_sequences_match_oracle(pool, elem, V, F_log2, ops, seed):
    G = gg()
    F = 1 << F_log2
    a, o = G.GGArray(pool, elem, V, F), Oracle(elem, V, F)
    rng = np.random.default_rng(seed)
    thr = wl.poisson_thresholds(3, 16)
    try:
        for step, op in enumerate(ops):
            kind = op[0]
            if kind == "buffer":
                n, p, with_flags = op[1], op[2], op[3]
                vals, flags = wl.random_round(rng, n, p, elem)
                if with_flags:
                    a.insert(G.to_device(vals), G.to_device(flags))
                    o.insert(vals, flags)
                else:
                    a.insert(G.to_device(vals))
                    o.insert(vals, np.ones(n, np.uint8))
            elif kind == "bernoulli":
                a.insert_gen(G.make_gen(G.GEN_BERNOULLI, seed=op[2], round=step), op[1])
                o.insert_gen(oracle.GEN_BERNOULLI, op[1], seed=op[2], round=step)
            elif kind == "round_tag":
                a.insert_gen(G.make_gen(G.GEN_ROUND_TAG, round=op[2], tag_shift=20), op[1])
                o.insert_gen(oracle.GEN_ROUND_TAG, op[1], round=op[2], tag_shift=20)
            elif kind == "keyed":
                a.insert_gen(G.make_gen(G.GEN_KEYED, seed=op[2] & 255, round=step, tag=op[2]), op[1])
                o.insert_gen(oracle.GEN_KEYED, op[1], seed=op[2] & 255, round=step, tag=op[2])
            elif kind == "counts":
                n, mx = op[1], op[2]
                counts = rng.integers(0, mx + 1, size=n).astype(np.uint8)
                if elem == 4:
                    vals = rng.integers(0, 1 << 32, size=n * mx, dtype=np.uint64).astype(np.uint32)
                else:
                    vals = rng.integers(0, np.iinfo(np.uint64).max, size=n * mx, dtype=np.uint64)
                a.insert_counts(G.to_device(vals), G.to_device(counts), mx)
                o.insert_counts(vals, counts, mx)
            elif kind == "poisson":
                a.insert_gen(G.make_gen(G.GEN_POISSON, seed=1, round=op[2], max_count=16, thresholds=thr), op[1])
                o.insert_gen(oracle.GEN_POISSON, op[1], seed=1, round=op[2], max_count=16, thresholds=thr)
            elif kind == "shrink":
                num, den = min(op[1], op[2]), op[2]
                a.shrink(num, den)
                o.shrink(num, den)
            elif kind == "fused":  # a round and its shrink in one call
                n, keyed, num, den = op[1], op[2], min(op[3], op[4]), op[4]
                if keyed:
                    a.insert_gen_shrink(G.make_gen(G.GEN_KEYED, seed=9, round=step, tag=5), n, num, den)
                    o.insert_gen(oracle.GEN_KEYED, n, seed=9, round=step, tag=5)
                else:
                    a.insert_gen_shrink(G.make_gen(G.GEN_ROUND_TAG, round=step, tag_shift=20), n, num, den)
                    o.insert_gen(oracle.GEN_ROUND_TAG, n, round=step, tag_shift=20)
                o.shrink(num, den)
            elif kind == "rounds":  # several rounds, each with the same shrink, in one call
                ns, keyed, num, den = op[1], op[2], min(op[3], op[4]), op[4]
                rs = [16 * step + k for k in range(len(ns))]
                if keyed:
                    a.insert_gen_rounds([G.make_gen(G.GEN_KEYED, seed=9, round=r, tag=5) for r in rs], ns, num, den)
                else:
                    a.insert_gen_rounds([G.make_gen(G.GEN_ROUND_TAG, round=r, tag_shift=20) for r in rs], ns,
                                        num, den)
                for r, n in zip(rs, ns):
                    if keyed:
                        o.insert_gen(oracle.GEN_KEYED, n, seed=9, round=r, tag=5)
                    else:
                        o.insert_gen(oracle.GEN_ROUND_TAG, n, round=r, tag_shift=20)
                    if num:
                        o.shrink(num, den)
            else:
                a.rw(op[1])
                o.rw(op[1])
            assert_same(a, o, f"step {step} {op}")
    finally:
        a.close()
        o.close()


BATCH_OPS = st.one_of(
    st.tuples(st.just("keyed"), st.lists(st.integers(0, 40000), min_size=8, max_size=8), st.integers(0, 255)),
    st.tuples(st.just("round_tag"), st.lists(st.integers(0, 40000), min_size=8, max_size=8), st.integers(0, 255)),
    st.tuples(st.just("bernoulli"), st.lists(st.integers(0, 40000), min_size=8, max_size=8), st.integers(0, 255)),
    st.tuples(st.just("shrink"), st.integers(0, 5), st.integers(1, 5)),
    st.tuples(st.just("rw"), st.integers(0, 2)),
    st.tuples(st.just("single"), st.integers(0, 7), st.integers(0, 30000)),  # one member alone, then batch again
)


@settings(max_examples=15, deadline=None, suppress_health_check=[HealthCheck.function_scoped_fixture])
@given(elem=st.sampled_from([4, 8]),
       shapes=st.lists(st.tuples(st.sampled_from([1, 3, 16, 200, 1024]), st.integers(0, 11)), min_size=1, max_size=8),
       ops=st.lists(BATCH_OPS, min_size=1, max_size=6), grid=st.sampled_from([0, 1, 5, 4096]))
def test_random_batch_sequences_match_oracle(pool, elem, shapes, ops, grid):
    """Batches of up to 8 arrays of random shapes through random sequences of batched
    rounds, shrinks and r/w passes (and single-array calls on members in between);
    after each operation every array, and the batch flatten with its offsets, must
    equal the oracles."""
    import torch

    G = gg()
    arrays = [G.GGArray(pool, elem, V, 1 << f) for V, f in shapes]
    oracles = [Oracle(elem, V, 1 << f) for V, f in shapes]
    b = G.Batch(arrays)
    b.set_grid(grid)
    n = len(arrays)
    dt = torch.int32 if elem == 4 else torch.int64
    try:
        for step, op in enumerate(ops):
            kind = op[0]
            if kind in ("keyed", "round_tag", "bernoulli"):
                counts = [int(c) for c in op[1][:n]]
                if kind == "keyed":
                    b.insert_gen(G.make_gen(G.GEN_KEYED, seed=op[2], round=step, tag=3), counts)
                    for i, o in enumerate(oracles):
                        o.insert_gen(oracle.GEN_KEYED, counts[i], seed=op[2], round=step, tag=3 + i)
                elif kind == "round_tag":
                    b.insert_gen(G.make_gen(G.GEN_ROUND_TAG, round=op[2], tag_shift=20), counts)
                    for i, o in enumerate(oracles):
                        o.insert_gen(oracle.GEN_ROUND_TAG, counts[i], round=op[2], tag_shift=20)
                else:
                    b.insert_gen(G.make_gen(G.GEN_BERNOULLI, seed=op[2], round=step), counts)
                    for i, o in enumerate(oracles):
                        o.insert_gen(oracle.GEN_BERNOULLI, counts[i], seed=op[2], round=step)
            elif kind == "shrink":
                num, den = min(op[1], op[2]), op[2]
                b.shrink(num, den)
                for o in oracles:
                    o.shrink(num, den)
            elif kind == "rw":
                b.rw(op[1])
                for o in oracles:
                    o.rw(op[1])
            else:
                i = op[1] % n
                arrays[i].insert_gen(G.make_gen(G.GEN_ROUND_TAG, round=200 + step, tag_shift=20), op[2])
                oracles[i].insert_gen(oracle.GEN_ROUND_TAG, op[2], round=200 + step, tag_shift=20)
            total = sum(int(o.size()) for o in oracles)
            out = torch.zeros(max(total, 1), dtype=dt, device="cuda")
            b.flatten_into(out)
            offs = b.offsets().cpu().numpy()
            got = G.as_unsigned(out)
            assert b.last_error() == 0, f"step {step} {kind}: batch error"
            for i, o in enumerate(oracles):
                ref = o.flatten()
                assert offs[i + 1] - offs[i] == ref.size, f"step {step} {kind}: array {i} size"
                assert np.array_equal(got[offs[i]:offs[i + 1]], ref), f"step {step} {kind}: array {i}"
                assert_same(arrays[i], o, f"step {step} {kind}: array {i}")
    finally:
        b.close()
        for a, o in zip(arrays, oracles):
            a.close()
            o.close()
