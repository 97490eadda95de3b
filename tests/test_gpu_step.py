"""GPU parity of the persistent step (gga_batch_step: insertion rounds, r/w and
flatten of every array of a batch in one launch): bit-exact against the CPU
oracle and against the per-round batch calls on twin arrays, for the
configuration-1 shape, uneven batches of keyed rounds, uint64 round-tag rounds,
more LFVectors than the step's prefix chunks (several LFVectors per chunk),
several tiles per LFVector, a step on a non-empty state, a step without r/w or
flatten, a too-small output, replays of a captured step, and the step with a
clear in the same launch against a clear followed by the step."""
import numpy as np
import pytest
import torch

import oracle
from oracle import Oracle
from paper_2209_00103_amd import workloads as wl
from tests.gpu_util import gg, gpu_flat, gpu_sizes

pytestmark = pytest.mark.gpu
MiB = 1 << 20


@pytest.fixture
def pool():
    p = gg().Pool(2048 * MiB)
    yield p
    p.close()


def _oracle_rounds(oracles, kind, gens, counts, elem_op=oracle.OP_ADD1, rw=True):
    for r, g in enumerate(gens):
        for i, o in enumerate(oracles):
            if kind[r] == "keyed":
                o.insert_gen(oracle.GEN_KEYED, counts[r][i], seed=g.seed, round=g.round, tag=g.tag + i,
                             tag_shift=g.tag_shift)
            elif kind[r] == "bern":
                o.insert_gen(oracle.GEN_BERNOULLI, counts[r][i], seed=g.seed, round=g.round)
            else:
                o.insert_gen(oracle.GEN_ROUND_TAG, counts[r][i], round=g.round, tag_shift=g.tag_shift)
    if rw:
        for o in oracles:
            o.rw(elem_op)


def _check_flat(out, oracles, what):
    ref = np.concatenate([o.flatten() for o in oracles])
    got = gg().as_unsigned(out[:ref.size])
    if not np.array_equal(got, ref):
        bad = np.nonzero(got != ref)[0]
        raise AssertionError(f"{what}: {bad.size} elements differ, first at {bad[:8]}")


def test_step_configuration_1_matches_oracle(pool):
    """256 LFVectors, first bucket 1024, uint32, 2^18 threads per round with
    probability 1/2 over 4 rounds, r/w x + 1, flatten; then a second step on top."""
    G = gg()
    cfg = wl.CFG1
    a = G.GGArray(pool, 4, cfg["V"], cfg["F"])
    o = Oracle(4, cfg["V"], cfg["F"])
    b = G.Batch([a])
    n = cfg["n_threads"]
    out = torch.empty(2 * cfg["rounds"] * n, dtype=torch.int32, device="cuda")
    for step in range(2):
        print(f"case step cfg1 pass {step}", flush=True)
        gens = [G.make_gen(G.GEN_BERNOULLI, seed=1, round=4 * step + r) for r in range(cfg["rounds"])]
        b.step(gens, [[n]] * cfg["rounds"], G.ADD1, out)
        _oracle_rounds([o], ["bern"] * 4, gens, [[n]] * 4)
        assert b.last_error() == 0 and a.last_error() == 0
        np.testing.assert_array_equal(gpu_sizes(a), o.vector_sizes())
        _check_flat(out, [o], f"pass {step}")
        np.testing.assert_array_equal(gpu_flat(a), o.flatten())
        assert a.capacity() == o.capacity()
    b.close()
    a.close()


SHAPES = [(1, 64), (4, 1024), (16, 256), (1, 16384), (64, 128), (7, 2048), (3, 1), (200, 8)]  # (V, F)


def test_step_keyed_batch_matches_rounds_and_oracle(pool):
    G = gg()
    arrays = [G.GGArray(pool, 4, V, F) for V, F in SHAPES]
    twins = [G.GGArray(pool, 4, V, F) for V, F in SHAPES]
    oracles = [Oracle(4, V, F) for V, F in SHAPES]
    b, bt = G.Batch(arrays), G.Batch(twins)
    rng = np.random.default_rng(11)
    counts = []
    for r in range(4):
        n = [int(x) for x in rng.integers(0, 30000, size=len(SHAPES))]
        n[r % len(n)] = 0  # an array that skips the round
        n[-1] = int(rng.integers(0, 150))  # fewer threads than LFVectors
        counts.append(n)
    gens = [G.make_gen(G.GEN_KEYED, seed=5, round=r, tag=100) for r in range(4)]
    total = sum(sum(c) for c in counts)
    out = torch.full((total + 17,), -1, dtype=torch.int32, device="cuda")
    b.step(gens, counts, G.ADD1, out)
    for r in range(4):
        bt.insert_gen(gens[r], counts[r])
    bt.rw(G.ADD1)
    out2 = torch.empty(total, dtype=torch.int32, device="cuda")
    bt.flatten_into(out2)
    _oracle_rounds(oracles, ["keyed"] * 4, gens, counts)
    assert b.last_error() == 0
    assert torch.equal(out[:total], out2)
    assert int((out[total:] == -1).sum()) == 17  # nothing past the flatten
    _check_flat(out, oracles, "step")
    for i, (a, t, o) in enumerate(zip(arrays, twins, oracles)):
        np.testing.assert_array_equal(gpu_sizes(a), o.vector_sizes(), err_msg=f"array {i}")
        assert a.capacity() == t.capacity() == o.capacity(), f"array {i}"
    # the per-round calls continue from the step's state
    b.insert_gen(G.make_gen(G.GEN_KEYED, seed=5, round=9, tag=100), counts[0])
    _oracle_rounds(oracles, ["keyed"], [G.make_gen(G.GEN_KEYED, seed=5, round=9, tag=100)], [counts[0]], rw=False)
    for i, (a, o) in enumerate(zip(arrays, oracles)):
        np.testing.assert_array_equal(gpu_flat(a), o.flatten(), err_msg=f"array {i} after a round")
    b.close()
    bt.close()
    for a in arrays + twins:
        a.close()


def test_step_round_tag_u64_many_lfvectors_and_tiles(pool):
    """uint64 round-tag rounds over 3000 + 4 LFVectors (more than the step's 1024
    prefix chunks) and an array whose LFVectors get several tiles per round."""
    G = gg()
    shapes = [(1500, 16), (4, 1), (1500, 64)]
    arrays = [G.GGArray(pool, 8, V, F) for V, F in shapes]
    oracles = [Oracle(8, V, F) for V, F in shapes]
    b = G.Batch(arrays)
    counts = [[1500 * 37 + 5, 4 * 2500 + 3, 1500 * 3], [0, 4 * 1024, 1500 * 40 + 1], [777, 13, 1500]]
    gens = [G.make_gen(G.GEN_ROUND_TAG, round=r, tag_shift=40) for r in range(3)]
    total = sum(sum(c) for c in counts)
    out = torch.empty(total, dtype=torch.int64, device="cuda")
    b.step(gens, counts, G.MUL3ADD1, out)
    _oracle_rounds(oracles, ["tag"] * 3, gens, counts, elem_op=oracle.OP_MUL3ADD1)
    assert b.last_error() == 0
    _check_flat(out, oracles, "u64 step")
    for i, (a, o) in enumerate(zip(arrays, oracles)):
        np.testing.assert_array_equal(gpu_sizes(a), o.vector_sizes(), err_msg=f"array {i}")
    b.close()
    for a in arrays:
        a.close()


def test_step_without_rw_or_flatten_and_too_small_output(pool):
    G = gg()
    arrays = [G.GGArray(pool, 4, V, F) for V, F in SHAPES[:4]]
    oracles = [Oracle(4, V, F) for V, F in SHAPES[:4]]
    b = G.Batch(arrays)
    counts = [[5000, 100, 20000, 3]]
    gens = [G.make_gen(G.GEN_BERNOULLI, seed=7, round=0)]
    b.step(gens, counts, G.RW_NONE, None)
    _oracle_rounds(oracles, ["bern"], gens, counts, rw=False)
    assert b.last_error() == 0
    for a, o in zip(arrays, oracles):
        np.testing.assert_array_equal(gpu_flat(a), o.flatten())
    total = sum(o.size() for o in oracles)
    small = torch.full((total - 1,), -1, dtype=torch.int32, device="cuda")
    b.step([], [], G.ADD1, small)  # r/w only, then a flatten that does not fit
    for o in oracles:
        o.rw(oracle.OP_ADD1)
    assert b.last_error() == G.ERANGE
    assert int((small == -1).sum()) == total - 1  # nothing written
    for a, o in zip(arrays, oracles):
        np.testing.assert_array_equal(gpu_flat(a), o.flatten())
    b.close()
    for a in arrays:
        a.close()


def test_step_graph_replays(pool):
    """A captured clear + step, replayed several times with eager work between
    the replays, gives the eager step's result every time."""
    G = gg()
    shapes = SHAPES[:6]
    arrays = [G.GGArray(pool, 4, V, F) for V, F in shapes]
    b = G.Batch(arrays)
    counts = [[3000, 9000, 400, 0, 12000, 700]] * 3
    gens = [G.make_gen(G.GEN_KEYED, seed=2, round=r, tag=7) for r in range(3)]
    total = sum(sum(c) for c in counts)
    ref = torch.empty(total, dtype=torch.int32, device="cuda")
    out = torch.empty(total, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b.shrink(1, 1)
        b.step(gens, counts, G.ADD1, ref)  # eager: uploads the counts table
        s.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            b.shrink(1, 1)
            b.step(gens, counts, G.ADD1, out)
        for k in range(4):
            out.fill_(-1)
            g.replay()
            s.synchronize()
            assert torch.equal(out, ref), f"replay {k}"
            junk = torch.arange(1 << 20, device="cuda").sum()  # eager work between replays
            assert int(junk) > 0
    assert b.last_error() == 0
    b.close()
    for a in arrays:
        a.close()


@pytest.mark.parametrize("elem", [4, 8])
def test_step_per_wave_many_lfvectors(pool, elem):
    """More than 4096 LFVectors (each wave takes its own LFVectors): keyed,
    Bernoulli and round-tag rounds, some giving an LFVector several 1024-candidate
    tiles or several buckets, then r/w and flatten; bit-exact against the
    per-round calls and the oracle."""
    G = gg()
    shapes = [(3000, 4), (1, 64), (1200, 1), (900, 256)]
    arrays = [G.GGArray(pool, elem, V, F) for V, F in shapes]
    twins = [G.GGArray(pool, elem, V, F) for V, F in shapes]
    oracles = [Oracle(elem, V, F) for V, F in shapes]
    b, bt = G.Batch(arrays), G.Batch(twins)
    counts = [[3000 * 7 + 11, 5000, 1200 * 3, 900 * 2500 + 7],
              [3000 * 2, 0, 1200 * 40 + 3, 900 * 1100],
              [12345, 70000, 1199, 900 * 3]]
    gens = [G.make_gen(G.GEN_KEYED, seed=3, round=0, tag=40),
            G.make_gen(G.GEN_BERNOULLI, seed=3, round=1),
            G.make_gen(G.GEN_ROUND_TAG, round=2, tag_shift=24)]
    kinds = ["keyed", "bern", "tag"]
    dt = torch.int32 if elem == 4 else torch.int64
    cap = sum(sum(c) for c in counts) + sum(counts[0])  # both steps' elements
    out = torch.empty(cap, dtype=dt, device="cuda")
    print(f"case step per wave elem={elem}", flush=True)
    b.step(gens, counts, G.MUL3ADD1, out)
    for r in range(3):
        bt.insert_gen(gens[r], counts[r])
    bt.rw(G.MUL3ADD1)
    _oracle_rounds(oracles, kinds, gens, counts, elem_op=oracle.OP_MUL3ADD1)
    assert b.last_error() == 0
    _check_flat(out, oracles, "per-wave step")
    for i, (a, t, o) in enumerate(zip(arrays, twins, oracles)):
        np.testing.assert_array_equal(gpu_sizes(a), o.vector_sizes(), err_msg=f"array {i}")
        np.testing.assert_array_equal(gpu_flat(t), o.flatten(), err_msg=f"twin {i}")
        assert a.capacity() == o.capacity(), f"array {i}"
    # a second step on top, without r/w
    b.step(gens[:1], counts[:1], G.RW_NONE, out)
    _oracle_rounds(oracles, kinds[:1], gens[:1], counts[:1], rw=False)
    assert b.last_error() == 0
    _check_flat(out, oracles, "second step")
    b.close()
    bt.close()
    for a in arrays + twins:
        a.close()


def _pool_counts(p):
    st = p.stats()
    return st["in_use"], st["allocs"], st["frees"]


@pytest.mark.parametrize("shapes", [[(256, 1024)], [(3000, 4), (1, 64), (1200, 1), (900, 256)]],
                         ids=["workgroup-per-lfvector", "wave-per-lfvector"])
def test_step_clear_equals_shrink_then_step(shapes):
    """gga_batch_step_clear against gga_batch_shrink(1, 1) + gga_batch_step on twin
    arrays in pools of their own, over passes that grow, shrink and grow again (so
    held buckets are taken again, left unreached and released, or joined by new
    ones): sizes, flatten, capacity and the pools' in-use bytes, allocation and
    release counts are equal, and both equal the oracle's clear and rounds."""
    G = gg()
    pa, pb = G.Pool(1024 * MiB), G.Pool(1024 * MiB)
    arrays = [G.GGArray(pa, 4, V, F) for V, F in shapes]
    twins = [G.GGArray(pb, 4, V, F) for V, F in shapes]
    oracles = [Oracle(4, V, F) for V, F in shapes]
    b, bt = G.Batch(arrays), G.Batch(twins)
    # per pass: thread counts per round, in units of V; the last pass takes the
    # buckets of the one before again round by round (reuse beyond bucket 0)
    scale = [[7, 3, 11], [1, 1, 1], [30, 2, 9], [12, 4, 20]]
    out = torch.empty(sum(V * 45 for V, _ in shapes), dtype=torch.int32, device="cuda")
    out_t = torch.empty_like(out)
    for p, sc in enumerate(scale):
        print(f"case step clear {len(shapes)} arrays pass {p}", flush=True)
        counts = [[V * k + (i % 5) for i, (V, _) in enumerate(shapes)] for k in sc]
        gens = [G.make_gen(G.GEN_KEYED, seed=7, round=3 * p, tag=0),
                G.make_gen(G.GEN_BERNOULLI, seed=7, round=3 * p + 1),
                G.make_gen(G.GEN_ROUND_TAG, round=3 * p + 2, tag_shift=24)]
        b.step(gens, counts, G.ADD1, out, clear=True)
        bt.shrink(1, 1)
        bt.step(gens, counts, G.ADD1, out_t)
        for o in oracles:
            o.shrink(1, 1)
        _oracle_rounds(oracles, ["keyed", "bern", "tag"], gens, counts)
        assert b.last_error() == 0 and bt.last_error() == 0
        _check_flat(out, oracles, f"clear pass {p}")
        _check_flat(out_t, oracles, f"twin pass {p}")
        for i, (a, t, o) in enumerate(zip(arrays, twins, oracles)):
            np.testing.assert_array_equal(gpu_sizes(a), o.vector_sizes(), err_msg=f"array {i} pass {p}")
            assert a.capacity() == t.capacity() == o.capacity(), f"array {i} pass {p}"
        assert _pool_counts(pa) == _pool_counts(pb), f"pass {p}: {pa.stats()} vs {pb.stats()}"
    b.close()
    bt.close()
    for a in arrays + twins:
        a.close()
    pa.close()
    pb.close()


def test_step_clear_under_fault_injection_matches_shrink_then_step():
    """One LFVector, one bucket per round (F = 64, rounds of 64, 128, 256 and 512
    round-tag threads), so allocation attempts come in bucket order.  A failure
    injected at the third attempt of the second pass freezes the LFVector at the
    size before that round, with the same buckets held and the same pool counts
    as the shrink-then-step twin; the next clear gives every bucket back."""
    G = gg()
    pa, pb = G.Pool(64 * MiB), G.Pool(64 * MiB)
    a, t = G.GGArray(pa, 4, 1, 64), G.GGArray(pb, 4, 1, 64)
    b, bt = G.Batch([a]), G.Batch([t])
    counts = [[64], [128], [256], [512]]
    out = torch.empty(1024, dtype=torch.int32, device="cuda")
    for p in range(3):
        print(f"case step clear fault pass {p}", flush=True)
        gens = [G.make_gen(G.GEN_ROUND_TAG, round=4 * p + r, tag_shift=20) for r in range(4)]
        if p == 1:
            pa.set_fault(pa.stats()["attempts"] + 3)
            pb.set_fault(pb.stats()["attempts"] + 3)
        b.step(gens, counts, G.RW_NONE, out, clear=True)
        bt.shrink(1, 1)
        bt.step(gens, counts, G.RW_NONE, out)
        pa.set_fault(0)
        pb.set_fault(0)
        want_err = G.ENOMEM if p >= 1 else 0
        assert a.last_error() == want_err and t.last_error() == want_err, f"pass {p}"
        want = 960 if p == 0 else (192 if p == 1 else 0)
        assert a.size(check_error=False) == t.size(check_error=False) == want, f"pass {p}"
        assert a.capacity(check_error=False) == t.capacity(check_error=False), f"pass {p}"
        assert _pool_counts(pa) == _pool_counts(pb), f"pass {p}: {pa.stats()} vs {pb.stats()}"
    assert pa.stats()["in_use"] == 0
    b.close()
    bt.close()
    a.close()
    t.close()
    pa.close()
    pb.close()
