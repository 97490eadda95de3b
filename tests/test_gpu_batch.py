"""GPU parity of batches (one launch per phase for many arrays) and of HIP-graph
replays, against the CPU oracle and against eager single-array calls."""
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
    p = gg().Pool(1024 * MiB)
    yield p
    p.close()


SHAPES = [(1, 64), (4, 1024), (16, 256), (1, 16384), (64, 128), (7, 2048), (3, 1)]  # (V, F)


def _sizes(rng, k):
    return [int(x) for x in rng.integers(0, 60000, size=k)]


def test_batch_keyed_rounds_match_oracle(pool):
    G = gg()
    arrays = [G.GGArray(pool, 4, V, F) for V, F in SHAPES]
    oracles = [Oracle(4, V, F) for V, F in SHAPES]
    b = G.Batch(arrays)
    rng = np.random.default_rng(3)
    for r in range(4):
        n = _sizes(rng, len(arrays))
        n[r % len(n)] = 0  # an array that skips the round
        b.insert_gen(G.make_gen(G.GEN_KEYED, seed=5, round=r, tag=100), n)
        for i, o in enumerate(oracles):
            o.insert_gen(oracle.GEN_KEYED, n[i], seed=5, round=r, tag=100 + i)
    b.rw(G.ADD1)
    for o in oracles:
        o.rw(oracle.OP_ADD1)
    for i, (a, o) in enumerate(zip(arrays, oracles)):
        np.testing.assert_array_equal(gpu_sizes(a), o.vector_sizes(), err_msg=f"array {i}")
        np.testing.assert_array_equal(gpu_flat(a), o.flatten(), err_msg=f"array {i}")
        assert a.capacity() == o.capacity()
    offs = b.offsets().cpu().numpy()
    total = int(offs[-1])
    out = torch.empty(total, dtype=torch.int32, device="cuda")
    b.flatten_into(out)
    assert b.last_error() == 0
    got = G.as_unsigned(out)
    ref = np.concatenate([o.flatten() for o in oracles])
    np.testing.assert_array_equal(got, ref)
    np.testing.assert_array_equal(offs, np.concatenate([[0], np.cumsum([o.size() for o in oracles])]))
    small = torch.empty(total - 1, dtype=torch.int32, device="cuda")
    b.flatten_into(small)
    assert b.last_error() == G.ERANGE
    b.close()
    for a in arrays:
        a.close()


def test_batch_round_tag_and_bernoulli_match_single_calls(pool):
    G = gg()
    a1 = [G.GGArray(pool, 8, V, F) for V, F in SHAPES]
    a2 = [G.GGArray(pool, 8, V, F) for V, F in SHAPES]
    b = G.Batch(a1)
    rng = np.random.default_rng(9)
    for r in range(3):
        n = _sizes(rng, len(a1))
        g = G.make_gen(G.GEN_BERNOULLI if r % 2 else G.GEN_ROUND_TAG, seed=3, round=r, tag_shift=40)
        b.insert_gen(g, n)
        for i, a in enumerate(a2):
            a.insert_gen(g, n[i])
    for x, y in zip(a1, a2):
        np.testing.assert_array_equal(gpu_flat(x), gpu_flat(y))
    b.close()
    for a in a1 + a2:
        a.close()


def _graph_step(G, arrays, b, rounds, out):
    for a in arrays:
        a.shrink(1, 1)
    for r, n in enumerate(rounds):
        b.insert_gen(G.make_gen(G.GEN_KEYED, seed=1, round=r, tag=0), n)
    b.rw(G.ADD1)
    b.flatten_into(out)


def test_batch_graph_replays_equal_eager(pool):
    """Capture clear + 4 batched rounds + r/w + flatten once; every replay gives the
    eager result (replays interleaved with eager work and synchronisations)."""
    G = gg()
    arrays = [G.GGArray(pool, 4, V, F) for V, F in SHAPES]
    b = G.Batch(arrays)
    rng = np.random.default_rng(1)
    rounds = [_sizes(rng, len(arrays)) for _ in range(4)]
    total = sum(sum(r[i] for r in rounds) for i in range(len(arrays)))
    out = torch.zeros(total, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        _graph_step(G, arrays, b, rounds, out)  # eager: sizes every table and status buffer
    s.synchronize()
    eager = G.as_unsigned(out).copy()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        _graph_step(G, arrays, b, rounds, out)
    for rep in range(3):
        out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(G.as_unsigned(out), eager, err_msg=f"replay {rep}")
        tmp = G.GGArray(pool, 4, 3, 8)  # unrelated eager work between replays
        tmp.insert_gen(G.make_gen(G.GEN_ROUND_TAG, round=rep, tag_shift=20), 9999)
        tmp.close()
    assert b.last_error() == 0
    b.close()
    for a in arrays:
        a.close()


def test_single_array_graph_replays_equal_eager(pool):
    """The configuration-2 step (12 rounds with shrink, r/w, flatten) at 1/64 scale,
    captured and replayed."""
    G = gg()
    V = 8
    a = G.GGArray(pool, 4, V, 1024)
    rounds = [n // 64 for n in wl.cfg2_round_threads()]
    gens = [G.make_gen(G.GEN_ROUND_TAG, round=r, tag_shift=27) for r in range(12)]
    o = Oracle(4, V, 1024)
    for r, n in enumerate(rounds):
        o.insert_gen(oracle.GEN_ROUND_TAG, n, round=r, tag_shift=27)
        o.shrink(1, 10)
    o.rw(oracle.OP_MUL3ADD1)
    ref = o.flatten()
    out = torch.zeros(ref.size, dtype=torch.int32, device="cuda")
    pre = torch.zeros(V + 1, dtype=torch.int64, device="cuda")

    def step():
        a.shrink(1, 1)
        for r, n in enumerate(rounds):
            a.insert_gen(gens[r], n)
            a.shrink(1, 10)
        a.prefix_into(pre)
        a.rw(G.MUL3ADD1)
        a.flatten_into(out)

    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        step()
    s.synchronize()
    np.testing.assert_array_equal(G.as_unsigned(out), ref)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        step()
    for rep in range(3):
        out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(G.as_unsigned(out), ref, err_msg=f"replay {rep}")
    assert a.last_error() == 0
    a.close()


def test_results_do_not_depend_on_launch_shape(pool):
    """The same batched rounds, r/w and flatten under every streaming grid (1
    workgroup up to 131072, and the default) give identical outputs; so do single
    arrays that differ only in their first-bucket size."""
    G = gg()
    rng = np.random.default_rng(5)
    rounds = [_sizes(rng, len(SHAPES)) for _ in range(3)]
    total = sum(sum(r[i] for r in rounds) for i in range(len(SHAPES)))
    ref = None
    for grid in (0, 1, 3, 4096, 131072):
        arrays = [G.GGArray(pool, 4, V, F) for V, F in SHAPES]
        b = G.Batch(arrays)
        b.set_grid(grid)
        for r, n in enumerate(rounds):
            b.insert_gen(G.make_gen(G.GEN_KEYED, seed=2, round=r, tag=7), n)
        b.rw(G.MUL3ADD1)
        out = torch.zeros(total, dtype=torch.int32, device="cuda")
        b.flatten_into(out)
        got = G.as_unsigned(out).copy()
        assert b.last_error() == 0
        if ref is None:
            ref = got
        else:
            assert np.array_equal(got, ref), f"grid {grid}"
        b.close()
        for a in arrays:
            a.close()
    flats = []
    for F in (1, 64, 4096):
        a = G.GGArray(pool, 8, 9, F)
        for r in range(3):
            a.insert_gen(G.make_gen(G.GEN_BERNOULLI, seed=4, round=r), 70001)
        a.shrink(2, 7)
        a.rw(G.ADD1)
        flats.append(gpu_flat(a))
        a.close()
    assert all(np.array_equal(flats[0], f) for f in flats[1:])
