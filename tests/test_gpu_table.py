"""The tile table that r/w and flatten of a large array (2^23 elements or more)
stream through: results equal the oracle whether the table covers the array or
not (graphs captured before the array outgrew it), and graphs captured earlier
stay correct after the library outgrows and retires its buffers."""
import numpy as np
import pytest
import torch

import oracle
from oracle import Oracle
from paper_2209_00103_amd import workloads as wl
from tests.gpu_util import gg

pytestmark = pytest.mark.gpu
MiB = 1 << 20
BIG = 1 << 23  # elements from which r/w and flatten use a tile table (2048 tiles of 16 KiB, u32)


@pytest.fixture
def pool():
    p = gg().Pool(2048 * MiB)
    yield p
    p.close()


def _check(G, out, o, what):
    ref = o.flatten()
    got = G.as_unsigned(out[:ref.size])
    assert np.array_equal(got, ref), f"{what}: {np.count_nonzero(got != ref)} elements differ"


@pytest.mark.parametrize("elem", [4, 8])
def test_graph_growing_past_the_table_it_was_captured_with(pool, elem):
    """The table is sized eagerly for a small array; the captured step grows the
    array far past it on every replay, so the replays stream without a table."""
    G = gg()
    V, F = 6, 16
    a, o = G.GGArray(pool, elem, V, F), Oracle(elem, V, F)
    dt = torch.int32 if elem == 4 else torch.int64
    a.insert_gen(G.make_gen(G.GEN_ROUND_TAG, round=0, tag_shift=26), BIG + 300)
    o.insert_gen(oracle.GEN_ROUND_TAG, BIG + 300, round=0, tag_shift=26)
    big = BIG
    out = torch.zeros(BIG + 300 + 3 * big, dtype=dt, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        a.rw(G.ADD1)  # eager: builds a table for this size
        a.flatten_into(out)
    s.synchronize()
    o.rw(oracle.OP_ADD1)
    _check(G, out, o, "eager")
    gen = G.make_gen(G.GEN_ROUND_TAG, round=1, tag_shift=26)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        a.insert_gen(gen, big)
        a.rw(G.MUL3ADD1)
        a.flatten_into(out)
    for rep in range(3):
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        o.insert_gen(oracle.GEN_ROUND_TAG, big, round=1, tag_shift=26)
        o.rw(oracle.OP_MUL3ADD1)
        _check(G, out, o, f"replay {rep}")
    assert a.last_error() == 0
    a.close()
    o.close()


def test_graph_of_rw_alone_sees_later_eager_growth(pool):
    """A graph of r/w + flatten captured on an array of 2^23 elements, replayed
    after eager insertions (and eager calls that grow, and retire, the tile table)."""
    G = gg()
    V, F = 5, 64
    a, o = G.GGArray(pool, 4, V, F), Oracle(4, V, F)
    a.insert_gen(G.make_gen(G.GEN_KEYED, seed=3, round=0, tag=1), BIG)
    o.insert_gen(oracle.GEN_KEYED, BIG, seed=3, round=0, tag=1)
    out = torch.zeros(BIG + (1 << 24) + 5000 + 400000 + 3000000, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        a.rw(G.ADD1)
    s.synchronize()
    o.rw(oracle.OP_ADD1)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        a.rw(G.ADD1_X30)
        a.flatten_into(out)
    for rep, n in enumerate((0, 5000, 3000000, 1 << 24)):
        if n:
            a.insert_gen(G.make_gen(G.GEN_KEYED, seed=3, round=rep, tag=1), n)
            o.insert_gen(oracle.GEN_KEYED, n, seed=3, round=rep, tag=1)
            a.rw(G.ADD1)  # eager: rebuilds (and grows) the table
            o.rw(oracle.OP_ADD1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        o.rw(oracle.OP_ADD1_X30)
        _check(G, out, o, f"replay after {n} more")
    assert a.last_error() == 0
    a.close()
    o.close()


def test_tile_table_on_many_small_and_empty_vectors(pool):
    """3000 LFVectors with first bucket 2 (many partial tiles per LFVector), buffer
    rounds of 2^22 threads with random flags, shrinks, r/w and flatten."""
    G = gg()
    V, F = 3000, 2
    a, o = G.GGArray(pool, 4, V, F), Oracle(4, V, F)
    rng = np.random.default_rng(11)
    out = torch.zeros(1 << 24, dtype=torch.int32, device="cuda")
    for r in range(4):
        n = (1 << 22) - int(rng.integers(0, 1000))
        vals, flags = wl.random_round(rng, n, float(rng.uniform(0.5, 0.95)), 4)
        a.insert(G.to_device(vals), G.to_device(flags))
        o.insert(vals, flags)
        a.rw(G.MUL3ADD1)
        o.rw(oracle.OP_MUL3ADD1)
        a.flatten_into(out)
        _check(G, out, o, f"round {r}")
        a.shrink(1, 5)
        o.shrink(1, 5)
    a.flatten_into(out)
    _check(G, out, o, "after the last shrink")
    assert a.last_error() == 0
    a.close()
    o.close()


def test_batch_table_and_its_graph(pool):
    """A batch above the table threshold (three arrays, 2^23 + elements in all):
    batched r/w and flatten against the oracles, eagerly and as a graph whose
    replays grow the batch past the table it was captured with."""
    G = gg()
    shapes = [(64, 1024), (3, 16), (700, 2)]
    arrays = [G.GGArray(pool, 4, V, F) for V, F in shapes]
    oracles = [Oracle(4, V, F) for V, F in shapes]
    b = G.Batch(arrays)
    first = [BIG // 2, 3 * BIG // 8, BIG // 4]
    b.insert_gen(G.make_gen(G.GEN_KEYED, seed=9, round=0, tag=4), first)
    for i, o in enumerate(oracles):
        o.insert_gen(oracle.GEN_KEYED, first[i], seed=9, round=0, tag=4 + i)
    grow = [1 << 20, 1 << 19, 3 << 19]
    total = sum(first) + 4 * sum(grow)
    out = torch.zeros(total, dtype=torch.int32, device="cuda")
    grow_gen = G.make_gen(G.GEN_KEYED, seed=9, round=1, tag=4)

    def grow_oracles():
        for i, o in enumerate(oracles):
            o.insert_gen(oracle.GEN_KEYED, grow[i], seed=9, round=1, tag=4 + i)

    def check(what):
        torch.cuda.synchronize()
        offs = b.offsets().cpu().numpy()
        got = G.as_unsigned(out)
        for i, o in enumerate(oracles):
            ref = o.flatten()
            assert offs[i + 1] - offs[i] == ref.size, f"{what}: array {i} size"
            assert np.array_equal(got[offs[i]:offs[i + 1]], ref), f"{what}: array {i} differs"

    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b.rw(G.ADD1)
        b.flatten_into(out)
    for o in oracles:
        o.rw(oracle.OP_ADD1)
    check("eager")
    with torch.cuda.stream(s):
        b.insert_gen(grow_gen, grow)  # eager round of this shape: its launch table exists before capture
    grow_oracles()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        b.insert_gen(grow_gen, grow)
        b.rw(G.MUL3ADD1)
        b.flatten_into(out)
    for rep in range(3):
        g.replay()
        grow_oracles()
        for o in oracles:
            o.rw(oracle.OP_MUL3ADD1)
        check(f"replay {rep}")
    assert b.last_error() == 0
    b.close()
    for a, o in zip(arrays, oracles):
        a.close()
        o.close()


@pytest.mark.parametrize("elem", [4, 8])
def test_repeated_rw_through_the_table(pool, elem):
    """r/w directly after r/w (streamed with non-temporal loads), then after a
    flatten and after an insertion (loads through the cache), on an array above
    the table threshold."""
    G = gg()
    a, o = G.GGArray(pool, elem, 32, 1024), Oracle(elem, 32, 1024)
    a.insert_gen(G.make_gen(G.GEN_KEYED, seed=6, round=0, tag=2), BIG + 12345)
    o.insert_gen(oracle.GEN_KEYED, BIG + 12345, seed=6, round=0, tag=2)
    dt = torch.int32 if elem == 4 else torch.int64
    out = torch.zeros(BIG + 12345 + 999, dtype=dt, device="cuda")
    for op in (G.ADD1, G.MUL3ADD1, G.ADD1_X30):
        a.rw(op)
        o.rw(op)
    a.flatten_into(out)
    _check(G, out, o, "after three r/w")
    a.rw(G.MUL3ADD1)
    o.rw(oracle.OP_MUL3ADD1)
    a.insert_gen(G.make_gen(G.GEN_KEYED, seed=6, round=1, tag=2), 999)
    o.insert_gen(oracle.GEN_KEYED, 999, seed=6, round=1, tag=2)
    a.rw(G.ADD1)
    o.rw(oracle.OP_ADD1)
    a.flatten_into(out)
    _check(G, out, o, "after flatten, r/w, insertion, r/w")
    assert a.last_error() == 0
    a.close()
    o.close()


def test_footprint_reports_metadata_lookback_and_tables(pool):
    G = gg()
    a = G.GGArray(pool, 4, 8, 1024)
    fp = a.footprint()
    assert fp["metadata"] >= 8 * (8 + 8 * 40) and fp["lookback"] == 0 and fp["tile_tables"] == 0
    vals = torch.zeros(40000, dtype=torch.int32, device="cuda")
    a.insert(vals, torch.ones(40000, dtype=torch.uint8, device="cuda"))  # 5000 threads per LFVector: look-back
    assert a.footprint()["lookback"] > 0
    a.insert_gen(G.make_gen(G.GEN_ROUND_TAG, round=1, tag_shift=24), BIG)
    a.rw(G.ADD1)  # above the threshold: builds a tile table
    assert a.footprint()["tile_tables"] >= 16 * (BIG // 4096)
    assert a.last_error() == 0
    a.close()


@pytest.mark.parametrize("elem", [4, 8])
def test_one_capture_reuses_its_prefix_and_table(pool, elem):
    """A captured step that calls r/w, flatten and prefix several times around an
    insertion: each replay's results equal the oracle, and eager calls made before
    the first replay and between replays see the array as it really is then."""
    G = gg()
    V, F = 7, 32
    a, o = G.GGArray(pool, elem, V, F), Oracle(elem, V, F)
    dt = torch.int32 if elem == 4 else torch.int64
    n_small = 70000
    a.insert_gen(G.make_gen(G.GEN_KEYED, seed=5, round=0, tag=2), BIG + 123)
    o.insert_gen(oracle.GEN_KEYED, BIG + 123, seed=5, round=0, tag=2)
    a.insert_gen(G.make_gen(G.GEN_KEYED, seed=5, round=1, tag=2), n_small)  # sizes the look-back eagerly
    o.insert_gen(oracle.GEN_KEYED, n_small, seed=5, round=1, tag=2)
    cap = BIG + 123 + 5 * n_small
    out1 = torch.zeros(cap, dtype=dt, device="cuda")
    out2 = torch.zeros(cap, dtype=dt, device="cuda")
    pre = torch.zeros(V + 1, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        a.rw(G.ADD1)  # eager prefix and table
    s.synchronize()
    o.rw(oracle.OP_ADD1)
    gen = G.make_gen(G.GEN_ROUND_TAG, round=9, tag_shift=26)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        a.rw(G.MUL3ADD1)
        a.flatten_into(out1)
        a.insert_gen(gen, n_small)
        a.rw(G.ADD1)
        a.rw(G.ADD1_X30)
        a.prefix_into(pre)
        a.flatten_into(out2)
    torch.cuda.synchronize()
    _check(G, a.flatten(), o, "eager flatten after capture, before any replay")
    for rep in range(3):
        if rep == 1:
            a.rw(G.ADD1)  # eager work between replays
            o.rw(oracle.OP_ADD1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        o.rw(oracle.OP_MUL3ADD1)
        _check(G, out1, o, f"replay {rep}: first flatten")
        o.insert_gen(oracle.GEN_ROUND_TAG, n_small, round=9, tag_shift=26)
        o.rw(oracle.OP_ADD1)
        o.rw(oracle.OP_ADD1_X30)
        assert np.array_equal(pre.cpu().numpy().astype(np.uint64), o.prefix().astype(np.uint64)), f"replay {rep}: prefix"
        _check(G, out2, o, f"replay {rep}: second flatten")
        _check(G, a.flatten(), o, f"replay {rep}: eager flatten")
    assert a.last_error() == 0
    a.close()
    o.close()


@pytest.mark.parametrize("base", [1000, BIG])
def test_graph_of_insertion_alone_then_eager_calls(pool, base):
    """A graph that only inserts changes the sizes on every replay behind the
    host's back: eager r/w, flatten and prefix calls between replays (each
    following an eager call that left a valid prefix and table) see them."""
    G = gg()
    V, F = 9, 64
    a, o = G.GGArray(pool, 4, V, F), Oracle(4, V, F)
    n = 30000
    a.insert_gen(G.make_gen(G.GEN_KEYED, seed=1, round=0, tag=7), base)
    o.insert_gen(oracle.GEN_KEYED, base, seed=1, round=0, tag=7)
    gen = G.make_gen(G.GEN_BERNOULLI, seed=4, round=2)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        a.insert_gen(gen, n)  # eager round of this shape: its look-back exists before capture
    s.synchronize()
    o.insert_gen(oracle.GEN_BERNOULLI, n, seed=4, round=2)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        a.insert_gen(gen, n)
    torch.cuda.synchronize()
    for rep in range(3):
        a.rw(G.ADD1)
        o.rw(oracle.OP_ADD1)
        _check(G, a.flatten(), o, f"before replay {rep}")
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        o.insert_gen(oracle.GEN_BERNOULLI, n, seed=4, round=2)
        assert np.array_equal(a.prefix().cpu().numpy().astype(np.uint64), o.prefix()), f"replay {rep}: prefix"
        a.rw(G.MUL3ADD1)
        o.rw(oracle.OP_MUL3ADD1)
        _check(G, a.flatten(), o, f"after replay {rep}")
    assert a.last_error() == 0
    a.close()
    o.close()


def test_batch_graph_of_insertion_alone_then_eager_calls(pool):
    """The same for a batch: eager batched r/w and flatten between replays of a
    graph holding only a batched insertion round."""
    G = gg()
    shapes = [(64, 1024), (3, 16), (700, 2)]
    arrays = [G.GGArray(pool, 4, V, F) for V, F in shapes]
    oracles = [Oracle(4, V, F) for V, F in shapes]
    b = G.Batch(arrays)
    first = [BIG // 2, 3 * BIG // 8, BIG // 4]
    grow = [40000, 3, 70000]
    gen = G.make_gen(G.GEN_KEYED, seed=2, round=1, tag=1)
    b.insert_gen(G.make_gen(G.GEN_KEYED, seed=2, round=0, tag=1), first)
    b.insert_gen(gen, grow)
    for i, o in enumerate(oracles):
        o.insert_gen(oracle.GEN_KEYED, first[i], seed=2, round=0, tag=1 + i)
        o.insert_gen(oracle.GEN_KEYED, grow[i], seed=2, round=1, tag=1 + i)
    out = torch.zeros(sum(first) + 5 * sum(grow), dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        b.insert_gen(gen, grow)

    def check(what):
        torch.cuda.synchronize()
        offs = b.offsets().cpu().numpy()
        got = G.as_unsigned(out)
        for i, o in enumerate(oracles):
            ref = o.flatten()
            assert offs[i + 1] - offs[i] == ref.size, f"{what}: array {i} size"
            assert np.array_equal(got[offs[i]:offs[i + 1]], ref), f"{what}: array {i} differs"

    for rep in range(3):
        b.rw(G.ADD1)
        b.flatten_into(out)
        for o in oracles:
            o.rw(oracle.OP_ADD1)
        check(f"before replay {rep}")
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, o in enumerate(oracles):
            o.insert_gen(oracle.GEN_KEYED, grow[i], seed=2, round=1, tag=1 + i)
        b.rw(G.MUL3ADD1)
        b.flatten_into(out)
        for o in oracles:
            o.rw(oracle.OP_MUL3ADD1)
        check(f"after replay {rep}")
    assert b.last_error() == 0
    b.close()
    for a, o in zip(arrays, oracles):
        a.close()
        o.close()


def test_kernel_timing_events(pool):
    """The measurement aid: r/w and flatten dispatches record events at the kernel's
    own start and end; results are unchanged, durations are positive, and asking
    before any timed kernel (or after timing is switched off) is an error."""
    G = gg()
    a, o = G.GGArray(pool, 4, 16, 1024), Oracle(4, 16, 1024)
    a.insert_gen(G.make_gen(G.GEN_KEYED, seed=1, round=0, tag=1), BIG)
    o.insert_gen(oracle.GEN_KEYED, BIG, seed=1, round=0, tag=1)
    with pytest.raises(G.GGAError):
        a.kernel_ms(0)
    a.kernel_timing(True)
    with pytest.raises(G.GGAError):
        a.kernel_ms(1)
    a.rw(G.ADD1)
    o.rw(oracle.OP_ADD1)
    out = torch.zeros(BIG, dtype=torch.int32, device="cuda")
    a.flatten_into(out)
    rw_ms, fl_ms = a.kernel_ms(0), a.kernel_ms(1)
    assert 0.0 < rw_ms < 1000.0 and 0.0 < fl_ms < 1000.0
    _check(G, out, o, "timed r/w and flatten")
    # a round of 8 tiles per LFVector is one launch and is timed; one of 128 tiles is not
    a.insert_gen_shrink(G.make_gen(G.GEN_ROUND_TAG, round=1, tag_shift=26), 16 * 4096 * 8, 1, 10)
    o.insert_gen(oracle.GEN_ROUND_TAG, 16 * 4096 * 8, round=1, tag_shift=26)
    o.shrink(1, 10)
    assert 0.0 < a.kernel_ms(2) < 1000.0
    a.insert_gen(G.make_gen(G.GEN_ROUND_TAG, round=2, tag_shift=26), BIG)
    o.insert_gen(oracle.GEN_ROUND_TAG, BIG, round=2, tag_shift=26)
    with pytest.raises(G.GGAError):
        a.kernel_ms(2)
    out = torch.zeros(o.flatten().size, dtype=torch.int32, device="cuda")
    a.flatten_into(out)
    _check(G, out, o, "after timed and untimed rounds")
    a.kernel_timing(False)
    with pytest.raises(G.GGAError):
        a.kernel_ms(0)
    a.close()
    o.close()


def test_flagged_round_captured_before_its_buffer_exists(pool):
    """A round from buffers with flags over several tiles per LFVector runs in two
    passes through a per-array buffer; captured in a graph before that buffer
    exists (it cannot grow under capture) it runs as one launch with tickets and
    the decoupled look-back.  Replays of the captured round and eager rounds of
    the same inputs between them (two passes) all equal the oracle."""
    from tests.gpu_util import dev

    G = gg()
    V, F, n = 3, 64, 50000  # 16667 threads per LFVector: 5 tiles of 4096
    a, o = G.GGArray(pool, 4, V, F), Oracle(4, V, F)
    rng = np.random.default_rng(11)
    vals, flags = wl.random_round(rng, n, 0.7, 4)
    dv, df = dev(vals), dev(flags)
    gen = G.make_gen(G.GEN_BERNOULLI, seed=4, round=2)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        a.insert_gen(gen, n)  # a generated round of this shape grows the look-back words
    s.synchronize()
    o.insert_gen(oracle.GEN_BERNOULLI, n, seed=4, round=2)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        a.insert(dv, df)
    torch.cuda.synchronize()
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        o.insert(vals, flags)
        _check(G, a.flatten(), o, f"after replay {rep}")
        a.insert(dv, df)  # eager: two passes
        o.insert(vals, flags)
        _check(G, a.flatten(), o, f"after eager round {rep}")
    assert a.last_error() == 0
    a.close()
    o.close()


@pytest.mark.parametrize("elem", [4, 8])
@pytest.mark.parametrize("F", [64, 1 << 16])
@pytest.mark.parametrize("case", ["blocked", "odd_count", "payloads_unaligned", "flags_unaligned"])
def test_flagged_rounds_in_both_mask_layouts(pool, elem, F, case):
    """Rounds from buffers with flags over several tiles per LFVector (two passes)
    keep lane-blocked masks when every tile starts and ends on a whole 16-byte
    payload vector and both buffers are aligned for the vector loads (a ragged
    last LFVector included), and the slot layout otherwise: a thread count that
    is not a multiple of the vector, payloads or flags off their alignment.  With
    first buckets of 64 elements a tile's kept elements cross several buckets;
    with 2^16 they land in one.  Every round's flatten equals the oracle."""
    from tests.gpu_util import dev

    G = gg()
    V = 5
    a, o = G.GGArray(pool, elem, V, F), Oracle(elem, V, F)
    rng = np.random.default_rng(23)
    dt = np.uint32 if elem == 4 else np.uint64
    sv = 1 if case == "payloads_unaligned" else 0
    sf = 1 if case == "flags_unaligned" else 0
    # 99996 threads: chunks of 20000 (5 tiles of 4096), the last LFVector 19996
    for r, (n, p) in enumerate([(99996, 0.6), (102400, 0.3), (99996, 0.95)]):
        if case == "odd_count":
            n += 1
        vals, flags = wl.random_round(rng, n, p, elem)
        dv = dev(np.concatenate([np.zeros(sv, dt), vals]))[sv:]
        df = dev(np.concatenate([np.zeros(sf, np.uint8), flags]))[sf:]
        a.insert(dv, df)
        o.insert(vals, flags)
        _check(G, a.flatten(), o, f"{case}, round {r}")
    assert a.last_error() == 0
    a.close()
    o.close()


@pytest.mark.parametrize("n", [99996, 99997], ids=["lane-blocked", "slot-layout"])
def test_two_pass_flagged_round_in_a_graph(pool, n):
    """A flagged round from buffers captured after an eager round of its shape has
    grown the per-array buffer: the capture holds the two passes (mask pass, scan,
    grow, copy; lane-blocked masks when the chunk and the thread count are whole
    16-byte vectors, the slot layout otherwise), and every replay, with eager
    rounds and shrinks between replays, equals the oracle."""
    from tests.gpu_util import dev

    G = gg()
    V, F = 5, 64  # chunks of 20000 threads: 5 tiles of 4096 per LFVector
    a, o = G.GGArray(pool, 4, V, F), Oracle(4, V, F)
    rng = np.random.default_rng(5)
    vals, flags = wl.random_round(rng, n, 0.6, 4)
    dv, df = dev(vals), dev(flags)
    s = torch.cuda.Stream()
    try:
        with torch.cuda.stream(s):
            a.insert(dv, df, stream=s)  # eager: grows the buffer of the two passes
        s.synchronize()
        o.insert(vals, flags)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            a.insert(dv, df, stream=s)
        torch.cuda.synchronize()
        for rep in range(3):
            g.replay()
            torch.cuda.synchronize()
            o.insert(vals, flags)
            _check(G, a.flatten(), o, f"after replay {rep}")
            a.insert(dv, df)
            a.shrink(1, 3)
            o.insert(vals, flags)
            o.shrink(1, 3)
            _check(G, a.flatten(), o, f"after eager round {rep}")
        assert a.last_error() == 0
    finally:
        a.close()
        o.close()
