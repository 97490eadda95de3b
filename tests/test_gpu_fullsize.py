"""GPU parity at the workloads' full sizes, in the launch configurations the
benchmark times, element by element against the list-form oracle: configuration
2 whole; configuration 3 whole (all 65536 LFVectors); configuration 4 every one
of the 512 arrays; configuration 5 every array's final state after 2^20 served
requests and, on a 2^16-request prefix with an arena that never wraps, every
flatten output.  The oracle runs per array in a thread pool (its C calls release
the GIL)."""
import concurrent.futures as cf
import os

import numpy as np
import pytest
import torch

import oracle
from oracle import Oracle
from paper_2209_00103_amd import workloads as wl
from paper_2209_00103_amd.autotune import CANDIDATES, predicted_ratio
from tests.gpu_util import gg

pytestmark = pytest.mark.gpu
GiB = 1 << 30


def _first_diff(got, ref):
    bad = np.nonzero(got != ref)[0]
    return f"{bad.size} differ, first at {bad[:4]}"


@pytest.mark.parametrize("V,mode", [(512, "rounds"), (512, "fused"), (512, "unfused"), (256, "rounds"),
                                    (256, "fused"), (32, "unfused")])
def test_config2_full_size_exact(V, mode):
    """2^28 insertions over 12 rounds with shrink 1/10 after each, r/w x = 3x + 1,
    flatten: every element against the list-form oracle.  "rounds": all twelve in
    one ggarray_insert_gen_rounds call, as the benchmark's step runs them (one
    launch at V = 512; at V = 256 the rounds of more than 8 tiles per LFVector
    keep it round by round); "fused": each round and its shrink one
    ggarray_insert_gen_shrink call (one launch per round at V = 512, two for
    those larger rounds at V = 256); "unfused": insert, then shrink."""
    G = gg()
    rounds = wl.cfg2_round_threads()
    pool = G.Pool(4 * GiB)
    a = G.GGArray(pool, 4, V, 1024)
    o = Oracle(4, V, 1024, forms=oracle.FORM_LIST)
    try:
        gens = [G.make_gen(G.GEN_ROUND_TAG, round=r, tag_shift=27) for r in range(len(rounds))]
        if mode == "rounds":
            a.insert_gen_rounds(gens, rounds, 1, 10)
        for r, n in enumerate(rounds):
            if mode == "fused":
                a.insert_gen_shrink(gens[r], n, 1, 10)
            elif mode == "unfused":
                a.insert_gen(gens[r], n)
                a.shrink(1, 10)
            o.insert_gen(oracle.GEN_ROUND_TAG, n, round=r, tag_shift=27)
            o.shrink(1, 10)
        a.rw(G.MUL3ADD1)
        o.rw(oracle.OP_MUL3ADD1)
        np.testing.assert_array_equal(a.vector_sizes().cpu().numpy().astype(np.uint64), o.vector_sizes())
        got, ref = G.as_unsigned(a.flatten()), o.flatten()
        assert got.size == ref.size == a.size()
        assert np.array_equal(got, ref), _first_diff(got, ref)
        assert a.capacity() == o.capacity() and a.last_error() == 0
    finally:
        o.close()
        a.close()
        pool.close()



@pytest.mark.parametrize("source", ["buffers", "generated"])
def test_config2_sparse_full_size_exact(source):
    """The configuration-2 round sizes with Bernoulli(1/2) insertion at V = 512,
    as the benchmark's sparse legs run them: from buffers of uint32 payloads and
    flag bytes (a round of several tiles per LFVector takes the two passes with
    lane-blocked masks, a smaller one the one-launch kernel), or drawn by the
    producer (the scan with per-LFVector tickets and the decoupled look-back);
    shrink 1/10 after each round, r/w x = 3x + 1, flatten: every element against
    the list-form oracle."""
    G = gg()
    rounds = wl.cfg2_round_threads()
    pool = G.Pool(4 * GiB)
    a = G.GGArray(pool, 4, 512, 1024)
    o = Oracle(4, 512, 1024, forms=oracle.FORM_LIST)
    rng = np.random.default_rng(2209)
    try:
        for r, n in enumerate(rounds):
            print(f"case sparse full size, {source}, round {r}, {n} threads", flush=True)
            if source == "buffers":
                vals, flags = wl.random_round(rng, n, 0.5, 4)
                a.insert(G.to_device(vals), G.to_device(flags))
                o.insert(vals, flags)
                del vals, flags
            else:
                a.insert_gen(G.make_gen(G.GEN_BERNOULLI, seed=1, round=r), n)
                o.insert_gen(oracle.GEN_BERNOULLI, n, seed=1, round=r)
            a.shrink(1, 10)
            o.shrink(1, 10)
        a.rw(G.MUL3ADD1)
        o.rw(oracle.OP_MUL3ADD1)
        np.testing.assert_array_equal(a.vector_sizes().cpu().numpy().astype(np.uint64), o.vector_sizes())
        got, ref = G.as_unsigned(a.flatten()), o.flatten()
        assert got.size == ref.size == a.size()
        assert np.array_equal(got, ref), _first_diff(got, ref)
        assert a.capacity() == o.capacity() and a.last_error() == 0
    finally:
        o.close()
        a.close()
        pool.close()

def test_config3_full_size_exact():
    """2^26 threads, Poisson(3) counts capped at 16, u64 payloads, V = 65536,
    4 insert phases each followed by r/w +1, flatten: every element of every
    LFVector against the oracle fed the same generated rounds."""
    G = gg()
    thr = wl.poisson_thresholds(3, 16)
    V, n, F = 65536, 1 << 26, 1024
    pool = G.Pool(16 * GiB)
    a = G.GGArray(pool, 8, V, F)
    o = Oracle(8, V, F, forms=oracle.FORM_LIST)
    try:
        for i in range(4):
            a.insert_gen(G.make_gen(G.GEN_POISSON, seed=1, round=i, max_count=16, thresholds=thr), n)
            a.rw(G.ADD1)
            o.insert_gen(oracle.GEN_POISSON, n, seed=1, round=i, max_count=16, thresholds=thr)
            o.rw(oracle.OP_ADD1)
        np.testing.assert_array_equal(a.vector_sizes().cpu().numpy().astype(np.uint64), o.vector_sizes())
        total = o.size()
        assert a.size() == total
        assert a.capacity() == o.capacity() <= 2 * total + V * (F - 1)
        got = G.as_unsigned(a.flatten())
        ref = o.flatten()
        assert np.array_equal(got, ref), _first_diff(got, ref)
        assert a.last_error() == 0
    finally:
        o.close()
        a.close()
        pool.close()


def _pool_map(fn, items):
    workers = min(16, os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(fn, items))


def test_config4_full_size_batched_exact():
    """512 arrays of log-uniform size 2^10..2^24, one launch per phase (4 keyed
    rounds, r/w +1, flatten to per-array offsets), first buckets spread over every
    candidate the tuner may pick; every array against the oracle, all offsets."""
    G = gg()
    n_arr = 512
    sizes = [int(x) for x in wl.cfg4_sizes(1, n_arr)]
    vecs = [wl.cfg4_vectors(s) for s in sizes]
    rounds = [wl.cfg4_round_threads(s, 4) for s in sizes]
    firsts = []
    for i, s in enumerate(sizes):
        ok = [F for F in CANDIDATES if predicted_ratio(s, vecs[i], F, rounds[i]) <= 2.0] or [CANDIDATES[0]]
        firsts.append(ok[i % len(ok)])
    total = sum(sizes)
    pool = G.Pool(int(4 * total * 2.2) + GiB)
    arrays = [G.GGArray(pool, 4, vecs[i], firsts[i]) for i in range(n_arr)]
    b = G.Batch(arrays)
    try:
        for r in range(4):
            b.insert_gen(G.make_gen(G.GEN_KEYED, seed=1, round=r, tag=0), [rounds[i][r] for i in range(n_arr)])
        b.rw(G.ADD1)
        out = torch.empty(total, dtype=torch.int32, device="cuda")
        b.flatten_into(out)
        offs = b.offsets().cpu().numpy()
        assert b.last_error() == 0
        np.testing.assert_array_equal(offs, np.concatenate([[0], np.cumsum(sizes)]))
        flat = G.as_unsigned(out)

        def check(i):
            o = Oracle(4, vecs[i], firsts[i], forms=oracle.FORM_LIST)
            for r in range(4):
                o.insert_gen(oracle.GEN_KEYED, rounds[i][r], seed=1, round=r, tag=i)
            o.rw(oracle.OP_ADD1)
            ref = o.flatten()
            o.close()
            got = flat[int(offs[i]):int(offs[i + 1])]
            return None if np.array_equal(got, ref) else f"array {i} (n={sizes[i]}, F={firsts[i]}): " + _first_diff(got, ref)

        bad = [m for m in _pool_map(check, range(n_arr)) if m]
        assert not bad, bad[:4]
        cap = sum(a.capacity() for a in arrays)
        assert cap <= 2 * total + sum(v * f for v, f in zip(vecs, firsts))
    finally:
        b.close()
        for a in arrays:
            a.close()
        pool.close()


def _served_setup(G, n_req):
    cfg = wl.CFG5
    seed, n_arr = 1, cfg["n_arrays"]
    sizes = [int(x) for x in wl.cfg5_sizes(seed, n_arr, cfg["median_log2"], cfg["sigma"], cfg["size_cap_log2"])]
    vecs = [wl.cfg4_vectors(s) for s in sizes]
    firsts = [wl.cfg5_first_bucket(s, v) for s, v in zip(sizes, vecs)]
    tr = wl.cfg5_trace(seed, n_req, n_arr, cfg["append_median_log2"], cfg["append_cap_log2"], cfg["mix"])
    final_live = sum(sizes) + int(tr["length"].sum())
    pool = G.Pool(4 * (2 * final_live + sum(v * f for v, f in zip(vecs, firsts))) + GiB)
    arrays = [G.GGArray(pool, 4, v, f) for v, f in zip(vecs, firsts)]
    fill = G.Batch(arrays)
    fill.insert_gen(G.make_gen(G.GEN_KEYED, seed=seed, round=cfg["fill_round"], tag=0), sizes)
    fill.close()
    return cfg, seed, sizes, vecs, firsts, tr, pool, arrays


def _requests_by_array(tr, n_arr):
    """For each array, the indices of its requests in trace order."""
    order = np.argsort(tr["target"], kind="stable")
    bounds = np.searchsorted(tr["target"][order], np.arange(n_arr + 1))
    return [order[bounds[a]:bounds[a + 1]] for a in range(n_arr)]


def _replay(cfg, seed, a, size, V, F, tr, reqs, on_flatten=None):
    """Array a's requests of the trace (reqs, in order) on a one-array oracle."""
    o = Oracle(4, V, F, forms=oracle.FORM_LIST)
    o.insert_gen(oracle.GEN_KEYED, size, seed=seed, round=cfg["fill_round"], tag=a)
    for r in reqs:
        k = tr["kind"][r]
        if k == wl.REQ_APPEND:
            o.insert_gen(oracle.GEN_KEYED, int(tr["length"][r]), seed=seed, round=cfg["append_round"],
                         tag_shift=cfg["append_shift"], tag=int(r))
        elif k == wl.REQ_RW:
            o.rw(oracle.OP_ADD1)
        elif on_flatten is not None:
            msg = on_flatten(int(r), o.flatten())
            if msg:
                o.close()
                return msg
    ref = o.flatten()
    o.close()
    return ref


def test_config5_full_size_served_exact():
    """4096 resident arrays (lognormal sizes, median 2^16), 2^20 requests all queued
    at t = 0, served with continuous batching as the benchmark runs it: every
    array's final state against the oracle replaying that array's requests in
    order, every flatten's length against the host replay."""
    G = gg()
    n = wl.CFG5["n_requests"]
    cfg, seed, sizes, vecs, firsts, tr, pool, arrays = _served_setup(G, n)
    try:
        arena = torch.empty(GiB // 4, dtype=torch.int32, device="cuda")
        out_len = torch.zeros(n, dtype=torch.int64, device="cuda")
        sv = G.Server(arrays, arena, cfg["cap_bytes"], mode=G.SERVE_BATCHED, lanes=2, max_step=1024, seed=seed,
                      append_round=cfg["append_round"], append_shift=cfg["append_shift"], rw_op=G.ADD1)
        res = sv.run(np.zeros(n, np.uint64), tr["kind"], tr["target"], tr["length"], out_len)
        sv.close()
        assert (res["status"] == 0).all() and res["issued"] == n
        lens = out_len.cpu().numpy()
        size = list(sizes)
        for r in range(n):
            a = int(tr["target"][r])
            if tr["kind"][r] == wl.REQ_APPEND:
                size[a] += int(tr["length"][r])
            elif tr["kind"][r] == wl.REQ_FLATTEN:
                assert int(lens[r]) == size[a], f"flatten request {r}"
        b = G.Batch(arrays)
        total = sum(size)
        out = torch.empty(total, dtype=torch.int32, device="cuda")
        b.flatten_into(out)
        offs = b.offsets().cpu().numpy()
        assert b.last_error() == 0
        b.close()
        flat = G.as_unsigned(out)
        del out

        by_array = _requests_by_array(tr, len(arrays))

        def check(a):
            ref = _replay(cfg, seed, a, sizes[a], vecs[a], firsts[a], tr, by_array[a])
            got = flat[int(offs[a]):int(offs[a + 1])]
            return None if np.array_equal(got, ref) else f"array {a}: " + _first_diff(got, ref)

        bad = [m for m in _pool_map(check, range(len(arrays))) if m]
        assert not bad, bad[:4]
        assert all(x.last_error() == 0 for x in arrays)
    finally:
        for a in arrays:
            a.close()
        pool.close()


def test_config5_every_flatten_output():
    """The same 4096 arrays and the first 2^16 requests of the trace, served with
    continuous batching into an arena large enough never to wrap: every flatten
    request's output, at its offset in the arena, against the oracle's flatten of
    that array at that point of its request sequence; then every final state."""
    G = gg()
    n = 1 << 16
    cfg, seed, sizes, vecs, firsts, tr, pool, arrays = _served_setup(G, n)
    try:
        size = list(sizes)
        flat_bytes = 0
        for r in range(n):
            a = int(tr["target"][r])
            if tr["kind"][r] == wl.REQ_APPEND:
                size[a] += int(tr["length"][r])
            elif tr["kind"][r] == wl.REQ_FLATTEN:
                flat_bytes += 4 * size[a] + 256
        arena_elems = (flat_bytes + (64 << 20)) // 4
        arena = torch.empty(arena_elems, dtype=torch.int32, device="cuda")
        out_len = torch.zeros(n, dtype=torch.int64, device="cuda")
        sv = G.Server(arrays, arena, cfg["cap_bytes"], mode=G.SERVE_BATCHED, lanes=3, max_step=1024, seed=seed,
                      append_round=cfg["append_round"], append_shift=cfg["append_shift"], rw_op=G.ADD1)
        res = sv.run(np.zeros(n, np.uint64), tr["kind"], tr["target"], tr["length"], out_len)
        sv.close()
        assert (res["status"] == 0).all() and res["issued"] == n and res["arena_wraps"] == 0
        host_arena = G.as_unsigned(arena)
        del arena
        offs_b = res["out_offset"]
        lens = out_len.cpu().numpy()
        n_flat = int((tr["kind"] == wl.REQ_FLATTEN).sum())
        assert n_flat > 1000

        b = G.Batch(arrays)
        out = torch.empty(sum(size), dtype=torch.int32, device="cuda")
        b.flatten_into(out)
        offs = b.offsets().cpu().numpy()
        b.close()
        flat = G.as_unsigned(out)
        del out

        by_array = _requests_by_array(tr, len(arrays))

        def check(a):
            def on_flatten(r, ref):
                e0 = int(offs_b[r]) // 4
                got = host_arena[e0:e0 + int(lens[r])]
                return None if np.array_equal(got, ref) else f"flatten request {r} (array {a}): " + _first_diff(got, ref)

            ref = _replay(cfg, seed, a, sizes[a], vecs[a], firsts[a], tr, by_array[a], on_flatten)
            if isinstance(ref, str):
                return ref
            got = flat[int(offs[a]):int(offs[a + 1])]
            return None if np.array_equal(got, ref) else f"array {a} final: " + _first_diff(got, ref)

        bad = [m for m in _pool_map(check, range(len(arrays))) if m]
        assert not bad, bad[:4]
    finally:
        for a in arrays:
            a.close()
        pool.close()
