"""GPU parity at the workloads' full sizes, in the launch configurations the
benchmark times: exact comparison where the oracle finishes in seconds
(configuration 2), otherwise sampled LFVectors / arrays that the oracle computes
one by one plus properties that hold at any size (configurations 3, 4, 5)."""
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


@pytest.mark.parametrize("V,fused", [(512, True), (512, False), (256, True), (32, False)])
def test_config2_full_size_exact(V, fused):
    """2^28 insertions over 12 rounds with shrink 1/10 after each, r/w x = 3x + 1,
    flatten: every element against the list-form oracle.  With `fused` each round
    and its shrink are one ggarray_insert_gen_shrink call, as the benchmark runs
    them (one launch per round at V = 512; at V = 256 the rounds of more than 8
    tiles per LFVector take two)."""
    G = gg()
    rounds = wl.cfg2_round_threads()
    pool = G.Pool(4 * GiB)
    a = G.GGArray(pool, 4, V, 1024)
    o = Oracle(4, V, 1024, forms=oracle.FORM_LIST)
    try:
        for r, n in enumerate(rounds):
            gen = G.make_gen(G.GEN_ROUND_TAG, round=r, tag_shift=27)
            if fused:
                a.insert_gen_shrink(gen, n, 1, 10)
            else:
                a.insert_gen(gen, n)
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


def _config3_vector_oracle(v, chunk, thr, F):
    """LFVector v of configuration 3 on its own: the threads of its chunk, their
    Poisson counts and payloads from the workload generator, inserted in thread
    order into a one-vector oracle, r/w +1 after every phase."""
    o = Oracle(8, 1, F, forms=oracle.FORM_LIST)
    g0 = v * chunk
    for i in range(4):
        c = wl.poisson_counts(1, i, chunk, thr, gid0=g0)
        gid = np.repeat(np.arange(g0, g0 + chunk, dtype=np.uint64), 16)
        j = np.tile(np.arange(16, dtype=np.uint64), chunk)
        vals = wl.poisson_payload(1, i, gid, j)
        o.insert_counts(vals, c, 16)
        o.rw(oracle.OP_ADD1)
    out = o.flatten()
    o.close()
    return out


def test_config3_full_size_sampled():
    """2^26 threads, Poisson(3) counts capped at 16, u64 payloads, V = 65536,
    4 insert phases each followed by r/w +1, flatten.  Per-vector sizes are checked
    for all 65536 vectors; the contents of 16 vectors element by element."""
    G = gg()
    thr = wl.poisson_thresholds(3, 16)
    V, n, F = 65536, 1 << 26, 1024
    chunk = n // V
    pool = G.Pool(16 * GiB)
    a = G.GGArray(pool, 8, V, F)
    try:
        expect = np.zeros(V, dtype=np.uint64)
        for i in range(4):
            a.insert_gen(G.make_gen(G.GEN_POISSON, seed=1, round=i, max_count=16, thresholds=thr), n)
            a.rw(G.ADD1)
            expect += wl.poisson_counts(1, i, n, thr).reshape(V, chunk).sum(axis=1, dtype=np.uint64)
        sizes = a.vector_sizes().cpu().numpy().astype(np.uint64)
        np.testing.assert_array_equal(sizes, expect)
        total = int(expect.sum())
        assert a.size() == total
        assert a.capacity() <= 2 * total + V * (F - 1)
        flat = a.flatten()
        pre = a.prefix().cpu().numpy()
        rng = np.random.default_rng(11)
        sample = sorted(set([0, 1, V // 2, V - 1] + [int(x) for x in rng.integers(0, V, 12)]))
        for v in sample:
            got = G.as_unsigned(flat[int(pre[v]):int(pre[v + 1])])
            ref = _config3_vector_oracle(v, chunk, thr, F)
            assert np.array_equal(got, ref), f"vector {v}: " + _first_diff(got, ref)
        assert a.last_error() == 0
        del flat
    finally:
        a.close()
        pool.close()


def test_config4_full_size_batched_sampled():
    """512 arrays of log-uniform size 2^10..2^24, one launch per phase (4 keyed
    rounds, r/w +1, flatten to per-array offsets), first buckets spread over every
    candidate the tuner may pick; 16 arrays against the oracle, all offsets exact."""
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
        order = sorted(range(n_arr), key=lambda i: sizes[i])
        sample = sorted(set(order[:: n_arr // 14] + [order[0], order[-1]]))
        for i in sample:
            o = Oracle(4, vecs[i], firsts[i], forms=oracle.FORM_LIST)
            for r in range(4):
                o.insert_gen(oracle.GEN_KEYED, rounds[i][r], seed=1, round=r, tag=i)
            o.rw(oracle.OP_ADD1)
            got = G.as_unsigned(out[int(offs[i]):int(offs[i + 1])])
            ref = o.flatten()
            o.close()
            assert np.array_equal(got, ref), f"array {i} (n={sizes[i]}, F={firsts[i]}): " + _first_diff(got, ref)
        cap = sum(a.capacity() for a in arrays)
        assert cap <= 2 * total + sum(v * f for v, f in zip(vecs, firsts))
    finally:
        b.close()
        for a in arrays:
            a.close()
        pool.close()


def test_config5_full_size_served_sampled():
    """4096 resident arrays (lognormal sizes, median 2^16), 2^20 requests all queued
    at t = 0, served with continuous batching as the benchmark runs it; 8 arrays
    replayed by the oracle, and every flatten's length against the host replay."""
    G = gg()
    cfg = wl.CFG5
    seed, n_arr, n = 1, cfg["n_arrays"], cfg["n_requests"]
    sizes = [int(x) for x in wl.cfg5_sizes(seed, n_arr, cfg["median_log2"], cfg["sigma"], cfg["size_cap_log2"])]
    vecs = [wl.cfg4_vectors(s) for s in sizes]
    firsts = [wl.cfg5_first_bucket(s, v) for s, v in zip(sizes, vecs)]
    tr = wl.cfg5_trace(seed, n, n_arr, cfg["append_median_log2"], cfg["append_cap_log2"], cfg["mix"])
    final_live = sum(sizes) + int(tr["length"].sum())
    pool = G.Pool(4 * (2 * final_live + sum(v * f for v, f in zip(vecs, firsts))) + GiB)
    arrays = [G.GGArray(pool, 4, v, f) for v, f in zip(vecs, firsts)]
    try:
        fill = G.Batch(arrays)
        fill.insert_gen(G.make_gen(G.GEN_KEYED, seed=seed, round=cfg["fill_round"], tag=0), sizes)
        fill.close()
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
        rng = np.random.default_rng(5)
        for a in sorted(set(int(x) for x in rng.integers(0, n_arr, 8))):
            o = Oracle(4, vecs[a], firsts[a], forms=oracle.FORM_LIST)
            o.insert_gen(oracle.GEN_KEYED, sizes[a], seed=seed, round=cfg["fill_round"], tag=a)
            for r in np.nonzero(tr["target"] == a)[0]:
                k = tr["kind"][r]
                if k == wl.REQ_APPEND:
                    o.insert_gen(oracle.GEN_KEYED, int(tr["length"][r]), seed=seed, round=cfg["append_round"],
                                 tag_shift=cfg["append_shift"], tag=int(r))
                elif k == wl.REQ_RW:
                    o.rw(oracle.OP_ADD1)
            ref = o.flatten()
            o.close()
            got = G.as_unsigned(arrays[a].flatten())
            assert np.array_equal(got, ref), f"array {a}: " + _first_diff(got, ref)
            assert arrays[a].last_error() == 0
    finally:
        for a in arrays:
            a.close()
        pool.close()
