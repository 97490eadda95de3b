"""GPU tests of the served mode: every request's result is the same in the mix
(continuous batching, several steps in flight) as alone (one request at a time
with the single-array calls), and both equal the CPU oracle replaying each
array's requests in arrival order."""
import numpy as np
import pytest
import torch

from oracle import Oracle
import oracle
from paper_2209_00103_amd import workloads as wl
from tests.gpu_util import gg

pytestmark = pytest.mark.gpu
MiB = 1 << 20
SEED = 3
ELEM = 4


def _shapes(sizes):
    V = [wl.cfg4_vectors(int(s)) for s in sizes]
    F = [wl.cfg5_first_bucket(int(s), v) for s, v in zip(sizes, V)]
    return V, F


def _resident(pool, sizes):
    """Arrays holding their initial contents (one keyed round each, in one launch)."""
    G = gg()
    V, F = _shapes(sizes)
    arrays = [G.GGArray(pool, ELEM, v, f) for v, f in zip(V, F)]
    b = G.Batch(arrays)
    b.insert_gen(G.make_gen(G.GEN_KEYED, seed=SEED, round=wl.CFG5["fill_round"], tag=0),
                 [int(s) for s in sizes])
    b.close()
    torch.cuda.synchronize()
    return arrays


def _flatten_bytes(sizes, tr, skip=()):
    """Arena bytes that hold every flatten output of the trace without reuse."""
    size = [int(s) for s in sizes]
    total = 0
    for r in range(tr["kind"].size):
        if r in skip:
            continue
        a = int(tr["target"][r])
        if tr["kind"][r] == wl.REQ_APPEND:
            size[a] += int(tr["length"][r])
        elif tr["kind"][r] == wl.REQ_FLATTEN:
            total += -(-size[a] * ELEM // 256) * 256
    return total


def _oracle_replay(sizes, tr, arrays_idx, skip=()):
    """CPU oracle: per array, its initial round then its requests in arrival order.
    Returns ({request: flatten output}, {array: final contents})."""
    V, F = _shapes(sizes)
    outs, finals = {}, {}
    for a in arrays_idx:
        o = Oracle(ELEM, V[a], F[a], forms=oracle.FORM_LIST)
        o.insert_gen(oracle.GEN_KEYED, int(sizes[a]), seed=SEED, round=wl.CFG5["fill_round"], tag=a)
        for r in np.nonzero(tr["target"] == a)[0]:
            r = int(r)
            if r in skip:
                continue
            k = tr["kind"][r]
            if k == wl.REQ_APPEND:
                o.insert_gen(oracle.GEN_KEYED, int(tr["length"][r]), seed=SEED,
                             round=wl.CFG5["append_round"], tag_shift=wl.CFG5["append_shift"], tag=r)
            elif k == wl.REQ_RW:
                o.rw(oracle.OP_ADD1)
            else:
                outs[r] = o.flatten()
        finals[a] = o.flatten()
        o.close()
    return outs, finals


def _run(arrays, tr, arrival, arena_bytes, cap, **kw):
    G = gg()
    n = tr["kind"].size
    arena = torch.zeros(max(arena_bytes, 256) // 4, dtype=torch.int32, device="cuda")
    out_len = torch.full((n,), -1, dtype=torch.int64, device="cuda")
    sv = G.Server(arrays, arena, cap, seed=SEED, **kw)
    try:
        res = sv.run(arrival, tr["kind"], tr["target"], tr["length"], out_len)
    finally:
        sv.close()
    res["arena"] = G.as_unsigned(arena)
    res["out_len"] = out_len.cpu().numpy()
    return res


def _outputs(res, tr):
    outs = {}
    for r in np.nonzero(tr["kind"] == wl.REQ_FLATTEN)[0]:
        r = int(r)
        if res["status"][r] != 0:
            continue
        off, n = int(res["out_offset"][r]) // ELEM, int(res["out_len"][r])
        outs[r] = res["arena"][off:off + n].copy()
    return outs


def _finals(arrays):
    return {a: gg().as_unsigned(arr.flatten()) for a, arr in enumerate(arrays)}


def _scenario(n_arr, n_req, seed_sizes=SEED):
    sizes = wl.cfg5_sizes(seed_sizes, n_arr, median_log2=10, sigma=1.0, cap_log2=16)
    tr = wl.cfg5_trace(SEED, n_req, n_arr, append_median_log2=6, append_cap_log2=14)
    return sizes, tr


@pytest.mark.parametrize("rate", [0.0, 2e6, 2e5])
def test_served_mix_equals_alone_and_oracle(rate):
    """Batched (2 lanes, steps of <= 16) vs per-request with nothing else in flight."""
    G = gg()
    sizes, tr = _scenario(48, 1500)
    arrival = wl.cfg5_arrivals_ns(tr["gap"], rate)
    arena_bytes = _flatten_bytes(sizes, tr) + 4096
    cap = 1 << 40
    pools = [G.Pool(256 * MiB), G.Pool(256 * MiB)]
    try:
        mix_arrays = _resident(pools[0], sizes)
        mix = _run(mix_arrays, tr, arrival, arena_bytes, cap, mode=G.SERVE_BATCHED, lanes=2, max_step=16)
        alone_arrays = _resident(pools[1], sizes)
        alone = _run(alone_arrays, tr, arrival, arena_bytes, cap, mode=G.SERVE_PER_REQUEST, depth=1)
        for res in (mix, alone):
            assert (res["status"] == 0).all()
            assert res["arena_wraps"] == 0 and res["rejected"] == 0
            assert (res["t_done_ns"] >= res["t_issue_ns"]).all()
            assert (res["t_issue_ns"] >= arrival).all()
        assert mix["issued"] == 1500 and mix["largest_step"] <= 16
        assert alone["steps"] == 1500
        mo, ao = _outputs(mix, tr), _outputs(alone, tr)
        assert mo.keys() == ao.keys()
        for r in mo:
            assert np.array_equal(mo[r], ao[r]), f"flatten request {r}: mix != alone"
        mf, af = _finals(mix_arrays), _finals(alone_arrays)
        for a in mf:
            assert np.array_equal(mf[a], af[a]), f"array {a}: mix != alone"
        # the oracle on a third of the arrays (every flatten of those, and their final state)
        sample = list(range(0, 48, 3))
        oo, of = _oracle_replay(sizes, tr, sample)
        for r, ref in oo.items():
            assert int(mix["out_len"][r]) == ref.size
            assert np.array_equal(mo[r], ref), f"flatten request {r}: mix != oracle"
        for a, ref in of.items():
            assert np.array_equal(mf[a], ref), f"array {a}: final != oracle"
        for arr in mix_arrays + alone_arrays:
            assert arr.last_error() == 0
            arr.close()
    finally:
        for p in pools:
            p.close()


def _expected_rejections(sizes, tr, cap):
    """The admission rule replayed in arrival order with nothing else in flight:
    an append of L elements is charged 2 L elem bytes against the capacity bounds
    elem (2 s_a + V_a F_a); a flatten needs its output bytes on top."""
    V, F = _shapes(sizes)
    size = [int(s) for s in sizes]
    charged = sum(ELEM * (2 * s + v * f) for s, v, f in zip(size, V, F))
    rej = set()
    for r in range(tr["kind"].size):
        a, k = int(tr["target"][r]), tr["kind"][r]
        if k == wl.REQ_APPEND:
            need = 2 * int(tr["length"][r]) * ELEM
            if charged + need > cap:
                rej.add(r)
            else:
                charged += need
                size[a] += int(tr["length"][r])
        elif k == wl.REQ_FLATTEN:
            if charged + -(-size[a] * ELEM // 256) * 256 > cap:
                rej.add(r)
    return rej


def test_served_admission_rejects_past_cap():
    G = gg()
    sizes, tr = _scenario(24, 600)
    V, F = _shapes(sizes)
    charged0 = sum(ELEM * (2 * int(s) + v * f) for s, v, f in zip(sizes, V, F))
    appended = int(tr["length"].sum())
    cap = charged0 + ELEM * appended  # about half the appends fit
    arrival = np.zeros(tr["kind"].size, dtype=np.uint64)
    expect = _expected_rejections(sizes, tr, cap)
    assert 0 < len(expect) < tr["kind"].size // 2
    arena_bytes = _flatten_bytes(sizes, tr, skip=expect) + 4096
    pool = G.Pool(128 * MiB)
    try:
        arrays = _resident(pool, sizes)
        res = _run(arrays, tr, arrival, arena_bytes, cap, mode=G.SERVE_PER_REQUEST, depth=1)
        got = set(int(r) for r in np.nonzero(res["status"] != 0)[0])
        assert got == expect
        assert (res["status"][sorted(got)] == G.ENOMEM).all()
        assert res["rejected"] == len(expect) and res["peak_charged_bytes"] <= cap
        oo, of = _oracle_replay(sizes, tr, range(24), skip=expect)
        outs = _outputs(res, tr)
        assert outs.keys() == oo.keys()
        for r in oo:
            assert np.array_equal(outs[r], oo[r])
        fin = _finals(arrays)
        for a in of:
            assert np.array_equal(fin[a], of[a])
        for arr in arrays:
            arr.close()
    finally:
        pool.close()


def test_served_batched_admission_and_small_arena():
    """Batched mode under a tight budget and a small arena that must wrap: the
    arrays equal the oracle replay without the rejected requests, every flatten
    reports the size its array had, and the budget is never exceeded."""
    G = gg()
    sizes, tr = _scenario(24, 600)
    V, F = _shapes(sizes)
    charged0 = sum(ELEM * (2 * int(s) + v * f) for s, v, f in zip(sizes, V, F))
    cap = charged0 + ELEM * int(tr["length"].sum())
    arrival = wl.cfg5_arrivals_ns(tr["gap"], 1e6)
    size, one = [int(x) for x in sizes], 0
    for r in range(tr["kind"].size):  # largest single flatten output, ignoring rejections
        a = int(tr["target"][r])
        if tr["kind"][r] == wl.REQ_APPEND:
            size[a] += int(tr["length"][r])
        elif tr["kind"][r] == wl.REQ_FLATTEN:
            one = max(one, -(-size[a] * ELEM // 256) * 256)
    arena_bytes = 2 * one  # room for a few outputs at a time
    pool = G.Pool(128 * MiB)
    try:
        arrays = _resident(pool, sizes)
        n = tr["kind"].size
        arena = torch.zeros(arena_bytes // 4, dtype=torch.int32, device="cuda")
        out_len = torch.zeros(n, dtype=torch.int64, device="cuda")
        sv = G.Server(arrays, arena, cap, seed=SEED, mode=G.SERVE_BATCHED, lanes=3, max_step=8)
        res = sv.run(arrival, tr["kind"], tr["target"], tr["length"], out_len)
        sv.close()
        rej = set(int(r) for r in np.nonzero(res["status"] != 0)[0])
        assert (res["status"][sorted(rej)] == G.ENOMEM).all()
        assert res["peak_charged_bytes"] <= cap and res["rejected"] == len(rej) > 0
        if _flatten_bytes(sizes, tr, skip=rej) > 2 * arena_bytes:
            assert res["arena_wraps"] > 0
        _, of = _oracle_replay(sizes, tr, range(24), skip=rej)
        fin = _finals(arrays)
        for a in of:
            assert np.array_equal(fin[a], of[a])
        lens = out_len.cpu().numpy()
        size = [int(s) for s in sizes]
        for r in range(n):
            a = int(tr["target"][r])
            if tr["kind"][r] == wl.REQ_APPEND and r not in rej:
                size[a] += int(tr["length"][r])
            elif tr["kind"][r] == wl.REQ_FLATTEN and r not in rej:
                assert int(lens[r]) == size[a]
        for arr in arrays:
            arr.close()
    finally:
        pool.close()


def test_served_flatten_larger_than_arena_is_rejected():
    G = gg()
    sizes = np.array([5000, 10], dtype=np.int64)
    tr = dict(kind=np.array([wl.REQ_FLATTEN, wl.REQ_FLATTEN, wl.REQ_APPEND, wl.REQ_FLATTEN], np.uint8),
              target=np.array([0, 1, 1, 1], np.uint32), length=np.array([0, 0, 7, 0], np.uint32))
    pool = G.Pool(64 * MiB)
    try:
        arrays = _resident(pool, sizes)
        res = _run(arrays, tr, np.zeros(4, np.uint64), 4096, 1 << 40, mode=G.SERVE_BATCHED)
        assert list(res["status"]) == [G.ENOMEM, 0, 0, 0]
        oo, _ = _oracle_replay(sizes, tr, [1])
        outs = _outputs(res, tr)
        assert np.array_equal(outs[1], oo[1]) and np.array_equal(outs[3], oo[3])
        for arr in arrays:
            arr.close()
    finally:
        pool.close()


def test_served_invalid_arguments():
    G = gg()
    pool = G.Pool(16 * MiB)
    try:
        arrays = _resident(pool, np.array([100, 200], dtype=np.int64))
        arena = torch.zeros(1024, dtype=torch.int32, device="cuda")
        for kw in (dict(lanes=0), dict(lanes=9), dict(max_step=0), dict(append_shift=0),
                   dict(append_shift=48), dict(rw_op=7), dict(seed=256), dict(depth=0)):
            with pytest.raises(G.GGAError):
                G.Server(arrays, arena, 1 << 30, **kw)
        with pytest.raises(G.GGAError):
            G.Server([arrays[0], arrays[0]], arena, 1 << 30)
        sv = G.Server(arrays, arena, 1 << 30, append_shift=4)
        z = np.zeros(2, np.uint64)
        bad = [
            (z, [0, 0], [0, 2], [1, 1]),                                  # target out of range
            (z, [3, 0], [0, 1], [1, 1]),                                  # unknown kind
            (z, [0, 0], [0, 1], [0, 1]),                                  # empty append
            (z, [0, 0], [0, 1], [17, 1]),                                 # longer than 2^shift
            (np.array([5, 4], np.uint64), [1, 1], [0, 1], [0, 0]),        # arrivals out of order
        ]
        for arr_ns, kind, target, length in bad:
            with pytest.raises(G.GGAError):
                sv.run(arr_ns, np.array(kind, np.uint8), np.array(target, np.uint32),
                       np.array(length, np.uint32))
        res = sv.run(z, np.array([0, 1], np.uint8), np.array([0, 1], np.uint32), np.array([16, 0], np.uint32))
        assert list(res["status"]) == [0, 0]
        sv.close()
        for arr in arrays:
            arr.close()
    finally:
        pool.close()


def test_served_step_wider_than_fused_limit():
    """A step with more r/w and flatten requests than one workgroup's offset table
    holds (4096) takes the two-launch path; results equal the oracle."""
    G = gg()
    n_arr = 4500
    sizes = np.array([1 + (a * 37) % 300 for a in range(n_arr)], dtype=np.int64)
    kind = np.array([wl.REQ_RW] * n_arr + [wl.REQ_FLATTEN] * n_arr + [wl.REQ_APPEND] * n_arr, np.uint8)
    target = np.tile(np.arange(n_arr, dtype=np.uint32), 3)
    length = np.where(kind == wl.REQ_APPEND, 5, 0).astype(np.uint32)
    tr = dict(kind=kind, target=target, length=length)
    pool = G.Pool(256 * MiB)
    try:
        arrays = _resident(pool, sizes)
        res = _run(arrays, tr, np.zeros(kind.size, np.uint64), _flatten_bytes(sizes, tr) + 4096, 1 << 40,
                   mode=G.SERVE_BATCHED, lanes=1, max_step=8192)  # one lane: every ready request joins its step
        assert (res["status"] == 0).all() and res["largest_step"] > 4096
        outs = _outputs(res, tr)
        fin = _finals(arrays)
        for a in range(0, n_arr, 97):
            o = Oracle(ELEM, *[x[a] for x in _shapes(sizes)], forms=oracle.FORM_LIST)
            o.insert_gen(oracle.GEN_KEYED, int(sizes[a]), seed=SEED, round=wl.CFG5["fill_round"], tag=a)
            o.rw(oracle.OP_ADD1)
            assert np.array_equal(outs[n_arr + a], o.flatten()), f"flatten of array {a}"
            o.insert_gen(oracle.GEN_KEYED, 5, seed=SEED, round=wl.CFG5["append_round"],
                         tag_shift=wl.CFG5["append_shift"], tag=2 * n_arr + a)
            assert np.array_equal(fin[a], o.flatten()), f"array {a}"
            o.close()
        for arr in arrays:
            arr.close()
    finally:
        pool.close()
