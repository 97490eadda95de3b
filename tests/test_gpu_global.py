"""GPU parity of access by global index (rw_g of Sec. VI-B): r/w by global index
gives exactly the r/w result, and gather returns the element at each global
index, against the CPU oracle."""
import numpy as np
import pytest
import torch

import oracle
from oracle import Oracle
from paper_2209_00103_amd import workloads as wl
from tests.gpu_util import assert_same, gg

pytestmark = pytest.mark.gpu
MiB = 1 << 20


@pytest.fixture
def pool():
    p = gg().Pool(512 * MiB)
    yield p
    p.close()


@pytest.mark.parametrize("elem,V,F", [(4, 37, 4), (8, 5, 1), (4, 512, 1024), (8, 1, 64)])
def test_rw_global_matches_oracle(pool, elem, V, F):
    G = gg()
    a, o = G.GGArray(pool, elem, V, F), Oracle(elem, V, F)
    rng = np.random.default_rng(V + F)
    for r, (n, p) in enumerate([(50, 0.5), (0, 0.5), (70000, 0.7), (3, 1.0), (200001, 0.4)]):
        vals, flags = wl.random_round(rng, n, p, elem)
        a.insert(G.to_device(vals), G.to_device(flags))
        o.insert(vals, flags)
        a.shrink(1, 5)
        o.shrink(1, 5)
        op = [G.ADD1, G.MUL3ADD1, G.ADD1_X30][r % 3]
        a.rw_global(op)
        o.rw(op)
        assert_same(a, o, f"round {r}")
    a.close()
    o.close()


def test_gather_matches_oracle(pool):
    G = gg()
    V, F = 300, 16
    a, o = G.GGArray(pool, 4, V, F), Oracle(4, V, F)
    for r, n in enumerate([1 << 16, 12345, 0, 99999]):  # sizes leave some LFVectors empty
        a.insert_gen(G.make_gen(G.GEN_BERNOULLI, seed=4, round=r), n)
        o.insert_gen(oracle.GEN_BERNOULLI, n, seed=4, round=r)
    a.shrink(1, 3)
    o.shrink(1, 3)
    size = o.size()
    assert a.size() == size
    rng = np.random.default_rng(8)
    idx = np.concatenate([rng.integers(0, size, 50000, dtype=np.uint64),
                          np.arange(size, dtype=np.uint64)[:: 97], np.array([0, size - 1], np.uint64)])
    ref, rc = o.gather(idx)
    assert rc == oracle.OK
    got = G.as_unsigned(a.gather(torch.from_numpy(idx.view(np.int64)).cuda()))
    assert np.array_equal(got, ref)
    assert a.last_error() == 0
    # past the end: those entries stay untouched, the others are written, ERANGE is sticky
    bad = np.array([size, 3, size + 1000, 1 << 60, size - 2], dtype=np.uint64)
    ref, rc = o.gather(bad, fill=0x5A5A5A5A)
    assert rc == oracle.ERANGE
    out = torch.full((bad.size,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
    a.gather(torch.from_numpy(bad.view(np.int64)).cuda(), out)
    assert np.array_equal(G.as_unsigned(out), ref)
    assert a.last_error() == G.ERANGE
    a.close()
    o.close()


def test_gather_empty_and_config2_full_size():
    """Gather on an empty array (only out-of-range) and, at the full configuration-2
    state (2.2e8 elements), 2^20 random indices against the oracle's flatten."""
    G = gg()
    pool = G.Pool(4 << 30)
    a = G.GGArray(pool, 4, 512, 1024)
    out = torch.full((2,), 7, dtype=torch.int32, device="cuda")
    a.gather(torch.zeros(2, dtype=torch.int64, device="cuda"), out)
    assert a.last_error() == G.ERANGE and (G.as_unsigned(out) == 7).all()
    a.close()
    a = G.GGArray(pool, 4, 512, 1024)
    o = Oracle(4, 512, 1024, forms=oracle.FORM_LIST)
    for r, n in enumerate(wl.cfg2_round_threads()):
        a.insert_gen(G.make_gen(G.GEN_ROUND_TAG, round=r, tag_shift=27), n)
        a.shrink(1, 10)
        o.insert_gen(oracle.GEN_ROUND_TAG, n, round=r, tag_shift=27)
        o.shrink(1, 10)
    a.rw_global(G.MUL3ADD1)
    o.rw(oracle.OP_MUL3ADD1)
    flat = o.flatten()
    idx = np.random.default_rng(1).integers(0, flat.size, 1 << 20, dtype=np.uint64)
    got = G.as_unsigned(a.gather(torch.from_numpy(idx.view(np.int64)).cuda()))
    assert np.array_equal(got, flat[idx])
    assert np.array_equal(G.as_unsigned(a.flatten()), flat)
    assert a.last_error() == 0
    o.close()
    a.close()
    pool.close()
