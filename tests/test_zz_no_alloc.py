"""GPU check of ggarray_insert_packed_noalloc, the packed insertion round that
allocates nothing (its tile offsets and look-back words live in the library's
static device scratch).  Through the C ABI, against ggarray_insert_packed on a
twin array and against the CPU oracle, bit-exact, on calls in a row whose inputs
shrink (several tiles per LFVector, then fewer, then one), with another array's
rounds in between sharing the scratch; a round beyond the scratch's 65536 tiles
is refused with GGA_ERANGE before anything is queued."""
import numpy as np
import pytest
import torch

import oracle
from oracle import Oracle
from paper_2209_00103_amd import workloads as wl
from tests.gpu_util import assert_same, dev, gg, gpu_flat, gpu_sizes

pytestmark = pytest.mark.gpu

MiB = 1 << 20
TILE = 1024


@pytest.fixture
def pool():
    p = gg().Pool(1024 * MiB)
    yield p
    p.close()


def _same_arrays(a, b, what):
    assert a.last_error() == 0 and b.last_error() == 0, what
    np.testing.assert_array_equal(gpu_sizes(b), gpu_sizes(a), err_msg=f"{what}: sizes")
    fa, fb = gpu_flat(a), gpu_flat(b)
    assert fa.shape == fb.shape and np.array_equal(fa, fb), f"{what}: contents differ"
    assert a.capacity() == b.capacity(), f"{what}: capacity"


@pytest.mark.parametrize("elem,V,F", [(8, 4, 1024), (4, 3, 1), (8, 64, 16)])
def test_noalloc_matches_packed(pool, elem, V, F):
    G = gg()
    print(f"case noalloc elem={elem} V={V} F={F}", flush=True)
    rng = np.random.default_rng(1000 + V * 7 + F)
    ref = G.GGArray(pool, elem, V, F)      # the allocating entry point
    na = G.GGArray(pool, elem, V, F)       # the allocation-free one
    o = Oracle(elem, V, F)
    other = G.GGArray(pool, elem, 2, F)    # shares the scratch between the calls
    o_other = Oracle(elem, 2, F)
    # calls in a row, each with fewer threads than the one before: 6, 2, then 1
    # tiles per LFVector (the later calls find the earlier calls' words)
    for k, chunk in enumerate([5 * TILE + 999, TILE + 17, 300]):
        n = V * chunk
        counts = rng.integers(0, 17, size=n, dtype=np.uint8)
        if k == 1:
            counts[rng.random(n) < 0.5] = 0
        total = int(counts.sum(dtype=np.uint64))
        vals, _ = wl.random_round(rng, total, 1.0, elem)
        dv, dc = dev(vals), dev(counts)
        ref.insert_packed(dv, dc)
        na.insert_packed_noalloc(dv, dc)
        assert o.insert_packed(vals, counts) == oracle.OK
        _same_arrays(ref, na, f"call {k}")
        assert_same(na, o, f"call {k} against the oracle")
        # another array's ticketed round through the same scratch
        oc = rng.integers(0, 9, size=2 * (3 * TILE + 5), dtype=np.uint8)
        ov, _ = wl.random_round(rng, int(oc.sum(dtype=np.uint64)), 1.0, elem)
        other.insert_packed_noalloc(dev(ov), dev(oc))
        assert o_other.insert_packed(ov, oc) == oracle.OK
        assert_same(other, o_other, f"other array after call {k}")
    # the allocation-free calls never grew the array's own look-back or offset words
    assert na.footprint()["lookback"] == 0
    assert other.footprint()["lookback"] == 0
    for x in (ref, na, other):
        x.close()
    o.close()
    o_other.close()


def test_noalloc_limit(pool):
    G = gg()
    V = 8
    a = G.GGArray(pool, 4, V, 1024)
    n = V * 8193 * TILE  # 65544 tiles: beyond the scratch
    counts = torch.zeros(n, dtype=torch.uint8, device="cuda")
    vals = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(G.GGAError) as e:
        a.insert_packed_noalloc(vals, counts)
    assert e.value.status == G.ERANGE
    assert a.size() == 0
    # exactly at the limit (65536 tiles): accepted; one round into an empty array
    # flattens to the first sum(counts) values
    m = V * 8192 * TILE
    c = counts[:m]
    c[::4096] = 1
    v = torch.arange(m // 4096, dtype=torch.int32, device="cuda")
    a.insert_packed_noalloc(v, c)
    assert a.last_error() == 0
    got = G.as_unsigned(a.flatten())
    assert np.array_equal(got, np.arange(m // 4096, dtype=np.uint32))
    a.close()
