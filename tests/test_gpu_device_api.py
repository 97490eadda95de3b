"""GPU tests of the device-side API: user kernels that grow a GGArray from inside
with gga::block_push_back (the block-cooperative push_back of Alg. 1), against the
CPU oracle."""
import ctypes
import os

import numpy as np
import pytest
import torch

import oracle
from oracle import Oracle
from tests.conftest import ROOT
from tests.gpu_util import gg, gpu_sizes

pytestmark = pytest.mark.gpu
MiB = 1 << 20
KLIB = os.path.join(ROOT, "tests", "device", "libggtest.so")


@pytest.fixture(scope="module")
def K():
    assert os.path.exists(KLIB), f"{KLIB} missing: run __graft_entry__.build()"
    L = ctypes.CDLL(KLIB)
    L.ggt_bernoulli_push.argtypes = [ctypes.c_char_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                     ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                     ctypes.c_void_p]
    L.ggt_bernoulli_push.restype = ctypes.c_int
    L.ggt_ref_bytes.restype = ctypes.c_uint64
    return L


def _push(K, arr, blocks, threads, seed, round0, rounds):
    nb = int(K.ggt_ref_bytes())
    ref = arr.device_ref(nb)
    s = torch.cuda.current_stream().cuda_stream
    assert K.ggt_bernoulli_push(ref, nb, arr.elem_bytes, blocks, threads, seed, round0, rounds, s) == 0
    arr.device_done()


@pytest.mark.parametrize("elem,V,F,threads,rounds", [(4, 64, 16, 256, 3), (8, 33, 1, 64, 5),
                                                     (4, 8, 1024, 1024, 2), (4, 5, 2, 128, 9)])
def test_one_block_per_lfvector_matches_oracle(K, elem, V, F, threads, rounds):
    """Block b owns LFVector b: the order is fixed (thread order, rounds in order),
    so the result equals the oracle's Bernoulli rounds exactly."""
    G = gg()
    pool = G.Pool(256 * MiB)
    a, o = G.GGArray(pool, elem, V, F), Oracle(elem, V, F)
    try:
        _push(K, a, V, threads, 3, 0, rounds)          # several rounds in one kernel
        _push(K, a, V, threads, 3, rounds, 1)          # and one more launch
        for r in range(rounds + 1):
            o.insert_gen(oracle.GEN_BERNOULLI, V * threads, seed=3, round=r)
        a.rw(G.ADD1)  # the library's own kernels see the new sizes
        o.rw(oracle.OP_ADD1)
        np.testing.assert_array_equal(gpu_sizes(a), o.vector_sizes())
        assert np.array_equal(G.as_unsigned(a.flatten()), o.flatten())
        assert a.capacity() == o.capacity() and a.last_error() == 0
    finally:
        a.close()
        o.close()
        pool.close()


def test_many_blocks_per_lfvector_multisets(K):
    """Eight blocks share each LFVector: the ranges come in atomic order, so each
    LFVector holds the union of its blocks' elements (compared as a multiset), and
    the bucket allocation of concurrently growing blocks stays consistent."""
    G = gg()
    V, blocks, threads, rounds = 16, 128, 256, 4
    pool = G.Pool(256 * MiB)
    a = G.GGArray(pool, 4, V, 4)
    o = Oracle(4, blocks, 4)  # one oracle LFVector per block
    try:
        _push(K, a, blocks, threads, 9, 0, rounds)
        for r in range(rounds):
            o.insert_gen(oracle.GEN_BERNOULLI, blocks * threads, seed=9, round=r)
        flat = G.as_unsigned(a.flatten())
        pre = a.prefix().cpu().numpy()
        ob = o.flatten()
        opre = o.prefix()
        for v in range(V):
            want = np.sort(np.concatenate([ob[opre[b]:opre[b + 1]] for b in range(v, blocks, V)]))
            got = np.sort(flat[pre[v]:pre[v + 1]])
            assert np.array_equal(got, want), f"LFVector {v}"
        sizes = gpu_sizes(a)
        cap = a.capacity()
        nb = [int(oracle.lib().orc_nbuckets_for(4, int(s))) for s in sizes]
        assert cap == sum(4 * ((1 << k) - 1) for k in nb)
        assert a.last_error() == 0
    finally:
        a.close()
        o.close()
        pool.close()


def test_device_push_out_of_memory_is_reported(K):
    G = gg()
    pool = G.Pool(3 * MiB)  # 1 MiB of buckets
    a = G.GGArray(pool, 4, 4, 1024)
    try:
        _push(K, a, 4, 1024, 1, 0, 200)  # about 100 k elements per LFVector: 2 MB of buckets in all
        assert a.last_error() == G.ENOMEM
    finally:
        a.close()
        pool.close()
