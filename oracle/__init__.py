"""CPU oracle for the GGArray hot path (Python side of ``ggoracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline leg
of the benchmark may import this package.  The product library never imports,
links or calls it.  It shares no code with the HIP path; the only module both
sides consume is the seeded workload generator, which holds none of the data
structure's arithmetic.

Parity pins: every function here is pinned by ``tests/test_oracle_pins.py``
against closed forms, brute force, textbook special cases (stream compaction)
and published SplitMix64 output, never against the HIP path.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ggoracle.c")
_LIB = os.path.join(_HERE, "libggoracle.so")

OK, EINVAL, ENOMEM, ERANGE = 0, -1, -2, -3
FORM_LIST, FORM_BUCKETS = 1, 2
OP_ADD1, OP_MUL3ADD1, OP_ADD1_X30 = 0, 1, 2
GEN_BERNOULLI, GEN_ROUND_TAG, GEN_POISSON, GEN_KEYED = 1, 2, 3, 4


def build(force: bool = False) -> str:
    """Compile the oracle with the host C compiler (plain C99, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-shared", "-fPIC",
                        _SRC, "-o", tmp], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        u32, u64, i32, vp = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p
        sig = {
            "orc_splitmix64": (u64, [u64]),
            "orc_K": (u64, [u64, u64, u64]),
            "orc_walk": (None, [u64, u64, ctypes.POINTER(u32), ctypes.POINTER(u64)]),
            "orc_walk_many": (None, [u64, vp, u64, vp, vp]),
            "orc_bucket_start": (u64, [u64, u32]),
            "orc_nbuckets_for": (u32, [u64, u64]),
            "orc_create": (vp, [u32, u32, u64, i32]),
            "orc_destroy": (None, [vp]),
            "orc_insert": (i32, [vp, vp, vp, u64]),
            "orc_insert_counts": (i32, [vp, vp, vp, u32, u64]),
            "orc_insert_segments": (i32, [vp, vp, vp, u64]),
            "orc_insert_packed": (i32, [vp, vp, u64, vp, u64]),
            "orc_insert_gen": (i32, [vp, u32, u64, u32, u32, u32, vp, u64, u64]),
            "orc_shrink": (i32, [vp, u32, u32]),
            "orc_rw": (i32, [vp, u32]),
            "orc_size": (u64, [vp]),
            "orc_vector_sizes": (None, [vp, vp]),
            "orc_prefix": (None, [vp, vp]),
            "orc_capacity": (u64, [vp]),
            "orc_vector_nbuckets": (None, [vp, vp]),
            "orc_alloc_count": (u64, [vp]),
            "orc_free_count": (u64, [vp]),
            "orc_flatten": (i32, [vp, vp, u64]),
            "orc_at": (i32, [vp, u64, ctypes.POINTER(u64)]),
            "orc_gather": (i32, [vp, vp, u64, vp]),
            "orc_check": (ctypes.c_int64, [vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def splitmix64(x: int) -> int:
    return int(lib().orc_splitmix64(x))


def K(seed: int, a: int, b: int) -> int:
    return int(lib().orc_K(seed, a, b))


def walk(F: int, idx: int) -> tuple[int, int]:
    """(bucket, offset) of local index idx by walking bucket starts."""
    b, off = ctypes.c_uint32(), ctypes.c_uint64()
    lib().orc_walk(F, idx, ctypes.byref(b), ctypes.byref(off))
    return b.value, off.value


def walk_many(F: int, idx: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    idx = np.ascontiguousarray(idx, dtype=np.uint64)
    b = np.zeros(idx.size, dtype=np.uint32)
    off = np.zeros(idx.size, dtype=np.uint64)
    lib().orc_walk_many(F, _ptr(idx), idx.size, _ptr(b), _ptr(off))
    return b, off


def bucket_start(F: int, b: int) -> int:
    return int(lib().orc_bucket_start(F, b))


def nbuckets_for(F: int, s: int) -> int:
    return int(lib().orc_nbuckets_for(F, s))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"oracle {what} failed with status {status}")
        self.status = status


class Oracle:
    """One GGArray state held by the CPU oracle."""

    def __init__(self, elem_bytes: int, n_vectors: int, first_bucket: int,
                 forms: int = FORM_LIST | FORM_BUCKETS):
        self.elem_bytes = elem_bytes
        self.n_vectors = n_vectors
        self.first_bucket = first_bucket
        self.dtype = np.uint32 if elem_bytes == 4 else np.uint64
        self._h = lib().orc_create(elem_bytes, n_vectors, first_bucket, forms)
        if not self._h:
            raise OracleError(EINVAL, "create")

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st, what):
        if st != OK:
            raise OracleError(st, what)

    def insert(self, values: np.ndarray, flags: np.ndarray | None = None):
        values = np.ascontiguousarray(values, dtype=self.dtype)
        if flags is not None:
            flags = np.ascontiguousarray(flags, dtype=np.uint8)
            assert flags.shape == values.shape
        self._chk(lib().orc_insert(self._h, _ptr(values), _ptr(flags), values.size), "insert")

    def insert_counts(self, values: np.ndarray, counts: np.ndarray, max_count: int):
        values = np.ascontiguousarray(values, dtype=self.dtype)
        counts = np.ascontiguousarray(counts, dtype=np.uint8)
        assert values.size == counts.size * max_count
        self._chk(lib().orc_insert_counts(self._h, _ptr(values), _ptr(counts), max_count,
                                          counts.size), "insert_counts")

    def insert_packed(self, values: np.ndarray, counts: np.ndarray) -> int:
        """Thread g inserts counts[g] elements, the next ones of `values` in thread
        order; returns the status (ERANGE when the counts need more values)."""
        values = np.ascontiguousarray(values, dtype=self.dtype)
        counts = np.ascontiguousarray(counts, dtype=np.uint8)
        return int(lib().orc_insert_packed(self._h, _ptr(values), values.size, _ptr(counts), counts.size))

    def insert_segments(self, values: np.ndarray, prefix: np.ndarray) -> int:
        """LFVector v appends values[prefix[v]:prefix[v + 1]]; returns the status
        (ERANGE for an invalid segment, whose LFVector is left unchanged)."""
        values = np.ascontiguousarray(values, dtype=self.dtype)
        prefix = np.ascontiguousarray(prefix, dtype=np.uint64)
        assert prefix.size == self.n_vectors + 1
        return int(lib().orc_insert_segments(self._h, _ptr(values), _ptr(prefix), values.size))

    def insert_gen(self, kind: int, n_threads: int, seed: int = 0, round: int = 0,
                   tag_shift: int | None = None, max_count: int = 0,
                   thresholds: np.ndarray | None = None, tag: int = 0):
        if tag_shift is None:
            tag_shift = 32 if kind == GEN_KEYED else 0
        thr = None if thresholds is None else np.ascontiguousarray(thresholds, dtype=np.uint64)
        self._chk(lib().orc_insert_gen(self._h, kind, seed, round, tag_shift, max_count,
                                       _ptr(thr), n_threads, tag), "insert_gen")

    def shrink(self, num: int, den: int):
        self._chk(lib().orc_shrink(self._h, num, den), "shrink")

    def rw(self, op: int):
        self._chk(lib().orc_rw(self._h, op), "rw")

    def size(self) -> int:
        return int(lib().orc_size(self._h))

    def capacity(self) -> int:
        return int(lib().orc_capacity(self._h))

    def vector_sizes(self) -> np.ndarray:
        out = np.zeros(self.n_vectors, dtype=np.uint64)
        lib().orc_vector_sizes(self._h, _ptr(out))
        return out

    def prefix(self) -> np.ndarray:
        out = np.zeros(self.n_vectors + 1, dtype=np.uint64)
        lib().orc_prefix(self._h, _ptr(out))
        return out

    def vector_nbuckets(self) -> np.ndarray:
        out = np.zeros(self.n_vectors, dtype=np.uint32)
        lib().orc_vector_nbuckets(self._h, _ptr(out))
        return out

    def alloc_count(self) -> int:
        return int(lib().orc_alloc_count(self._h))

    def free_count(self) -> int:
        return int(lib().orc_free_count(self._h))

    def flatten(self, out_cap: int | None = None) -> np.ndarray:
        n = self.size()
        cap = n if out_cap is None else out_cap
        out = np.zeros(max(cap, 1), dtype=self.dtype)
        self._chk(lib().orc_flatten(self._h, _ptr(out), cap), "flatten")
        return out[:n]

    def at(self, i: int) -> int | None:
        """Element at global index i (None past the end)."""
        e = ctypes.c_uint64()
        rc = int(lib().orc_at(self._h, i, ctypes.byref(e)))
        return None if rc == ERANGE else e.value

    def gather(self, idx: np.ndarray, fill: int = 0) -> tuple[np.ndarray, int]:
        """(out, status): out[k] = element at idx[k]; out of range leaves fill."""
        idx = np.ascontiguousarray(idx, dtype=np.uint64)
        out = np.full(max(idx.size, 1), fill, dtype=self.dtype)
        rc = int(lib().orc_gather(self._h, _ptr(idx), idx.size, _ptr(out)))
        return out[:idx.size], rc

    def flatten_status(self, out: np.ndarray) -> int:
        return int(lib().orc_flatten(self._h, _ptr(out), out.size))

    def check(self) -> int:
        return int(lib().orc_check(self._h))
