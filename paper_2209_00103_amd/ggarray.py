"""ctypes binding of ``libggarray.so`` (the C ABI in ``include/ggarray.h``).

Argument marshalling only: every operation runs in the library's HIP kernels.
PyTorch supplies device memory (tensors) and streams (the current stream unless
one is given).  Elements live in int32 / int64 tensors that hold the unsigned
bit patterns; ``as_unsigned`` views them as numpy uint32 / uint64.

The library must be built in-tree (``__graft_entry__.build()``); importing this
module raises if it is missing, there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libggarray.so")

OK, EINVAL, ENOMEM, ERANGE, EHIP, EBUSY = 0, -1, -2, -3, -4, -5
ADD1, MUL3ADD1, ADD1_X30 = 0, 1, 2
RW_NONE = 0xFFFFFFFF  # a step without r/w
GEN_BERNOULLI, GEN_ROUND_TAG, GEN_POISSON, GEN_KEYED = 1, 2, 3, 4
REQ_APPEND, REQ_RW, REQ_FLATTEN = 0, 1, 2
SERVE_BATCHED, SERVE_PER_REQUEST = 0, 1

_u32, _u64, _i32, _vp = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p
_P = ctypes.POINTER


class GenSpec(ctypes.Structure):
    _fields_ = [("kind", _u32), ("round", _u32), ("seed", _u64), ("tag_shift", _u32),
                ("max_count", _u32), ("thresholds", _u64 * 16), ("tag", _u64)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("cap_bytes", _u64), ("mode", _u32), ("lanes", _u32), ("max_step", _u32),
                ("depth", _u32), ("seed", _u64), ("append_round", _u32), ("append_shift", _u32),
                ("rw_op", _u32)]


class Trace(ctypes.Structure):
    _fields_ = [("n", _u64), ("arrival_ns", _vp), ("kind", _vp), ("target", _vp), ("length", _vp)]


# name -> argtypes (every entry point returns int status unless listed in _RES)
_SIGS = {
    "gga_last_hip_error": [],
    "gga_strerror": [_i32],
    "gga_pool_create": [_P(_vp), _vp, _u64, _vp],
    "gga_pool_destroy": [_vp],
    "gga_pool_stats": [_vp, _P(_u64), _vp],
    "gga_pool_set_fault": [_vp, _u64, _vp],
    "ggarray_create": [_P(_vp), _vp, _u32, _u32, _u64, _vp],
    "ggarray_destroy": [_vp, _vp],
    "ggarray_insert": [_vp, _vp, _vp, _u64, _vp],
    "ggarray_insert_counts": [_vp, _vp, _vp, _u32, _u64, _vp],
    "ggarray_insert_packed": [_vp, _vp, _u64, _vp, _u64, _vp],
    "ggarray_insert_packed_noalloc": [_vp, _vp, _u64, _vp, _u64, _vp],
    "ggarray_insert_gen": [_vp, _P(GenSpec), _u64, _vp],
    "ggarray_shrink": [_vp, _u32, _u32, _vp],
    "ggarray_insert_gen_shrink": [_vp, _P(GenSpec), _u64, _u32, _u32, _vp],
    "ggarray_insert_gen_rounds": [_vp, _P(GenSpec), _P(ctypes.c_uint64), _u32, _u32, _u32, _u32, _vp],
    "ggarray_kernel_timing": [_vp, _u32],
    "ggarray_set_spin_limit": [_vp, _u32],
    "ggarray_kernel_ms": [_vp, _u32, _P(ctypes.c_float)],
    "ggarray_rw": [_vp, _u32, _vp],
    "ggarray_flatten": [_vp, _vp, _u64, _vp],
    "ggarray_rw_global": [_vp, _u32, _vp],
    "ggarray_device_ref": [_vp, _vp, _u64],
    "ggarray_device_done": [_vp, _vp],
    "ggarray_gather": [_vp, _vp, _u64, _vp, _vp],
    "ggarray_size": [_vp, _P(_u64), _vp],
    "ggarray_capacity": [_vp, _P(_u64), _vp],
    "ggarray_footprint": [_vp, _P(_u64)],
    "ggarray_insert_segments": [_vp, _vp, _vp, _u64, _vp],
    "ggarray_vector_sizes": [_vp, _vp, _vp],
    "ggarray_prefix": [_vp, _vp, _vp],
    "ggarray_last_error": [_vp, _vp],
    "gga_static_create": [_P(_vp), _vp, _u64, _u32, _vp],
    "gga_static_destroy": [_vp, _vp],
    "gga_static_insert": [_vp, _vp, _vp, _u64, _vp],
    "gga_static_insert_gen": [_vp, _P(GenSpec), _u64, _vp],
    "gga_static_insert_gen_atomic": [_vp, _P(GenSpec), _u64, _vp],
    "gga_static_rw": [_vp, _u32, _vp],
    "gga_static_size": [_vp, _P(_u64), _vp],
    "gga_static_last_error": [_vp, _vp],
    "gga_static_clear": [_vp, _vp],
    "gga_static_set_size": [_vp, _u64, _vp],
    "gga_batch_create": [_P(_vp), _vp, _u32, _vp],
    "gga_batch_destroy": [_vp, _vp],
    "gga_batch_insert_gen": [_vp, _P(GenSpec), _vp, _vp],
    "gga_batch_step": [_vp, _vp, _u32, _vp, _u32, _vp, _u64, _vp],
    "gga_batch_step_clear": [_vp, _vp, _u32, _vp, _u32, _vp, _u64, _vp],
    "gga_batch_shrink": [_vp, _u32, _u32, _vp],
    "gga_batch_rw": [_vp, _u32, _vp],
    "gga_batch_flatten": [_vp, _vp, _u64, _vp],
    "gga_batch_set_grid": [_vp, _u32],
    "gga_batch_offsets": [_vp, _vp, _vp],
    "gga_batch_last_error": [_vp, _vp],
    "gga_semi_create": [_P(_vp), _u32, _u64, _vp],
    "gga_semi_destroy": [_vp, _vp],
    "gga_semi_insert": [_vp, _vp, _vp, _u64, _vp],
    "gga_semi_insert_gen": [_vp, _P(GenSpec), _u64, _vp],
    "gga_semi_rw": [_vp, _u32, _vp],
    "gga_semi_size": [_vp, _P(_u64), _vp],
    "gga_semi_data": [_vp, _P(_vp), _P(_u64)],
    "gga_semi_resizes": [_vp, _P(_u64)],
    "gga_mapped_create": [_P(_vp), _u32, _u64, _vp],
    "gga_mapped_destroy": [_vp, _vp],
    "gga_mapped_insert": [_vp, _vp, _vp, _u64, _vp],
    "gga_mapped_insert_gen": [_vp, _P(GenSpec), _u64, _vp],
    "gga_mapped_rw": [_vp, _u32, _vp],
    "gga_mapped_size": [_vp, _P(_u64), _vp],
    "gga_mapped_data": [_vp, _P(_vp), _P(_u64)],
    "gga_mapped_maps": [_vp, _P(_u64)],
    "gga_server_create": [_P(_vp), _vp, _u32, _vp, _u64, _P(ServerConfig)],
    "gga_server_destroy": [_vp],
    "gga_server_run": [_vp, _P(Trace), _vp, _vp, _vp, _vp, _vp, _vp],
}
_RES = {"gga_strerror": ctypes.c_char_p, "gga_last_hip_error": ctypes.c_char_p}

_lib = None


def lib() -> ctypes.CDLL:
    """Load the HIP library (raises ImportError when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = _RES.get(name, _i32)
        _lib = L
    return _lib


class GGAError(RuntimeError):
    def __init__(self, status: int, what: str):
        msg = lib().gga_strerror(status).decode()
        if status == EHIP:
            detail = lib().gga_last_hip_error().decode()
            if detail:
                msg += f" [{detail}]"
        super().__init__(f"{what}: {msg} ({status})")
        self.status = status


def _check(status: int, what: str) -> None:
    if status != OK:
        raise GGAError(status, what)


def _stream(stream) -> ctypes.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dtype(elem_bytes: int) -> torch.dtype:
    return torch.int32 if elem_bytes == 4 else torch.int64


def _dev_ptr(t: torch.Tensor | None, what: str, min_numel: int = 0, itemsize: int | None = None):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{what} must be a contiguous device tensor")
    if itemsize is not None and t.element_size() != itemsize:
        raise ValueError(f"{what} must have {itemsize}-byte elements")
    if t.numel() < min_numel:
        raise ValueError(f"{what} holds {t.numel()} elements, needs {min_numel}")
    return ctypes.c_void_p(t.data_ptr())


def to_device(a: np.ndarray, device="cuda") -> torch.Tensor:
    """numpy uint32/uint64/uint8 array -> device tensor with the same bits."""
    a = np.ascontiguousarray(a)
    view = {np.dtype(np.uint32): np.int32, np.dtype(np.uint64): np.int64,
            np.dtype(np.uint8): np.uint8}[a.dtype]
    return torch.from_numpy(a.view(view)).to(device)


def as_unsigned(t: torch.Tensor) -> np.ndarray:
    """Device or host int32/int64 tensor -> numpy uint32/uint64 array."""
    a = t.detach().cpu().numpy()
    return a.view(np.uint32 if a.dtype == np.int32 else np.uint64)


def make_gen(kind: int, seed: int = 0, round: int = 0, tag_shift: int | None = None, max_count: int = 0,
             thresholds=None, tag: int = 0) -> GenSpec:
    if tag_shift is None:
        tag_shift = 32 if kind == GEN_KEYED else 0
    g = GenSpec()
    g.kind, g.round, g.seed, g.tag_shift, g.max_count, g.tag = kind, round, seed, tag_shift, max_count, tag
    if thresholds is not None:
        thr = [int(x) for x in np.asarray(thresholds, dtype=np.uint64)]
        for k, x in enumerate(thr[:16]):
            g.thresholds[k] = x
    return g


class Pool:
    """Device bucket pool over a caller-owned HBM tensor."""

    def __init__(self, nbytes: int, device="cuda", stream=None):
        self.mem = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
        self._h = _vp()
        _check(lib().gga_pool_create(ctypes.byref(self._h), self.mem.data_ptr(), int(nbytes),
                                     _stream(stream)), "gga_pool_create")

    @property
    def handle(self):
        return self._h

    def stats(self, stream=None) -> dict:
        out = (_u64 * 7)()
        _check(lib().gga_pool_stats(self._h, out, _stream(stream)), "gga_pool_stats")
        keys = ("in_use", "high_water", "allocs", "frees", "bump", "limit", "attempts")
        return dict(zip(keys, [int(x) for x in out]))

    def set_fault(self, fault_at: int, stream=None):
        _check(lib().gga_pool_set_fault(self._h, int(fault_at), _stream(stream)), "gga_pool_set_fault")

    def close(self):
        if self._h:
            _check(lib().gga_pool_destroy(self._h), "gga_pool_destroy")
            self._h = _vp()


class GGArray:
    """An array of LFVectors on the GPU (see include/ggarray.h)."""

    def __init__(self, pool: Pool, elem_bytes: int, n_vectors: int, first_bucket: int, stream=None):
        self.pool = pool
        self.elem_bytes = elem_bytes
        self.n_vectors = n_vectors
        self.first_bucket = first_bucket
        self.dtype = _dtype(elem_bytes)
        self._h = _vp()
        _check(lib().ggarray_create(ctypes.byref(self._h), pool.handle, elem_bytes, n_vectors,
                                    first_bucket, _stream(stream)), "ggarray_create")

    def insert(self, values: torch.Tensor, flags: torch.Tensor | None = None, n_threads=None,
               stream=None):
        n = values.numel() if n_threads is None else int(n_threads)
        vp = _dev_ptr(values, "values", n, self.elem_bytes)
        fp = _dev_ptr(flags, "flags", n, 1)
        _check(lib().ggarray_insert(self._h, vp, fp, n, _stream(stream)), "ggarray_insert")

    def insert_counts(self, values: torch.Tensor, counts: torch.Tensor, max_count: int, stream=None):
        n = counts.numel()
        vp = _dev_ptr(values, "values", n * max_count, self.elem_bytes)
        cp = _dev_ptr(counts, "counts", n, 1)
        _check(lib().ggarray_insert_counts(self._h, vp, cp, max_count, n, _stream(stream)),
               "ggarray_insert_counts")

    def insert_gen(self, gen: GenSpec, n_threads: int, stream=None):
        _check(lib().ggarray_insert_gen(self._h, ctypes.byref(gen), int(n_threads), _stream(stream)),
               "ggarray_insert_gen")

    def insert_packed(self, values: torch.Tensor, counts: torch.Tensor, n_values=None, stream=None):
        """Thread g inserts counts[g] elements, the next ones of `values` (packed in thread order)."""
        n = counts.numel()
        nv = values.numel() if n_values is None else int(n_values)
        vp = _dev_ptr(values, "values", nv, self.elem_bytes) if nv else None
        cp = _dev_ptr(counts, "counts", n, 1)
        _check(lib().ggarray_insert_packed(self._h, vp, nv, cp, n, _stream(stream)), "ggarray_insert_packed")

    def insert_packed_noalloc(self, values: torch.Tensor, counts: torch.Tensor, n_values=None, stream=None):
        """insert_packed through the entry point that allocates nothing (library scratch, at most 65536 tiles)."""
        n = counts.numel()
        nv = values.numel() if n_values is None else int(n_values)
        vp = _dev_ptr(values, "values", nv, self.elem_bytes) if nv else None
        cp = _dev_ptr(counts, "counts", n, 1)
        _check(lib().ggarray_insert_packed_noalloc(self._h, vp, nv, cp, n, _stream(stream)),
               "ggarray_insert_packed_noalloc")

    def shrink(self, num: int, den: int, stream=None):
        _check(lib().ggarray_shrink(self._h, num, den, _stream(stream)), "ggarray_shrink")

    def kernel_timing(self, on: bool):
        """Measurement aid: r/w and flatten dispatches record events at their own start and end."""
        _check(lib().ggarray_kernel_timing(self._h, 1 if on else 0), "ggarray_kernel_timing")

    def kernel_ms(self, kind: int) -> float:
        """Duration of the last timed r/w (0) or flatten (1) kernel, in ms."""
        ms = ctypes.c_float()
        _check(lib().ggarray_kernel_ms(self._h, int(kind), ctypes.byref(ms)), "ggarray_kernel_ms")
        return float(ms.value)

    def insert_gen_shrink(self, gen: GenSpec, n_threads: int, num: int, den: int, stream=None):
        """insert_gen then shrink(num, den), as one launch where the round allows it."""
        _check(lib().ggarray_insert_gen_shrink(self._h, ctypes.byref(gen), int(n_threads), num, den,
                                               _stream(stream)), "ggarray_insert_gen_shrink")

    def insert_gen_rounds(self, gens, n_threads, num: int = 0, den: int = 1, clear_first: bool = False,
                          stream=None):
        """With clear_first, shrink(1, 1) first; then rounds r = 0.. of n_threads[r]
        threads with gens[r], each followed by shrink(num, den) when num > 0; one
        launch where the rounds allow it."""
        n = len(gens)
        if len(n_threads) != n:
            raise ValueError("one thread count per generator")
        ga = (GenSpec * max(n, 1))(*gens)
        na = (ctypes.c_uint64 * max(n, 1))(*[int(x) for x in n_threads])
        _check(lib().ggarray_insert_gen_rounds(self._h, ga, na, n, num, den, int(bool(clear_first)),
                                               _stream(stream)),
               "ggarray_insert_gen_rounds")

    def rw(self, op: int, stream=None):
        _check(lib().ggarray_rw(self._h, op, _stream(stream)), "ggarray_rw")

    def device_ref(self, nbytes: int) -> bytes:
        """The array's device descriptor (for user kernels that push elements)."""
        buf = ctypes.create_string_buffer(nbytes)
        _check(lib().ggarray_device_ref(self._h, buf, nbytes), "ggarray_device_ref")
        return buf.raw

    def device_done(self, stream=None):
        _check(lib().ggarray_device_done(self._h, _stream(stream)), "ggarray_device_done")

    def rw_global(self, op: int, stream=None):
        _check(lib().ggarray_rw_global(self._h, op, _stream(stream)), "ggarray_rw_global")

    def gather(self, idx: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """out[k] = element at global index idx[k] (idx: device int64 tensor)."""
        n = idx.numel()
        if out is None:
            out = torch.zeros(n, dtype=_dtype(self.elem_bytes), device=idx.device)
        _check(lib().ggarray_gather(self._h, _dev_ptr(idx, "idx", n, 8), n,
                                    _dev_ptr(out, "out", n, self.elem_bytes), _stream(stream)),
               "ggarray_gather")
        return out

    def flatten_into(self, out: torch.Tensor, stream=None):
        _check(lib().ggarray_flatten(self._h, _dev_ptr(out, "out", 0, self.elem_bytes), out.numel(),
                                     _stream(stream)), "ggarray_flatten")

    def flatten(self, stream=None) -> torch.Tensor:
        """Flattened copy of the committed contents (also after a sticky pool error)."""
        n = self.size(stream, check_error=False)
        out = torch.empty(max(n, 1), dtype=self.dtype, device=self.pool.mem.device)
        self.flatten_into(out[:n] if n else out[:0], stream)
        return out[:n]

    def size(self, stream=None, check_error: bool = True) -> int:
        """Global size.  With check_error=False a sticky ENOMEM / ERANGE does not raise
        (the size of the committed contents is still returned)."""
        v = _u64()
        st = lib().ggarray_size(self._h, ctypes.byref(v), _stream(stream))
        if check_error or st not in (OK, ENOMEM, ERANGE):
            _check(st, "ggarray_size")
        return int(v.value)

    def capacity(self, stream=None, check_error: bool = True) -> int:
        """Elements held by the allocated buckets (check_error as for size())."""
        v = _u64()
        st = lib().ggarray_capacity(self._h, ctypes.byref(v), _stream(stream))
        if check_error or st not in (OK, ENOMEM, ERANGE):
            _check(st, "ggarray_capacity")
        return int(v.value)

    def insert_segments(self, values: torch.Tensor, prefix: torch.Tensor, stream=None):
        """LFVector v appends values[prefix[v]:prefix[v + 1]] (prefix: V + 1 int64 on
        the device); with prefix_into and flatten_into, restores a flat snapshot."""
        if prefix.numel() != self.n_vectors + 1:
            raise ValueError(f"prefix needs {self.n_vectors + 1} entries")
        _check(lib().ggarray_insert_segments(self._h, _dev_ptr(values, "values", 0, self.elem_bytes) if values.numel() else None,
                                             _dev_ptr(prefix, "prefix", 0, 8), values.numel(), _stream(stream)),
               "ggarray_insert_segments")

    def footprint(self) -> dict:
        """Device bytes besides the buckets (host state, no synchronisation)."""
        out = (_u64 * 3)()
        _check(lib().ggarray_footprint(self._h, out), "ggarray_footprint")
        return {"metadata": int(out[0]), "lookback": int(out[1]), "tile_tables": int(out[2])}

    def vector_sizes(self, stream=None) -> torch.Tensor:
        out = torch.empty(self.n_vectors, dtype=torch.int64, device=self.pool.mem.device)
        _check(lib().ggarray_vector_sizes(self._h, _dev_ptr(out, "out"), _stream(stream)),
               "ggarray_vector_sizes")
        return out

    def prefix(self, stream=None) -> torch.Tensor:
        out = torch.empty(self.n_vectors + 1, dtype=torch.int64, device=self.pool.mem.device)
        self.prefix_into(out, stream)
        return out

    def prefix_into(self, out: torch.Tensor, stream=None):
        _check(lib().ggarray_prefix(self._h, _dev_ptr(out, "out", self.n_vectors + 1, 8),
                                    _stream(stream)), "ggarray_prefix")

    def last_error(self, stream=None) -> int:
        return int(lib().ggarray_last_error(self._h, _stream(stream)))

    def set_spin_limit(self, polls: int):
        _check(lib().ggarray_set_spin_limit(self._h, int(polls)), "ggarray_set_spin_limit")

    def close(self, stream=None):
        if self._h:
            _check(lib().ggarray_destroy(self._h, _stream(stream)), "ggarray_destroy")
            self._h = _vp()


class Batch:
    """Many GGArrays driven with one launch per phase (see include/ggarray.h)."""

    def __init__(self, arrays, stream=None):
        self.arrays = list(arrays)
        self.n = len(self.arrays)
        handles = (_vp * self.n)(*[a._h.value for a in self.arrays])
        self._h = _vp()
        _check(lib().gga_batch_create(ctypes.byref(self._h), handles, self.n, _stream(stream)),
               "gga_batch_create")
        self._counts = {}

    def insert_gen(self, gen: GenSpec, n_threads, stream=None):
        key = tuple(int(x) for x in n_threads)
        arr = self._counts.get(key)
        if arr is None:  # keep the host array alive: a captured graph never reads it, but tidy
            arr = (_u64 * self.n)(*key)
            self._counts[key] = arr
        _check(lib().gga_batch_insert_gen(self._h, ctypes.byref(gen), arr, _stream(stream)),
               "gga_batch_insert_gen")

    def step(self, gens, n_threads, op: int, out: torch.Tensor | None = None, stream=None, clear: bool = False):
        """One persistent launch: rounds gens[r] with n_threads[r][i] threads on array i,
        r/w op (RW_NONE: none), then the flatten into out (None: no flatten).  With
        clear, every array is first emptied (shrink 1/1) in the same launch."""
        rounds = len(gens)
        flat = tuple(int(x) for row in n_threads for x in row)
        if len(flat) != rounds * self.n:
            raise ValueError("n_threads needs one row of n counts per round")
        key = ("step", flat)
        arr = self._counts.get(key)
        if arr is None:
            arr = (_u64 * max(1, len(flat)))(*flat)
            self._counts[key] = arr
        g = (GenSpec * max(1, rounds))(*gens)
        op_ = _dev_ptr(out, "out", 0, self.arrays[0].elem_bytes) if out is not None else None
        fn, name = (lib().gga_batch_step_clear, "gga_batch_step_clear") if clear else \
            (lib().gga_batch_step, "gga_batch_step")
        _check(fn(self._h, g, rounds, arr, op, op_, 0 if out is None else out.numel(), _stream(stream)), name)

    def shrink(self, num: int, den: int, stream=None):
        _check(lib().gga_batch_shrink(self._h, num, den, _stream(stream)), "gga_batch_shrink")

    def rw(self, op: int, stream=None):
        _check(lib().gga_batch_rw(self._h, op, _stream(stream)), "gga_batch_rw")

    def flatten_into(self, out: torch.Tensor, stream=None):
        _check(lib().gga_batch_flatten(self._h, _dev_ptr(out, "out", 0, self.arrays[0].elem_bytes),
                                       out.numel(), _stream(stream)), "gga_batch_flatten")

    def set_grid(self, stream_blocks: int):
        _check(lib().gga_batch_set_grid(self._h, int(stream_blocks)), "gga_batch_set_grid")

    def offsets(self, stream=None) -> torch.Tensor:
        out = torch.empty(self.n + 1, dtype=torch.int64, device="cuda")
        _check(lib().gga_batch_offsets(self._h, _dev_ptr(out, "out"), _stream(stream)), "gga_batch_offsets")
        return out

    def last_error(self, stream=None) -> int:
        return int(lib().gga_batch_last_error(self._h, _stream(stream)))

    def close(self, stream=None):
        if self._h:
            _check(lib().gga_batch_destroy(self._h, _stream(stream)), "gga_batch_destroy")
            self._h = _vp()


class Server:
    """Request loop over resident arrays (see include/ggarray.h, serving).

    ``arena`` is a device tensor that receives flatten outputs (a ring)."""

    STATS = ("steps", "largest_step", "issued", "rejected", "memory_waits", "peak_charged_bytes",
             "elapsed_ns", "arena_wraps")

    def __init__(self, arrays, arena: torch.Tensor, cap_bytes: int, mode: int = SERVE_BATCHED,
                 lanes: int = 2, max_step: int = 1024, depth: int = 256, seed: int = 1,
                 append_round: int = 0xA0, append_shift: int = 20, rw_op: int = ADD1):
        self.arrays = list(arrays)
        self.arena = arena
        handles = (_vp * len(self.arrays))(*[a._h.value for a in self.arrays])
        cfg = ServerConfig(int(cap_bytes), mode, lanes, max_step, depth, seed, append_round,
                           append_shift, rw_op)
        self._h = _vp()
        nbytes = arena.numel() * arena.element_size()
        _check(lib().gga_server_create(ctypes.byref(self._h), handles, len(self.arrays),
                                       _dev_ptr(arena, "arena"), nbytes, ctypes.byref(cfg)),
               "gga_server_create")

    def run(self, arrival_ns, kind, target, length, out_len: torch.Tensor | None = None) -> dict:
        """Replay a trace (numpy arrays); returns per-request host arrays and stats."""
        arrival_ns = np.ascontiguousarray(arrival_ns, dtype=np.uint64)
        kind = np.ascontiguousarray(kind, dtype=np.uint8)
        target = np.ascontiguousarray(target, dtype=np.uint32)
        length = np.ascontiguousarray(length, dtype=np.uint32)
        n = arrival_ns.size
        assert kind.size == n and target.size == n and length.size == n
        tr = Trace(n, arrival_ns.ctypes.data, kind.ctypes.data, target.ctypes.data, length.ctypes.data)
        t_issue = np.zeros(n, dtype=np.uint64)
        t_done = np.zeros(n, dtype=np.uint64)
        status = np.zeros(n, dtype=np.int32)
        out_off = np.zeros(n, dtype=np.uint64)
        stats = (_u64 * 8)()
        dev_len = _dev_ptr(out_len, "out_len", n, 8)
        _check(lib().gga_server_run(self._h, ctypes.byref(tr), t_issue.ctypes.data, t_done.ctypes.data,
                                    status.ctypes.data, out_off.ctypes.data, dev_len, stats),
               "gga_server_run")
        res = dict(zip(self.STATS, (int(x) for x in stats)))
        res.update(t_issue_ns=t_issue, t_done_ns=t_done, status=status, out_offset=out_off)
        return res

    def close(self):
        if self._h:
            _check(lib().gga_server_destroy(self._h), "gga_server_destroy")
            self._h = _vp()


class StaticArray:
    """Pre-allocated flat array baseline (caller-owned buffer of cap elements)."""

    def __init__(self, cap: int, elem_bytes: int, device="cuda", stream=None, buf: torch.Tensor | None = None):
        self.elem_bytes = elem_bytes
        if buf is None:
            buf = torch.empty(max(int(cap), 1), dtype=_dtype(elem_bytes), device=device)
        elif buf.numel() < cap or buf.element_size() != elem_bytes or not buf.is_contiguous():
            raise ValueError("buf must be a contiguous tensor of at least cap elements of elem_bytes each")
        self.buf = buf
        self.cap = int(cap)
        self._h = _vp()
        _check(lib().gga_static_create(ctypes.byref(self._h), self.buf.data_ptr(), self.cap,
                                       elem_bytes, _stream(stream)), "gga_static_create")

    def insert(self, values, flags=None, stream=None):
        n = values.numel()
        _check(lib().gga_static_insert(self._h, _dev_ptr(values, "values", n, self.elem_bytes),
                                       _dev_ptr(flags, "flags", n, 1), n, _stream(stream)),
               "gga_static_insert")

    def insert_gen(self, gen: GenSpec, n_threads: int, stream=None):
        _check(lib().gga_static_insert_gen(self._h, ctypes.byref(gen), int(n_threads), _stream(stream)),
               "gga_static_insert_gen")

    def insert_gen_atomic(self, gen: GenSpec, n_threads: int, stream=None):
        """Per-element atomic strategy (the scan's comparison point)."""
        _check(lib().gga_static_insert_gen_atomic(self._h, ctypes.byref(gen), int(n_threads), _stream(stream)),
               "gga_static_insert_gen_atomic")

    def rw(self, op: int, stream=None):
        _check(lib().gga_static_rw(self._h, op, _stream(stream)), "gga_static_rw")

    def size(self, stream=None) -> int:
        v = _u64()
        _check(lib().gga_static_size(self._h, ctypes.byref(v), _stream(stream)), "gga_static_size")
        return int(v.value)

    def last_error(self, stream=None) -> int:
        return int(lib().gga_static_last_error(self._h, _stream(stream)))

    def data(self, stream=None) -> torch.Tensor:
        return self.buf[: self.size(stream)]

    def clear(self, stream=None):
        _check(lib().gga_static_clear(self._h, _stream(stream)), "gga_static_clear")

    def set_size(self, n: int, stream=None):
        _check(lib().gga_static_set_size(self._h, int(n), _stream(stream)), "gga_static_set_size")

    def close(self, stream=None):
        if self._h:
            _check(lib().gga_static_destroy(self._h, _stream(stream)), "gga_static_destroy")
            self._h = _vp()


class SemiStaticArray:
    """Host-resized doubling array baseline."""

    def __init__(self, elem_bytes: int, initial_cap: int, stream=None):
        self.elem_bytes = elem_bytes
        self.dtype = _dtype(elem_bytes)
        self._h = _vp()
        _check(lib().gga_semi_create(ctypes.byref(self._h), elem_bytes, int(initial_cap),
                                     _stream(stream)), "gga_semi_create")

    def insert(self, values, flags=None, stream=None):
        n = values.numel()
        _check(lib().gga_semi_insert(self._h, _dev_ptr(values, "values", n, self.elem_bytes),
                                     _dev_ptr(flags, "flags", n, 1), n, _stream(stream)),
               "gga_semi_insert")

    def insert_gen(self, gen: GenSpec, n_threads: int, stream=None):
        _check(lib().gga_semi_insert_gen(self._h, ctypes.byref(gen), int(n_threads), _stream(stream)),
               "gga_semi_insert_gen")

    def rw(self, op: int, stream=None):
        _check(lib().gga_semi_rw(self._h, op, _stream(stream)), "gga_semi_rw")

    def size(self, stream=None) -> int:
        v = _u64()
        _check(lib().gga_semi_size(self._h, ctypes.byref(v), _stream(stream)), "gga_semi_size")
        return int(v.value)

    def resizes(self) -> int:
        v = _u64()
        _check(lib().gga_semi_resizes(self._h, ctypes.byref(v)), "gga_semi_resizes")
        return int(v.value)

    def data(self, stream=None) -> torch.Tensor:
        """Copy of the live elements (device tensor)."""
        n = self.size(stream)
        p, cap = _vp(), _u64()
        _check(lib().gga_semi_data(self._h, ctypes.byref(p), ctypes.byref(cap)), "gga_semi_data")
        out = torch.empty(max(n, 1), dtype=self.dtype, device="cuda")
        if n:
            torch.cuda.current_stream().synchronize()
            _copy_from_ptr(out, p.value, n * self.elem_bytes)
        return out[:n]

    def close(self, stream=None):
        if self._h:
            _check(lib().gga_semi_destroy(self._h, _stream(stream)), "gga_semi_destroy")
            self._h = _vp()


class MappedArray:
    """Host-grown array over a reserved virtual range (memMap baseline)."""

    def __init__(self, elem_bytes: int, max_elems: int, stream=None):
        self.elem_bytes = elem_bytes
        self.dtype = _dtype(elem_bytes)
        self._h = _vp()
        _check(lib().gga_mapped_create(ctypes.byref(self._h), elem_bytes, int(max_elems), _stream(stream)),
               "gga_mapped_create")

    def insert(self, values, flags=None, stream=None):
        n = values.numel()
        _check(lib().gga_mapped_insert(self._h, _dev_ptr(values, "values", n, self.elem_bytes),
                                       _dev_ptr(flags, "flags", n, 1), n, _stream(stream)),
               "gga_mapped_insert")

    def insert_gen(self, gen: GenSpec, n_threads: int, stream=None):
        _check(lib().gga_mapped_insert_gen(self._h, ctypes.byref(gen), int(n_threads), _stream(stream)),
               "gga_mapped_insert_gen")

    def rw(self, op: int, stream=None):
        _check(lib().gga_mapped_rw(self._h, op, _stream(stream)), "gga_mapped_rw")

    def size(self, stream=None) -> int:
        v = _u64()
        _check(lib().gga_mapped_size(self._h, ctypes.byref(v), _stream(stream)), "gga_mapped_size")
        return int(v.value)

    def maps(self) -> int:
        v = _u64()
        _check(lib().gga_mapped_maps(self._h, ctypes.byref(v)), "gga_mapped_maps")
        return int(v.value)

    def data(self, stream=None) -> torch.Tensor:
        """Copy of the live elements (device tensor)."""
        n = self.size(stream)
        p, cap = _vp(), _u64()
        _check(lib().gga_mapped_data(self._h, ctypes.byref(p), ctypes.byref(cap)), "gga_mapped_data")
        out = torch.empty(max(n, 1), dtype=self.dtype, device="cuda")
        if n:
            torch.cuda.current_stream().synchronize()
            _copy_from_ptr(out, p.value, n * self.elem_bytes)
        return out[:n]

    def close(self, stream=None):
        if self._h:
            _check(lib().gga_mapped_destroy(self._h, _stream(stream)), "gga_mapped_destroy")
            self._h = _vp()


def _copy_from_ptr(out: torch.Tensor, src_ptr: int, nbytes: int):
    """Device-to-device copy from a raw device pointer into `out` (HIP runtime)."""
    hip = _hip_runtime()
    rc = hip.hipMemcpy(ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(src_ptr), ctypes.c_size_t(nbytes),
                       ctypes.c_int(3))
    if rc != 0:
        raise GGAError(EHIP, "hipMemcpy")


_hip = None


def _hip_runtime():
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.restype = ctypes.c_int
    return _hip
