"""Helpers shared by the GPU parity tests: run the same operations on the HIP
library (through the C ABI binding) and on the CPU oracle, and compare."""
import numpy as np

import oracle
from oracle import Oracle


def gg():
    from paper_2209_00103_amd import ggarray
    return ggarray


def gpu_sizes(arr) -> np.ndarray:
    return arr.vector_sizes().cpu().numpy().astype(np.uint64)


def gpu_flat(arr) -> np.ndarray:
    return gg().as_unsigned(arr.flatten())


def assert_same(arr, o: Oracle, what: str = ""):
    """Bit-exact comparison of sizes, contents, prefix and capacity."""
    assert arr.last_error() == 0, f"{what}: device error {arr.last_error()}"
    np.testing.assert_array_equal(gpu_sizes(arr), o.vector_sizes(), err_msg=f"{what}: sizes")
    flat = gpu_flat(arr)
    ref = o.flatten()
    assert flat.shape == ref.shape, f"{what}: size {flat.shape} vs {ref.shape}"
    if not np.array_equal(flat, ref):
        bad = np.nonzero(flat != ref)[0]
        raise AssertionError(f"{what}: {bad.size} elements differ, first at {bad[:8]}: "
                             f"gpu {flat[bad[:8]]} oracle {ref[bad[:8]]}")
    pre = arr.prefix().cpu().numpy().astype(np.uint64)
    np.testing.assert_array_equal(pre, o.prefix(), err_msg=f"{what}: prefix")
    assert arr.capacity() == o.capacity(), f"{what}: capacity"


def both(elem, V, F, pool):
    G = gg()
    return G.GGArray(pool, elem, V, F), Oracle(elem, V, F)


def dev(a):
    return gg().to_device(a)


def oracle_mod():
    return oracle
