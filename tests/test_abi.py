"""C ABI checks that need no GPU: the library loads, exports every function that
include/ggarray.h declares, and rejects invalid arguments on the host before any
HIP call is made."""
import ctypes
import os
import re
import subprocess

import pytest

from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "ggarray.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return re.findall(r"^\s*(?:const\s+char\s*\*|int)\s*(\w+)\s*\(", text, re.M)


@pytest.fixture(scope="module")
def G():
    from paper_2209_00103_amd import ggarray
    return ggarray


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("ggarray_create", "ggarray_insert", "ggarray_rw", "ggarray_flatten", "ggarray_size",
                 "ggarray_destroy", "ggarray_shrink", "gga_pool_create", "gga_static_insert",
                 "gga_semi_insert", "gga_strerror"):
        assert must in names
    assert len(names) == len(set(names))


def test_library_exports_every_declared_symbol(G):
    L = G.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", G.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r" T (\w+)$", out, re.M))
    assert set(declared_functions()) <= exported


def test_binding_covers_every_symbol(G):
    assert set(declared_functions()) == set(G._SIGS)


def test_strerror(G):
    L = G.lib()
    assert L.gga_strerror(0) == b"ok"
    assert L.gga_strerror(G.ENOMEM) == b"bucket pool exhausted"
    assert L.gga_strerror(-99) == b"unknown status"


def test_host_side_validation(G):
    L = G.lib()
    h = ctypes.c_void_p()
    EINVAL = G.EINVAL
    assert L.ggarray_create(None, None, 4, 1, 1, None) == EINVAL
    assert L.ggarray_create(ctypes.byref(h), None, 4, 1, 1, None) == EINVAL
    assert L.gga_pool_create(ctypes.byref(h), None, 1 << 30, None) == EINVAL
    assert L.gga_pool_create(ctypes.byref(h), 0x1001, 1 << 30, None) == EINVAL  # unaligned
    assert L.gga_pool_create(ctypes.byref(h), 0x100000, 1000, None) == EINVAL   # too small
    assert L.ggarray_insert(None, None, None, 0, None) == EINVAL
    assert L.ggarray_insert_gen(None, None, 0, None) == EINVAL
    assert L.ggarray_shrink(None, 1, 2, None) == EINVAL
    assert L.ggarray_insert_gen_rounds(None, None, None, 0, 1, 10, 0, None) == EINVAL
    assert L.ggarray_rw(None, 0, None) == EINVAL
    assert L.ggarray_flatten(None, None, 0, None) == EINVAL
    assert L.ggarray_size(None, None, None) == EINVAL
    assert L.ggarray_last_error(None, None) == EINVAL
    assert L.ggarray_destroy(None, None) == EINVAL
    assert L.gga_pool_destroy(None) == EINVAL
    assert L.gga_static_create(ctypes.byref(h), None, 10, 4, None) == EINVAL
    assert L.gga_static_create(ctypes.byref(h), 0x1008, 10, 4, None) == EINVAL  # not 16-aligned
    assert L.gga_semi_create(ctypes.byref(h), 3, 10, None) == EINVAL
    assert L.gga_semi_create(ctypes.byref(h), 4, 0, None) == EINVAL


def test_product_has_no_oracle_dependency():
    """The HIP library and its binding never reach the oracle."""
    pkg = os.path.join(ROOT, "paper_2209_00103_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "ggoracle" not in text, f
