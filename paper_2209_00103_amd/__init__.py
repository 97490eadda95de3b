"""GGArray for MI355X (gfx950): a dynamically growable GPU array built as an array
of per-block LFVectors, with block-cooperative insertion, in-kernel bucket growth
from a device sub-allocator, bucket-aligned read/write and a prefix-sum flatten.

The compute path is the HIP library ``libggarray.so`` behind the C ABI declared in
``include/ggarray.h``; ``paper_2209_00103_amd.ggarray`` is its ctypes binding.
"""
