"""kx: Kronecker-product exact exchange on AMD MI355X (gfx950).

The compute path is the HIP library ``libkx.so`` (C ABI in include/kx.h);
``paper_2406_16998_amd.kx`` is its ctypes binding.
"""
