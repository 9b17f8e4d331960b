"""Bitsliced Method of Four Russians over F_3, F_5, F_7 and GF(4) on AMD MI355X.

The compute path is the HIP library ``libgfq.so`` (C ABI in include/gfq.h); the module
``paper_0901_1413_amd.gfq`` binds it with ctypes and takes torch tensors as device buffers.
Importing the package loads nothing; the library is loaded on first use and a missing
library raises instead of falling back to anything else.
"""
