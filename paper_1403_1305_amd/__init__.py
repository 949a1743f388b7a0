"""Aho-Corasick multi-pattern scanning on AMD Instinct MI355X (gfx950).

The library proper is the C ABI in include/ac.h (libac.so, built from csrc/);
``paper_1403_1305_amd.ac`` is its ctypes binding. Importing this package does
not load the library; ``from paper_1403_1305_amd import ac`` does.
"""
__all__ = ["ac"]
