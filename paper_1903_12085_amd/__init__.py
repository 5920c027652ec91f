"""MI355X-native phased single-source shortest paths (Kainer & Traff, arXiv 1903.12085).

The product is the C-ABI library libsssp.so (include/sssp.h) built from the
HIP sources in csrc/; ``binding`` is its thin ctypes binding and ``build``
compiles it for gfx950.
"""
__all__ = ["binding", "build"]
