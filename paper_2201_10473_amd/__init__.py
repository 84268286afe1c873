"""MI355X-native multiplication in F2[X] and F2[X]/(X^n - 1).

The compute path is the HIP library ``libgf2x.so`` (built from ``csrc/``)
behind the C ABI declared in ``include/gf2x.h``; ``gf2x`` is its thin ctypes
binding.  ``inputs`` draws seeded synthetic operands.
"""
__all__ = ["gf2x", "inputs"]
