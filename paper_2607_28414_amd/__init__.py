"""MI355X (gfx950) reduced Kelvin-Voigt shear-wave solver.

The solver lives in the HIP library ``libkvs.so`` (C ABI in include/kvs.h);
``paper_2607_28414_amd.kvs`` is its ctypes binding.  Importing the package
does not load the library; the first binding call does, and raises when the
library is not built.
"""
__all__ = ["kvs"]
