"""MI355X-native (gfx950) Lagrangian particle-deposition step.

The compute path is the HIP library ``libdepo.so`` built from ``csrc/`` and
declared in ``include/depo.h``; :mod:`paper_2205_04979_amd.depo` is a thin
ctypes binding with the same entry points.  Importing the package loads
nothing; the library is opened on first use and a missing library is an
error, never a fallback.
"""

__all__ = ["depo", "build"]
