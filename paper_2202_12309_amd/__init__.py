"""MI355X-native hot path of Parthenon-hydro's block-AMR Euler cycle.

The compute path is the HIP library ``libpkhydro.so`` (``csrc/``), reached
through the C-ABI declared in ``include/pkhydro.h``; :mod:`.binding` is its
thin ctypes binding. Importing this package loads nothing: the library is
loaded on first use and raises if it is missing.
"""
__all__ = ["inputs"]
