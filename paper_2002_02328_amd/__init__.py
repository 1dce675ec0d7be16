"""MI355X-native hot path of block distributed 3MG (BD3MG) deblurring.

The compute path is the HIP library ``libbd3mg.so`` (sources under ``csrc/``,
C interface in ``include/bd3mg.h``); ``binding`` is a thin ctypes layer with the
same function names.  ``inputs`` draws the seeded synthetic workloads.
"""
__all__ = ["inputs", "binding"]
