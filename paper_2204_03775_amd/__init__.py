"""MI355X-native 25-point acoustic wave propagator (arXiv 2204.03775 hot path).

The compute path is ``libwave.so`` (hand-written HIP for gfx950 behind a C
ABI, declared in ``include/wave.h``); ``paper_2204_03775_amd.wave`` is its
thin ctypes binding and ``paper_2204_03775_amd.inputs`` generates seeded
synthetic workloads.  Importing this package loads nothing; the binding
loads the library on first use and raises if it is missing.
"""
__all__ = ["wave", "inputs"]
