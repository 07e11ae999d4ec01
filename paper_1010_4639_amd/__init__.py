"""MI355X-native conjugate-gradient / SpMV path for sparse SPD systems.

The compute path lives in the HIP shared library built from ``csrc/`` and is
reached through :mod:`paper_1010_4639_amd.cgmi` (ctypes).  Nothing is imported
eagerly, so the input generator in :mod:`paper_1010_4639_amd.workload` can be
used on machines without a GPU.
"""
__all__ = ["workload", "cgmi"]
