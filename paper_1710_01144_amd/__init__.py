"""MI355X-native Greedy++ group-closeness maximisation.

The computation lives in libgc.so (HIP kernels for gfx950 behind the C ABI of
include/gc.h); ``gc`` is its ctypes binding.  Build with
``python -m paper_1710_01144_amd.build``.
"""
from .gc import Graph, GCError, load_library, library_path  # noqa: F401
