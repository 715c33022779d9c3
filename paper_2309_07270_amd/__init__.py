"""MI355X-native batched X-drop seed-and-extend.

The computation runs in ``libxdrop.so`` (hand-written HIP for gfx950 behind a
C ABI declared in ``include/xdrop.h``); ``paper_2309_07270_amd.xdrop`` is the
thin ctypes binding and ``paper_2309_07270_amd.workload`` draws seeded
synthetic inputs.  Importing the package loads nothing native.
"""
__all__ = ["workload", "xdrop"]
