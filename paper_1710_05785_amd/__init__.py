"""MI355X-native DAIC (delta-based accumulative iterative computation) hot path.

The compute lives in ``libdaic.so`` (HIP kernels for gfx950 behind the C ABI
declared in ``include/daic.h``); ``paper_1710_05785_amd.daic`` is its ctypes
binding. Importing this package loads nothing: the library is opened on first
use and its absence is an error, never a fallback.
"""
