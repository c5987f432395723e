"""MI355X-native ray casting of deep-octree volumetric canvases.

The compute path is the C-ABI library ``lib/libcvx.so`` (HIP kernels for
gfx950, entry points declared in ``include/cvx.h``); ``cvx`` is its ctypes
binding with the same function names.
"""
