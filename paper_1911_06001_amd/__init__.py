"""Animated sparse-voxel-octree ray traversal for MI355X (gfx950).

The compute path is libsvo.so (HIP kernels behind the C ABI of
include/svo.h); ``svo`` is its ctypes binding.
"""
from . import svo  # noqa: F401
