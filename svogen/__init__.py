"""Seeded synthetic inputs (scenes, pools, transforms, rays) for the animated-SVO
tracer and its oracle.  Holds no traversal, ray-transform or inversion
arithmetic: it only produces the bytes both sides read."""
from . import camera, hashing, noise, octree, scenes, xforms  # noqa: F401
