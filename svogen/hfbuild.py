"""ctypes wrapper of csrc/hfbuild.c: breadth-first heightfield pools built in
C (input generation only), identical node for node to build_tree with
heightfield_classifier and the height-band colours."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC_PATH = os.path.join(_HERE, "csrc", "hfbuild.c")
LIB_PATH = os.path.join(_HERE, "libhfbuild.so")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-Wall", "-o", tmp, SRC_PATH])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=True)
        L = ctypes.CDLL(LIB_PATH)
        P, I64 = ctypes.c_void_p, ctypes.c_int64
        L.svogen_hf_count.restype = I64
        L.svogen_hf_count.argtypes = [ctypes.c_int, P, P]
        L.svogen_hf_build.restype = I64
        L.svogen_hf_build.argtypes = [ctypes.c_int, P, I64, P, I64, P, I64]
        _lib = L
    return _lib


FAR = 0xFFFFFF


def build_heightfield_pool(H: np.ndarray, K: int, seed: int, far_from: int = FAR):
    """(nodes uint64 [n], nodes per level int64 [K + 1]) for columns H[x, z].
    far_from < 2^24 - 1 writes far pointers for smaller offsets too (tests)."""
    n = 1 << K
    Hc = np.ascontiguousarray(np.asarray(H).reshape(n, n), np.int32)
    counts = np.zeros(K + 1, np.int64)
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    total = lib().svogen_hf_count(K, P(Hc), P(counts))
    if total < 0:
        raise RuntimeError("heightfield pool: bad arguments or out of memory")
    nodes = np.empty(total, np.uint64)
    if total:
        got = lib().svogen_hf_build(K, P(Hc), int(seed), P(nodes), total, P(counts), int(far_from))
        if got != total:
            raise RuntimeError("heightfield pool build failed (%d)" % got)
    return nodes, counts
