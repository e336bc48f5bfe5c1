"""FP64 CPU oracle for animated-SVO first-hit tracing (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``liboracle.so``, built from
``svo_oracle.c`` with plain gcc; it shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "svo_oracle.c")
NONE = 0xFFFFFFFF


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
                               "-o", tmp, SRC_PATH, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=True)
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.oracle_trace.restype = ctypes.c_int
        L.oracle_trace.argtypes = [P, ctypes.c_uint64, ctypes.c_uint32, P, ctypes.c_double, ctypes.c_uint32,
                                   P, P, P, P, ctypes.c_uint64, P, P, P, P, P, P, P, P, P, P,
                                   ctypes.c_double, ctypes.c_int]
        L.oracle_trace_paper_form.restype = ctypes.c_int
        L.oracle_trace_paper_form.argtypes = [P, ctypes.c_uint64, ctypes.c_uint32, P, ctypes.c_double,
                                              ctypes.c_uint32, P, P, P, P, P, P, P, ctypes.c_uint64,
                                              P, P, P, P, ctypes.c_int]
        L.oracle_frames.restype = ctypes.c_int
        L.oracle_frames.argtypes = [P, ctypes.c_uint64, ctypes.c_uint32, P, ctypes.c_double, ctypes.c_uint32,
                                    P, P, P, P, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Hits:
    """Oracle results per ray.  margin: the id margin (gaps that can change
    which leaf is hit); margin_n: the normal margin (also the entry-face
    gaps).  nnode / nframe: node records read and frames entered, lower bound
    (frames entered by the final hit, each cut at it); nnode_hi / nframe_hi:
    upper bound (every frame the segment meets, each to its own first hit)."""
    id: np.ndarray
    inst: np.ndarray
    t: np.ndarray
    normal: np.ndarray
    margin: Optional[np.ndarray] = None
    margin_n: Optional[np.ndarray] = None
    nnode: Optional[np.ndarray] = None
    nframe: Optional[np.ndarray] = None
    nnode_hi: Optional[np.ndarray] = None
    nframe_hi: Optional[np.ndarray] = None


def _scene_args(nodes, root, root_min, root_size, slot_child, slot_cell):
    nodes = np.ascontiguousarray(nodes, dtype=np.uint64)
    rmin = np.ascontiguousarray(np.asarray(root_min, np.float64).reshape(3))
    sc = np.ascontiguousarray(np.asarray(slot_child, np.uint32).reshape(-1))
    cell = np.ascontiguousarray(np.asarray(slot_cell, np.float64).reshape(-1, 4))
    return nodes, rmin, sc, cell


def trace(nodes, root, root_min, root_size, slot_child, slot_cell, fwd, rays, margin=False, counters=False,
          nthreads=0, margin_eps=1e-6, fwd_f64=False) -> Hits:
    """First hits of rays [n, 8] (float32); fwd = [S, 12] parent-relative forward maps,
    rounded to float32 (the precision transform slots carry) unless ``fwd_f64``."""
    nodes, rmin, sc, cell = _scene_args(nodes, root, root_min, root_size, slot_child, slot_cell)
    S = sc.shape[0]
    fdt = np.float64 if fwd_f64 else np.float32
    fw = np.ascontiguousarray(np.asarray(fwd, fdt).astype(np.float64).reshape(S, 12)) if S else np.zeros((0, 12))
    r = np.ascontiguousarray(np.asarray(rays, np.float32).reshape(-1, 8))
    n = r.shape[0]
    out = Hits(np.empty(n, np.uint32), np.empty(n, np.uint32), np.empty(n, np.float64), np.empty((n, 3), np.float64))
    if margin:
        out.margin = np.empty(n, np.float64)
        out.margin_n = np.empty(n, np.float64)
    if counters:
        out.nnode = np.empty(n, np.uint32)
        out.nframe = np.empty(n, np.uint32)
        out.nnode_hi = np.empty(n, np.uint32)
        out.nframe_hi = np.empty(n, np.uint32)
    rc = lib().oracle_trace(_p(nodes), nodes.shape[0], int(root), _p(rmin), float(root_size), S, _p(sc), _p(cell),
                            _p(fw), _p(r), n, _p(out.id), _p(out.inst), _p(out.t), _p(out.normal), _p(out.margin),
                            _p(out.margin_n), _p(out.nnode), _p(out.nnode_hi), _p(out.nframe), _p(out.nframe_hi),
                            float(margin_eps), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_trace failed with %d" % rc)
    return out


def trace_scene(scene, rays, frame=0, static=False, margin=False, counters=False, fwd=None, nthreads=0,
                margin_eps=1e-6, fwd_f64=False) -> Hits:
    """Convenience wrapper over a generated scene (svogen.scenes.Scene)."""
    nodes = scene.static_pool() if static else scene.nodes
    if fwd is None:
        fwd = scene.xform(frame) if scene.n_slots else np.zeros((0, 12), np.float32)
    return trace(nodes, scene.root, scene.root_min, scene.root_size, scene.slot_child, scene.slot_cell, fwd, rays,
                 margin=margin, counters=counters, nthreads=nthreads, margin_eps=margin_eps, fwd_f64=fwd_f64)


def trace_paper_form(nodes, root, root_min, root_size, slot_child, slot_cell, rot, scale, pivot, tau, rays,
                     nthreads=0) -> Hits:
    nodes, rmin, sc, cell = _scene_args(nodes, root, root_min, root_size, slot_child, slot_cell)
    S = sc.shape[0]
    R = np.ascontiguousarray(np.asarray(rot, np.float64).reshape(S, 9))
    Sc = np.ascontiguousarray(np.asarray(scale, np.float64).reshape(S, 3))
    Pv = np.ascontiguousarray(np.asarray(pivot, np.float64).reshape(S, 3))
    Tu = np.ascontiguousarray(np.asarray(tau, np.float64).reshape(S, 3))
    r = np.ascontiguousarray(np.asarray(rays, np.float32).reshape(-1, 8))
    n = r.shape[0]
    out = Hits(np.empty(n, np.uint32), np.empty(n, np.uint32), np.empty(n, np.float64), np.empty((n, 3), np.float64))
    rc = lib().oracle_trace_paper_form(_p(nodes), nodes.shape[0], int(root), _p(rmin), float(root_size), S, _p(sc),
                                       _p(cell), _p(R), _p(Sc), _p(Pv), _p(Tu), _p(r), n, _p(out.id), _p(out.inst),
                                       _p(out.t), _p(out.normal), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_trace_paper_form failed with %d" % rc)
    return out


def frames(nodes, root, root_min, root_size, slot_child, slot_cell, fwd):
    """(n_frames, parent slot per slot, composed world<-local maps [S,12])."""
    nodes, rmin, sc, cell = _scene_args(nodes, root, root_min, root_size, slot_child, slot_cell)
    S = sc.shape[0]
    fw = np.ascontiguousarray(np.asarray(fwd, np.float32).astype(np.float64).reshape(S, 12)) if S else np.zeros((0, 12))
    par = np.empty(S, np.uint32)
    W = np.empty((S, 12), np.float64)
    nf = lib().oracle_frames(_p(nodes), nodes.shape[0], int(root), _p(rmin), float(root_size), S, _p(sc), _p(cell),
                             _p(fw), _p(par), _p(W))
    if nf < 0:
        raise ValueError("oracle_frames failed with %d" % nf)
    return nf, par, W


def shade(nodes, prim_id, ao_id, width, height, samples, k, ambient_permille, background, pixel_index):
    """Composite hits into an RGBA8 image (the colour field of the paper's hit
    buffer, Sec. 4.3), written from its definition in integers.

    pixel_index[p]: flat row-major pixel of the p-th pixel in ray order (the
    input generator's order); samples consecutive rays per pixel, k
    consecutive AO rays per primary ray.  A sample whose id is a pool node
    takes that leaf's RGB (word1) with weight (F k + (1000 - F)(k - occ)) /
    (1000 k), occ = its blocked AO rays (weight 1 if k == 0); otherwise the
    background with weight 1.  Each channel is the mean over the samples,
    rounded half up; alpha 255.  Returns uint32 [height, width]."""
    nodes = np.asarray(nodes, np.uint64)
    ids = np.asarray(prim_id).astype(np.uint64).reshape(-1)
    npix = width * height
    S = int(samples)
    assert ids.shape[0] == npix * S
    hit = ids < np.uint64(nodes.shape[0])
    col = np.full(ids.shape[0], int(background) & 0xFFFFFFFF, np.uint64)
    col[hit] = nodes[ids[hit].astype(np.int64)] >> np.uint64(32)
    den = 1000 * max(int(k), 1)
    w = np.full(ids.shape[0], den, np.int64)
    if k:
        occ = (np.asarray(ao_id).astype(np.uint64).reshape(-1, k) != np.uint64(0xFFFFFFFF)).sum(1)
        wk = int(ambient_permille) * k + (1000 - int(ambient_permille)) * (k - occ.astype(np.int64))
        w[hit] = wk[hit]
    out = np.full(npix, 0xFF000000, np.uint64)
    total = den * S
    for c in range(3):
        ch = ((col >> np.uint64(8 * c)) & np.uint64(0xFF)).astype(np.int64)
        acc = (ch * w).reshape(npix, S).sum(1)
        out |= (((acc + total // 2) // total).astype(np.uint64) << np.uint64(8 * c))
    img = np.zeros(npix, np.uint64)
    img[np.asarray(pixel_index, np.int64)] = out
    return img.astype(np.uint32).reshape(height, width)
