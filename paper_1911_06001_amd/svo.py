"""ctypes binding of libsvo.so (the C ABI in include/svo.h).

Argument marshalling only: every step of the trace runs in the library's
HIP kernels.  torch supplies device memory (``tensor.data_ptr()``) and
streams (``torch.cuda.current_stream().cuda_stream``).  Importing this
module raises if the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsvo.so")

SVO_OK, SVO_EINVAL, SVO_ENOMEM, SVO_EDEVICE, SVO_ERANGE, SVO_EBUSY, SVO_ESTATE = 0, -1, -2, -3, -4, -5, -6
NONE = 0xFFFFFFFF
STEP_LIMIT = 0xFFFFFFFE
MAX_DEPTH = 20
MAX_SLOTS = 1023
MAX_INLINE_NEST = 4

# every symbol include/svo.h declares
EXPORTS = ("svo_abi_version", "svo_last_error", "svo_create", "svo_destroy", "svo_validate", "svo_upload",
           "svo_free_scene", "svo_scene_bytes", "svo_get_scene_stats", "svo_set_transforms", "svo_trace_rays",
           "svo_trace_batch", "svo_get_config", "svo_set_config", "svo_tune", "svo_generate_primary_rays",
           "svo_generate_ao_rays", "svo_trace_rays_reuse", "svo_shade", "svo_plan_create", "svo_plan_set_jobs",
           "svo_plan_launch", "svo_plan_destroy", "svo_trace_batch_static", "svo_trace_rays_counted",
           "svo_trace_camera")


class SvoError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("svo error %d: %s" % (code, msg))
        self.code = code


class PoolInfo(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_uint64), ("n_frames", ctypes.c_uint32), ("world_height", ctypes.c_uint32),
                ("max_height", ctypes.c_uint32), ("max_nesting", ctypes.c_uint32), ("n_shared", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class Camera(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_float * 3), ("forward", ctypes.c_float * 3), ("right", ctypes.c_float * 3),
                ("up", ctypes.c_float * 3), ("tan_half_fov", ctypes.c_float), ("width", ctypes.c_uint32),
                ("height", ctypes.c_uint32), ("samples", ctypes.c_uint32), ("seed", ctypes.c_uint32),
                ("jitter", ctypes.c_uint32), ("tiled", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class Job(ctypes.Structure):
    _fields_ = [("scene", ctypes.c_uint32), ("fwd_3x4", ctypes.c_void_p), ("rays", ctypes.c_void_p),
                ("n", ctypes.c_uint64), ("out_id", ctypes.c_void_p), ("out_inst", ctypes.c_void_p),
                ("out_t", ctypes.c_void_p), ("out_normal", ctypes.c_void_p), ("camera", ctypes.POINTER(Camera))]


def make_camera(eye, target, up, vfov_deg, width, height, samples=1, seed=0, jitter=False, tiled=True) -> Camera:
    """Camera record from eye / look-at / up (basis built in float64)."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, np.float64))
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    c = Camera()
    c.eye[:] = eye.astype(np.float32).tolist()
    c.forward[:] = f.astype(np.float32).tolist()
    c.right[:] = r.astype(np.float32).tolist()
    c.up[:] = u.astype(np.float32).tolist()
    c.tan_half_fov = float(np.tan(np.radians(vfov_deg) * 0.5))
    c.width, c.height, c.samples, c.seed = int(width), int(height), int(samples), int(seed) & 0xFFFFFFFF
    c.jitter, c.tiled = int(bool(jitter)), int(bool(tiled))
    return c


class PlanLimits(ctypes.Structure):
    _fields_ = [("max_jobs", ctypes.c_uint32), ("max_frames", ctypes.c_uint32), ("reserved", ctypes.c_uint32 * 2)]


class SceneStats(ctypes.Structure):
    _fields_ = [("device_bytes", ctypes.c_uint64), ("n_slots", ctypes.c_uint32), ("n_frames", ctypes.c_uint32),
                ("n_inline", ctypes.c_uint32), ("n_candidates", ctypes.c_uint32), ("stack_levels", ctypes.c_uint32),
                ("nest_levels", ctypes.c_uint32)]


class Config(ctypes.Structure):
    _fields_ = [("waves_per_block", ctypes.c_uint32), ("blocks_per_cu", ctypes.c_uint32),
                ("lds_cache_nodes", ctypes.c_uint32), ("refill_lanes", ctypes.c_uint32),
                ("step_limit", ctypes.c_uint32), ("claim_tiles", ctypes.c_uint32),
                ("sorted_candidates", ctypes.c_uint32), ("tile_order", ctypes.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


_lib = None


def lib():
    """Load libsvo.so (raises if it is missing: build it first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libsvo.so is not built (run paper_1911_06001_amd/build.py or __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    P, U32, U64, I = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    sig = {
        "svo_abi_version": (I, []),
        "svo_last_error": (ctypes.c_char_p, []),
        "svo_create": (I, [ctypes.POINTER(P), I]),
        "svo_destroy": (None, [P]),
        "svo_validate": (I, [P, U64, U32, U32, P, U32, ctypes.POINTER(PoolInfo)]),
        "svo_upload": (I, [P, P, U64, U32, P, ctypes.c_float, U32, P, P, U32, ctypes.POINTER(U32)]),
        "svo_free_scene": (I, [P, U32]),
        "svo_scene_bytes": (I, [P, U32, ctypes.POINTER(U64)]),
        "svo_get_scene_stats": (I, [P, U32, ctypes.POINTER(SceneStats)]),
        "svo_set_transforms": (I, [P, U32, U32, U32, P, P]),
        "svo_trace_rays": (I, [P, U32, P, U64, P, P, P, P, P]),
        "svo_trace_batch": (I, [P, ctypes.POINTER(Job), U32, P]),
        "svo_trace_batch_static": (I, [P, ctypes.POINTER(Job), U32, P]),
        "svo_trace_rays_reuse": (I, [P, U32, P, U64, P, P, P, P, P, P]),
        "svo_trace_rays_counted": (I, [P, U32, P, U64, P, P, P, P, P, P, U32, P]),
        "svo_trace_camera": (I, [P, U32, ctypes.POINTER(Camera), P, P, P, P, P]),
        "svo_shade": (I, [P, U32, P, P, U32, U32, U32, U32, U32, U32, U32, P, P]),
        "svo_tune": (I, [P, U32, P, U64, P, ctypes.POINTER(Config)]),
        "svo_generate_primary_rays": (I, [P, ctypes.POINTER(Camera), P, P]),
        "svo_generate_ao_rays": (I, [P, P, P, P, U64, U32, U32, ctypes.c_float, ctypes.c_float, P, P]),
        "svo_get_config": (I, [P, ctypes.POINTER(Config)]),
        "svo_set_config": (I, [P, ctypes.POINTER(Config)]),
        "svo_plan_create": (I, [P, P, U32, ctypes.POINTER(PlanLimits), ctypes.POINTER(P)]),
        "svo_plan_set_jobs": (I, [P, P, ctypes.POINTER(Job), U32]),
        "svo_plan_launch": (I, [P, P, P]),
        "svo_plan_destroy": (I, [P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def last_error() -> str:
    return lib().svo_last_error().decode(errors="replace")


def _check(rc: int):
    if rc != SVO_OK:
        raise SvoError(rc, last_error())


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def validate(nodes, root, max_depth, slot_child) -> PoolInfo:
    """Host-only pool check; returns what it learned, raises SvoError otherwise."""
    nodes = np.ascontiguousarray(nodes, dtype=np.uint64)
    sc = np.ascontiguousarray(np.asarray(slot_child, np.uint32).reshape(-1))
    info = PoolInfo()
    _check(lib().svo_validate(_np_ptr(nodes), nodes.shape[0], int(root), int(max_depth), _np_ptr(sc), sc.shape[0],
                              ctypes.byref(info)))
    return info


def _dptr(t, n_elems: int, name: str, itemsize: int = 4):
    """Device pointer of tensor t after checking that it can hold n_elems
    contiguous elements of itemsize bytes.  The library takes plain pointers
    and cannot see buffer sizes, so a short or strided tensor would be read
    or written out of bounds on the device.  None passes through."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.element_size() != itemsize:
        raise ValueError("%s must have %d-byte elements (has %d)" % (name, itemsize, t.element_size()))
    if t.numel() < n_elems:
        raise ValueError("%s holds %d elements, needs %d" % (name, t.numel(), n_elems))
    return t.data_ptr()


def _rays_ptr(r, name: str = "rays"):
    """(pointer, n) of a device ray tensor [n, 8] float32."""
    if r.dim() != 2 or r.shape[1] != 8:
        raise ValueError("%s must have shape [n, 8]" % name)
    return _dptr(r, 8 * r.shape[0], name), int(r.shape[0])


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


@dataclass
class Hits:
    id: "torch.Tensor"
    inst: "torch.Tensor"
    t: "torch.Tensor"
    normal: "torch.Tensor"


def _job_array(jobs):
    arr = (Job * max(len(jobs), 1))()
    keep = []
    for i, j in enumerate(jobs):
        fwd = j.get("fwd")
        if fwd is not None:
            fwd = np.ascontiguousarray(np.asarray(fwd, np.float32).reshape(-1, 12))
            keep.append(fwd)
        cam = j.get("camera")
        if cam is not None:
            # rays made in the trace kernel from the camera
            rp, n = None, int(cam.width) * int(cam.height) * int(cam.samples)
            keep.append(cam)
        else:
            rp, n = _rays_ptr(j["rays"], "job %d rays" % i)
        arr[i] = Job(int(j["scene"]), _np_ptr(fwd) if fwd is not None else None, rp, n,
                     _dptr(j["out_id"], n, "job %d out_id" % i), _dptr(j.get("out_inst"), n, "job %d out_inst" % i),
                     _dptr(j["out_t"], n, "job %d out_t" % i), _dptr(j.get("out_normal"), 3 * n, "job %d out_normal" % i),
                     ctypes.pointer(cam) if cam is not None else None)
    return arr, keep


class Plan:
    """svo_plan_*: fixed-argument batched launch.  set_jobs() packs jobs into
    the plan's pinned staging; launch() enqueues the staging copy and the
    persistent trace kernel and may be captured into a torch CUDA graph."""

    def __init__(self, ctx: "Context", scenes, max_jobs: int, max_frames: int):
        self.ctx = ctx
        hs = (ctypes.c_uint32 * len(scenes))(*[int(h) for h in scenes])
        lim = PlanLimits(int(max_jobs), int(max_frames))
        ptr = ctypes.c_void_p()
        _check(lib().svo_plan_create(ctx._ptr, hs, len(scenes), ctypes.byref(lim), ctypes.byref(ptr)))
        self._ptr = ptr

    def set_jobs(self, jobs):
        arr, keep = _job_array(jobs)
        _check(lib().svo_plan_set_jobs(self.ctx._ptr, self._ptr, arr, len(jobs)))

    def launch(self, stream=None):
        _check(lib().svo_plan_launch(self.ctx._ptr, self._ptr, _stream_handle(stream)))

    def close(self):
        if self._ptr and self.ctx._ptr:
            lib().svo_plan_destroy(self.ctx._ptr, self._ptr)
        self._ptr = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Context:
    """One device context (svo_create / svo_destroy)."""

    def __init__(self, device: int = 0):
        self._ptr = ctypes.c_void_p()
        self.device = int(device)
        _check(lib().svo_create(ctypes.byref(self._ptr), self.device))

    def close(self):
        if self._ptr:
            lib().svo_destroy(self._ptr)
            self._ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- configuration
    def get_config(self) -> Config:
        c = Config()
        _check(lib().svo_get_config(self._ptr, ctypes.byref(c)))
        return c

    def set_config(self, **kw) -> Config:
        c = self.get_config()
        for k, v in kw.items():
            setattr(c, k, int(v))
        _check(lib().svo_set_config(self._ptr, ctypes.byref(c)))
        return self.get_config()

    # -- scenes
    def upload(self, nodes, root, root_min, root_size, max_depth, slot_child, slot_cell) -> int:
        nodes = np.ascontiguousarray(nodes, dtype=np.uint64)
        rmin = np.ascontiguousarray(np.asarray(root_min, np.float32).reshape(3))
        sc = np.ascontiguousarray(np.asarray(slot_child, np.uint32).reshape(-1))
        cell = np.ascontiguousarray(np.asarray(slot_cell, np.float32).reshape(-1, 4))
        h = ctypes.c_uint32(0)
        _check(lib().svo_upload(self._ptr, _np_ptr(nodes), nodes.shape[0], int(root), _np_ptr(rmin),
                                float(root_size), int(max_depth), _np_ptr(sc), _np_ptr(cell), sc.shape[0],
                                ctypes.byref(h)))
        return int(h.value)

    def upload_scene(self, scene, static: bool = False) -> int:
        """Upload a generated scene (svogen.scenes.Scene) or its static twin."""
        nodes = scene.static_pool() if static else scene.nodes
        return self.upload(nodes, scene.root, scene.root_min, scene.root_size, scene.max_depth, scene.slot_child,
                           scene.slot_cell)

    def free_scene(self, scene: int):
        _check(lib().svo_free_scene(self._ptr, int(scene)))

    def scene_bytes(self, scene: int) -> int:
        b = ctypes.c_uint64(0)
        _check(lib().svo_scene_bytes(self._ptr, int(scene), ctypes.byref(b)))
        return int(b.value)

    def scene_stats(self, scene: int) -> SceneStats:
        st = SceneStats()
        _check(lib().svo_get_scene_stats(self._ptr, int(scene), ctypes.byref(st)))
        return st

    def set_transforms(self, scene: int, fwd, first: int = 0, stream=None):
        f = np.ascontiguousarray(np.asarray(fwd, np.float32).reshape(-1, 12))
        _check(lib().svo_set_transforms(self._ptr, int(scene), int(first), f.shape[0], _np_ptr(f),
                                        _stream_handle(stream)))

    def trace_into(self, scene: int, rays, out_id, out_t, out_inst=None, out_normal=None, stream=None):
        """Trace device rays [n, 8] float32 into preallocated device outputs."""
        rp, n = _rays_ptr(rays)
        _check(lib().svo_trace_rays(self._ptr, int(scene), rp, n, _dptr(out_id, n, "out_id"),
                                    _dptr(out_inst, n, "out_inst"), _dptr(out_t, n, "out_t"),
                                    _dptr(out_normal, 3 * n, "out_normal"), _stream_handle(stream)))

    def tune(self, scene: int, sample_rays, stream=None) -> Config:
        """Autotune the kernel configuration for `scene` on device sample rays."""
        c = Config()
        rp, n = _rays_ptr(sample_rays, "sample_rays")
        _check(lib().svo_tune(self._ptr, int(scene), rp, n, _stream_handle(stream), ctypes.byref(c)))
        return c

    def trace_camera(self, scene: int, cam: Camera, out: Optional[Hits] = None, stream=None,
                     normals: bool = True) -> Hits:
        """svo_trace_camera: trace the camera's primary rays, made in the
        trace kernel (no ray buffer)."""
        import torch
        n = cam.width * cam.height * cam.samples
        dev = "cuda:%d" % self.device
        if out is None:
            out = Hits(torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.int32, device=dev),
                       torch.empty(n, dtype=torch.float32, device=dev),
                       torch.empty((n, 3), dtype=torch.float32, device=dev) if normals else None)
        _check(lib().svo_trace_camera(self._ptr, int(scene), ctypes.byref(cam), _dptr(out.id, n, "out_id"),
                                      _dptr(out.inst, n, "out_inst"), _dptr(out.t, n, "out_t"),
                                      _dptr(out.normal, 3 * n, "out_normal"), _stream_handle(stream)))
        return out

    def primary_rays(self, cam: Camera, out=None, stream=None):
        """Generate cam.width * cam.height * cam.samples rays into a device tensor [n, 8]."""
        import torch
        n = cam.width * cam.height * cam.samples
        if out is None:
            out = torch.empty((n, 8), dtype=torch.float32, device="cuda:%d" % self.device)
        _check(lib().svo_generate_primary_rays(self._ptr, ctypes.byref(cam), _dptr(out, 8 * n, "out"),
                                               _stream_handle(stream)))
        return out

    def ao_rays(self, rays, hits: "Hits", k: int, seed: int, radius: float, offset: float = 1e-3, out=None,
                stream=None):
        """k cosine-weighted AO rays per primary ray, as a device tensor [n * k, 8]."""
        import torch
        rp, n = _rays_ptr(rays)
        if out is None:
            out = torch.empty((n * k, 8), dtype=torch.float32, device=rays.device)
        if hits.normal is None:
            raise ValueError("AO rays need the primary hits' normals")
        _check(lib().svo_generate_ao_rays(self._ptr, rp, _dptr(hits.t, n, "hits.t"), _dptr(hits.normal, 3 * n, "hits.normal"),
                                          n, int(k), int(seed) & 0xFFFFFFFF, float(radius), float(offset),
                                          _dptr(out, 8 * n * int(k), "out"), _stream_handle(stream)))
        return out

    def trace_reuse(self, scene: int, rays, hits: "Hits", retraced=None, stream=None):
        """Update `hits` (the previous trace of these rays on this scene) for
        the scene's current transforms, retracing only rays that can change.
        retraced: optional int64 device tensor [1] the retraced count is added to."""
        rp, n = _rays_ptr(rays)
        _check(lib().svo_trace_rays_reuse(self._ptr, int(scene), rp, n, _dptr(hits.id, n, "hits.id"),
                                          _dptr(hits.inst, n, "hits.inst"), _dptr(hits.t, n, "hits.t"),
                                          _dptr(hits.normal, 3 * n, "hits.normal"),
                                          _dptr(retraced, 1, "retraced", itemsize=8), _stream_handle(stream)))
        return hits

    def shade(self, scene: int, prim_id, width: int, height: int, samples: int = 1, tiled: bool = True, ao_id=None,
              k: int = 0, ambient_permille: int = 200, background=0xFF402010, out=None, stream=None):
        """RGBA8 image [height, width] (uint32, R in the low byte) from hit ids."""
        import torch
        if out is None:
            out = torch.empty((height, width), dtype=torch.int32, device=prim_id.device)
        n = int(width) * int(height) * int(samples)
        _check(lib().svo_shade(self._ptr, int(scene), _dptr(prim_id, n, "prim_id"),
                               _dptr(ao_id, n * int(k), "ao_id") if k else None,
                               int(width), int(height), int(samples), int(bool(tiled)), int(k), int(ambient_permille),
                               int(background) & 0xFFFFFFFF, _dptr(out, int(width) * int(height), "out"),
                               _stream_handle(stream)))
        return out

    def trace_batch(self, jobs, stream=None):
        """jobs: sequence of dicts with keys scene, rays (device [n, 8]), out_id,
        out_t, and optionally out_inst, out_normal, fwd (host [n_slots, 12])."""
        arr, keep = _job_array(jobs)
        _check(lib().svo_trace_batch(self._ptr, arr, len(jobs), _stream_handle(stream)))

    def trace_counted(self, scene: int, rays, trail_cap: int = 0, stream=None):
        """svo_trace_rays_counted: (hits, counts [3, n] int32 tensor, trail
        [trail_cap, n] int32 tensor or None)."""
        import torch
        if not rays.is_cuda or rays.dtype != torch.float32 or rays.dim() != 2 or rays.shape[1] != 8:
            raise ValueError("rays must be a float32 device tensor of shape [n, 8]")
        rays = rays.contiguous()
        n = rays.shape[0]
        dev = rays.device
        h = Hits(torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.int32, device=dev),
                 torch.empty(n, dtype=torch.float32, device=dev), torch.empty((n, 3), dtype=torch.float32, device=dev))
        counts = torch.zeros((3, n), dtype=torch.int32, device=dev)
        trail = torch.zeros((trail_cap, n), dtype=torch.int32, device=dev) if trail_cap else None
        _check(lib().svo_trace_rays_counted(self._ptr, int(scene), rays.data_ptr(), n, h.id.data_ptr(),
                                            h.inst.data_ptr(), h.t.data_ptr(), h.normal.data_ptr(), counts.data_ptr(),
                                            trail.data_ptr() if trail is not None else None, int(trail_cap),
                                            _stream_handle(stream)))
        return h, counts, trail

    def trace_batch_static(self, jobs, stream=None):
        """As trace_batch, through the allocation-free entry point (the
        library's per-device scratch; calls on one device must not overlap)."""
        arr, keep = _job_array(jobs)
        _check(lib().svo_trace_batch_static(self._ptr, arr, len(jobs), _stream_handle(stream)))

    def plan(self, scenes, max_jobs: int = 64, max_frames: int = 512) -> "Plan":
        """A reusable (graph-capturable) batched launch for jobs on `scenes`."""
        return Plan(self, scenes, max_jobs, max_frames)

    def trace(self, scene: int, rays, stream=None, normals: bool = True) -> Hits:
        import torch
        if not rays.is_cuda or rays.dtype != torch.float32 or rays.dim() != 2 or rays.shape[1] != 8:
            raise ValueError("rays must be a float32 device tensor of shape [n, 8]")
        rays = rays.contiguous()
        n = rays.shape[0]
        dev = rays.device
        out_id = torch.empty(n, dtype=torch.int32, device=dev)
        out_inst = torch.empty(n, dtype=torch.int32, device=dev)
        out_t = torch.empty(n, dtype=torch.float32, device=dev)
        out_n = torch.empty((n, 3), dtype=torch.float32, device=dev) if normals else None
        self.trace_into(scene, rays, out_id, out_t, out_inst, out_n, stream)
        return Hits(out_id, out_inst, out_t, out_n)
