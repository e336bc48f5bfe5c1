"""Serving loop: render requests of uneven resolution and scene, continuously
batched into persistent trace launches, admitted by device-memory footprint.

Each request asks for one frame (an animation frame index) of one resident
scene at some resolution and rays per pixel.  Pools and transform tables stay
resident and are counted against the device-memory budget first
(svo_scene_bytes); a request only brings its ray and output buffers, admitted
against what is left.

  batched  requests are admitted while their footprint fits the budget;
           every step packs up to `max_rays_per_step` rays from the admitted
           requests (large requests are split across steps, unless one is
           the only request with work: then up to `solo_rays_per_step`) into one
           persistent launch, each job with its own scene and animation
           frame; two steps are kept in flight, on two streams, so the host
           prepares step k+1 while the device runs step k, and step k+1's
           launch takes the CUs that step k frees while its last rays drain.
           With graph=True each in-flight slot owns a launch plan (svo_plan_*)
           whose launch was captured once into a HIP graph; a step writes its
           jobs into the plan's staging and replays the graph.  Otherwise a
           step is one svo_trace_batch call.
  single   the baseline: one request per svo_trace_rays launch, first come,
           first served, the next one starting when the previous finished.

Latency = completion - arrival, with completion read from device events on
the launch stream (the device clock, aligned with the host clock at start).
The loop itself is host Python; every step of the trace runs in libsvo.so.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np

from . import svo

RAY_BYTES = 32
OUT_BYTES = 4 + 4 + 4 + 12  # id, inst, t, normal


@dataclass
class Request:
    rid: int
    arrival: float      # seconds after the start of the run
    scene: str
    frame: int
    width: int
    height: int
    samples: int
    seed: int = 0
    ao: int = 0               # ambient-occlusion rays per primary ray (0: primary rays only)
    ao_radius: float = 64.0

    @property
    def rays(self) -> int:
        """Primary rays."""
        return self.width * self.height * self.samples

    @property
    def total_rays(self) -> int:
        return self.rays * (1 + self.ao)

    @property
    def footprint(self) -> int:
        return self.total_rays * (RAY_BYTES + OUT_BYTES)


@dataclass
class SceneEntry:
    handle: int
    xform: Callable[[int], np.ndarray]   # frame -> [n_slots, 12] forward maps
    camera: dict


@dataclass
class Result:
    req: Request
    admitted: float = 0.0
    completed: float = 0.0
    out: Optional[dict] = None           # device tensors, kept when keep_outputs

    @property
    def latency(self) -> float:
        return self.completed - self.req.arrival


@dataclass
class _Active:
    req: Request
    res: Result
    rays: "object"
    out: dict
    fwd: np.ndarray
    next_ray: int = 0        # first ray of the current phase not yet submitted
    pending_chunks: int = 0  # submitted chunks not yet complete
    frames: int = 1          # frame records one chunk of this request takes
    n: int = -1              # rays of the current phase (primary, then AO)
    phase: int = 0           # 0: primary rays; 1: AO rays from the primary hits
    primary_out: Optional[dict] = None
    ready: "object" = None   # device event after which the current phase's rays exist
    step_events: list = field(default_factory=list)   # events of the steps holding this phase's chunks
    done_at: float = 0.0     # latest completion of its retired steps (steps on two streams may end out of order)

    def __post_init__(self):
        if self.n < 0:
            self.n = self.req.rays


class Scheduler:
    """The batching policy, free of device calls (so it can be tested alone).

    admit(): move waiting requests (first come, first served) into the
    active set while their footprint fits the budget.  plan(): pick the next
    step's chunks, at most `max_rays` rays, `max_jobs` chunks and `max_frames`
    frame records (a launch's limits):
      fifo  oldest admitted request first, each taking what is left of the
            step's rays in turn;
      fair  the step's rays are shared evenly among the requests with work
            left (at least `min_chunk` each), so a small request admitted
            behind a large one finishes in the next step instead of waiting
            for the large one to drain (processor sharing: large requests
            are stretched by everything that arrives while they run);
      edf   earliest deadline first, deadline = arrival + slack x rays /
            ref_rate: a small request overtakes large ones that arrived a
            little earlier, but no request is passed by work that arrived
            after its deadline, which bounds the stretch of large requests.
    A request that is the only one with work left may take up to
    `solo_rays` rays in one step (0: no exception): there is nothing to
    interleave with it, and every extra step costs a launch and its drain.
    For the same reason a chunk takes the rest of its request's phase when
    that rest is at most a quarter of the step cap and the chunk stays
    within 1.25 step caps.
    """

    def __init__(self, budget: int, max_rays: int, policy: str = "edf", min_chunk: int = 1 << 16,
                 max_jobs: int = 256, max_frames: int = 2047, slack: float = 3.0, ref_rate: float = 4e9,
                 solo_rays: int = 0):
        if policy not in ("fifo", "fair", "edf"):
            raise ValueError(policy)
        self.slack = float(slack)
        self.ref_rate = float(ref_rate)
        self.budget = int(budget)
        self.max_rays = int(max_rays)
        self.policy = policy
        self.min_chunk = int(min_chunk)
        self.max_jobs = int(max_jobs)
        self.max_frames = int(max_frames)
        self.solo_rays = int(solo_rays)
        self.used = 0
        self.max_used = 0

    def admit(self, waiting: "collections.deque", on_admit: Callable[[Request], object],
              frames_of: Optional[Callable[[Request], int]] = None) -> list:
        """frames_of(req): frame records one chunk of req takes; a request that
        could never fit a step is rejected instead of waiting forever."""
        if frames_of is not None:
            for req in waiting:
                if frames_of(req) > self.max_frames:
                    raise ValueError("request %d needs %d frame records per step, the limit is %d" %
                                     (req.rid, frames_of(req), self.max_frames))
        admitted = []
        while waiting and self.used + waiting[0].footprint <= self.budget:
            req = waiting.popleft()
            self.used += req.footprint
            self.max_used = max(self.max_used, self.used)
            admitted.append(on_admit(req))
        if waiting and waiting[0].footprint > self.budget:
            raise ValueError("request %d needs %d bytes, more than the budget %d" %
                             (waiting[0].rid, waiting[0].footprint, self.budget))
        return admitted

    def release(self, req: Request):
        self.used -= req.footprint

    def plan(self, active: list) -> list:
        """[(active, lo, hi)] within the step limits; advances next_ray."""
        work = [a for a in active if a.n > a.next_ray]
        if self.policy == "edf":
            work.sort(key=lambda a: a.req.arrival + self.slack * a.req.total_rays / self.ref_rate)
        left = self.max_rays
        if len(work) == 1:
            # splitting lets other requests interleave; with none to interleave
            # it only adds a launch (and its drain) per extra step
            left = max(left, self.solo_rays)
        chunks, frames = [], 0
        share = left
        if self.policy == "fair" and work:
            share = max(self.min_chunk, left // min(len(work), self.max_jobs))
        for a in work:
            if left <= 0 or len(chunks) >= self.max_jobs or frames + a.frames > self.max_frames:
                break
            k = min(a.n - a.next_ray, share, left)
            rest = a.n - a.next_ray - k
            if 0 < rest <= self.max_rays // 4 and k + rest <= self.max_rays + self.max_rays // 4:
                # a remainder this small would cost a step (and its drain) of
                # its own: it rides along, the chunk exceeding the step cap by
                # at most a quarter
                k += rest
            chunks.append((a, a.next_ray, a.next_ray + k))
            a.next_ray += k
            a.pending_chunks += 1
            left -= k
            frames += a.frames
        return chunks


def poisson_requests(n: int, rate: float, seed: int, scenes: List[str], frames: int = 60,
                     resolutions=((256, 256), (1280, 720), (1920, 1080), (2048, 1152)),
                     samples=(1, 5), shapes: Optional[Dict[str, tuple]] = None) -> List[Request]:
    """Seeded Poisson arrival trace with uniformly drawn scene, frame,
    resolution and rays per pixel; `shapes` fixes (width, height, samples,
    AO rays per primary ray) per scene instead."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(n):
        W, H = resolutions[rng.integers(0, len(resolutions))]
        sc = scenes[rng.integers(0, len(scenes))]
        f = int(rng.integers(0, frames))
        spp = int(rng.integers(samples[0], samples[1] + 1))
        sd = int(rng.integers(0, 2**31))
        ao = 0
        if shapes is not None:
            W, H, spp, ao = shapes[sc]
        out.append(Request(i, float(t[i]), sc, f, int(W), int(H), int(spp), sd, int(ao)))
    return out


class Server:
    def __init__(self, ctx: svo.Context, scenes: Dict[str, SceneEntry], hbm_budget: int,
                 max_rays_per_step: int = 1 << 23, solo_rays_per_step: int = 1 << 24, inflight_steps: int = 2,
                 keep_outputs: bool = False,
                 policy: str = "edf", graph: bool = False, max_jobs: int = 16, max_frames: int = 64):
        import torch
        self.torch = torch
        self.ctx = ctx
        self.scenes = scenes
        self.budget = int(hbm_budget)
        self.max_rays = int(max_rays_per_step)
        self.solo_rays = int(solo_rays_per_step)
        self.inflight_steps = int(inflight_steps)
        self.keep = keep_outputs
        self.policy = policy
        self.stream = torch.cuda.current_stream()
        self.dev = torch.device("cuda:%d" % ctx.device)
        # one stream per in-flight step (default priority): the next step's
        # launch takes the CUs that the previous launch frees while it drains,
        # instead of waiting behind its slowest rays
        self.step_streams = [torch.cuda.Stream(device=self.dev) for _ in range(self.inflight_steps)]
        self.frames = {k: 1 + ctx.scene_stats(e.handle).n_slots for k, e in scenes.items()}
        # the resident pools and transform tables come out of the budget
        # first; requests are admitted against what is left
        self.resident_bytes = sum(ctx.scene_bytes(e.handle) for e in scenes.values())
        if self.resident_bytes >= self.budget:
            raise ValueError("resident scenes take %d bytes, the budget is %d" % (self.resident_bytes, self.budget))
        self.max_jobs = int(max_jobs)
        # room for at least two jobs of the largest scene per step
        self.max_frames = max(int(max_frames), 2 * max(self.frames.values()))
        self.graph = bool(graph)
        self._plans = []
        self._graphs = []
        if self.graph:
            self._capture()

    def _capture(self):
        """One plan per in-flight slot, its launch captured into a graph."""
        t = self.torch
        handles = [e.handle for e in self.scenes.values()]
        # the scene with the most pool nodes first: its prefix sizes the LDS cache
        handles.sort(key=lambda h: -self.ctx.scene_stats(h).device_bytes)
        for _ in range(self.inflight_steps):
            plan = self.ctx.plan(handles, max_jobs=self.max_jobs, max_frames=self.max_frames)
            plan.set_jobs([])
            g = t.cuda.CUDAGraph()
            side = t.cuda.Stream()
            side.wait_stream(t.cuda.current_stream())
            with t.cuda.graph(g, stream=side):
                plan.launch(t.cuda.current_stream())
            self._plans.append(plan)
            self._graphs.append(g)
        t.cuda.synchronize()

    def close(self):
        self.torch.cuda.synchronize()
        self._graphs = []
        for p in self._plans:
            p.close()
        self._plans = []

    # -- helpers
    def _camera(self, req: Request):
        c = self.scenes[req.scene].camera
        return svo.make_camera(c["eye"], c["target"], c["up"], c["fov"], req.width, req.height, samples=req.samples,
                               seed=req.seed, jitter=req.samples > 1, tiled=True)

    def _buffers(self, n: int):
        t = self.torch
        return dict(out_id=t.empty(n, dtype=t.int32, device=self.dev), out_inst=t.empty(n, dtype=t.int32, device=self.dev),
                    out_t=t.empty(n, dtype=t.float32, device=self.dev),
                    out_normal=t.empty((n, 3), dtype=t.float32, device=self.dev))

    def _start_ao(self, a: "_Active", stream):
        """Second phase of a request: AO rays from its primary hits, generated
        on the device.  Called once the request's last primary chunk has been
        enqueued: the generation waits on `stream` for every step that holds
        a primary chunk, and the steps of the AO phase wait for it."""
        from .svo import Hits
        for e in a.step_events:
            stream.wait_event(e)
        hits = Hits(a.out["out_id"], a.out["out_inst"], a.out["out_t"], a.out["out_normal"])
        ao = self.ctx.ao_rays(a.rays, hits, k=a.req.ao, seed=a.req.seed, radius=a.req.ao_radius, stream=stream)
        a.ready = self.torch.cuda.Event()
        a.ready.record(stream)
        a.step_events = []
        a.primary_out, a.primary_rays = a.out, a.rays
        a.rays, a.out = ao, self._buffers(ao.shape[0])
        a.phase, a.n, a.next_ray = 1, ao.shape[0], 0

    def run(self, requests: List[Request], mode: str = "batched") -> List[Result]:
        if mode == "batched":
            return self._run_batched(requests)
        if mode == "single":
            return self._run_single(requests)
        raise ValueError(mode)

    # -- continuous batching
    def _run_batched(self, requests: List[Request]) -> List[Result]:
        t = self.torch
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting = collections.deque()
        active: List[_Active] = []
        inflight = collections.deque()   # (event, [(active, n_rays)])
        results: List[Result] = []
        sched = Scheduler(self.budget - self.resident_bytes, self.max_rays, self.policy, max_jobs=self.max_jobs,
                          max_frames=self.max_frames, solo_rays=self.solo_rays)
        step = 0
        self.scheduler = sched
        t.cuda.synchronize()
        start_ev = t.cuda.Event(enable_timing=True)
        start_ev.record(self.stream)
        t0 = time.perf_counter()

        def on_admit(req):
            entry = self.scenes[req.scene]
            rays = self.ctx.primary_rays(self._camera(req), stream=self.stream)
            res = Result(req, admitted=time.perf_counter() - t0)
            a = _Active(req, res, rays, self._buffers(req.rays), np.ascontiguousarray(entry.xform(req.frame), np.float32),
                        frames=self.frames[req.scene])
            a.ready = t.cuda.Event()
            a.ready.record(self.stream)
            active.append(a)
            return a

        while pending or waiting or active or inflight:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            # retire finished steps (in submission order)
            while inflight and inflight[0][0].query():
                ev, chunks = inflight.popleft()
                done_at = start_ev.elapsed_time(ev) * 1e-3
                for a, _, _ in chunks:
                    a.pending_chunks -= 1
                    a.done_at = max(a.done_at, done_at)
                    if a.pending_chunks == 0 and a.next_ray >= a.n and (a.phase == 1 or not a.req.ao):
                        a.res.completed = a.done_at
                        if self.keep:
                            a.res.out = a.primary_out or a.out
                            a.res.out["rays"] = a.primary_rays if a.phase else a.rays
                            if a.phase:
                                a.res.out["ao"] = dict(a.out, rays=a.rays)
                        results.append(a.res)
                        active.remove(a)
                        sched.release(a.req)
            sched.admit(waiting, on_admit, lambda r: self.frames[r.scene])
            # submit one step when a slot is free and there is work
            if len(inflight) < self.inflight_steps:
                chunks = sched.plan(active)
                if chunks:
                    jobs = [dict(scene=self.scenes[a.req.scene].handle, fwd=a.fwd, rays=a.rays[lo:hi],
                                 out_id=a.out["out_id"][lo:hi], out_inst=a.out["out_inst"][lo:hi],
                                 out_t=a.out["out_t"][lo:hi], out_normal=a.out["out_normal"][lo:hi])
                            for a, lo, hi in chunks]
                    k = step % self.inflight_steps
                    st = self.step_streams[k]
                    for a in {id(a): a for a, _, _ in chunks}.values():
                        st.wait_event(a.ready)     # its rays exist (generated on another stream)
                    if self.graph:
                        # this slot's previous replay has retired (steps
                        # retire in order and at most inflight_steps - 1 are
                        # still in flight)
                        self._plans[k].set_jobs(jobs)
                        with t.cuda.stream(st):
                            self._graphs[k].replay()
                    else:
                        self.ctx.trace_batch(jobs, stream=st)
                    step += 1
                    ev = t.cuda.Event(enable_timing=True)
                    ev.record(st)
                    inflight.append((ev, chunks))
                    for a, _, _ in chunks:
                        a.step_events.append(ev)
                    # a request whose last primary chunk is in this step gets
                    # its AO rays generated behind it, so its AO phase can go
                    # into the next step without waiting for this one to retire
                    for a in {id(a): a for a, _, _ in chunks}.values():
                        if a.phase == 0 and a.req.ao and a.next_ray >= a.n:
                            self._start_ao(a, st)
                    continue
            # nothing to submit: wait for the device or the next arrival
            if inflight:
                if not (pending and pending[0].arrival <= time.perf_counter() - t0):
                    time.sleep(0)
            elif pending and not waiting:
                dt = pending[0].arrival - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(min(dt, 0.001))
        t.cuda.synchronize()
        return sorted(results, key=lambda r: r.req.rid)

    # -- one request per launch
    def _run_single(self, requests: List[Request]) -> List[Result]:
        t = self.torch
        queue = sorted(requests, key=lambda r: r.arrival)
        results = []
        t.cuda.synchronize()
        start_ev = t.cuda.Event(enable_timing=True)
        start_ev.record(self.stream)
        t0 = time.perf_counter()
        for req in queue:
            now = time.perf_counter() - t0
            if req.arrival > now:
                time.sleep(req.arrival - now)
            entry = self.scenes[req.scene]
            res = Result(req, admitted=time.perf_counter() - t0)
            rays = self.ctx.primary_rays(self._camera(req), stream=self.stream)
            out = self._buffers(req.rays)
            self.ctx.set_transforms(entry.handle, entry.xform(req.frame), stream=self.stream)
            self.ctx.trace_into(entry.handle, rays, out["out_id"], out["out_t"], out["out_inst"], out["out_normal"],
                                stream=self.stream)
            if req.ao:
                from .svo import Hits
                hits = Hits(out["out_id"], out["out_inst"], out["out_t"], out["out_normal"])
                ao = self.ctx.ao_rays(rays, hits, k=req.ao, seed=req.seed, radius=req.ao_radius, stream=self.stream)
                ao_out = self._buffers(ao.shape[0])
                self.ctx.trace_into(entry.handle, ao, ao_out["out_id"], ao_out["out_t"], ao_out["out_inst"],
                                    ao_out["out_normal"], stream=self.stream)
                out["ao"] = dict(ao_out, rays=ao)
            ev = t.cuda.Event(enable_timing=True)
            ev.record(self.stream)
            ev.synchronize()
            res.completed = start_ev.elapsed_time(ev) * 1e-3
            if self.keep:
                out["rays"] = rays
                res.out = out
            results.append(res)
        return sorted(results, key=lambda r: r.req.rid)


def summarize(results: List[Result]) -> dict:
    lat = np.array([r.latency for r in results]) * 1e3
    rays = sum(r.req.total_rays for r in results)
    span = max(r.completed for r in results) - min(r.req.arrival for r in results)
    return dict(requests=len(results), p50_ms=round(float(np.percentile(lat, 50)), 3),
                p99_ms=round(float(np.percentile(lat, 99)), 3), mean_ms=round(float(lat.mean()), 3),
                mrays_per_s=round(rays / span / 1e6, 2) if span > 0 else None, rays=int(rays),
                makespan_s=round(span, 4))
