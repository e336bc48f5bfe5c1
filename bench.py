"""Benchmark: animated vs static SVO trace at 1080p on one MI355X.

Workload: depth-10 (1024^3) fBm heightfield, 8 level-3 subtrees
animated per frame (rotation + anisotropic scale 0.5..2), 1920x1080 primary
rays.  One step = one frame: upload that frame's transforms
(svo_set_transforms: FP64 compose/invert + 64-byte records) and trace all
2,073,600 rays (svo_trace_rays), rays and pool resident in HBM.  The static
twin (same pool, no transforms, same rays) is timed the same way.

Prints one JSON line.  value = animated Mrays/s over the timed steps.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mrays/s animated vs static SVO trace at 1080p; p50/p99 served frame latency"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_1911_06001_amd/csrc/svo_trace.hip", "paper_1911_06001_amd/csrc/svo_internal.h"]
PMC_SUMMARY = os.path.join(ROOT, "profiles", "trace_kernel_terrain1024_1080p_pmc.txt")


# The paper's own measurements (Sec. 5.1, Fig. 7: average render time per
# 1280x768 frame of a depth-11 car model, static camera), on NVIDIA GPUs.
# Context only, not a target: another model, resolution and machine, and the
# frame time may include display.  Mrays/s is derived here as 1280 * 768
# rays per frame (one ray per pixel) / render time.
def _paper_rate(ms):
    return round(1280 * 768 / (ms * 1e-3) / 1e6, 2)


PAPER_CONTEXT = {
    "source": "Sec. 5.1, Fig. 7 (render time per 1280x768 frame, depth-11 car, 1 ray/pixel derived)",
    "unit": "Mrays/s",
    "gpus": {
        gpu: {"static": _paper_rate(st), "animated": _paper_rate(an), "animated_opt": _paper_rate(op)}
        for gpu, st, an, op in (("Quadro T1000", 61.68, 80.78, 62.05), ("GeForce GTX 680", 42.86, 56.16, 40.18),
                                ("Quadro P5000", 16.74, 21.12, 14.77))
    },
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_counters():
    """Per-launch counter figures from the committed rocprofv3 summary, if it
    was taken on the current kernel source; else {}."""
    if not os.path.exists(PMC_SUMMARY):
        return {}
    vals = {}
    for line in open(PMC_SUMMARY):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_hash") != kernel_hash():
        return {}
    out = {}
    for k, v in vals.items():
        try:
            out[k] = float(v)
        except ValueError:
            pass
    return out


# VALU issue peak: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 instruction per
# SIMD every 4 cycles (16 lanes per cycle)
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4


def cpu_baseline(scene, rays, frames, budget_s):
    """The oracle as it stands, on the host cores, over whole frames of the
    same workload until ``budget_s`` seconds have been spent."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    done = 0
    spent = 0.0
    bytes_sum = 0.0
    frame_list = []
    nnode = []
    nnode_hi = []
    nframe = []
    f = 0
    while spent < budget_s and f < frames:
        t0 = time.perf_counter()
        h = oracle.trace_scene(scene, rays, frame=f, counters=True, nthreads=threads)
        spent += time.perf_counter() - t0
        done += rays.shape[0]
        # algorithmic bytes per ray: 8 B per node record, 64 B per frame
        # record, 32 B ray in, 24 B hit out; the node and frame counts are the
        # oracle's lower bound (frames entered by the hit, each cut at it)
        bytes_sum += float((8.0 * h.nnode.astype(np.float64) + 64.0 * h.nframe + 32.0 + 24.0).sum())
        nnode.append(h.nnode)
        nnode_hi.append(h.nnode_hi)
        nframe.append(h.nframe)
        frame_list.append(f)
        f += 1
    nn = np.concatenate(nnode) if nnode else np.zeros(1)
    nh = np.concatenate(nnode_hi) if nnode_hi else np.zeros(1)
    nf = np.concatenate(nframe) if nframe else np.zeros(1)
    return dict(rays=done, seconds=spent, threads=threads, frames=frame_list, bytes_per_ray=bytes_sum / max(done, 1),
                n_node_mean=float(nn.mean()), n_node_p99=float(np.percentile(nn, 99)), n_frame_mean=float(nf.mean()),
                n_node_hi_mean=float(nh.mean()))


def replay_ceiling(ctx, handle, sc, fwd, rays, kc, n_cu, reps=5, max_cap=512):
    """The trace's own ceiling: one frame traced by the counting build with a
    trail of its node loads, then those loads replayed in order, with the
    trace's dependence and grid and none of its arithmetic (plus each ray's
    32-byte read and 24-byte write).  Returns the replay and trace times of
    that frame (HIP events on the launch stream)."""
    import torch
    from paper_1911_06001_amd import ceiling
    stream = torch.cuda.current_stream()
    ctx.set_transforms(handle, fwd, stream=stream)
    _, counts, _ = ctx.trace_counted(handle, rays)
    c = counts.cpu().numpy().view(np.uint32)
    loads = (c[0] - c[1]).astype(np.int64)
    cap = int(min(loads.max(), max_cap))
    _, counts, trail = ctx.trace_counted(handle, rays, trail_cap=cap)
    nodes = torch.from_numpy(sc.nodes.view(np.int64)).cuda()
    n = rays.shape[0]
    out = torch.empty(6 * n, dtype=torch.int32, device=rays.device)
    blocks, threads = n_cu * kc["blocks_per_cu"], 64 * kc["waves_per_block"]
    sink = torch.empty(blocks * threads, dtype=torch.int64, device=rays.device)
    n_lds = int(min(kc["lds_cache_nodes"], 16384, sc.nodes.shape[0]))
    t_rep = ceiling._time(lambda: ceiling.replay(nodes, n_lds, trail, counts, rays, out, blocks, threads, sink,
                                                 stream), reps)
    hits = ctx.trace(handle, rays)
    t_tr = ceiling._time(lambda: ctx.trace_into(handle, rays, hits.id, hits.t, hits.inst, hits.normal, stream=stream),
                         reps)
    del trail, nodes, out, sink
    torch.cuda.empty_cache()
    return {"replay_ms": round(t_rep * 1e3, 4), "trace_ms_same_frame": round(t_tr * 1e3, 4), "grid": [blocks, threads],
            "lds_nodes": n_lds, "loads_per_ray_mean": round(float(loads.mean()), 3), "trail_cap": cap,
            "loads_truncated": int(np.maximum(loads - cap, 0).sum())}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def instances_throughput(ctx, steps, knobs=None):
    """Instanced scene (64 DAG-shared instances of 4 SVOs in a 4096^3 world):
    1080p primary rays, then 4 cosine-weighted AO rays per pixel from the
    primary hits (incoherent).  Mrays/s of each trace, kernel time from HIP
    events on the launch stream.  With ``knobs`` the kernel runs that
    configuration instead of the autotuner's."""
    import torch
    from svogen import scenes
    t0 = time.perf_counter()
    sc = scenes.instanced_scene()
    log("instanced scene: %d nodes (%.1f s)" % (sc.nodes.shape[0], time.perf_counter() - t0))
    h = ctx.upload_scene(sc)
    ctx.set_transforms(h, sc.xform(0))
    rays_np, _ = sc.rays()
    rays = torch.from_numpy(rays_np).cuda()
    n = rays.shape[0]
    prim = ctx.trace(h, rays)
    ao = ctx.ao_rays(rays, prim, k=4, seed=3, radius=64.0)
    if knobs:
        ctx.set_config(**knobs)
        cfg = ctx.get_config().as_dict()
    else:
        cfg = ctx.tune(h, rays).as_dict()
    out_ao = ctx.trace(h, ao)
    stream = torch.cuda.current_stream()
    res = {}
    for name, r, out in (("primary", rays, prim), ("ao", ao, out_ao)):
        for _ in range(2):
            ctx.trace_into(h, r, out.id, out.t, out.inst, out.normal, stream=stream)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        for a, b in evs:
            a.record(stream)
            ctx.trace_into(h, r, out.id, out.t, out.inst, out.normal, stream=stream)
            b.record(stream)
        torch.cuda.synchronize()
        ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
        res[name] = {"rays": int(r.shape[0]), "kernel_ms": round(ms, 4), "mrays_per_s": round(r.shape[0] / ms / 1e3, 2)}
    st = ctx.scene_stats(h)
    ctx.free_scene(h)
    log("instances: primary %.0f Mrays/s, AO %.0f Mrays/s" % (res["primary"]["mrays_per_s"], res["ao"]["mrays_per_s"]))
    res.update({"workload": "instances4096: 64 instances (sphere d8, noise blob d9, heightfield d10, box lattice d11) "
                            "at levels 1-3 of a 4096^3 world; 1920x1080 primary + 4 AO rays per pixel",
                "nodes": int(sc.nodes.shape[0]), "candidates": int(st.n_candidates), "inline": int(st.n_inline),
                "kernel": cfg})
    return res


def c5_throughput(ctx, steps, frames=60, knobs=None):
    """Depth-12 ridged terrain (4096^3, ~1.5e8 nodes = 1.2 GB pool, 256
    animated level-4 subtrees): per frame, upload that frame's transforms,
    trace 3840x2160 primary rays, generate 2 cosine-weighted AO rays per
    pixel on the device, trace them and composite the RGBA8 frame.  Kernel times from HIP events on the
    launch stream; algorithmic bytes per ray from the oracle's counters on a
    sample of the same rays (every 997th).  With ``knobs`` the kernel runs
    that configuration instead of the autotuner's."""
    import torch
    import oracle
    from svogen import scenes
    t0 = time.perf_counter()
    sc = scenes.ridged_terrain_d12(frames=frames)
    log("depth-12 terrain: %d nodes (%.1f s)" % (sc.nodes.shape[0], time.perf_counter() - t0))
    h = ctx.upload_scene(sc)
    rays_np, _ = sc.rays()
    n = rays_np.shape[0]
    rays = torch.from_numpy(rays_np).cuda()
    xf = [sc.xform(f) for f in range(frames)]
    ctx.set_transforms(h, xf[0])
    if knobs:
        ctx.set_config(**knobs)
        tuned = ctx.get_config().as_dict()
    else:
        tuned = ctx.tune(h, rays).as_dict()
    stream = torch.cuda.current_stream()
    prim = ctx.trace(h, rays)
    ao = ctx.ao_rays(rays, prim, k=2, seed=5, radius=64.0)
    out_ao = ctx.trace(h, ao)
    torch.cuda.synchronize()
    W5, H5 = sc.camera["W"], sc.camera["H"]
    img = ctx.shade(h, prim.id, W5, H5, ao_id=out_ao.id, k=2)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
    w0 = time.perf_counter()
    for k in range(steps):
        e = ev[k]
        ctx.set_transforms(h, xf[(7 * k) % frames], stream=stream)   # 7 is coprime with the 60-frame cycle
        e[0].record(stream)
        ctx.trace_into(h, rays, prim.id, prim.t, prim.inst, prim.normal, stream=stream)
        e[1].record(stream)
        ctx.ao_rays(rays, prim, k=2, seed=5 + k, radius=64.0, out=ao, stream=stream)
        e[2].record(stream)
        ctx.trace_into(h, ao, out_ao.id, out_ao.t, out_ao.inst, out_ao.normal, stream=stream)
        e[3].record(stream)
        ctx.shade(h, prim.id, W5, H5, ao_id=out_ao.id, k=2, out=img, stream=stream)
        e[4].record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - w0) / steps
    pm = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    am = float(np.mean([e[2].elapsed_time(e[3]) for e in ev]))
    sm = float(np.mean([e[3].elapsed_time(e[4]) for e in ev]))
    # algorithmic bytes of the primary trace from the oracle on a sample
    idx = np.arange(0, n, 997)
    hs = oracle.trace_scene(sc, rays_np[idx], frame=0, counters=True)
    bpr = float((8.0 * hs.nnode.astype(np.float64) + 64.0 * hs.nframe + 32.0 + 24.0).mean())
    achieved = bpr * n / (pm * 1e-3) / 1e9
    st = ctx.scene_stats(h)
    res = {"workload": "terrain4096: depth-12 (4096^3) ridged-fBm heightfield SVO, %d nodes (%.2f GB), 256 level-4 "
                       "subtrees animated by 4 jittered keyframes (slerp + log-scale lerp), 3840x2160 primary + 2 "
                       "AO rays per pixel" % (sc.nodes.shape[0], sc.nodes.nbytes / 1e9),
           "nodes": int(sc.nodes.shape[0]), "pool_bytes": int(sc.nodes.nbytes), "candidates": int(st.n_candidates),
           "inline": int(st.n_inline), "kernel": tuned, "steps": steps,
           "primary": {"rays": n, "kernel_ms": round(pm, 4), "mrays_per_s": round(n / pm / 1e3, 2)},
           "ao": {"rays": 2 * n, "kernel_ms": round(am, 4), "mrays_per_s": round(2 * n / am / 1e3, 2)},
           "shade_ms": round(sm, 4),
           "frame_ms_wall": round(wall * 1e3, 4),
           "roofline_primary": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": round(achieved / HBM_PEAK_GBS, 5), "bytes_per_ray": round(bpr, 2),
                                "sample_rays": int(idx.shape[0])}}
    log("depth-12 terrain: primary %.0f Mrays/s, AO %.0f Mrays/s, %.2f ms/frame" % (
        res["primary"]["mrays_per_s"], res["ao"]["mrays_per_s"], res["frame_ms_wall"]))
    del rays, prim, ao, out_ao, img
    torch.cuda.empty_cache()
    return res, sc, h


def serve_c5(ctx, c5_scene, c5_handle, n_requests, load):
    """The depth-12 terrain served beside an instanced-scene stream under a
    16 GiB device-memory budget: 3840x2160 requests with 2 AO rays per pixel
    and 1920x1080 requests with 4 AO rays per pixel (AO rays generated from
    each request's own primary hits, as a second phase), Poisson arrivals at
    `load` x the measured saturation rate; continuously batched vs one
    request per launch."""
    from paper_1911_06001_amd import serve
    from svogen import scenes
    inst = scenes.instanced_scene()
    hi = ctx.upload_scene(inst)
    ctx.set_transforms(hi, inst.xform(0))
    entries = {"terrain4096": serve.SceneEntry(c5_handle, c5_scene.xform, c5_scene.camera),
               "instances4096": serve.SceneEntry(hi, inst.xform, inst.camera)}
    shapes = {"terrain4096": (3840, 2160, 1, 2), "instances4096": (1920, 1080, 1, 4)}
    names = list(entries)
    budget = 16 << 30
    srv = serve.Server(ctx, entries, hbm_budget=budget)
    srv.run(serve.poisson_requests(4, 1e9, 60, names, shapes=shapes), "batched")
    burst = serve.poisson_requests(max(12, n_requests // 4), 1e9, 61, names, shapes=shapes)
    sat = serve.summarize(srv.run(burst, "batched"))
    rate = sat["requests"] / sat["makespan_s"]
    trace = serve.poisson_requests(n_requests, load * rate, 62, names, shapes=shapes)
    b = serve.summarize(srv.run(trace, "batched"))
    max_used = srv.scheduler.max_used
    s1 = serve.summarize(srv.run(trace, "single"))
    ctx.free_scene(hi)
    log("serving depth-12 + instances at %.1f load: batched p50 %.1f p99 %.1f ms, single p50 %.1f p99 %.1f ms, "
        "peak admitted %.1f GiB" % (load, b["p50_ms"], b["p99_ms"], s1["p50_ms"], s1["p99_ms"], max_used / 2**30))
    return {"requests": n_requests, "offered_load": load, "saturation_rps": round(rate, 2), "hbm_budget_bytes": budget,
            "resident_scene_bytes": int(srv.resident_bytes), "peak_admitted_bytes": int(max_used),
            "mix": "terrain4096 3840x2160 + 2 AO rays/pixel and instances4096 1920x1080 + 4 AO rays/pixel, "
                   "Poisson arrivals",
            "batched": b, "single": s1}


def serve_latency(ctx, terrain, terrain_handle, n_requests, loads, warm=100):
    """p50/p99 frame latency of Poisson request streams over the noisy-sphere
    and terrain scenes (resolutions 256^2 .. 2048x1152, 1-5 rays per pixel)
    at each offered load (a fraction of the batched saturation rate), under a
    16 GiB device-memory budget: continuously batched with the launch
    replayed from a captured HIP graph, continuously batched with eager
    launches, and one request per launch.  The first `warm` requests of each
    stream are excluded from the statistics."""
    from paper_1911_06001_amd import serve
    from svogen import scenes
    sph = scenes.noisy_sphere_d6()
    hs = ctx.upload_scene(sph)
    entries = {"sphere": serve.SceneEntry(hs, sph.xform, sph.camera),
               "terrain": serve.SceneEntry(terrain_handle, terrain.xform, terrain.camera)}
    budget = 16 << 30
    warm = min(warm, n_requests // 5)
    srv = serve.Server(ctx, entries, hbm_budget=budget)
    srv_g = serve.Server(ctx, entries, hbm_budget=budget, graph=True)
    names = ["sphere", "terrain"]
    srv_g.run(serve.poisson_requests(20, 1e9, 40, names), "batched")
    srv.run(serve.poisson_requests(20, 1e9, 40, names), "batched")
    burst = serve.poisson_requests(max(40, n_requests // 3), 1e9, 41, names)
    sat = serve.summarize(srv_g.run(burst, "batched"))
    rate = sat["requests"] / sat["makespan_s"]
    points = []
    for i, load in enumerate(loads):
        trace = serve.poisson_requests(n_requests, load * rate, 42 + i, names)
        keep = lambda res: [r for r in res if r.req.rid >= warm]
        pt = {"offered_load": load, "rate_rps": round(load * rate, 1),
              "batched_graph": serve.summarize(keep(srv_g.run(trace, "batched"))),
              "batched": serve.summarize(keep(srv.run(trace, "batched"))),
              "single": serve.summarize(keep(srv.run(trace, "single")))}
        log("serving load %.1f: graph p50 %.2f p99 %.2f | eager p50 %.2f p99 %.2f | single p50 %.2f p99 %.2f ms" % (
            load, pt["batched_graph"]["p50_ms"], pt["batched_graph"]["p99_ms"], pt["batched"]["p50_ms"],
            pt["batched"]["p99_ms"], pt["single"]["p50_ms"], pt["single"]["p99_ms"]))
        points.append(pt)
    srv_g.close()
    ctx.free_scene(hs)
    return {"requests": n_requests, "warmup_requests": warm, "saturation_rps": round(rate, 1),
            "hbm_budget_bytes": budget, "resident_scene_bytes": int(srv.resident_bytes), "policy": srv.policy,
            "max_rays_per_step": srv.max_rays,
            "solo_rays_per_step": srv.solo_rays, "step_streams": srv.inflight_steps,
            "mix": "sphere64 + terrain1024 scenes, 256^2/720p/1080p/2048x1152, 1-5 rays per pixel, Poisson arrivals",
            "points": points}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--frames", type=int, default=60, help="animation cycle length")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="CPU oracle budget (0 disables)")
    ap.add_argument("--width", type=int, default=1920)
    ap.add_argument("--height", type=int, default=1080)
    ap.add_argument("--waves-per-block", type=int, default=0)
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--lds-cache-nodes", type=int, default=-1)
    ap.add_argument("--refill", type=int, default=-1)
    ap.add_argument("--claim-tiles", type=int, default=0)
    ap.add_argument("--serve-requests", type=int, default=1000,
                    help="requests per offered load in the served-latency runs (0 disables)")
    ap.add_argument("--serve-loads", default="0.3,0.6,0.9", help="offered loads, fractions of saturation")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner")
    ap.add_argument("--no-instances", action="store_true", help="skip the instanced-scene measurement")
    ap.add_argument("--no-ceilings", action="store_true", help="skip the gather / stream ceiling kernels")
    ap.add_argument("--no-c5", action="store_true", help="skip the depth-12 terrain measurement")
    ap.add_argument("--no-hit-buffer", action="store_true", help="skip the hit-buffer (frame-to-frame reuse) run")
    ap.add_argument("--c5-only", action="store_true",
                    help="run only the depth-12 terrain leg (for profiling) and print its JSON")
    ap.add_argument("--instances-only", action="store_true",
                    help="run only the instanced-scene leg (for profiling) and print its JSON")
    ap.add_argument("--no-camera", action="store_true", help="skip the camera-ray (in-kernel generation) run")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (reference for HBM byte counters)")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch
        nb = args.copy_calibration << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nb, "copies": 5}), flush=True)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (rays would shard across GPUs "
              "with the pool replicated on each); rerun with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1911_06001_amd import svo
    from svogen import scenes

    knobs = {}
    if args.waves_per_block:
        knobs["waves_per_block"] = args.waves_per_block
    if args.blocks_per_cu:
        knobs["blocks_per_cu"] = args.blocks_per_cu
    if args.lds_cache_nodes >= 0:
        knobs["lds_cache_nodes"] = args.lds_cache_nodes
    if args.refill >= 0:
        knobs["refill_lanes"] = args.refill
    if args.claim_tiles:
        knobs["claim_tiles"] = args.claim_tiles
    if args.c5_only:
        ctx = svo.Context(0)
        res, _, h5 = c5_throughput(ctx, args.steps, knobs=knobs or None)
        ctx.free_scene(h5)
        ctx.close()
        print(json.dumps({"c5_only": res}), flush=True)
        return
    if args.instances_only:
        ctx = svo.Context(0)
        res = instances_throughput(ctx, args.steps, knobs=knobs or None)
        ctx.close()
        print(json.dumps({"instances_only": res}), flush=True)
        return

    t0 = time.perf_counter()
    sc = scenes.fbm_terrain_d10(frames=args.frames)
    rays_np, _ = sc.rays(W=args.width, H=args.height)
    n = rays_np.shape[0]
    log("scene: %d nodes, %d slots, %d rays (%.1f s)" % (sc.nodes.shape[0], sc.n_slots, n, time.perf_counter() - t0))

    dev = torch.device("cuda:0")
    rays = torch.from_numpy(rays_np).to(dev)
    out_id = torch.empty(n, dtype=torch.int32, device=dev)
    out_inst = torch.empty(n, dtype=torch.int32, device=dev)
    out_t = torch.empty(n, dtype=torch.float32, device=dev)
    out_n = torch.empty((n, 3), dtype=torch.float32, device=dev)
    ctx = svo.Context(0)
    cfg = ctx.set_config(**knobs).as_dict()
    log("kernel config", cfg)
    anim = ctx.upload_scene(sc)
    stat = ctx.upload_scene(sc, static=True)
    xf = [sc.xform(f) for f in range(args.frames)]
    stream = torch.cuda.current_stream()
    tuned = None
    if not args.no_tune and not knobs:
        # the autotuner times candidate configurations on this workload's rays
        ctx.set_transforms(anim, xf[0], stream=stream)
        tuned = ctx.tune(anim, rays).as_dict()
        ctx.tune(stat, rays)
        log("tuned config", tuned)

    # step k shows animation frame (stride * k) mod frames, stride coprime
    # with the cycle: any number of steps samples the whole cycle evenly
    stride = next(s for s in range(7, 7 + args.frames + 1) if math.gcd(s, args.frames) == 1)

    def frame_of(k):
        return (stride * k) % args.frames

    def step_anim(k):
        ctx.set_transforms(anim, xf[frame_of(k)], stream=stream)
        ctx.trace_into(anim, rays, out_id, out_t, out_inst, out_n, stream=stream)

    def step_static(k):
        ctx.trace_into(stat, rays, out_id, out_t, out_inst, out_n, stream=stream)

    def timed(step, K):
        # the wall time of K plain steps (a timing event around every trace
        # adds about 7 us per step), then the same K steps again with HIP
        # events around each trace for the kernel times
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for k in range(K):
            step(k)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
        for k in range(K):
            if step is step_anim:
                ctx.set_transforms(anim, xf[frame_of(k)], stream=stream)
                evs[k][0].record(stream)
                ctx.trace_into(anim, rays, out_id, out_t, out_inst, out_n, stream=stream)
                evs[k][1].record(stream)
            else:
                evs[k][0].record(stream)
                ctx.trace_into(stat, rays, out_id, out_t, out_inst, out_n, stream=stream)
                evs[k][1].record(stream)
        torch.cuda.synchronize()
        kms = [a.elapsed_time(b) for a, b in evs]
        return wall, kms

    for k in range(args.warmup):
        step_anim(k)
        step_static(k)
    torch.cuda.synchronize()
    log("warmup done")

    K = args.steps
    wall_a, kms_a = timed(step_anim, K)
    log("animated: %.3f ms/step wall, kernel mean %.3f ms" % (wall_a / K * 1e3, float(np.mean(kms_a))))
    wall_s, kms_s = timed(step_static, K)
    log("static: %.3f ms/step wall, kernel mean %.3f ms" % (wall_s / K * 1e3, float(np.mean(kms_s))))

    # The same frames with the primary rays made inside the trace kernel
    # from the camera (svo_trace_camera: no ray buffer read).  Reported
    # beside the headline, which reads its rays.
    camera_run = None
    c = sc.camera
    cam = svo.make_camera(c["eye"], c["target"], c["up"], c["fov"], args.width, args.height)
    cam_hits = svo.Hits(out_id, out_inst, out_t, out_n)
    n_cam_steps = 0 if args.no_camera else K
    if n_cam_steps:
        for k in range(3):
            ctx.set_transforms(anim, xf[frame_of(k)], stream=stream)
            ctx.trace_camera(anim, cam, out=cam_hits, stream=stream)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for k in range(K):
            ctx.set_transforms(anim, xf[frame_of(k)], stream=stream)
            ctx.trace_camera(anim, cam, out=cam_hits, stream=stream)
        torch.cuda.synchronize()
        cwall = time.perf_counter() - w0
        cevs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
        for k in range(K):
            ctx.set_transforms(anim, xf[frame_of(k)], stream=stream)
            cevs[k][0].record(stream)
            ctx.trace_camera(anim, cam, out=cam_hits, stream=stream)
            cevs[k][1].record(stream)
        torch.cuda.synchronize()
        ckms = float(np.mean([x.elapsed_time(y) for x, y in cevs]))
        camera_run = {"value": round(n * K / cwall / 1e6, 3), "unit": "Mrays/s",
                      "ms_per_step": round(cwall / K * 1e3, 4), "kernel_ms": round(ckms, 4),
                      "note": "same frames; rays made in the trace kernel from a 96-byte camera record "
                              "(svo_trace_camera)"}
        log("camera rays: %.3f ms/step wall, kernel %.3f ms" % (cwall / K * 1e3, ckms))

    # Two frames in flight: frame k traces on stream k mod 2 into its own
    # outputs, so the next frame's launch fills the CUs that this one frees
    # while its last tiles drain.  Reported beside the sequential figures
    # above, which stay the headline.
    pipe_streams = [torch.cuda.Stream(device=dev), torch.cuda.Stream(device=dev)]
    pipe_out = [(out_id, out_t, out_inst, out_n),
                (torch.empty_like(out_id), torch.empty_like(out_t), torch.empty_like(out_inst), torch.empty_like(out_n))]

    def pipelined(handle, animated, K):
        torch.cuda.synchronize()
        for st in pipe_streams:
            st.wait_stream(stream)
        w0 = time.perf_counter()
        for k in range(K):
            st = pipe_streams[k % 2]
            if animated:
                ctx.set_transforms(handle, xf[frame_of(k)], stream=st)
            o = pipe_out[k % 2]
            ctx.trace_into(handle, rays, o[0], o[1], o[2], o[3], stream=st)
        torch.cuda.synchronize()
        return time.perf_counter() - w0

    pipelined(anim, True, min(K, 10))
    pipelined(stat, False, min(K, 10))
    pwall_a = pipelined(anim, True, K)
    pwall_s = pipelined(stat, False, K)
    pipe = {"frames_in_flight": 2, "value": round(n * K / pwall_a / 1e6, 3), "unit": "Mrays/s",
            "ms_per_step": round(pwall_a / K * 1e3, 4), "static_value": round(n * K / pwall_s / 1e6, 3),
            "static_ms_per_step": round(pwall_s / K * 1e3, 4),
            "note": "same frames and rays; frame k on stream k mod 2 with its own outputs"}
    log("two frames in flight: animated %.3f ms/step (%.0f Mrays/s), static %.3f ms/step" % (
        pwall_a / K * 1e3, pipe["value"], pwall_s / K * 1e3))

    # the paper's hit buffer (Sec. 4.3): each frame updates the previous
    # frame's hits, retracing only rays a moved subtree can reach
    hb = None
    if not args.no_hit_buffer:
        hb_hits = ctx.trace(anim, rays)
        cnt = torch.zeros(1, dtype=torch.int64, device=dev)
        torch.cuda.synchronize()
        # frames follow one another across both passes: each trace updates
        # the previous frame's hits
        w0 = time.perf_counter()
        for k in range(K):
            ctx.set_transforms(anim, xf[(k + 1) % args.frames], stream=stream)
            ctx.trace_reuse(anim, rays, hb_hits, retraced=cnt, stream=stream)
        torch.cuda.synchronize()
        hwall = time.perf_counter() - w0
        hev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
        for k in range(K):
            ctx.set_transforms(anim, xf[(K + k + 1) % args.frames], stream=stream)
            hev[k][0].record(stream)
            ctx.trace_reuse(anim, rays, hb_hits, retraced=cnt, stream=stream)
            hev[k][1].record(stream)
        torch.cuda.synchronize()
        hk = float(np.mean([x.elapsed_time(y) for x, y in hev]))
        hb = {"value": round(n * K / hwall / 1e6, 3), "unit": "Mrays/s", "ms_per_step": round(hwall / K * 1e3, 4),
              "kernel_ms": round(hk, 4), "retraced_fraction": round(int(cnt.item()) / (2 * n * K), 4),
              "note": "svo_trace_rays_reuse: results identical to full traces (tested); rays whose previous hit is "
                      "in the static world and that no moved subtree can reach keep it"}
        log("hit buffer: %.3f ms/step wall, kernel %.3f ms, %.1f%% of rays retraced" % (
            hwall / K * 1e3, hk, 100 * hb["retraced_fraction"]))

    value = n * K / wall_a / 1e6
    static_value = n * K / wall_s / 1e6
    kmean_a = float(np.mean(kms_a)) * 1e-3

    cpu = None
    bytes_per_ray = None
    if args.cpu_seconds > 0:
        log("oracle baseline on host cores (budget %.0f s)" % args.cpu_seconds)
        cb = cpu_baseline(sc, rays_np, args.frames, args.cpu_seconds)
        bytes_per_ray = cb["bytes_per_ray"]
        cpu = {"value": round(cb["rays"] / cb["seconds"] / 1e6, 4), "unit": "Mrays/s", "cores": cb["threads"],
               "kind": "oracle", "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
               "sample": "animated terrain1024 frames %d..%d, all %d rays each (%d rays, %.1f s)" % (
                   cb["frames"][0], cb["frames"][-1], n, cb["rays"], cb["seconds"])}
    roof = None
    if bytes_per_ray is not None:
        achieved = bytes_per_ray * n / kmean_a / 1e9
        pmc = read_counters()
        traffic = pmc.get("hbm_bytes_per_launch")
        roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                "bytes_per_ray": round(bytes_per_ray, 2), "rays_per_launch": n,
                "kernel_ms": round(kmean_a * 1e3, 4),
                "n_node_mean": round(cb["n_node_mean"], 2), "n_node_p99": round(cb["n_node_p99"], 1),
                "n_node_upper_mean": round(cb["n_node_hi_mean"], 2),
                "n_frame_mean": round(cb["n_frame_mean"], 3)}
        if "valu_wave_insts_per_launch" in pmc:
            # instruction issue beside the byte roofline: the same launch's VALU
            # wave instructions (SQ_INSTS_VALU) over its live kernel time
            vi = pmc["valu_wave_insts_per_launch"]
            roof["valu_issue"] = {"wave_insts_per_launch": vi, "achieved_G_per_s": round(vi / kmean_a / 1e9, 1),
                                  "peak_G_per_s": VALU_ISSUE_PEAK / 1e9,
                                  "frac": round(vi / kmean_a / VALU_ISSUE_PEAK, 4),
                                  "lane_activity": pmc.get("valu_lane_activity")}

    ceilings = None
    if not args.no_ceilings:
        from paper_1911_06001_amd import ceiling
        kc = tuned or cfg
        n_cu = torch.cuda.get_device_properties(dev).multi_processor_count
        ceilings = ceiling.measure(int(sc.nodes.nbytes), n_cu * kc["blocks_per_cu"], 64 * kc["waves_per_block"])
        rep = replay_ceiling(ctx, anim, sc, xf[0], rays, kc, n_cu)
        ceilings["replay"] = rep
        log("ceilings", ceilings)
        if roof is not None:
            # the replay ceiling: the same algorithmic bytes over the replay's time
            ceilings["replay_GBps"] = round(bytes_per_ray * n / (rep["replay_ms"] * 1e-3) / 1e9, 1)
            ceilings["frac_replay"] = round(rep["replay_ms"] / rep["trace_ms_same_frame"], 4)
            for k in ("gather_independent_GBps", "gather_dependent_GBps", "stream_pool_GBps", "stream_hbm_GBps"):
                ceilings["frac_" + k[:-5]] = round(roof["achieved"] / ceilings[k], 4)
            roof["target_ceiling"] = "replay"
            roof["frac_of_target_ceiling"] = ceilings["frac_replay"]

    instances = None
    if not args.no_instances:
        instances = instances_throughput(ctx, max(5, K // 6))
    c5 = None
    c5_serving = None
    if not args.no_c5:
        c5, c5_scene, c5_h = c5_throughput(ctx, max(5, K // 6))
        if args.serve_requests > 0:
            c5_serving = serve_c5(ctx, c5_scene, c5_h, max(40, args.serve_requests // 5), 0.6)
        ctx.free_scene(c5_h)
        del c5_scene
    serving = None
    if args.serve_requests > 0:
        serving = serve_latency(ctx, sc, anim, args.serve_requests, [float(x) for x in args.serve_loads.split(",")])

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(wall_a / K * 1e3, 4),
        "timing": "wall clock over K steps (transform update + trace) with no timing events; kernel times from "
                  "HIP events in a second pass over K steps",
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "terrain1024: depth-10 (1024^3) fBm heightfield SVO, 8 level-3 subtrees animated per "
                               "frame (rotation + anisotropic scale 0.5-2), %dx%d primary rays, %d-frame cycle"
                               % (args.width, args.height, args.frames),
                   "rays_per_step": n, "nodes": int(sc.nodes.shape[0]), "slots": sc.n_slots,
                   "kernel": tuned or cfg},
        "static": {"value": round(static_value, 3), "unit": "Mrays/s", "ms_per_step": round(wall_s / K * 1e3, 4),
                   "kernel_ms": round(float(np.mean(kms_s)), 4)},
        "animated_over_static_time": round(wall_a / wall_s, 4),
        "animated_over_static_kernel_time": round(float(np.mean(kms_a)) / float(np.mean(kms_s)), 4),
        "two_frames_in_flight": pipe,
        "camera_rays": camera_run,
        "hit_buffer": hb,
        "roofline": roof,
        "ceilings": ceilings,
        "cpu_baseline": cpu,
        "paper_context": PAPER_CONTEXT,
        "serving": serving,
        "instances": instances,
        "terrain4096": c5,
        "serving_terrain4096_instances": c5_serving,
    }
    ctx.free_scene(anim)
    ctx.free_scene(stat)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
