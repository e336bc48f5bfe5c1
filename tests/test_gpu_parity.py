"""Device path vs the FP64 oracle on identical seeded inputs (needs the GPU).

Every call goes through the C ABI (libsvo.so via its ctypes binding).
"""
import sys

import numpy as np
import pytest

import oracle
import parity
from svogen import octree as ot
from svogen import scenes as S
from svogen import xforms as xf

pytestmark = pytest.mark.gpu
NONE = 0xFFFFFFFF


def _say(*a):
    print("[gpu-parity]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def ctx(torch_dev):
    from paper_1911_06001_amd import svo
    c = svo.Context(0)
    yield c
    c.close()


def _trace(ctx, torch, scene_h, rays):
    r = torch.from_numpy(np.ascontiguousarray(rays, np.float32)).cuda()
    h = ctx.trace(scene_h, r)
    torch.cuda.synchronize()
    return parity.to_numpy(h)


def _check_scene(ctx, torch, sc, rays, frame=0, static=False, fwd=None, max_rate=None, label=""):
    _say("case", label or sc.name, "rays", rays.shape[0], "frame", frame, "static", static)
    h = ctx.upload_scene(sc, static=static)
    try:
        if not static and sc.n_slots:
            ctx.set_transforms(h, sc.xform(frame) if fwd is None else fwd)
        g = _trace(ctx, torch, h, rays)
    finally:
        ctx.free_scene(h)
    ref = oracle.trace_scene(sc, rays, frame=frame, static=static, fwd=fwd, margin=True)
    st = parity.compare(g, ref, ref.margin, rays)
    _say(label or sc.name, st)
    parity.assert_parity(st, max_rate)
    return st


def test_sphere64_full(ctx, torch_dev):
    sc = S.noisy_sphere_d6()
    rays, _ = sc.rays()
    st = _check_scene(ctx, torch_dev, sc, rays, max_rate=1e-4, label="sphere64")
    assert st["hits"] > 2000


def test_sphere64_static_and_identity(ctx, torch_dev):
    sc = S.noisy_sphere_d6()
    rays, _ = sc.rays()
    _check_scene(ctx, torch_dev, sc, rays, static=True, max_rate=1e-4, label="sphere64-static")
    ident = xf.to_f32(xf.identity()).reshape(1, 12)
    _check_scene(ctx, torch_dev, sc, rays, fwd=ident, max_rate=1e-4, label="sphere64-identity")


def test_sphere64_rows_order_and_ragged(ctx, torch_dev):
    sc = S.noisy_sphere_d6()
    rays, _ = sc.rays(order="rows")
    for n in (1, 63, 64, 65, 1000, 4097):
        _check_scene(ctx, torch_dev, sc, rays[:n], label="sphere64-ragged-%d" % n)


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5, 6])
def test_tiny_nested(ctx, torch_dev, seed):
    sc = S.tiny_scene(seed, K=5 if seed % 2 else 4, n_slots=4, nested=True, translate=0.3)
    rays = S.random_rays(seed, 3000, 0.0, sc.root_size)
    _check_scene(ctx, torch_dev, sc, rays, label="tiny-%d" % seed)


def test_random_scenes_stress(ctx, torch_dev):
    """Many seeded random scenes: depth 4-6, 1-8 slots, nested or not,
    shrinking to growing scales and translations (contained, leaving and
    overlapping slots), camera-like and inside rays, some with a short tmax;
    each against the oracle.  Rare paths (in-place frames at several depths,
    candidates crossing each other, ties) get many chances to show up."""
    rng = np.random.default_rng(2024)
    cases = 0
    for seed in range(100, 116):
        K = int(rng.integers(4, 7))
        slots = int(rng.integers(1, 9))
        nested = bool(rng.integers(0, 2))
        lo_s, hi_s = sorted(rng.uniform(0.3, 2.2, 2))
        try:
            sc = S.tiny_scene(seed, K=K, n_slots=slots, nested=nested, scale_range=(lo_s, hi_s),
                              translate=float(rng.uniform(0.0, 0.5)))
        except ValueError:
            continue  # an empty random scene
        rays = np.concatenate([S.random_rays(seed, 2500, 0.0, sc.root_size),
                               S.random_rays(seed + 1000, 800, 0.0, sc.root_size, inside_frac=1.0)])
        short = np.arange(rays.shape[0]) % 5 == 0
        rays[short, 7] = np.float32(0.3 * sc.root_size)
        _check_scene(ctx, torch_dev, sc, rays, label="stress-%d K%d s%d %s" % (seed, K, slots,
                                                                              "nested" if nested else "flat"))
        cases += 1
    assert cases >= 12


def test_axis_aligned_and_inside(ctx, torch_dev):
    sc = S.tiny_scene(5, K=4, n_slots=2, nested=False, rotate=False, scale_range=(1.0, 1.0), translate=0.4)
    rng = np.random.default_rng(3)
    rays = []
    for k in range(2000):
        o = rng.uniform(-4, 20, 3)
        d = np.zeros(3)
        d[k % 3] = 1.0 if k % 2 else -1.0
        if k % 5 == 0:
            d[(k + 1) % 3] = 0.5
        rays.append([*o, 0.0, *(d / np.linalg.norm(d)), np.inf])
    _check_scene(ctx, torch_dev, sc, np.array(rays, np.float32), label="axis-aligned")


def test_terrain1024_reduced_frames(ctx, torch_dev):
    sc = S.fbm_terrain_d10()
    rays, _ = sc.rays(W=320, H=180)
    for f in (0, 17, 45):
        _check_scene(ctx, torch_dev, sc, rays, frame=f, max_rate=1e-4, label="terrain1024-320x180-f%d" % f)
    _check_scene(ctx, torch_dev, sc, rays, static=True, max_rate=1e-4, label="terrain1024-320x180-static")


def test_terrain1024_full_resolution_sampled(ctx, torch_dev):
    """1920x1080 in the benchmark's launch (the configuration the autotuner
    picks for these rays, as the benchmark does): every 17th ray plus one
    block of 4096 consecutive rays are checked against the oracle one by one,
    and the default configuration gives the same results bit for bit."""
    sc = S.fbm_terrain_d10()
    rays, pix = sc.rays()
    n = rays.shape[0]
    idx = np.unique(np.concatenate([np.arange(0, n, 17), np.arange(400 * 64, 400 * 64 + 4096)]))
    h = ctx.upload_scene(sc)
    try:
        ctx.set_transforms(h, sc.xform(30))
        g0 = _trace(ctx, torch_dev, h, rays)
        cfg = ctx.tune(h, torch_dev.from_numpy(rays).cuda())
        _say("tuned", cfg.as_dict())
        g = _trace(ctx, torch_dev, h, rays)
    finally:
        ctx.free_scene(h)
    for a, b in zip(g0, g):
        assert np.array_equal(a, b)
    ref = oracle.trace_scene(sc, rays[idx], frame=30, margin=True)
    st = parity.compare(tuple(a[idx] for a in g), ref, ref.margin, rays[idx])
    _say("terrain1024-1080p-sampled", st)
    parity.assert_parity(st, 1e-4)


def test_far_pointers(ctx, torch_dev):
    sc = S.tiny_scene(6, K=5, n_slots=3, nested=True)
    rays = S.random_rays(5, 2000, 0.0, sc.root_size)
    far = ot.force_far(sc.nodes, 2)
    h = ctx.upload(far, sc.root, sc.root_min, sc.root_size, sc.max_depth, sc.slot_child, sc.slot_cell)
    try:
        ctx.set_transforms(h, sc.xform(0))
        g = _trace(ctx, torch_dev, h, rays)
    finally:
        ctx.free_scene(h)
    ref = oracle.trace(far, sc.root, sc.root_min, sc.root_size, sc.slot_child, sc.slot_cell, sc.xform(0), rays,
                       margin=True)
    parity.assert_parity(parity.compare(g, ref, ref.margin, rays))


def test_degenerate_rays_and_worlds(ctx, torch_dev):
    torch = torch_dev
    sc = S.tiny_scene(2, K=4, n_slots=2, nested=False)
    bad = np.array([
        [np.nan, 1, 1, 0, 1, 0, 0, np.inf],
        [1, 1, 1, 0, 0, 0, 0, np.inf],          # zero direction
        [-3, 5, 5, 4, 1, 0, 0, 3],              # tmin > tmax
        [-3, 5, 5, 0, np.inf, 0, 0, np.inf],
        [-3, 5, 5, np.inf, 1, 0, 0, np.inf],
        [5, 5, 5, 0, 1, 0, 0, np.nan],
    ], np.float32)
    h = ctx.upload_scene(sc)
    try:
        g = _trace(ctx, torch, h, bad)
    finally:
        ctx.free_scene(h)
    assert np.all(g[0] == NONE) and np.all(np.isinf(g[2]))
    ref = oracle.trace_scene(sc, bad)
    assert np.all(ref.id == NONE)
    # empty world and a world that is one solid leaf
    rays = S.random_rays(9, 500, 0.0, 16.0)
    h = ctx.upload(np.zeros(0, np.uint64), NONE, (0, 0, 0), 16.0, 4, np.zeros(0, np.uint32), np.zeros((0, 4)))
    try:
        g = _trace(ctx, torch, h, rays)
    finally:
        ctx.free_scene(h)
    assert np.all(g[0] == NONE)
    leaf = np.array([np.uint64(0xFF0000FF) << np.uint64(32)], np.uint64)
    h = ctx.upload(leaf, 0, (0, 0, 0), 16.0, 4, np.zeros(0, np.uint32), np.zeros((0, 4)))
    try:
        g = _trace(ctx, torch, h, rays)
    finally:
        ctx.free_scene(h)
    ref = oracle.trace(leaf, 0, np.zeros(3), 16.0, np.zeros(0, np.uint32), np.zeros((0, 4)), np.zeros((0, 12)), rays,
                       margin=True)
    parity.assert_parity(parity.compare(g, ref, ref.margin, rays))


def test_zero_rays_and_repeated_launches(ctx, torch_dev):
    torch = torch_dev
    sc = S.noisy_sphere_d6()
    rays, _ = sc.rays()
    h = ctx.upload_scene(sc)
    try:
        ctx.set_transforms(h, sc.xform(0))
        r = torch.from_numpy(rays).cuda()
        z = torch.empty(0, dtype=torch.int32, device="cuda")
        zt = torch.empty(0, dtype=torch.float32, device="cuda")
        ctx.trace_into(h, r[:0], z, zt)
        first = ctx.trace(h, r)
        s2 = torch.cuda.Stream()
        outs = []
        for k in range(5):
            outs.append(ctx.trace(h, r, stream=s2 if k % 2 else None))
            torch.cuda.synchronize()
        for o in outs:
            assert torch.equal(o.id, first.id) and torch.equal(o.t, first.t)
    finally:
        ctx.free_scene(h)


def test_transform_updates_are_stream_ordered(ctx, torch_dev):
    torch = torch_dev
    sc = S.fbm_terrain_d10()
    rays, _ = sc.rays(W=160, H=90)
    r = torch.from_numpy(rays).cuda()
    h = ctx.upload_scene(sc)
    try:
        res = []
        for f in (3, 4, 5):
            ctx.set_transforms(h, sc.xform(f))
            res.append(ctx.trace(h, r))     # enqueued back to back, no host sync
        torch.cuda.synchronize()
    finally:
        ctx.free_scene(h)
    for f, hh in zip((3, 4, 5), res):
        ref = oracle.trace_scene(sc, rays, frame=f, margin=True)
        parity.assert_parity(parity.compare(parity.to_numpy(hh), ref, ref.margin, rays))


def test_small_scene_traces_keep_their_transforms_on_any_stream(ctx, torch_dev):
    """A scene of at most 8 slots carries its frame table in the arguments of
    the launches after a transform update: traces on two streams, each
    enqueued after a different update and with no host wait, see their own
    frame."""
    torch = torch_dev
    sc = S.fbm_terrain_d10()
    rays, _ = sc.rays(W=160, H=90)
    r = torch.from_numpy(rays).cuda()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    h = ctx.upload_scene(sc)
    frames = (3, 17, 29, 44)
    try:
        torch.cuda.synchronize()
        res = []
        for i, f in enumerate(frames):
            ctx.set_transforms(h, sc.xform(f))
            res.append(ctx.trace(h, r, stream=streams[i % 2]))
        torch.cuda.synchronize()
    finally:
        ctx.free_scene(h)
    for f, hh in zip(frames, res):
        ref = oracle.trace_scene(sc, rays, frame=f, margin=True)
        parity.assert_parity(parity.compare(parity.to_numpy(hh), ref, ref.margin, rays))


def test_large_scene_table_updates_wait_for_traces_on_other_streams(ctx, torch_dev):
    """A scene above 10 slots keeps two device tables.  A long trace on one
    stream reads the current table; two transform updates on another stream
    then rewrite first the other table and then the one that trace reads:
    the second copy waits for the trace on the device, so the trace still
    sees the transforms it was enqueued with (checked bit for bit against a
    trace of the same transforms alone), and the traces after the updates
    see theirs."""
    torch = torch_dev
    sc = S.instanced_scene()
    rays, _ = sc.rays()                       # 1080p: a launch long enough to overlap the copies
    r = torch.from_numpy(rays).cuda()
    h = ctx.upload_scene(sc)
    try:
        assert ctx.scene_stats(h).n_candidates > 16
        f0, f1, f2 = sc.xform(0), sc.xform(0).copy(), sc.xform(0).copy()
        f1[:, 3] += 1.5                        # translations only: the same slots stay valid
        f2[:, 7] -= 2.0
        refs = []
        for f in (f0, f1, f2):
            ctx.set_transforms(h, f)
            refs.append(ctx.trace(h, r))
        torch.cuda.synchronize()
        a, b = torch.cuda.Stream(), torch.cuda.Stream()
        ctx.set_transforms(h, f0, stream=a)
        a.synchronize()
        long_trace = ctx.trace(h, r, stream=a)
        ctx.set_transforms(h, f1, stream=b)    # the other table
        ctx.set_transforms(h, f2, stream=b)    # the table long_trace reads: waits for it
        after = ctx.trace(h, r, stream=b)
        torch.cuda.synchronize()
        for k in ("id", "inst", "t", "normal"):
            assert torch.equal(getattr(long_trace, k), getattr(refs[0], k)), k
            assert torch.equal(getattr(after, k), getattr(refs[2], k)), k
    finally:
        ctx.free_scene(h)


def test_rejected_transforms_change_nothing(ctx, torch_dev):
    """A call rejected for one slot's map (singular) stores none of its maps:
    a later call that uploads the table again still traces the old ones."""
    from paper_1911_06001_amd import svo
    sc = S.tiny_scene(7, K=5, n_slots=2, nested=False)
    fwd0 = sc.xform(0)
    bad = fwd0.copy()
    bad[0, 3] += np.float32(0.25 * sc.root_size)    # a valid, different map for slot 0 ...
    bad[1, [0, 1, 2, 4, 5, 6, 8, 9, 10]] = 0.0      # ... and a singular one for slot 1
    rays = S.random_rays(7, 3000, 0.0, sc.root_size)
    ref = oracle.trace_scene(sc, rays, fwd=fwd0, margin=True)
    moved = fwd0.copy()
    moved[0] = bad[0]
    assert np.count_nonzero(oracle.trace_scene(sc, rays, fwd=moved).id != ref.id) > 0
    h = ctx.upload_scene(sc)
    try:
        ctx.set_transforms(h, fwd0)
        with pytest.raises(svo.SvoError):
            ctx.set_transforms(h, bad)
        ctx.set_transforms(h, fwd0[1:], first=1)   # packs and uploads every slot's map
        g = _trace(ctx, torch_dev, h, rays)
    finally:
        ctx.free_scene(h)
    parity.assert_parity(parity.compare(g, ref, ref.margin, rays))


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_inline_contained_frames(ctx, torch_dev, seed):
    """Shrunk, rotated subtrees stay inside their static cells: the walk
    enters them in place (nested chains included), no candidate frames."""
    sc = S.tiny_scene(seed, K=5, n_slots=4, nested=True, scale_range=(0.3, 0.55))
    rays = S.random_rays(seed + 3, 4000, 0.0, sc.root_size)
    h = ctx.upload_scene(sc)
    try:
        ctx.set_transforms(h, sc.xform(0))
        st = ctx.scene_stats(h)
        _say("inline stats", dict(n_inline=st.n_inline, n_cand=st.n_candidates, nest=st.nest_levels,
                                  stack=st.stack_levels))
        assert st.n_inline == sc.n_slots and st.n_candidates == 0 and st.nest_levels >= 2
        g = _trace(ctx, torch_dev, h, rays)
    finally:
        ctx.free_scene(h)
    ref = oracle.trace_scene(sc, rays, margin=True)
    stt = parity.compare(g, ref, ref.margin, rays)
    if stt["worst_t"]:
        stt["worst_t"]["ray_data"] = rays[stt["worst_t"]["ray"]].tolist()
    _say("inline-%d" % seed, stt)
    parity.assert_parity(stt)
    assert (ref.inst[ref.id != NONE] != NONE).sum() > 10


def test_inline_and_candidates_mixed(ctx, torch_dev):
    """Per slot: contained ones in place, overflowing ones as candidates."""
    sc = S.tiny_scene(7, K=5, n_slots=4, nested=True, scale_range=(0.3, 1.6), translate=0.2)
    rays = S.random_rays(70, 4000, 0.0, sc.root_size)
    h = ctx.upload_scene(sc)
    try:
        seen_inline = seen_cand = 0
        for k in range(6):
            fwd = sc.xform(0).copy()
            # shrink a different subset of slots each time
            for s in range(sc.n_slots):
                if (k >> (s % 3)) & 1:
                    A = fwd[s].reshape(3, 4).astype(np.float64)
                    c = sc.slot_cell[s, :3].astype(np.float64) + sc.slot_cell[s, 3] / 2
                    L = A[:, :3] * (0.3 / np.abs(np.linalg.det(A[:, :3])) ** (1 / 3))
                    fwd[s] = xf.to_f32(xf.about_pivot(L, c)).reshape(12)
            ctx.set_transforms(h, fwd)
            st = ctx.scene_stats(h)
            seen_inline += st.n_inline
            seen_cand += st.n_candidates
            g = _trace(ctx, torch_dev, h, rays)
            ref = oracle.trace_scene(sc, rays, fwd=fwd, margin=True)
            stt = parity.compare(g, ref, ref.margin, rays)
            _say("mixed-%d" % k, dict(n_inline=st.n_inline, n_cand=st.n_candidates), stt)
            parity.assert_parity(stt)
    finally:
        ctx.free_scene(h)
    assert seen_inline > 0 and seen_cand > 0


def _outs(torch, n):
    return dict(out_id=torch.empty(n, dtype=torch.int32, device="cuda"),
                out_inst=torch.empty(n, dtype=torch.int32, device="cuda"),
                out_t=torch.empty(n, dtype=torch.float32, device="cuda"),
                out_normal=torch.empty((n, 3), dtype=torch.float32, device="cuda"))


def test_batch_equals_alone(ctx, torch_dev):
    """Rays of several requests, scenes and animation frames in one launch:
    every job's result is bit-identical to tracing it alone, and to a batch
    of that job alone."""
    torch = torch_dev
    sph = S.noisy_sphere_d6()
    ter = S.fbm_terrain_d10()
    tin = S.tiny_scene(3, K=5, n_slots=4, nested=True, scale_range=(0.3, 1.5))
    hs = {k: ctx.upload_scene(v) for k, v in (("sph", sph), ("ter", ter), ("tin", tin))}
    try:
        ctx.set_transforms(hs["sph"], sph.xform(0))
        ctx.set_transforms(hs["tin"], tin.xform(0))
        ctx.set_transforms(hs["ter"], ter.xform(5))
        specs = [("sph", sph.rays(W=100, H=77)[0], None),
                 ("ter", ter.rays(W=160, H=90)[0], None),            # scene's current transforms (frame 5)
                 ("ter", ter.rays(W=123, H=45)[0], ter.xform(33)),    # a different animation frame
                 ("tin", S.random_rays(4, 3001, 0.0, 32.0), None),
                 ("sph", sph.rays(W=8, H=1)[0], None)]
        jobs = []
        for name, rays, fwd in specs:
            r = torch.from_numpy(rays).cuda()
            j = dict(scene=hs[name], rays=r, fwd=fwd, **_outs(torch, rays.shape[0]))
            jobs.append(j)
        ctx.trace_batch(jobs)
        torch.cuda.synchronize()
        for (name, rays, fwd), j in zip(specs, jobs):
            if fwd is not None:
                ctx.set_transforms(hs[name], fwd)
            alone = ctx.trace(hs[name], j["rays"])
            torch.cuda.synchronize()
            if fwd is not None:
                ctx.set_transforms(hs[name], ter.xform(5))
            assert torch.equal(alone.id, j["out_id"]), name
            assert torch.equal(alone.inst, j["out_inst"]), name
            assert torch.equal(alone.t, j["out_t"]), name
            assert torch.equal(alone.normal, j["out_normal"]), name
        # a batch of one job (its own transforms) runs the single-job kernel:
        # the same results as that job in the larger batch
        one = [dict(scene=hs["ter"], rays=jobs[2]["rays"], fwd=specs[2][2], **_outs(torch, specs[2][1].shape[0]))]
        ctx.trace_batch(one)
        torch.cuda.synchronize()
        for k in ("out_id", "out_inst", "out_t", "out_normal"):
            assert torch.equal(one[0][k], jobs[2][k]), k
        # and against the oracle for the job with its own transforms
        ref = oracle.trace_scene(ter, specs[2][1], fwd=specs[2][2], margin=True)
        g = (jobs[2]["out_id"].cpu().numpy().view(np.uint32), jobs[2]["out_inst"].cpu().numpy().view(np.uint32),
             jobs[2]["out_t"].cpu().numpy().astype(np.float64), jobs[2]["out_normal"].cpu().numpy().astype(np.float64))
        parity.assert_parity(parity.compare(g, ref, ref.margin, specs[2][1]))
    finally:
        for h in hs.values():
            ctx.free_scene(h)


def test_results_independent_of_kernel_config(ctx, torch_dev):
    torch = torch_dev
    sc = S.fbm_terrain_d10()
    rays, _ = sc.rays(W=320, H=180)
    r = torch.from_numpy(rays).cuda()
    h = ctx.upload_scene(sc)
    base_cfg = ctx.get_config().as_dict()
    try:
        ctx.set_transforms(h, sc.xform(9))
        ref = ctx.trace(h, r)
        torch.cuda.synchronize()
        for cfg in (dict(waves_per_block=1, blocks_per_cu=1, lds_cache_nodes=0, refill_lanes=0),
                    dict(waves_per_block=8, blocks_per_cu=2, lds_cache_nodes=4096, refill_lanes=16),
                    dict(waves_per_block=2, blocks_per_cu=8, lds_cache_nodes=512, refill_lanes=1)):
            ctx.set_config(**cfg)
            o = ctx.trace(h, r)
            torch.cuda.synchronize()
            assert torch.equal(o.id, ref.id) and torch.equal(o.t, ref.t) and torch.equal(o.normal, ref.normal), cfg
    finally:
        ctx.set_config(**base_cfg)
        ctx.free_scene(h)


def test_results_independent_of_candidate_ordering(ctx, torch_dev):
    """sorted_candidates picks the per-lane sorted entry table or the box
    hierarchy for a job's candidate frames: both give bit-identical results,
    on a scene of 64 candidates (hierarchy by default, the sorted table up to
    64) and one of at most 12 (the sorted table by default, the hierarchy
    below its count)."""
    torch = torch_dev
    base_cfg = ctx.get_config().as_dict()
    cases = [(S.instanced_scene(), 0, None, 64),
             (S.tiny_scene(5, K=6, n_slots=12, nested=False, scale_range=(0.8, 1.6)), 3, "random", 1)]
    for sc, frame, kind, other in cases:
        rays = S.random_rays(4, 20000, 0.0, 64.0) if kind == "random" else sc.rays(W=320, H=180)[0]
        r = torch.from_numpy(rays).cuda()
        h = ctx.upload_scene(sc)
        try:
            ctx.set_transforms(h, sc.xform(frame))
            st = ctx.scene_stats(h)
            assert st.n_candidates > 1, st.n_candidates
            ctx.set_config(**base_cfg)
            ref = ctx.trace(h, r)
            ctx.set_config(sorted_candidates=other)
            o = ctx.trace(h, r)
            torch.cuda.synchronize()
            for k in ("id", "inst", "t", "normal"):
                assert torch.equal(getattr(o, k), getattr(ref, k)), (sc.name, k)
        finally:
            ctx.set_config(**base_cfg)
            ctx.free_scene(h)


def test_step_limit(ctx, torch_dev):
    """A ray whose walk needs more advances than step_limit reports
    SVO_STEP_LIMIT (no slot, t = +inf, zero normal); every other ray is
    exactly the unlimited result, and a larger limit caps a subset of the
    rays a smaller one caps (the walk is the same up to the cap)."""
    from paper_1911_06001_amd import svo
    torch = torch_dev
    cases = [(S.fbm_terrain_d10(), 9), (S.tiny_scene(3, K=6, n_slots=4, nested=True, scale_range=(0.6, 1.0)), 2)]
    base_cfg = ctx.get_config().as_dict()
    for sc, frame in cases:
        if sc.name == "terrain1024":
            rays, _ = sc.rays(W=320, H=180)
        else:
            rays = S.random_rays(3, 20000, 0.0, 64.0)
        r = torch.from_numpy(rays).cuda()
        h = ctx.upload_scene(sc)
        try:
            ctx.set_transforms(h, sc.xform(frame))
            full = ctx.trace(h, r)
            prev = None
            for limit in (2, 8, 32):
                ctx.set_config(step_limit=limit)
                o = ctx.trace(h, r)
                torch.cuda.synchronize()
                cap = o.id == (svo.STEP_LIMIT - (1 << 32))     # int32 view of the id
                keep = ~cap
                _say(sc.name, "step limit", limit, "capped", int(cap.sum()), "of", rays.shape[0])
                assert torch.all(o.inst[cap] == -1) and torch.all(torch.isinf(o.t[cap]))
                assert torch.all(o.normal[cap] == 0)
                for k in ("id", "inst", "t", "normal"):
                    assert torch.equal(getattr(o, k)[keep], getattr(full, k)[keep]), (limit, k)
                if prev is not None:
                    assert not torch.any(cap & ~prev)
                prev = cap
                if limit == 2:
                    assert int(cap.sum()) > 0
            assert int((~prev).sum()) > 0
        finally:
            ctx.set_config(**base_cfg)
            ctx.free_scene(h)


def _corner_rays(sc, fwd, per_slot=48, seed=0):
    """Rays through points just inside the leaf corners nearest each moved
    root cell's bounding sphere, in directions perpendicular to the radius:
    each ray passes at almost exactly the sphere's radius from its centre
    and still meets a solid leaf of that slot."""
    import bruteforce as bf
    rng = np.random.default_rng(seed)
    slots, ids, C = bf.world_boxes(sc, fwd)
    out = []
    for s in range(sc.n_slots):
        cell = sc.slot_cell[s].astype(np.float64)
        Wc = bf.apply_chain(cell[:3] + cell[3] * bf.CORNERS, s, fwd, sc.slot_parent)
        c = bf.apply_chain((cell[:3] + 0.5 * cell[3])[None], s, fwd, sc.slot_parent)[0]
        r = np.linalg.norm(Wc - c, axis=1).max()
        Cs = C[slots == s]
        if Cs.shape[0] == 0:
            continue
        dist = np.linalg.norm(Cs - c, axis=2)                 # [k, 8]
        far = dist.max(1)
        for j in np.argsort(-far)[:per_slot]:
            q = Cs[j, dist[j].argmax()]
            p = q + 0.05 * (Cs[j].mean(0) - q)                  # just inside the leaf
            u = rng.normal(size=3)
            v = p - c
            u -= v * (u @ v) / (v @ v)
            u /= np.linalg.norm(u)
            o = p + u * (2.0 * r)
            out.append([o[0], o[1], o[2], 0.0, -u[0], -u[1], -u[2], np.inf])
    return np.asarray(out, np.float32)


@pytest.mark.parametrize("which", ["terrain_sorted", "tiny_index_order"])
def test_sphere_cull_keeps_corner_hits(ctx, torch_dev, which):
    """The kernel's bounding-sphere test (Eq. 4) must not cull a candidate
    frame for rays that graze its sphere where the moved cell's corner
    voxels touch it: at most 16 candidates take the sorted path, more take
    the index-order path."""
    if which == "terrain_sorted":
        sc = S.fbm_terrain_d10()
        fwd = sc.xform(17)
    else:
        sc = S.tiny_scene(7, K=6, n_slots=20, nested=False, scale_range=(1.0, 2.0))
        fwd = sc.xform(0)
    rays = _corner_rays(sc, fwd)
    h = ctx.upload_scene(sc)
    try:
        ctx.set_transforms(h, fwd)
        st_dev = ctx.scene_stats(h)
        _say(which, "rays", rays.shape[0], "candidates", st_dev.n_candidates)
        assert st_dev.n_candidates >= (17 if which == "tiny_index_order" else 4)
        g = _trace(ctx, torch_dev, h, rays)
    finally:
        ctx.free_scene(h)
    ref = oracle.trace_scene(sc, rays, fwd=fwd, margin=True)
    st = parity.compare(g, ref, ref.margin, rays)
    _say(which, st, "slot hits", int((ref.inst != NONE).sum()))
    parity.assert_parity(st)
    assert (ref.inst != NONE).mean() > 0.3


@pytest.mark.parametrize("n_slots", [60, 150])
def test_hierarchy_over_many_candidates(ctx, torch_dev, n_slots):
    """More than 16 candidate frames go through the hierarchy of their world
    boxes: camera and random rays (incl. inside starts and short tmax) equal
    the oracle, alone, in a batch next to a sorted-path job, and in a plan."""
    torch = torch_dev
    sc = S.tiny_scene(11, K=7, n_slots=n_slots, nested=False, scale_range=(0.8, 2.0), translate=0.3)
    cam_rays = S.random_rays(3, 6000, -40.0, 168.0)
    ins = S.random_rays(4, 3000, 20.0, 108.0)
    ins[:, 7] = np.where(np.arange(ins.shape[0]) % 3 == 0, 9.0, np.inf).astype(np.float32)
    rays = np.concatenate([cam_rays, ins])
    st = _check_scene(ctx, torch, sc, rays, label="hierarchy-%d" % n_slots)
    assert st["hits"] > 0
    h = ctx.upload_scene(sc)
    sph = S.noisy_sphere_d6()
    hs = ctx.upload_scene(sph)
    try:
        ctx.set_transforms(h, sc.xform(0))
        ctx.set_transforms(hs, sph.xform(0))
        assert ctx.scene_stats(h).n_candidates > 16
        r = torch.from_numpy(rays).cuda()
        rs = torch.from_numpy(sph.rays(W=40, H=40)[0]).cuda()
        alone = ctx.trace(h, r)
        jobs = [dict(scene=hs, rays=rs, **_outs(torch, rs.shape[0])), dict(scene=h, rays=r, **_outs(torch, r.shape[0]))]
        ctx.trace_batch(jobs)
        plan = ctx.plan([h, hs], max_jobs=4, max_frames=2 * (n_slots + 2))
        pj = [dict(scene=hs, rays=rs, **_outs(torch, rs.shape[0])), dict(scene=h, rays=r, **_outs(torch, r.shape[0]))]
        plan.set_jobs(pj)
        plan.launch()
        torch.cuda.synchronize()
        plan.close()
        # a configuration too large for these tables' LDS: the launch drops
        # the node cache and waves per work-group until it fits
        base_cfg = ctx.get_config().as_dict()
        try:
            ctx.set_config(waves_per_block=16, blocks_per_cu=2, lds_cache_nodes=4096)
            # five jobs on the hierarchy scene: their tables alone leave no
            # room for 16 waves' stacks, so the batch drops waves too
            big = [dict(scene=hs, rays=rs, **_outs(torch, rs.shape[0]))] + \
                [dict(scene=h, rays=r, **_outs(torch, r.shape[0])) for _ in range(5)]
            ctx.trace_batch(big)
            # 800 frame records: with 16 (and 12) waves the plan's tables
            # exceed the LDS even without a node cache, so it drops to 8
            plan16 = ctx.plan([h, hs], max_jobs=4, max_frames=800)
            pj16 = [dict(scene=hs, rays=rs, **_outs(torch, rs.shape[0])), dict(scene=h, rays=r, **_outs(torch, r.shape[0]))]
            plan16.set_jobs(pj16)
            plan16.launch()
            torch.cuda.synchronize()
            plan16.close()
        finally:
            ctx.set_config(**base_cfg)
        for got in [jobs[1], pj[1], pj16[1]] + big[1:]:
            assert torch.equal(got["out_id"], alone.id) and torch.equal(got["out_t"], alone.t)
            assert torch.equal(got["out_inst"], alone.inst) and torch.equal(got["out_normal"], alone.normal)
    finally:
        ctx.free_scene(h)
        ctx.free_scene(hs)


def test_slow_tiles_first_hierarchy_and_camera(ctx, torch_dev):
    """Slow tiles first in the other single-job instantiations: the
    candidate hierarchy (more than 16 candidate frames, which keeps the plain
    issue priority) and the camera trace (rays made in the kernel from the
    camera record kept in LDS; its ray set is named by the camera).  Each ray
    set on its own (a queue keeps two sets' lists), traced repeatedly with
    the transforms changing between traces: tile_order 0 equals tile_order 1
    bit for bit."""
    torch = torch_dev
    from paper_1911_06001_amd import svo
    sc = S.tiny_scene(11, K=7, n_slots=60, nested=False, scale_range=(0.8, 2.0), translate=0.3)
    rays = torch.from_numpy(np.concatenate([S.random_rays(3, 20000, -40.0, 168.0),
                                            S.random_rays(4, 6000, 20.0, 108.0)])).cuda()
    ter = S.fbm_terrain_d10()
    h = ctx.upload_scene(sc)
    ht = ctx.upload_scene(ter)
    c = ter.camera
    cams = [svo.make_camera(c["eye"], c["target"], c["up"], c["fov"], 320, 184),
            svo.make_camera(c["eye"], c["target"], c["up"], c["fov"], 96, 40, samples=2, seed=5, jitter=True)]
    cases = [("hierarchy", h, sc, lambda: ctx.trace(h, rays))] + \
        [("camera%d" % i, ht, ter, (lambda cm: (lambda: ctx.trace_camera(ht, cm)))(cm)) for i, cm in enumerate(cams)]
    base_cfg = ctx.get_config().as_dict()
    try:
        ctx.set_transforms(h, sc.xform(0))
        assert ctx.scene_stats(h).n_candidates > 16
        frames = (0, 9, 18)
        for label, sh, scene, run in cases:
            ctx.set_config(waves_per_block=4, blocks_per_cu=2, lds_cache_nodes=1024, refill_lanes=0, tile_order=1)
            ref = {}
            for f in frames:
                ctx.set_transforms(sh, scene.xform(f))
                ref[f] = run()
            ctx.set_config(tile_order=0)
            for rep in range(3):
                for f in frames:
                    ctx.set_transforms(sh, scene.xform(f))
                    o = run()
                    torch.cuda.synchronize()
                    e = ref[f]
                    assert torch.equal(o.id, e.id) and torch.equal(o.inst, e.inst), (label, rep, f)
                    assert torch.equal(o.t, e.t) and torch.equal(o.normal, e.normal), (label, rep, f)
    finally:
        ctx.set_config(**base_cfg)
        ctx.free_scene(h)
        ctx.free_scene(ht)


def test_slow_tiles_first_keeps_results(ctx, torch_dev):
    """tile_order 0 hands the tiles that were slowest in the previous trace of
    the same rays (on the same stream) to the waves first; tile_order 1 keeps
    the plain claim order.  Two ray sets traced in turn, the transforms
    changing between traces: from the third trace of a set on, its own list
    is in use, and every result equals the plain order's bit for bit.  The
    counting build, ordered the same way, writes every ray exactly once."""
    torch = torch_dev
    sc = S.fbm_terrain_d10()
    sets = [torch.from_numpy(sc.rays(W=320, H=180)[0]).cuda(),
            torch.from_numpy(S.random_rays(9, 30000, 0.0, sc.root_size)).cuda()]
    h = ctx.upload_scene(sc)
    base_cfg = ctx.get_config().as_dict()
    try:
        frames = (0, 7, 14, 21, 28)
        ctx.set_config(waves_per_block=4, blocks_per_cu=2, lds_cache_nodes=1024, refill_lanes=0, tile_order=1)
        ref = {}
        for f in frames:
            ctx.set_transforms(h, sc.xform(f))
            for i, r in enumerate(sets):
                ref[f, i] = ctx.trace(h, r)
        ctx.set_config(tile_order=0)
        for rep in range(3):
            for f in frames:
                ctx.set_transforms(h, sc.xform(f))
                for i, r in enumerate(sets):
                    o = ctx.trace(h, r)
                    torch.cuda.synchronize()
                    e = ref[f, i]
                    assert torch.equal(o.id, e.id) and torch.equal(o.inst, e.inst), (rep, f, i)
                    assert torch.equal(o.t, e.t) and torch.equal(o.normal, e.normal), (rep, f, i)
        for i, r in enumerate(sets):
            hits, counts, _ = ctx.trace_counted(h, r)
            torch.cuda.synchronize()
            assert int(counts[2].min()) == 1 and int(counts[2].max()) == 1, i
            assert torch.equal(hits.id, ref[frames[-1], i].id), i
    finally:
        ctx.set_config(**base_cfg)
        ctx.free_scene(h)
