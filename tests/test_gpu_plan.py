"""Launch plans (svo_plan_*): a plan launch equals svo_trace_batch with the
same jobs, bit for bit; the launch captured once into a HIP graph (torch
CUDA graph) and replayed with new jobs in the staging equals the eager
result at every replay; capacity and ownership errors are reported."""
import sys

import numpy as np
import pytest

import oracle
import parity
from svogen import scenes as S

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-plan]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_1911_06001_amd import svo
    ctx = svo.Context(0)
    sph = S.noisy_sphere_d6()
    ter = S.fbm_terrain_d10()
    tin = S.tiny_scene(3, K=5, n_slots=4, nested=True, scale_range=(0.3, 1.5))
    hs = {k: ctx.upload_scene(v) for k, v in (("sph", sph), ("ter", ter), ("tin", tin))}
    ctx.set_transforms(hs["sph"], sph.xform(0))
    ctx.set_transforms(hs["tin"], tin.xform(0))
    ctx.set_transforms(hs["ter"], ter.xform(5))
    yield torch, svo, ctx, hs, dict(sph=sph, ter=ter, tin=tin)
    ctx.close()


def _outs(torch, n, fill=0):
    return dict(out_id=torch.full((n,), fill, dtype=torch.int32, device="cuda"),
                out_inst=torch.full((n,), fill, dtype=torch.int32, device="cuda"),
                out_t=torch.full((n,), float(fill), dtype=torch.float32, device="cuda"),
                out_normal=torch.full((n, 3), float(fill), dtype=torch.float32, device="cuda"))


def _jobs(torch, hs, sc, specs):
    jobs = []
    for name, rays, fwd in specs:
        r = torch.from_numpy(rays).cuda()
        jobs.append(dict(scene=hs[name], rays=r, fwd=fwd, **_outs(torch, rays.shape[0], -7)))
    return jobs


def _mix(sc, k):
    """Job mixes of different sizes, scenes and animation frames."""
    ter, sph, tin = sc["ter"], sc["sph"], sc["tin"]
    if k == 0:
        return [("sph", sph.rays(W=100, H=77)[0], None),
                ("ter", ter.rays(W=160, H=90)[0], None),
                ("ter", ter.rays(W=123, H=45)[0], ter.xform(33)),
                ("tin", S.random_rays(4, 3001, 0.0, 32.0), None)]
    if k == 1:
        return [("ter", ter.rays(W=97, H=61)[0], ter.xform(12)),
                ("sph", sph.rays(W=8, H=1)[0], None)]
    return [("tin", S.random_rays(5, 777, 0.0, 32.0), tin.xform(1)),
            ("ter", ter.rays(W=64, H=64)[0], ter.xform(47)),
            ("sph", sph.rays(W=33, H=17)[0], sph.xform(0)),
            ("ter", ter.rays(W=31, H=7)[0], None),
            ("sph", sph.rays(W=5, H=3)[0], None)]


def _equal(torch, a, b, label):
    for k in ("out_id", "out_inst", "out_t", "out_normal"):
        assert torch.equal(a[k], b[k]), (label, k)


def test_plan_equals_batch(env):
    torch, svo, ctx, hs, sc = env
    plan = ctx.plan([hs["ter"], hs["sph"], hs["tin"]], max_jobs=16, max_frames=64)
    try:
        for k in range(3):
            specs = _mix(sc, k)
            a = _jobs(torch, hs, sc, specs)
            b = _jobs(torch, hs, sc, specs)
            _say("eager mix", k, [r.shape[0] for _, r, _ in specs])
            ctx.trace_batch(a)
            plan.set_jobs(b)
            plan.launch()
            torch.cuda.synchronize()
            for ja, jb, (name, _, _) in zip(a, b, specs):
                _equal(torch, ja, jb, (k, name))
        # one job against the oracle
        specs = _mix(sc, 0)
        b = _jobs(torch, hs, sc, specs)
        plan.set_jobs(b)
        plan.launch()
        torch.cuda.synchronize()
        ref = oracle.trace_scene(sc["ter"], specs[2][1], fwd=specs[2][2], margin=True)
        g = (b[2]["out_id"].cpu().numpy().view(np.uint32), b[2]["out_inst"].cpu().numpy().view(np.uint32),
             b[2]["out_t"].cpu().numpy().astype(np.float64), b[2]["out_normal"].cpu().numpy().astype(np.float64))
        parity.assert_parity(parity.compare(g, ref, ref.margin, specs[2][1]))
    finally:
        plan.close()


def test_plan_graph_replays(env):
    """Capture one plan launch, then replay it with a different job mix in the
    staging each time, with eager work in between; every replay equals
    svo_trace_batch on the same jobs."""
    torch, svo, ctx, hs, sc = env
    plan = ctx.plan([hs["ter"], hs["sph"], hs["tin"]], max_jobs=16, max_frames=64)
    try:
        first = _jobs(torch, hs, sc, _mix(sc, 1))
        plan.set_jobs(first)
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        _say("capture")
        with torch.cuda.graph(g, stream=side):
            plan.launch(torch.cuda.current_stream())
        torch.cuda.synchronize()
        for rep, k in enumerate((0, 2, 1, 0, 2)):
            specs = _mix(sc, k)
            mine = _jobs(torch, hs, sc, specs)
            ref = _jobs(torch, hs, sc, specs)
            plan.set_jobs(mine)
            _say("replay", rep, "mix", k)
            g.replay()
            torch.cuda.synchronize()
            ctx.trace_batch(ref)            # eager work between replays
            torch.cuda.synchronize()
            for ja, jb, (name, _, _) in zip(mine, ref, specs):
                _equal(torch, ja, jb, (rep, k, name))
        # the first capture's outputs were never written by a replay with other jobs
        assert int(first[0]["out_id"][0]) == -7
        del g
        torch.cuda.synchronize()
    finally:
        plan.close()


def test_plan_empty_and_errors(env):
    torch, svo, ctx, hs, sc = env
    plan = ctx.plan([hs["sph"]], max_jobs=2, max_frames=4)
    try:
        # no jobs: the launch traces nothing
        plan.set_jobs([])
        plan.launch()
        j = _jobs(torch, hs, sc, [("sph", sc["sph"].rays(W=16, H=16)[0], None)])
        empty = dict(j[0])
        empty["rays"] = j[0]["rays"][:0]
        plan.set_jobs([empty])
        plan.launch()
        torch.cuda.synchronize()
        assert int((j[0]["out_id"] != -7).sum()) == 0
        # a scene outside the plan
        with pytest.raises(svo.SvoError) as e:
            plan.set_jobs(_jobs(torch, hs, sc, [("ter", sc["ter"].rays(W=8, H=8)[0], None)]))
        assert e.value.code == svo.SVO_EINVAL
        # more frame records than the plan holds (sphere: 2 per job, 3 jobs > 2 jobs / 4 frames)
        many = _jobs(torch, hs, sc, [("sph", sc["sph"].rays(W=8, H=8)[0], None)] * 3)
        with pytest.raises(svo.SvoError) as e:
            plan.set_jobs(many)
        assert e.value.code == svo.SVO_ERANGE
        # a plan's scene cannot be freed while the plan lives
        with pytest.raises(svo.SvoError) as e:
            ctx.free_scene(hs["sph"])
        assert e.value.code == svo.SVO_EBUSY
        # the plan still works after the failed calls
        ok = _jobs(torch, hs, sc, [("sph", sc["sph"].rays(W=16, H=16)[0], None)])
        plan.set_jobs(ok)
        plan.launch()
        alone = ctx.trace(hs["sph"], ok[0]["rays"])
        torch.cuda.synchronize()
        assert torch.equal(alone.id, ok[0]["out_id"]) and torch.equal(alone.t, ok[0]["out_t"])
    finally:
        plan.close()
    with pytest.raises(svo.SvoError) as e:
        svo.Plan(ctx, [hs["sph"]], 0, 4)
    assert e.value.code == svo.SVO_ERANGE
    with pytest.raises(svo.SvoError) as e:
        svo.Plan(ctx, [12345], 4, 4)
    assert e.value.code == svo.SVO_EINVAL
