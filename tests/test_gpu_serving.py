"""Serving loop on the device: continuous batching under an HBM budget, each
request's result equal alone and in the mix (needs the GPU)."""
import sys

import numpy as np
import pytest

import oracle
import parity
from svogen import scenes as S

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-serving]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    import torch
    assert torch.cuda.is_available()
    from paper_1911_06001_amd import serve, svo
    ctx = svo.Context(0)
    sph = S.noisy_sphere_d6()
    ter = S.fbm_terrain_d10()
    hs = {"sphere": ctx.upload_scene(sph), "terrain": ctx.upload_scene(ter)}
    entries = {"sphere": serve.SceneEntry(hs["sphere"], sph.xform, sph.camera),
               "terrain": serve.SceneEntry(hs["terrain"], ter.xform, ter.camera)}
    yield torch, ctx, entries, {"sphere": sph, "terrain": ter}
    for h in hs.values():
        ctx.free_scene(h)
    ctx.close()


@pytest.mark.parametrize("graph,solo", [(False, 0), (True, 0), (False, 1 << 24)])
def test_each_result_same_alone_and_in_the_mix(setup, graph, solo):
    """Continuous batching (eager batched launches, or a captured plan
    launch replayed per step; requests split across steps, or a lone one
    taken whole): every request's outputs equal tracing it alone."""
    torch, ctx, entries, scenes = setup
    from paper_1911_06001_amd import serve
    reqs = serve.poisson_requests(24, 4000.0, 3, ["sphere", "terrain"],
                                  resolutions=((64, 64), (160, 90), (256, 144), (96, 200)), samples=(1, 3))
    # the resident scenes come out of the budget first; room for three requests
    resident = sum(ctx.scene_bytes(e.handle) for e in entries.values())
    budget = resident + 3 * max(r.footprint for r in reqs)
    srv = serve.Server(ctx, entries, hbm_budget=budget, max_rays_per_step=60000, solo_rays_per_step=solo,
                       keep_outputs=True, graph=graph)
    try:
        res = srv.run(reqs, mode="batched")
    finally:
        srv.close()
    _say("served graph=%s" % graph, serve.summarize(res), "max_used", srv.scheduler.max_used, "budget", budget)
    assert len(res) == len(reqs) and srv.resident_bytes == resident
    assert srv.scheduler.max_used <= budget - resident
    for r in res:
        e = entries[r.req.scene]
        ctx.set_transforms(e.handle, e.xform(r.req.frame))
        alone = ctx.trace(e.handle, r.out["rays"])
        torch.cuda.synchronize()
        for k, v in (("out_id", alone.id), ("out_inst", alone.inst), ("out_t", alone.t), ("out_normal", alone.normal)):
            assert torch.equal(r.out[k], v), (r.req, k)
        assert r.completed >= r.admitted >= r.req.arrival - 1e-3
    # two served requests checked against the oracle on the very rays they used
    for r in res[:2]:
        sc = scenes[r.req.scene]
        rays = r.out["rays"].cpu().numpy()
        ref = oracle.trace_scene(sc, rays, frame=r.req.frame, margin=True)
        got = (r.out["out_id"].cpu().numpy().view(np.uint32), r.out["out_inst"].cpu().numpy().view(np.uint32),
               r.out["out_t"].cpu().numpy().astype(np.float64), r.out["out_normal"].cpu().numpy().astype(np.float64))
        parity.assert_parity(parity.compare(got, ref, ref.margin, rays), 1e-4)


def test_single_mode_baseline_runs(setup):
    torch, ctx, entries, scenes = setup
    from paper_1911_06001_amd import serve
    reqs = serve.poisson_requests(8, 2000.0, 5, ["sphere", "terrain"], resolutions=((64, 64), (128, 72)), samples=(1, 2))
    srv = serve.Server(ctx, entries, hbm_budget=1 << 30)
    res = srv.run(reqs, mode="single")
    st = serve.summarize(res)
    _say("single", st)
    assert st["requests"] == 8 and st["p99_ms"] >= st["p50_ms"] > 0


@pytest.mark.parametrize("graph", [False, True])
def test_requests_with_ao_phase(setup, graph):
    """Requests whose AO rays (from their own primary hits) form a second
    phase: both phases equal tracing them alone."""
    torch, ctx, entries, scenes = setup
    from paper_1911_06001_amd import serve
    shapes = {"sphere": (48, 40, 2, 3), "terrain": (120, 72, 1, 2)}
    reqs = serve.poisson_requests(12, 3000.0, 8, ["sphere", "terrain"], shapes=shapes)
    resident = sum(ctx.scene_bytes(e.handle) for e in entries.values())
    budget = resident + 3 * max(r.footprint for r in reqs)
    srv = serve.Server(ctx, entries, hbm_budget=budget, max_rays_per_step=20000, solo_rays_per_step=0,
                       keep_outputs=True, graph=graph)
    try:
        res = srv.run(reqs, mode="batched")
    finally:
        srv.close()
    _say("ao phase graph=%s" % graph, serve.summarize(res))
    assert len(res) == len(reqs) and srv.scheduler.max_used <= budget - resident
    for r in res:
        e = entries[r.req.scene]
        ctx.set_transforms(e.handle, e.xform(r.req.frame))
        prim = ctx.trace(e.handle, r.out["rays"])
        ao_rays = ctx.ao_rays(r.out["rays"], prim, k=r.req.ao, seed=r.req.seed, radius=r.req.ao_radius)
        ao = ctx.trace(e.handle, ao_rays)
        torch.cuda.synchronize()
        assert torch.equal(r.out["out_id"], prim.id) and torch.equal(r.out["out_t"], prim.t)
        assert torch.equal(r.out["ao"]["rays"], ao_rays)
        assert torch.equal(r.out["ao"]["out_id"], ao.id) and torch.equal(r.out["ao"]["out_t"], ao.t)
