"""Hit buffer (svo_trace_rays_reuse): updating the previous frame's hits for
new transforms gives exactly what a full trace gives, frame after frame,
while tracing only the rays that can change (needs the GPU)."""
import sys

import numpy as np
import pytest

import oracle
import parity
from svogen import scenes as S

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-reuse]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_1911_06001_amd import svo
    ctx = svo.Context(0)
    yield torch, ctx
    ctx.close()


def _run(torch, ctx, sc, rays_np, frames, label, check_oracle_at=None):
    h = ctx.upload_scene(sc)
    try:
        r = torch.from_numpy(rays_np).cuda()
        ctx.set_transforms(h, sc.xform(frames[0]))
        hits = ctx.trace(h, r)
        counts = []
        for f in frames[1:]:
            ctx.set_transforms(h, sc.xform(f))
            cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
            ctx.trace_reuse(h, r, hits, retraced=cnt)
            full = ctx.trace(h, r)
            torch.cuda.synchronize()
            for k in ("id", "inst", "t", "normal"):
                assert torch.equal(getattr(hits, k), getattr(full, k)), (label, f, k)
            counts.append(int(cnt.item()))
            if f == check_oracle_at:
                ref = oracle.trace_scene(sc, rays_np, frame=f, margin=True)
                parity.assert_parity(parity.compare(parity.to_numpy(hits), ref, ref.margin, rays_np))
        _say(label, "rays", rays_np.shape[0], "retraced per frame", counts)
        return counts
    finally:
        ctx.free_scene(h)


def test_terrain_frames(env):
    torch, ctx = env
    sc = S.fbm_terrain_d10()
    rays, _ = sc.rays(W=480, H=270)
    counts = _run(torch, ctx, sc, rays, [0, 1, 2, 17, 18, 40, 59], "terrain", check_oracle_at=17)
    assert max(counts) < 0.5 * rays.shape[0]          # most rays keep their hit
    assert min(counts) > 0


@pytest.mark.parametrize("seed", [2, 5])
def test_nested_in_place_frames(env, seed):
    torch, ctx = env
    sc = S.tiny_scene(seed, K=6, n_slots=4, nested=True, scale_range=(0.6, 1.0))
    rays = np.concatenate([S.random_rays(seed, 4000, 0.0, 64.0), S.random_rays(seed + 9, 1000, 8.0, 56.0)])
    _run(torch, ctx, sc, rays, [0, 1, 2, 3, 4], "nested-%d" % seed, check_oracle_at=3)


def test_instances_hierarchy_path(env):
    torch, ctx = env
    sc = S.instanced_scene()
    rays, _ = sc.rays(W=320, H=180)
    base = sc.xform(0)

    # the instances' transforms are static: animate them by re-posing a few
    def xform(f):
        x = base.copy()
        k = np.arange(0, x.shape[0], 7)
        x[k, 3] += np.float32(37.0 * f)
        x[k, 11] -= np.float32(21.0 * f)
        return x
    sc.xform = xform
    counts = _run(torch, ctx, sc, rays, [0, 1, 2, 3], "instances", check_oracle_at=2)
    assert max(counts) < rays.shape[0]
