"""Device ray generation and the autotuner, through the C ABI (needs the GPU)."""
import sys

import numpy as np
import pytest

import oracle
import parity
from svogen import camera as hostcam
from svogen import scenes as S

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-raygen]", *a, flush=True)
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


@pytest.mark.parametrize("W,H,tiled", [(128, 128, True), (101, 37, True), (64, 48, False)])
def test_primary_rays_match_host_camera(ctx, torch_dev, W, H, tiled):
    from paper_1911_06001_amd import svo
    sc = S.noisy_sphere_d6()
    c = sc.camera
    cam = svo.make_camera(c["eye"], c["target"], c["up"], c["fov"], W, H, tiled=tiled)
    g = ctx.primary_rays(cam)
    torch_dev.cuda.synchronize()
    g = g.cpu().numpy()
    h, _ = hostcam.pinhole_rays(c["eye"], c["target"], c["up"], c["fov"], W, H, order="tiles" if tiled else "rows")
    assert g.shape == h.shape
    np.testing.assert_array_equal(g[:, 0:4], h[:, 0:4])
    np.testing.assert_array_equal(g[:, 7], h[:, 7])
    np.testing.assert_allclose(g[:, 4:7], h[:, 4:7], atol=2e-6)


def test_jittered_rays_trace_like_the_oracle(ctx, torch_dev):
    from paper_1911_06001_amd import svo
    sc = S.noisy_sphere_d6()
    c = sc.camera
    cam = svo.make_camera(c["eye"], c["target"], c["up"], c["fov"], 96, 80, samples=3, seed=11, jitter=True)
    rays = ctx.primary_rays(cam)
    # jitter keeps every sample inside its pixel: same pixel grid, spread directions
    r = rays.cpu().numpy()
    assert r.shape[0] == 96 * 80 * 3
    assert np.unique(r[:, 4:7], axis=0).shape[0] > 0.99 * r.shape[0]
    h = ctx.upload_scene(sc)
    try:
        ctx.set_transforms(h, sc.xform(0))
        out = ctx.trace(h, rays)
        torch_dev.cuda.synchronize()
        got = parity.to_numpy(out)
    finally:
        ctx.free_scene(h)
    ref = oracle.trace_scene(sc, r, margin=True)
    st = parity.compare(got, ref, ref.margin, r)
    _say("jittered", st)
    parity.assert_parity(st, 1e-4)


def test_tune_picks_a_config_and_keeps_results(ctx, torch_dev):
    torch = torch_dev
    sc = S.fbm_terrain_d10()
    rays, _ = sc.rays(W=480, H=270)
    r = torch.from_numpy(rays).cuda()
    h = ctx.upload_scene(sc)
    try:
        ctx.set_transforms(h, sc.xform(12))
        before = ctx.trace(h, r)
        torch.cuda.synchronize()
        cfg = ctx.tune(h, r)
        _say("tuned", cfg.as_dict())
        # one of the tuner's candidates (svo_tune's search space)
        assert cfg.waves_per_block in (4, 8, 12, 16) and cfg.blocks_per_cu in (1, 2, 3, 4, 5, 6, 8)
        assert cfg.waves_per_block * cfg.blocks_per_cu <= 32
        assert cfg.lds_cache_nodes in (1024, 2048, 4096) and cfg.refill_lanes in (0, 48) and cfg.claim_tiles in (1, 2, 4)
        after = ctx.trace(h, r)
        torch.cuda.synchronize()
        assert torch.equal(before.id, after.id) and torch.equal(before.t, after.t)
    finally:
        ctx.free_scene(h)
