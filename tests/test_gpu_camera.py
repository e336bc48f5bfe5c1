"""Camera traces: primary rays made inside the trace kernel from a camera
record instead of read from a ray buffer (svo_trace_camera, svo_job.camera).
Results are bit-identical to generating the rays on the device and tracing
them, for whole-tile images (the fast pixel mapping) and for partial tiles,
several jittered samples per pixel and row order (the general one); camera
jobs mix with ray jobs in one batch and in a launch plan; and the terrain
camera trace matches the oracle (needs the GPU)."""
import sys

import numpy as np
import pytest

import oracle
import parity
from svogen import scenes as S

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-camera]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_1911_06001_amd import svo
    ctx = svo.Context(0)
    ter = S.fbm_terrain_d10()
    sph = S.noisy_sphere_d6()
    hs = dict(ter=ctx.upload_scene(ter), sph=ctx.upload_scene(sph))
    ctx.set_transforms(hs["ter"], ter.xform(9))
    ctx.set_transforms(hs["sph"], sph.xform(0))
    yield torch, svo, ctx, hs, dict(ter=ter, sph=sph)
    ctx.close()


def _cam(svo, sc, W, H, **kw):
    c = sc.camera
    return svo.make_camera(c["eye"], c["target"], c["up"], c["fov"], W, H, **kw)


def _equal(torch, a, b, label):
    for k in ("id", "inst", "t", "normal"):
        assert torch.equal(getattr(a, k), getattr(b, k)), (label, k)


@pytest.mark.parametrize("name,W,H,kw", [
    ("ter", 1920, 1080, {}),                                          # whole 8x8 tiles, one sample
    ("ter", 333, 101, dict(samples=3, seed=7, jitter=True)),          # partial tiles, jittered samples
    ("sph", 96, 50, dict(tiled=False, samples=2, seed=3, jitter=True)),  # row order
])
def test_camera_trace_equals_generated_rays(env, name, W, H, kw):
    torch, svo, ctx, hs, sc = env
    cam = _cam(svo, sc[name], W, H, **kw)
    rays = ctx.primary_rays(cam)
    ref = ctx.trace(hs[name], rays)
    got = ctx.trace_camera(hs[name], cam)
    torch.cuda.synchronize()
    _say(name, W, H, kw, "hits", int((got.id != -1).sum()))
    _equal(torch, got, ref, (name, W, H))


def test_camera_trace_matches_the_oracle(env):
    torch, svo, ctx, hs, sc = env
    ter = sc["ter"]
    cam = _cam(svo, ter, 1920, 1080)
    got = ctx.trace_camera(hs["ter"], cam)
    rays = ctx.primary_rays(cam).cpu().numpy()
    torch.cuda.synchronize()
    pix = np.arange(rays.shape[0])
    idx = parity.survey_sample(pix, 1920, 1080)
    ref = oracle.trace_scene(ter, rays[idx], fwd=ter.xform(9), margin=True)
    st = parity.compare(tuple(x[idx] for x in parity.to_numpy(got)), ref, ref.margin, rays[idx])
    _say("oracle", st)
    parity.assert_parity(st, 1e-4)


def _outs(torch, n):
    return dict(out_id=torch.full((n,), -3, dtype=torch.int32, device="cuda"),
                out_inst=torch.full((n,), -3, dtype=torch.int32, device="cuda"),
                out_t=torch.full((n,), -3.0, dtype=torch.float32, device="cuda"),
                out_normal=torch.full((n, 3), -3.0, dtype=torch.float32, device="cuda"))


def test_camera_jobs_in_batches_and_plans(env):
    torch, svo, ctx, hs, sc = env
    ter, sph = sc["ter"], sc["sph"]
    cams = [_cam(svo, ter, 160, 96), _cam(svo, sph, 72, 40, samples=2, seed=5, jitter=True),
            _cam(svo, ter, 64, 64)]
    fwd = [None, None, ter.xform(40)]
    names = ["ter", "sph", "ter"]
    ray_job = ter.rays(W=50, H=30)[0]
    # references: one camera trace per job (the job's own transforms set first)
    refs = []
    for c, f, nm in zip(cams, fwd, names):
        if f is not None:
            ctx.set_transforms(hs[nm], f)
        refs.append(ctx.trace_camera(hs[nm], c))
        if f is not None:
            ctx.set_transforms(hs[nm], ter.xform(9))
    r = torch.from_numpy(ray_job).cuda()
    ref_rays = ctx.trace(hs["ter"], r)
    torch.cuda.synchronize()

    def jobs():
        out = []
        for c, f, nm in zip(cams, fwd, names):
            n = c.width * c.height * c.samples
            out.append(dict(scene=hs[nm], camera=c, fwd=f, **_outs(torch, n)))
        out.insert(1, dict(scene=hs["ter"], rays=r, **_outs(torch, r.shape[0])))
        return out

    def check(js, label):
        refs_all = [refs[0], ref_rays, refs[1], refs[2]]
        for j, ref in zip(js, refs_all):
            for k, key in (("id", "out_id"), ("inst", "out_inst"), ("t", "out_t"), ("normal", "out_normal")):
                assert torch.equal(j[key], getattr(ref, k)), (label, key)

    a = jobs()
    ctx.trace_batch(a)
    torch.cuda.synchronize()
    check(a, "batch")
    # a single camera job (the camera in the kernel arguments)
    one = [dict(scene=hs["ter"], camera=cams[0], **_outs(torch, 160 * 96))]
    ctx.trace_batch(one)
    torch.cuda.synchronize()
    for k, key in (("id", "out_id"), ("t", "out_t")):
        assert torch.equal(one[0][key], getattr(refs[0], k)), ("single", key)
    plan = ctx.plan([hs["ter"], hs["sph"]], max_jobs=8, max_frames=64)
    try:
        b = jobs()
        plan.set_jobs(b)
        plan.launch()
        torch.cuda.synchronize()
        check(b, "plan")
    finally:
        plan.close()


def test_camera_job_errors(env):
    torch, svo, ctx, hs, sc = env
    cam = _cam(svo, sc["ter"], 16, 8)
    o = _outs(torch, 128)
    # a camera job with a ray buffer, and one whose n is not the camera's
    arr, keep = svo._job_array([dict(scene=hs["ter"], camera=cam, **o)])
    arr[0].rays = o["out_t"].data_ptr()
    assert svo.lib().svo_trace_batch(ctx._ptr, arr, 1, None) == svo.SVO_EINVAL
    arr, keep = svo._job_array([dict(scene=hs["ter"], camera=cam, **o)])
    arr[0].n = 127
    assert svo.lib().svo_trace_batch(ctx._ptr, arr, 1, None) == svo.SVO_EINVAL
    bad = _cam(svo, sc["ter"], 16, 8)
    bad.samples = 0
    with pytest.raises(svo.SvoError):
        ctx.trace_camera(hs["ter"], bad)
