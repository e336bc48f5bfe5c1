"""svo_trace_batch_static (the allocation-free batched launch: work queue
and tables in the library's per-device scratch) against svo_trace_batch on
the same jobs: bit-identical outputs on two calls in a row, the second with
a smaller batch, then a single small-scene job (its table in the kernel
arguments), and an oversized batch refused before anything is enqueued
(needs the GPU)."""
import sys

import numpy as np
import pytest

import oracle
import parity
from svogen import scenes as S

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-static]", *a, flush=True)
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


def _jobs(torch, hs, specs, fill):
    jobs = []
    for name, rays, fwd in specs:
        n = rays.shape[0]
        jobs.append(dict(scene=hs[name], rays=torch.from_numpy(rays).cuda(), fwd=fwd,
                         out_id=torch.full((n,), fill, dtype=torch.int32, device="cuda"),
                         out_inst=torch.full((n,), fill, dtype=torch.int32, device="cuda"),
                         out_t=torch.full((n,), float(fill), dtype=torch.float32, device="cuda"),
                         out_normal=torch.full((n, 3), float(fill), dtype=torch.float32, device="cuda")))
    return jobs


def _equal(torch, a, b, label):
    for k in ("out_id", "out_inst", "out_t", "out_normal"):
        assert torch.equal(a[k], b[k]), (label, k)


def test_static_batch_equals_batch(env):
    torch, svo, ctx, hs, sc = env
    ter, sph, tin = sc["ter"], sc["sph"], sc["tin"]
    calls = [
        # larger batch first: every job kind, tables in the scratch
        [("sph", sph.rays(W=100, H=77)[0], None),
         ("ter", ter.rays(W=160, H=90)[0], None),
         ("ter", ter.rays(W=123, H=45)[0], ter.xform(33)),
         ("tin", S.random_rays(4, 3001, 0.0, 32.0), None)],
        # then a smaller one on the same scratch
        [("ter", ter.rays(W=97, H=61)[0], ter.xform(12)),
         ("sph", sph.rays(W=8, H=1)[0], None)],
        # one job of a small scene: table in the kernel arguments, queue in the scratch
        [("sph", sph.rays(W=37, H=29)[0], sph.xform(0))],
    ]
    for k, specs in enumerate(calls):
        a = _jobs(torch, hs, specs, -7)
        b = _jobs(torch, hs, specs, -5)
        _say("call", k, [r.shape[0] for _, r, _ in specs])
        ctx.trace_batch(a)
        ctx.trace_batch_static(b)
        torch.cuda.synchronize()
        for ja, jb, (name, _, _) in zip(a, b, specs):
            _equal(torch, ja, jb, (k, name))
        if k == 1:
            # the animated terrain job of the smaller call against the oracle
            name, rays, fwd = specs[0]
            ref = oracle.trace_scene(ter, rays, fwd=fwd, margin=True)
            g = (b[0]["out_id"].cpu().numpy().view(np.uint32), b[0]["out_inst"].cpu().numpy().view(np.uint32),
                 b[0]["out_t"].cpu().numpy().astype(np.float64), b[0]["out_normal"].cpu().numpy().astype(np.float64))
            st = parity.compare(g, ref, ref.margin, rays)
            _say("oracle", st)
            parity.assert_parity(st)


def test_static_batch_refuses_oversized_tables(env):
    torch, svo, ctx, hs, sc = env
    # 160 jobs of the 8-slot terrain: 1,440 frame records, about 290 KiB of
    # tables (above the scratch's 256 KiB) but within the launch's LDS
    rays = sc["ter"].rays(W=8, H=1)[0][:1]
    specs = [("ter", rays, None)] * 160
    b = _jobs(torch, hs, specs, -5)
    with pytest.raises(svo.SvoError) as e:
        ctx.trace_batch_static(b)
    assert e.value.code == svo.SVO_ERANGE
    assert "allocation-free" in str(e.value), str(e.value)
    torch.cuda.synchronize()
    assert all(int(j["out_id"][0]) == -5 for j in b)
    # the regular entry point takes the same batch
    ctx.trace_batch(b)
    torch.cuda.synchronize()
    assert all(int(j["out_id"][0]) != -5 for j in b)
