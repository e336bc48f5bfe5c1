"""Instanced scene (64 DAG-shared instances of 4 SVOs in a 4096^3 world) with
ambient-occlusion rays, against the oracle (needs the GPU)."""
import sys

import numpy as np
import pytest

import oracle
import parity
from svogen import scenes as S

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-instances]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_1911_06001_amd import svo
    _say("building the instanced scene")
    sc = S.instanced_scene()
    ctx = svo.Context(0)
    h = ctx.upload_scene(sc)
    ctx.set_transforms(h, sc.xform(0))
    st = ctx.scene_stats(h)
    _say("stats", dict(n_inline=st.n_inline, n_cand=st.n_candidates, stack=st.stack_levels, bytes=st.device_bytes))
    yield torch, ctx, sc, h
    ctx.free_scene(h)
    ctx.close()


def test_primary_rays(env):
    torch, ctx, sc, h = env
    rays, _ = sc.rays(W=320, H=180)
    out = ctx.trace(h, torch.from_numpy(rays).cuda())
    torch.cuda.synchronize()
    ref = oracle.trace_scene(sc, rays, margin=True)
    st = parity.compare(parity.to_numpy(out), ref, ref.margin, rays)
    _say("primary", st)
    parity.assert_parity(st, 1e-4)
    assert len(np.unique(ref.inst[ref.id != 0xFFFFFFFF])) > 40


def test_ao_rays(env):
    torch, ctx, sc, h = env
    rays, _ = sc.rays(W=160, H=90)
    r = torch.from_numpy(rays).cuda()
    prim = ctx.trace(h, r)
    ao = ctx.ao_rays(r, prim, k=4, seed=3, radius=64.0)
    out = ctx.trace(h, ao)
    torch.cuda.synchronize()
    a = ao.cpu().numpy()
    t = prim.t.cpu().numpy()
    nrm = prim.normal.cpu().numpy()
    hit = np.repeat(np.isfinite(t) & (np.abs(nrm).sum(1) > 0), 4)
    assert a.shape == (rays.shape[0] * 4, 8)
    d = a[hit, 4:7].astype(np.float64)
    n4 = np.repeat(nrm, 4, axis=0)[hit].astype(np.float64)
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-5)
    cos = (d * n4).sum(1)
    assert cos.min() > -1e-5
    assert abs(cos.mean() - 2.0 / 3.0) < 0.02          # cosine-weighted hemisphere
    assert np.all(a[~hit, 3] > a[~hit, 7])              # misses give empty rays
    ref = oracle.trace_scene(sc, a, margin=True)
    st = parity.compare(parity.to_numpy(out), ref, ref.margin, a)
    _say("ao", st, "occluded", float((ref.id[hit] != 0xFFFFFFFF).mean()))
    parity.assert_parity(st, 1e-4)


@pytest.mark.timeout(600)
def test_full_resolution_in_the_benchmark_launch(env):
    """1920x1080 primary rays and 4 AO rays per pixel under the configuration
    the autotuner picks (as the benchmark runs them): every 17th pixel plus a
    64x64-pixel block (about 126 k primary and 503 k AO rays) checked against
    the oracle one by one, at an id mismatch rate of at most 1e-4."""
    torch, ctx, sc, h = env
    rays, pix = sc.rays()
    r = torch.from_numpy(rays).cuda()
    cfg = ctx.tune(h, r)
    _say("tuned", cfg.as_dict())
    prim = ctx.trace(h, r)
    ao = ctx.ao_rays(r, prim, k=4, seed=3, radius=64.0)
    out = ctx.trace(h, ao)
    torch.cuda.synchronize()
    idx = parity.survey_sample(pix, 1920, 1080)
    g = parity.to_numpy(prim)
    ref = oracle.trace_scene(sc, rays[idx], margin=True)
    st = parity.compare(tuple(x[idx] for x in g), ref, ref.margin, rays[idx])
    _say("primary 1080p sampled", st)
    parity.assert_parity(st, 1e-4)
    aidx = (4 * idx[:, None] + np.arange(4)[None, :]).reshape(-1)
    a = ao[torch.from_numpy(aidx).cuda()].cpu().numpy()
    ga = parity.to_numpy(out)
    refa = oracle.trace_scene(sc, a, margin=True)
    sta = parity.compare(tuple(x[aidx] for x in ga), refa, refa.margin, a)
    _say("ao sampled", sta)
    parity.assert_parity(sta, 1e-4)
