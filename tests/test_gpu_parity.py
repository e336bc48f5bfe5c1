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
    st = parity.compare(g, ref, ref.margin)
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
    """1920x1080 in the benchmark's launch: every 17th ray plus one 64x64 tile
    block of rays are checked against the oracle one by one."""
    sc = S.fbm_terrain_d10()
    rays, pix = sc.rays()
    n = rays.shape[0]
    idx = np.unique(np.concatenate([np.arange(0, n, 17), np.arange(400 * 64, 400 * 64 + 4096)]))
    h = ctx.upload_scene(sc)
    try:
        ctx.set_transforms(h, sc.xform(30))
        g = _trace(ctx, torch_dev, h, rays)
    finally:
        ctx.free_scene(h)
    ref = oracle.trace_scene(sc, rays[idx], frame=30, margin=True)
    st = parity.compare(tuple(a[idx] for a in g), ref, ref.margin)
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
    parity.assert_parity(parity.compare(g, ref, ref.margin))


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
    parity.assert_parity(parity.compare(g, ref, ref.margin))


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
        parity.assert_parity(parity.compare(parity.to_numpy(hh), ref, ref.margin))
