"""Pins for the FP64 oracle: each checks it against something other than itself.

P1 brute force (world-space parallelepipeds, forward maps only), P2 identity
transforms reproduce the static tree, P3 lattice-preserving transforms equal
the re-voxelised static scene, P4 translation equals a shifted origin, P5 the
paper's own form (rotate/translate the ray, scale the octree extents, Sec.
3.1-3.2) equals the general affine inverse, P6 closed forms, P8 t scales
with 1/|d| (Eq. 2: the local ray keeps the world parameter t).
"""
import numpy as np
import pytest

import bruteforce as bf
import oracle
from svogen import octree as ot
from svogen import scenes as S
from svogen import xforms as xf

NONE = 0xFFFFFFFF


def _ok(h, thr=1e-9):
    return h.margin >= thr


# ---------------------------------------------------------------- P1 brute force

@pytest.mark.parametrize("seed", range(1, 9))
def test_p1_bruteforce_nested(seed, oracle_lib):
    sc = S.tiny_scene(seed, K=5 if seed % 2 else 4, n_slots=4, nested=True, translate=0.3)
    assert (sc.slot_parent != NONE).any(), "scene must exercise nested frames"
    fwd = sc.xform(0)
    rays = S.random_rays(seed, 800, 0.0, sc.root_size)
    h = oracle.trace_scene(sc, rays, margin=True)
    bid, binst, bt, bn = bf.trace(sc, fwd, rays)
    ok = _ok(h)
    assert ok.mean() > 0.97
    assert (h.id != NONE).sum() > 100
    np.testing.assert_array_equal(h.id[ok], bid[ok])
    np.testing.assert_array_equal(h.inst[ok], binst[ok])
    fin = ok & np.isfinite(bt)
    np.testing.assert_allclose(h.t[fin], bt[fin], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(h.normal[ok], bn[ok], atol=1e-9)


def test_p1_axis_aligned_and_inside_rays(oracle_lib):
    sc = S.tiny_scene(5, K=4, n_slots=2, nested=False, rotate=False, scale_range=(1.0, 1.0), translate=0.4)
    fwd = sc.xform(0)
    st_rays = []
    rng = np.random.default_rng(3)
    for k in range(600):
        o = rng.uniform(-4, 20, 3).astype(np.float32)
        d = np.zeros(3, np.float32)
        a = k % 3
        d[a] = 1.0 if k % 2 else -1.0
        if k % 5 == 0:
            d[(a + 1) % 3] = 0.5
        st_rays.append([*o, 0.0, *(d / np.linalg.norm(d)), np.inf])
    rays = np.array(st_rays, np.float32)
    h = oracle.trace_scene(sc, rays, margin=True)
    bid, binst, bt, bn = bf.trace(sc, fwd, rays)
    ok = _ok(h)
    assert ok.mean() > 0.9
    np.testing.assert_array_equal(h.id[ok], bid[ok])
    fin = ok & np.isfinite(bt)
    np.testing.assert_allclose(h.t[fin], bt[fin], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(h.normal[ok], bn[ok], atol=1e-9)


def test_p1_noisy_sphere_d6(oracle_lib):
    sc = S.noisy_sphere_d6()
    rays, _ = sc.rays(W=48, H=48)
    h = oracle.trace_scene(sc, rays, margin=True)
    bid, binst, bt, bn = bf.trace(sc, sc.xform(0), rays)
    ok = _ok(h)
    np.testing.assert_array_equal(h.id[ok], bid[ok])
    np.testing.assert_array_equal(h.inst[ok], binst[ok])
    assert (h.inst == 0).sum() > 20 and ((h.id != NONE) & (h.inst == NONE)).sum() > 20


def test_frames_match_generator(oracle_lib):
    for seed in range(1, 6):
        sc = S.tiny_scene(seed, K=5, n_slots=4, nested=True)
        nf, par, W = oracle.frames(sc.nodes, sc.root, sc.root_min, sc.root_size, sc.slot_child, sc.slot_cell,
                                   sc.xform(0))
        assert nf == sc.n_slots + 1
        np.testing.assert_array_equal(par, sc.slot_parent)
        # composed map applied to points == forward chain applied map by map
        pts = np.random.default_rng(seed).uniform(0, 32, (20, 3))
        for s in range(sc.n_slots):
            A = W[s].reshape(3, 4)
            np.testing.assert_allclose(pts @ A[:, :3].T + A[:, 3], bf.apply_chain(pts, s, sc.xform(0), sc.slot_parent),
                                       rtol=1e-12, atol=1e-10)


# ---------------------------------------------------------------- P2 identity

@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_p2_identity_equals_static(seed, oracle_lib):
    sc = S.tiny_scene(seed, K=5, n_slots=4, nested=True)
    ident = np.tile(xf.to_f32(xf.identity()).reshape(1, 12), (sc.n_slots, 1))
    rays = S.random_rays(seed + 10, 1500, 0.0, sc.root_size)
    ha = oracle.trace_scene(sc, rays, fwd=ident, margin=True)
    hs = oracle.trace_scene(sc, rays, static=True, margin=True)
    ok = _ok(ha) & _ok(hs)
    assert ok.mean() > 0.97
    np.testing.assert_array_equal(ha.id[ok], hs.id[ok])
    np.testing.assert_array_equal(ha.t[ok], hs.t[ok])
    np.testing.assert_array_equal(ha.normal[ok], hs.normal[ok])
    assert (hs.inst == NONE).all()
    assert (ha.inst[ok & (ha.id != NONE)] != NONE).any()


def test_p2_sphere64_identity(oracle_lib):
    sc = S.noisy_sphere_d6()
    rays, _ = sc.rays()
    ident = xf.to_f32(xf.identity()).reshape(1, 12)
    ha = oracle.trace_scene(sc, rays, fwd=ident, margin=True)
    hs = oracle.trace_scene(sc, rays, static=True, margin=True)
    ok = _ok(ha) & _ok(hs)
    np.testing.assert_array_equal(ha.id[ok], hs.id[ok])
    np.testing.assert_array_equal(ha.t[ok], hs.t[ok])


# ---------------------------------------------------------------- P3 pre-transformed voxels

def _revoxelise(occ, level, xyz, A):
    """Static occupancy with the cell's voxels moved by the lattice map A."""
    n = occ.shape[0]
    K = int(np.log2(n))
    s = 1 << (K - level)
    lo = np.asarray(xyz) * s
    out = occ.copy()
    block = occ[lo[0]:lo[0] + s, lo[1]:lo[1] + s, lo[2]:lo[2] + s].copy()
    out[lo[0]:lo[0] + s, lo[1]:lo[1] + s, lo[2]:lo[2] + s] = False
    M = A[:, :3]
    scale = int(round(abs(np.linalg.det(M)) ** (1.0 / 3.0)))
    vox = np.argwhere(block) + lo
    for v in vox:
        for dx in range(scale):
            for dy in range(scale):
                for dz in range(scale):
                    # image of sub-cell centres of voxel v under A
                    c = v + (np.array([dx, dy, dz]) + 0.5) / scale
                    w = M @ c + A[:, 3]
                    q = np.floor(w).astype(int)
                    assert np.all(q >= 0) and np.all(q < n), "moved voxel leaves the grid"
                    out[q[0], q[1], q[2]] = True
    return out


def _lattice_cases():
    R90y = np.array([[0, 0, 1], [0, 1, 0], [-1, 0, 0]], float)
    R90x = np.array([[1, 0, 0], [0, 0, -1], [0, 1, 0]], float)
    R180z = np.array([[-1, 0, 0], [0, -1, 0], [0, 0, 1]], float)
    R270y = R90y.T
    return [("rot90y", R90y, (0, 0, 0), 1), ("rot90x", R90x, (0, 0, 0), 1), ("rot180z", R180z, (0, 0, 0), 1),
            ("rot270y_shift", R270y, (2, -3, 1), 1), ("shift", np.eye(3), (3, 1, -2), 1),
            ("scale2", 2 * np.eye(3), (0, 0, 0), 2)]


@pytest.mark.parametrize("case", _lattice_cases(), ids=lambda c: c[0])
def test_p3_pretransformed_voxels(case, oracle_lib):
    name, M, shift, scale = case
    K = 5
    level = 2  # cells of 8 voxels
    s = 1 << (K - level)
    # sparse world, and a denser pattern in the transformed cell so its moved copy is visible
    occ = S.blob_occupancy(K, 7, 0.15)
    xyz = (1, 1, 1) if scale == 1 else (1, 0, 1)
    block = S.blob_occupancy(3, 8, 0.5)
    assert 0 < block.sum() < block.size
    occ[xyz[0] * s:(xyz[0] + 1) * s, xyz[1] * s:(xyz[1] + 1) * s, xyz[2] * s:(xyz[2] + 1) * s] = block
    lo = np.asarray(xyz, float) * s
    pivot = lo + s / 2.0 if scale == 1 else lo
    A = xf.about_pivot(M, pivot, shift)
    moved = _revoxelise(occ, level, xyz, A)
    anim = S.from_occupancy(occ, [(level, xyz)], xf.to_f32(A).reshape(1, 12))
    stat = S.from_occupancy(moved, [], np.zeros((0, 12)))
    corners = lo + s * bf.CORNERS
    img = corners @ A[:, :3].T + A[:, 3]
    rays = S.random_rays(11, 2000, 0.0, 32.0, target_lo=img.min(0) - 1, target_hi=img.max(0) + 1)
    ha = oracle.trace_scene(anim, rays, margin=True)
    hs = oracle.trace_scene(stat, rays, margin=True)
    ok = _ok(ha) & _ok(hs)
    assert ok.mean() > 0.95
    np.testing.assert_array_equal(ha.id[ok] == NONE, hs.id[ok] == NONE)
    hit = ok & (ha.id != NONE)
    np.testing.assert_allclose(ha.t[hit], hs.t[hit], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(ha.normal[hit], hs.normal[hit], atol=1e-12)
    assert (ha.inst[hit] == 0).sum() > 30


# ---------------------------------------------------------------- P4 translation

def test_p4_translation_is_shifted_origin(oracle_lib):
    K, level = 5, 1
    occ = S.blob_occupancy(K, 9, 0.4)
    tree = ot.build_tree(K, ot.dense_classifier(occ)[0])
    cands = [tuple(int(v) for v in tree.coord[j]) for j in np.nonzero((tree.level == level) & (tree.kind == ot.PARTIAL))[0]]
    xyz = cands[0]
    s = 1 << (K - level)
    tau = np.array([1.375, -2.25, 0.625])  # dyadic: o - tau stays exact in float32
    A = xf.about_pivot(np.eye(3), np.zeros(3), tau)
    anim = S.from_occupancy(occ, [(level, xyz)], xf.to_f32(A).reshape(1, 12))
    lo = np.asarray(xyz) * s
    sub = occ[lo[0]:lo[0] + s, lo[1]:lo[1] + s, lo[2]:lo[2] + s]
    alone = ot.build_tree(K - level, ot.dense_classifier(sub)[0])
    rng = np.random.default_rng(4)
    n = 1500
    o = np.round(rng.uniform(-16, 48, (n, 3)) * 64) / 64
    tgt = rng.uniform(0, 32, (n, 3))
    d = (tgt - o)
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    rays = np.zeros((n, 8), np.float32)
    rays[:, :3] = o
    rays[:, 4:7] = d
    rays[:, 7] = np.inf
    shifted = rays.copy()
    shifted[:, :3] = (o - tau).astype(np.float32)
    assert np.all(shifted[:, :3].astype(np.float64) == o - tau)
    ha = oracle.trace_scene(anim, rays, margin=True)
    hc = oracle.trace(alone.nodes, 0, lo.astype(np.float64), float(s), np.zeros(0, np.uint32), np.zeros((0, 4)),
                      np.zeros((0, 12)), shifted, margin=True)
    ok = _ok(ha) & _ok(hc)
    inslot = ok & (ha.inst == 0)
    assert inslot.sum() > 50
    np.testing.assert_allclose(ha.t[inslot], hc.t[inslot], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(ha.normal[inslot], hc.normal[inslot], atol=1e-12)
    other = ok & (ha.inst != 0) & np.isfinite(hc.t)
    assert np.all(hc.t[other] >= ha.t[other] - 1e-9)


# ---------------------------------------------------------------- P5 the paper's form

@pytest.mark.parametrize("seed", [1, 2, 3, 5, 8])
def test_p5_paper_form_equals_affine_inverse(seed, oracle_lib):
    K = 5
    occ = S.blob_occupancy(K, seed, 0.4)
    tree = ot.build_tree(K, ot.dense_classifier(occ)[0])
    st = S.Stream(seed, 99)
    cands = np.nonzero((tree.kind == ot.PARTIAL) & (tree.level == 2))[0]
    picks = []
    for j in cands[st.integers(12, 0, cands.shape[0])]:
        if int(j) not in picks:
            picks.append(int(j))
        if len(picks) == 3:
            break
    cells = [(2, tuple(int(v) for v in tree.coord[j])) for j in picks]
    rot, scl, piv, tau, fwd = [], [], [], [], []
    for (l, xyz) in cells:
        R = xf.random_rotation(st)
        sc_ = 2.0 ** st.uniform(3, -1.0, 1.0)
        c = (np.asarray(xyz, float) + 0.5) * 8.0
        t = st.uniform(3, -3, 3)
        A = np.zeros((3, 4))
        A[:, :3] = R * sc_[None, :]          # x -> R S (x - c) + c + t
        A[:, 3] = c + t - A[:, :3] @ c
        rot.append(R.reshape(9)); scl.append(sc_); piv.append(c); tau.append(t)
        fwd.append(A.reshape(12))
    anim = S.from_occupancy(occ, cells, np.zeros((len(cells), 12)))
    rays = S.random_rays(seed + 40, 2000, 0.0, 32.0)
    # both sides take the same float64 data: forward R S for the general inverse,
    # R, S, c, t for the paper form
    h = oracle.trace_scene(anim, rays, fwd=np.array(fwd), fwd_f64=True, margin=True)
    hp = oracle.trace_paper_form(anim.nodes, 0, anim.root_min, anim.root_size, anim.slot_child, anim.slot_cell,
                                 np.array(rot), np.array(scl), np.array(piv), np.array(tau), rays)
    ok = _ok(h)
    assert ok.mean() > 0.95
    np.testing.assert_array_equal(h.id[ok], hp.id[ok])
    np.testing.assert_array_equal(h.inst[ok], hp.inst[ok])
    fin = ok & (h.id != NONE)
    assert (h.inst[fin] != NONE).sum() > 50
    np.testing.assert_allclose(h.t[fin], hp.t[fin], rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(h.normal[fin], hp.normal[fin], atol=1e-11)


# ---------------------------------------------------------------- P6 closed forms

def _leaf_pool():
    return np.array([np.uint64(0xFF00FF00) << np.uint64(32)], dtype=np.uint64)


def _one(o, d, tmin=0.0, tmax=np.inf, root_min=(0.0, 0.0, 0.0), size=8.0):
    r = np.array([[*o, tmin, *d, tmax]], np.float32)
    h = oracle.trace(_leaf_pool(), 0, np.asarray(root_min, float), size, np.zeros(0, np.uint32), np.zeros((0, 4)),
                     np.zeros((0, 12)), r)
    return h.id[0], h.t[0], h.normal[0]


def test_p6_single_box_closed_forms(oracle_lib):
    assert _one((-3, 2.5, 4.25), (1, 0, 0))[1:2] == (3.0,)
    i, t, n = _one((-3, 2.5, 4.25), (1, 0, 0))
    assert i == 0 and t == 3.0 and tuple(n) == (-1.0, 0.0, 0.0)
    i, t, n = _one((10, 1, 1), (-1, 0, 0))
    assert t == 2.0 and tuple(n) == (1.0, 0.0, 0.0)
    i, t, n = _one((4, 20, 4), (0, -2, 0))
    assert t == 6.0 and tuple(n) == (0.0, 1.0, 0.0)
    i, t, n = _one((4, 4, 4), (0.6, 0.0, 0.8))        # origin inside: t = tmin, no normal
    assert t == 0.0 and tuple(n) == (0.0, 0.0, 0.0)
    assert _one((-3, 9, 4), (1, 0, 0))[0] == NONE      # passes above
    assert _one((-3, 2.5, 4.25), (1, 0, 0), tmax=2.5)[0] == NONE
    assert _one((-3, 2.5, 4.25), (1, 0, 0), tmax=3.0)[1] == 3.0   # closed box, t = tmax
    assert _one((-3, 2.5, 4.25), (1, 0, 0), tmin=12.0)[0] == NONE
    i, t, n = _one((-3, 2.5, 4.25), (1, 0, 0), tmin=5.0)          # starts inside at tmin
    assert t == 5.0 and tuple(n) == (0.0, 0.0, 0.0)
    # box [1,5]x[0,4]x[2,6]: x entry at 6/0.8 = 7.5, z entry at 5/0.6 = 8.33 -> enters through z = 2
    i, t, n = _one((-5, 1, -3), (0.8, 0.0, 0.6), root_min=(1.0, 0.0, 2.0), size=4.0)
    assert abs(t - 5.0 / float(np.float32(0.6))) < 1e-12 and tuple(n) == (0.0, 0.0, -1.0)
    # non-finite and degenerate rays miss
    assert _one((np.nan, 0, 0), (1, 0, 0))[0] == NONE
    assert _one((0, 0, 0), (0, 0, 0))[0] == NONE
    assert _one((-3, 2.5, 4.25), (1, 0, 0), tmin=4.0, tmax=3.0)[0] == NONE


def test_p6_heightfield_columns_exact(oracle_lib):
    K = 5
    n = 1 << K
    rng = np.random.default_rng(12)
    H = rng.integers(0, n, (n, n))
    tree = ot.build_tree(K, ot.heightfield_classifier(H, K))
    xs, zs = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    xs, zs = xs.ravel(), zs.ravel()
    top = 40.0
    rays = np.zeros((xs.size, 8), np.float32)
    rays[:, 0] = xs + 0.5
    rays[:, 1] = top
    rays[:, 2] = zs + 0.5
    rays[:, 5] = -1.0
    rays[:, 7] = np.inf
    h = oracle.trace(tree.nodes, 0, np.zeros(3), float(n), np.zeros(0, np.uint32), np.zeros((0, 4)), np.zeros((0, 12)), rays)
    Hc = H[xs, zs]
    hit = Hc > 0
    assert np.all(h.id[~hit] == NONE)
    np.testing.assert_array_equal(h.t[hit], top - Hc[hit])
    np.testing.assert_array_equal(h.normal[hit], np.tile([0.0, 1.0, 0.0], (hit.sum(), 1)))
    # the same columns traced upwards from below the ground hit y = 0 ... only if H > 0
    up = rays.copy()
    up[:, 1] = -3.0
    up[:, 5] = 1.0
    hu = oracle.trace(tree.nodes, 0, np.zeros(3), float(n), np.zeros(0, np.uint32), np.zeros((0, 4)), np.zeros((0, 12)), up)
    np.testing.assert_array_equal(hu.t[hit], np.full(hit.sum(), 3.0))


def test_p6_voxelised_sphere_bounds(oracle_lib):
    K, R = 6, 24.0
    n = 1 << K
    g = np.arange(n) + 0.5
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    occ = np.sqrt((X - 32) ** 2 + (Y - 32) ** 2 + (Z - 32) ** 2) < R
    tree = ot.build_tree(K, ot.dense_classifier(occ)[0])
    sc = S.noisy_sphere_d6()
    rays, _ = sc.rays(W=96, H=96)
    h = oracle.trace(tree.nodes, 0, np.zeros(3), float(n), np.zeros(0, np.uint32), np.zeros((0, 4)), np.zeros((0, 12)), rays)
    o = rays[:, :3].astype(np.float64)
    d = rays[:, 4:7].astype(np.float64)
    c = np.array([32.0, 32.0, 32.0])

    def sphere_t(rad):
        oc = o - c
        b = np.einsum("ij,ij->i", oc, d)
        cc = np.einsum("ij,ij->i", oc, oc) - rad * rad
        aa = np.einsum("ij,ij->i", d, d)
        disc = b * b - aa * cc
        with np.errstate(invalid="ignore"):
            return np.where(disc >= 0, (-b - np.sqrt(np.maximum(disc, 0))) / aa, np.inf)

    half_diag = np.sqrt(3.0) / 2
    t_in = sphere_t(R - half_diag)
    t_out = sphere_t(R + half_diag)
    hit = h.id != NONE
    assert np.all(hit[np.isfinite(t_in)])
    assert not np.any(hit[~np.isfinite(t_out)])
    assert np.all(h.t[hit] >= t_out[hit] - 1e-9)
    assert np.all(h.t[np.isfinite(t_in)] <= t_in[np.isfinite(t_in)] + 1e-9)
    p = o[hit] + h.t[hit][:, None] * d[hit]
    r = np.linalg.norm(p - c, axis=1)
    assert np.all(r >= R - half_diag - 1e-9) and np.all(r <= R + half_diag + 1e-9)


# ---------------------------------------------------------------- P8 t scaling

def test_p8_t_scales_inversely_with_direction(oracle_lib):
    sc = S.tiny_scene(4, K=5, n_slots=3, nested=True, translate=0.2)
    rays = S.random_rays(77, 1500, 0.0, sc.root_size)
    rays[:, 4:7] = np.round(rays[:, 4:7] * 1024) / 1024      # few mantissa bits: 3 d is exact
    scaled = rays.copy()
    scaled[:, 4:7] = rays[:, 4:7] * 3.0
    assert np.all(scaled[:, 4:7].astype(np.float64) == 3.0 * rays[:, 4:7].astype(np.float64))
    h1 = oracle.trace_scene(sc, rays, margin=True)
    h3 = oracle.trace_scene(sc, scaled, margin=True)
    ok = _ok(h1) & _ok(h3)
    np.testing.assert_array_equal(h1.id[ok], h3.id[ok])
    fin = ok & (h1.id != NONE)
    np.testing.assert_allclose(h3.t[fin] * 3.0, h1.t[fin], rtol=1e-12)
    np.testing.assert_allclose(h3.normal[fin], h1.normal[fin], atol=1e-12)


# ---------------------------------------------------------------- grazing margin

def test_margin_flags_edge_rays(oracle_lib):
    i_leaf = _leaf_pool()
    rays = np.array([
        [-3, 2.5, 4.25, 0, 1, 0, 0, np.inf],     # through the middle of a face
        [-3, 8.0, 4.0, 0, 1, 0, 0, np.inf],      # along the top face plane (touches)
        [-3, 8.000002, 4.0, 0, 1, 0, 0, np.inf],  # one float32 ulp pair above: near miss
        [-3, -3, 4.0, 0, 0.70710678, 0.70710678, 0, np.inf],  # through the edge x=0,y=0
    ], np.float32)
    h = oracle.trace(i_leaf, 0, np.zeros(3), 8.0, np.zeros(0, np.uint32), np.zeros((0, 4)), np.zeros((0, 12)), rays,
                     margin=True)
    assert h.margin[0] > 1e-6 and h.margin_n[0] > 1e-6
    assert h.margin[1] < 1e-6 and h.id[1] == 0
    assert h.margin[2] < 1e-6 and h.id[2] == NONE
    # through the edge into the interior: one box either way, so the id is
    # not in doubt, only the entry face (normal)
    assert h.id[3] == 0 and h.margin[3] > 1e-6 and h.margin_n[3] < 1e-6


def test_p6_closed_box_edge_contact_hits(oracle_lib):
    s = np.float32(np.sqrt(0.5))
    # enters through the edge x = 0, y = 0 and crosses the interior
    i, t, n = _one((-3, -3, 4), (s, s, 0))
    assert i == 0 and t == 3.0 / float(s)
    assert tuple(n) == (-1.0, 0.0, 0.0)        # entry-axis tie goes to the lower axis
    # touches the box only at the edge x = 0, y = 0: a closed box still counts it
    i, t, n = _one((-3, 3, 4), (s, -s, 0))
    assert i == 0 and t == 3.0 / float(s)
    assert tuple(n) == (-1.0, 0.0, 0.0)
    # the same line shifted by one float32 step misses
    assert _one((-3, np.nextafter(np.float32(3), np.float32(0)), 4), (s, -s, 0))[0] == NONE


def test_far_pointers_decode_identically(oracle_lib):
    sc = S.tiny_scene(6, K=5, n_slots=3, nested=True)
    rays = S.random_rays(5, 1500, 0.0, sc.root_size)
    h = oracle.trace_scene(sc, rays)
    for every in (1, 3):
        far = ot.force_far(sc.nodes, every)
        assert np.any(far != sc.nodes)
        hf = oracle.trace(far, sc.root, sc.root_min, sc.root_size, sc.slot_child, sc.slot_cell, sc.xform(0), rays)
        np.testing.assert_array_equal(hf.id, h.id)
        np.testing.assert_array_equal(hf.t, h.t)


def _eq4_rejects(c, r, o, d, tmin, tmax):
    """Eq. 4 (Sec. 4.1) as read for an unnormalised direction: the squared
    distance of the ray line from the centre is l.l - (l.d)^2 / (d.d) with
    l = c - o; a sphere is rejected when that exceeds r^2, or when its chord
    lies wholly before tmin or after tmax."""
    l = c - o
    dd = (d * d).sum(-1)
    tca = (l * d).sum(-1)
    perp2 = np.maximum((l * l).sum(-1) - tca * tca / dd, 0.0)
    miss = perp2 > r * r
    half = np.sqrt(np.maximum(r * r - perp2, 0.0) / dd)
    tc = tca / dd
    return miss | (tc + half < tmin) | (tc - half > tmax)


def _segment_meets(C, o, d, tmin, tmax):
    """Exact segment vs parallelepiped (corners C [8, 3]) by clipping against
    its six face planes."""
    P, N = bf._faces(C[None])
    P, N = P[0], N[0]
    dn = d @ N.T                                   # [n, 6]
    num = np.einsum("fk,nfk->nf", N, P[None] - o[:, None, :])
    with np.errstate(divide="ignore", invalid="ignore"):
        tt = num / dn
    tn = np.where(dn < 0, tt, -np.inf).max(1)
    tf = np.where(dn > 0, tt, np.inf).min(1)
    par_out = ((dn == 0) & (num < 0)).any(1)
    return ~par_out & (np.maximum(tn, tmin) <= np.minimum(tf, tmax))


def test_p7_eq4_sphere_never_drops_a_hit():
    """P7: the bounding-sphere cull (centre = image of the cell centre,
    radius = distance to the farthest image corner) never rejects a ray
    segment that meets the moved cell, over random affine maps (rotation,
    anisotropic scale, shear, translation) and random rays, many of them
    aimed at the cell's corners.  The other reading of the centre (the map's
    translation, i.e. the image of the cell's origin corner) does drop hits."""
    rng = np.random.default_rng(17)
    hits = rejected = dropped_other = 0
    for trial in range(300):
        A = rng.normal(size=(3, 3)) * rng.uniform(0.3, 3.0, size=3)
        if abs(np.linalg.det(A)) < 1e-2:
            continue
        b = rng.uniform(-50, 50, 3)
        lo = rng.uniform(-8, 8, 3)
        size = rng.uniform(0.5, 16)
        C = (lo + size * bf.CORNERS) @ A.T + b
        c = (lo + 0.5 * size) @ A.T + b
        r = np.linalg.norm(C - c, axis=1).max()
        n = 256
        # half aimed at points near the corners (inside the cell), half random
        k = rng.integers(0, 8, n)
        w = rng.uniform(0.0, 0.05, (n, 1))
        target = C[k] * (1 - w) + c * w
        rand = rng.uniform(-2, 2, (n, 3)) * r + c
        target[n // 2:] = rand[n // 2:]
        d = rng.normal(size=(n, 3)) * rng.uniform(0.1, 10.0, (n, 1))
        back = rng.uniform(0.1, 4.0, (n, 1)) * r / np.linalg.norm(d, axis=1, keepdims=True)
        o = target - back * d
        tmin = np.where(rng.random(n) < 0.3, rng.uniform(0, 2, n) * back[:, 0], 0.0)
        tmax = np.where(rng.random(n) < 0.3, rng.uniform(0, 3, n) * back[:, 0], np.inf)
        meet = _segment_meets(C, o, d, tmin, tmax)
        rej = _eq4_rejects(c, r, o, d, tmin, tmax)
        assert not (meet & rej).any(), trial
        hits += int(meet.sum())
        rejected += int(rej.sum())
        dropped_other += int((meet & _eq4_rejects(b + lo @ A.T, r, o, d, tmin, tmax)).sum())
    assert hits > 10000 and rejected > 10000     # neither side of the test is vacuous
    assert dropped_other > 0


def test_shade_hand_worked_example():
    """Shading pin, worked by hand: leaf colour (200, 100, 50); a pixel with
    two samples, one a miss on black, one a hit with 1 of k = 2 AO rays
    blocked and F = 200 per mille: weight (200*2 + 800*1)/2000 = 0.6, so the
    hit sample is (120, 60, 30) and the pixel mean (60, 30, 15)."""
    leaf = np.uint64((0xFF << 24 | 50 << 16 | 100 << 8 | 200)) << np.uint64(32)
    nodes = np.array([np.uint64(0x1), leaf], np.uint64)         # node 1: a leaf (mask 0)
    NONE = 0xFFFFFFFF
    # 1x1 image, 2 samples: sample 0 misses, sample 1 hits node 1
    img = oracle.shade(nodes, [NONE, 1], [0, 0, 0, NONE], 1, 1, 2, 2, 200, 0xFF000000, [0])
    assert int(img[0, 0]) == (0xFF << 24 | 15 << 16 | 30 << 8 | 60)
    # no AO: the leaf colour itself; all AO blocked: colour * F / 1000 (rounded half up)
    assert int(oracle.shade(nodes, [1], None, 1, 1, 1, 0, 200, 0, [0])[0, 0]) == (0xFF << 24 | 50 << 16 | 100 << 8 | 200)
    img = oracle.shade(nodes, [1], [3, 4, 5], 1, 1, 1, 3, 333, 0, [0])
    assert int(img[0, 0]) == (0xFF << 24 | 17 << 16 | 33 << 8 | 67)   # 200*.333=66.6, 100*.333=33.3, 50*.333=16.65
    # a step-limit id is no node: background
    assert int(oracle.shade(nodes, [0xFFFFFFFE], None, 1, 1, 1, 0, 200, 0xFF0A0B0C, [0])[0, 0]) == 0xFF0A0B0C


def test_shade_places_pixels_in_tile_order():
    from svogen import camera as cam
    W, H = 13, 10
    pix = cam.pixel_order(W, H, "tiles")
    nodes = np.zeros(W * H, np.uint64)
    nodes[:] = (np.arange(W * H, dtype=np.uint64) | np.uint64(0xFF000000)) << np.uint64(32)   # colour = node index
    img = oracle.shade(nodes, np.arange(W * H), None, W, H, 1, 0, 0, 0, pix)
    # ray p hit node p, whose colour encodes p: the pixel at pix[p] holds p
    flat = img.reshape(-1) & 0xFFFFFF
    assert np.array_equal(flat[pix], np.arange(W * H))
