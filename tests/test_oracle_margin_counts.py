"""Pins for the oracle's grazing margins inside moved frames and for its node
and frame counters.

Margins.  The margin of a ray is a t gap divided by the frame's coordinate
scale S = max(|o_F|inf, |o_F + t d_F|inf, 1) / |d_F|inf, computed in the
local coordinates of the frame the gap belongs to (Eq. 2: the local ray keeps
the world parameter t).  Each case below is designed in the local frame of a
rotated, anisotropically scaled and translated slot, where the gap is known
by construction (a ray passing a chosen distance from a moved voxel's face,
two parallel faces a chosen t apart, two entry planes a chosen t apart); the
world ray is the forward image of that local ray, rounded to float32.  The
oracle maps it back with its own inverse, and its margin must equal the
designed gap over the designed S to 1 %.  A term dropped from S (the hit
point, the local origin, the direction norm), S taken in world instead of
local coordinates, or a near miss skipped inside a slot frame changes the
value by far more than that.

The id margin (gaps that can change which leaf is hit) and the normal margin
(which also holds the entry-face gaps) are checked apart.

Counters.  On a hand-drawn depth-2 tree, node records read and frames entered
are counted by hand for each ray: a frame entered counts its root record,
then its front-to-back descent reads one record per occupied child cell the
ray meets, up to its first leaf (transformed children are read and skipped);
the lower bound counts only frames entered by the final hit and cuts each at
it, the upper bound every frame the segment meets, each to its own first hit.
"""
import numpy as np
import pytest

import oracle
from svogen import scenes as S
from svogen import xforms as xf

NONE = 0xFFFFFFFF

# a slot at level 2 of a 16^3 world: static (and local root) cell [4, 8)^3,
# leaves of one unit
LEVEL, XYZ = 2, (1, 1, 1)
CENTRE = np.array([6.0, 6.0, 6.0])


def _general_map():
    R = xf.rot_axis_angle((1.0, 2.0, 3.0), 0.4)
    L = R @ np.diag([1.5, 0.75, 1.25])
    return xf.about_pivot(L, CENTRE, (0.3, -0.2, 0.1))


def _scene(voxels, A, world_voxels=()):
    occ = np.zeros((16, 16, 16), bool)
    for v in list(voxels) + list(world_voxels):
        occ[v] = True
    return S.from_occupancy(occ, [(LEVEL, XYZ)], xf.to_f32(A).reshape(1, 12))


def _world_ray(A, o_loc, d_loc, tmin=0.0, tmax=np.inf):
    """The forward image of a local ray, rounded to float32 (the ray the
    caller would pass)."""
    L, b = A[:, :3], A[:, 3]
    o = L @ np.asarray(o_loc, float) + b
    d = L @ np.asarray(d_loc, float)
    return np.array([[*o, tmin, *d, tmax]], np.float32)


def _trace(sc, ray, eps):
    return oracle.trace_scene(sc, ray, margin=True, margin_eps=eps)


def _scale(o_loc, d_loc, t):
    """max(|o_F|inf, |o_F + t d_F|inf, 1), the numerator of S, in the frame's
    local units; the gaps below are local distances, so margin = gap / this."""
    o = np.asarray(o_loc, float)
    d = np.asarray(d_loc, float)
    m = np.abs(o).max()
    if np.isfinite(t):
        m = max(m, np.abs(o + t * d).max())
    return max(m, 1.0)


def test_g1_hit_voxel_depth_in_moved_frame():
    """The ray runs through a moved voxel delta above its bottom face: the
    voxel can shrink by delta before the ray misses it."""
    A = _general_map()
    sc = _scene([(6, 4, 4)], A)
    delta = 0.01
    o_loc, d_loc = (2.0, 4.0 + delta, 4.5), (0.75, 0.0, 0.0)
    h = _trace(sc, _world_ray(A, o_loc, d_loc), 1e-2)
    assert h.inst[0] == 0 and h.id[0] != NONE
    t_hit = (6.0 - 2.0) / 0.75
    assert abs(h.t[0] - t_hit) < 1e-5
    want = delta / _scale(o_loc, d_loc, t_hit)             # the hit point (6, ...) sets the scale, not the origin
    np.testing.assert_allclose(h.margin[0], want, rtol=0.01)
    np.testing.assert_allclose(h.margin_n[0], want, rtol=0.01)


def test_g3_near_miss_in_moved_frame_missing_ray():
    """The ray passes a moved voxel delta below its bottom face and hits
    nothing: the near miss sets the margin, with the scale taken where the
    ray leaves the frame's root cell."""
    A = _general_map()
    sc = _scene([(6, 5, 4)], A)
    delta = 0.004
    o_loc, d_loc = (2.0, 5.0 - delta, 4.5), (0.75, 0.0, 0.0)
    h = _trace(sc, _world_ray(A, o_loc, d_loc), 1e-2)
    assert h.id[0] == NONE
    t_exit = (8.0 - 2.0) / 0.75                             # x = 8, the root cell's far face
    want = delta / _scale(o_loc, d_loc, t_exit)
    np.testing.assert_allclose(h.margin[0], want, rtol=0.01)
    # the same ray 10 delta further away: the gap is no longer resolved at
    # this eps, then resolved at a larger one
    o_far = (2.0, 5.0 - 10 * delta, 4.5)
    h2 = _trace(sc, _world_ray(A, o_far, d_loc), 1e-4)
    assert h2.margin[0] == np.inf
    h3 = _trace(sc, _world_ray(A, o_far, d_loc), 1e-1)
    np.testing.assert_allclose(h3.margin[0], 10 * delta / _scale(o_far, d_loc, t_exit), rtol=0.01)


def test_g2_runner_up_in_moved_frame():
    """A world voxel is hit first; a moved voxel is entered tau later through
    a parallel face (the slot rotates about x and scales x by 1.5, so its x
    faces stay parallel to the world's).  The runner-up gap is measured with
    the moved frame's own scale at the hit."""
    theta, sx = 0.5, 1.5
    c, s_ = np.cos(theta), np.sin(theta)
    Rx = np.array([[1, 0, 0], [0, c, -s_], [0, s_, c]])
    L = Rx @ np.diag([sx, 0.75, 1.25])
    tau = 2.0 ** -7
    wx = 3.0                                               # world voxel [3, 4) in x, outside the static cell
    # M = local [6, 7] x [4, 5] x [4, 5]; its x = 6 face lands at world x = 6 + tx
    tx = wx - 6.0 + tau
    # place M's cross-section centre (local y = z = 4.5) on a world voxel centre
    yz = Rx[1:, 1:] @ (np.diag([0.75, 1.25]) @ (np.array([4.5, 4.5]) - 6.0)) + 6.0
    ty, tz = np.floor(yz) + 0.5 - yz
    A = xf.about_pivot(L, CENTRE, (tx, ty, tz))
    wv = (int(wx), int(np.floor(yz[0] + ty)), int(np.floor(yz[1] + tz)))
    sc = _scene([(6, 4, 4)], A, world_voxels=[wv])
    # local ray along local x through M's cross-section centre, starting where
    # the world x is 0: world direction (1, 0, 0) exactly
    u = 6.0 - (6.0 + tx) / sx
    o_loc, d_loc = (u, 4.5, 4.5), (1.0 / sx, 0.0, 0.0)
    ray = _world_ray(A, o_loc, d_loc)
    np.testing.assert_array_equal(ray[0, 4:7], [1.0, 0.0, 0.0])
    h = _trace(sc, ray, 1e-2)
    assert h.inst[0] == NONE and h.id[0] != NONE           # the world voxel
    t_w = wx - float(ray[0, 0])
    np.testing.assert_allclose(h.t[0], t_w, atol=1e-6)
    want = (tau * (1.0 / sx)) / _scale(o_loc, d_loc, t_w)  # t gap times |d_F|inf over the moved frame's scale
    np.testing.assert_allclose(h.margin[0], want, rtol=0.01)


def test_g5_entry_axis_tie_only_lowers_the_normal_margin():
    """The ray enters a moved voxel through its x face tau after entering its
    y slab: the entry face is ambiguous at that scale, the voxel is not."""
    A = _general_map()
    sc = _scene([(6, 4, 4)], A)
    tau = 0.02
    d_loc = (0.75, 0.3, 0.0)
    t_x = (6.0 - 2.0) / 0.75
    o_loc = (2.0, 4.0 - 0.3 * (t_x - tau), 4.5)            # y slab entered at t_x - tau
    h = _trace(sc, _world_ray(A, o_loc, d_loc), 1e-2)
    assert h.inst[0] == 0 and h.id[0] != NONE
    np.testing.assert_allclose(h.t[0], t_x, rtol=1e-6)
    want = tau * 0.75 / _scale(o_loc, d_loc, t_x)          # t gap times |d_F|inf over the scale
    np.testing.assert_allclose(h.margin_n[0], want, rtol=0.01)
    assert h.margin[0] > 10 * want                         # the id margin does not see it


def test_g4_start_near_entry_face_only_lowers_the_normal_margin():
    """tmin falls tau before the ray enters the moved voxel: whether the ray
    enters through a face or starts inside is ambiguous at that scale (the
    normal), which voxel it hits is not."""
    A = _general_map()
    sc = _scene([(6, 4, 4)], A)
    tau = 0.02
    o_loc, d_loc = (2.0, 4.5, 4.5), (0.75, 0.0, 0.0)
    t_x = (6.0 - 2.0) / 0.75
    h = _trace(sc, _world_ray(A, o_loc, d_loc, tmin=t_x - tau), 1e-2)
    assert h.inst[0] == 0 and h.id[0] != NONE
    want = tau * 0.75 / _scale(o_loc, d_loc, t_x)
    np.testing.assert_allclose(h.margin_n[0], want, rtol=0.01)
    assert h.margin[0] > 10 * want


# ---------------------------------------------------------------- counters

def _count_scene(slot_map=None):
    """Depth 2 (4^3 world, unit leaves).  Octant 0 of the root ([0,2)^3) is
    solid and collapses to one leaf; octant 1 ([2,4)x[0,2)x[0,2)) holds the
    single voxel (3,0,0); octant 7 ([2,4)^3) is transformed node slot 0 with
    voxels (2,2,2) and (3,3,3); the other octants are empty."""
    occ = np.zeros((4, 4, 4), bool)
    occ[0:2, 0:2, 0:2] = True
    occ[3, 0, 0] = True
    occ[2, 2, 2] = True
    occ[3, 3, 3] = True
    A = xf.identity() if slot_map is None else slot_map
    return S.from_occupancy(occ, [(1, (1, 1, 1))], xf.to_f32(A).reshape(1, 12))


def _rays(spec):
    return np.array([[*o, tmin, *d, tmax] for o, d, tmin, tmax in spec], np.float32)


def test_count_pool_shape():
    sc = _count_scene()
    nodes = sc.nodes
    # root, its three children (leaf, interior, transformed), the voxel of
    # octant 1, the two voxels of the slot
    assert nodes.shape[0] == 7
    assert int(nodes[0]) & 0xFF == 0b10000011


@pytest.mark.parametrize("slot_map", [None, xf.about_pivot(np.eye(3), (3.0, 3.0, 3.0), (0.0, 0.0, 0.0))])
def test_counts_by_hand(slot_map):
    sc = _count_scene(slot_map)
    inf = np.inf
    rays = _rays([
        # 1: +x at y = z = 0.5 from x = -1: world root (1) + octant-0 leaf (1), a hit at t = 1; the slot's
        #    root cell [2,4)^3 is never met
        ((-1.0, 0.5, 0.5), (1.0, 0.0, 0.0), 0.0, inf),
        # 2: starts inside octant 1 at x = 2.5: root (1) + octant 1 (1) + voxel (3,0,0) (1), a hit at t = 0.5
        ((2.5, 0.5, 0.5), (1.0, 0.0, 0.0), 0.0, inf),
        # 3: +x at y = z = 2.5: world root (1) + the transformed octant 7 (1, read and skipped); slot root (1)
        #    + voxel (2,2,2) (1), a hit at t = 3 in the slot; both frames entered by then
        ((-1.0, 2.5, 2.5), (1.0, 0.0, 0.0), 0.0, inf),
        # 4: diagonal: hits the octant-0 leaf at t = 1 (root + leaf = 2); the slot is entered only at t = 3,
        #    past the hit (upper bound: + slot root + voxel (2,2,2) = 4, 2 frames)
        ((-1.0, -0.8, -0.9), (1.0, 1.0, 1.0), 0.0, inf),
        # 5: +z at x = 2.5, y = 0.5: root (1) + octant 1 (1), whose occupied voxel the ray never meets; a miss
        ((2.5, 0.5, -1.0), (0.0, 0.0, 1.0), 0.0, inf),
        # 6: ray 1 stopped before the world: nothing entered
        ((-1.0, 0.5, 0.5), (1.0, 0.0, 0.0), 0.0, 0.5),
        # 7: starts inside the world, heading down: the world descent reads the transformed octant 7 at t = 1,
        #    where the slot's voxel (2,2,2) is hit (slot root + voxel = 2); past t = 1 the world would go on to
        #    octant 1 (t = 1.5) and its voxel (3,0,0) (t = 2.5): lower 2 + 2, upper 4 + 2
        ((1.0, 3.5, 3.3), (1.0, -1.0, -1.0), 0.0, inf),
    ])
    h = oracle.trace_scene(sc, rays, counters=True)
    np.testing.assert_array_equal(h.nnode, [2, 3, 4, 2, 2, 0, 4])
    np.testing.assert_array_equal(h.nnode_hi, [2, 3, 4, 4, 2, 0, 6])
    np.testing.assert_array_equal(h.nframe, [1, 1, 2, 1, 1, 0, 2])
    np.testing.assert_array_equal(h.nframe_hi, [1, 1, 2, 2, 1, 0, 2])
    np.testing.assert_array_equal(h.id == NONE, [False, False, False, False, True, True, False])
    np.testing.assert_array_equal(h.inst[[0, 1, 2, 3, 6]], [NONE, NONE, 0, NONE, 0])
    np.testing.assert_allclose(h.t[[0, 1, 2, 3, 6]], [1.0, 0.5, 3.0, 1.0, 1.0], rtol=1e-6)


def test_counts_bound_each_other_and_single_frame_coincide():
    """lower <= upper always; on the static twin (one frame) they coincide."""
    sc = S.tiny_scene(3, K=5, n_slots=4, nested=True)
    rays = S.random_rays(21, 2000, 0.0, sc.root_size)
    h = oracle.trace_scene(sc, rays, counters=True)
    assert np.all(h.nnode <= h.nnode_hi) and np.all(h.nframe <= h.nframe_hi)
    assert np.any(h.nnode < h.nnode_hi)
    hs = oracle.trace_scene(sc, rays, static=True, counters=True)
    np.testing.assert_array_equal(hs.nnode, hs.nnode_hi)
    np.testing.assert_array_equal(hs.nframe, hs.nframe_hi)
    assert np.all(hs.nframe <= 1)
