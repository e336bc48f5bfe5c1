"""Brute-force ray vs every transformed voxel, in world space (test helper).

Independent of the oracle's arithmetic: no matrix is inverted or composed.
Each solid leaf box is turned into its world-space parallelepiped by pushing
its 8 corners through the chain of forward (local -> parent) maps one map at
a time, and the ray is clipped against the parallelepiped's 6 face planes
(Cyrus-Beck), with plane normals from cross products of its edges.
"""
from __future__ import annotations

import numpy as np

NONE = 0xFFFFFFFF
CORNERS = np.array([[i & 1, (i >> 1) & 1, (i >> 2) & 1] for i in range(8)], dtype=np.float64)


def apply_chain(points, slot, fwd, slot_parent):
    """Map local points of frame ``slot`` to world by applying each forward map."""
    p = points
    s = slot
    while s != NONE:
        A = np.asarray(fwd[s], np.float64).reshape(3, 4)
        p = p @ A[:, :3].T + A[:, 3]
        s = int(slot_parent[s])
    return p


def world_boxes(scene, fwd):
    """Per leaf: (frame slot or NONE, node index, corners [8,3] in world)."""
    out_slot, out_id, out_corners = [], [], []
    for f, (idx, mn, sz) in scene.frame_leaves().items():
        loc = mn[:, None, :] + sz[:, None, None] * CORNERS[None, :, :]
        w = apply_chain(loc.reshape(-1, 3), f, fwd, scene.slot_parent).reshape(-1, 8, 3) if f != NONE else loc
        out_slot.append(np.full(idx.shape[0], f, dtype=np.int64))
        out_id.append(idx.astype(np.int64))
        out_corners.append(w)
    return np.concatenate(out_slot), np.concatenate(out_id), np.concatenate(out_corners)


def _faces(C):
    """Outward face planes of parallelepipeds C [m,8,3]: points P [m,6,3], normals N [m,6,3]."""
    centre = C.mean(axis=1)
    P = np.empty((C.shape[0], 6, 3))
    N = np.empty((C.shape[0], 6, 3))
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        for side in range(2):
            k0 = side << a
            p0 = C[:, k0]
            u = C[:, k0 | (1 << b)] - p0
            v = C[:, k0 | (1 << c)] - p0
            n = np.cross(u, v)
            flip = np.einsum("ij,ij->i", n, p0 - centre) < 0
            n[flip] = -n[flip]
            P[:, 2 * a + side] = p0
            N[:, 2 * a + side] = n
    return P, N


def trace(scene, fwd, rays, chunk=256):
    """Nearest hit per ray by exhaustive clipping: (id, inst, t, normal)."""
    slots, ids, C = world_boxes(scene, fwd)
    P, N = _faces(C)
    m = ids.shape[0]
    rays = np.asarray(rays, np.float32).astype(np.float64)
    n = rays.shape[0]
    out_id = np.full(n, NONE, np.uint32)
    out_inst = np.full(n, NONE, np.uint32)
    out_t = np.full(n, np.inf)
    out_n = np.zeros((n, 3))
    inst_key = np.where(slots == NONE, NONE, slots).astype(np.int64)
    for a in range(0, n, chunk):
        r = rays[a:a + chunk]
        o = r[:, None, None, 0:3]
        d = r[:, None, None, 4:7]
        tmin = r[:, 3][:, None]
        tmax = r[:, 7][:, None]
        dn = np.einsum("bmfk,mfk->bmf", np.broadcast_to(d, (r.shape[0], m, 6, 3)), N)
        num = np.einsum("mfk,bmfk->bmf", N, P[None] - o)
        with np.errstate(divide="ignore", invalid="ignore"):
            tt = num / dn
        enter = dn < 0
        leave = dn > 0
        par_out = (dn == 0) & (num < 0)
        tn_f = np.where(enter, tt, -np.inf)
        tf_f = np.where(leave, tt, np.inf)
        tn = tn_f.max(axis=2)
        face = tn_f.argmax(axis=2)
        tf = tf_f.min(axis=2)
        ok = ~par_out.any(axis=2)
        te = np.maximum(tn, tmin)
        tx = np.minimum(tf, tmax)
        ok &= te <= tx
        te = np.where(ok, te, np.inf)
        # lexicographic min over (t, inst, id)
        order_t = te.min(axis=1)
        for b in range(r.shape[0]):
            if not np.isfinite(order_t[b]):
                continue
            cand = np.nonzero(ok[b] & (te[b] == order_t[b]))[0]
            key = np.lexsort((ids[cand], inst_key[cand]))
            j = cand[key[0]]
            out_id[a + b] = ids[j]
            out_inst[a + b] = slots[j] if slots[j] != NONE else NONE
            out_t[a + b] = te[b, j]
            if tn[b, j] >= r[b, 3]:
                nv = N[j, face[b, j]]
                out_n[a + b] = nv / np.linalg.norm(nv)
    return out_id, out_inst, out_t, out_n
