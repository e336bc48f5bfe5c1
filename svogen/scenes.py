"""Seeded synthetic scenes standing in for the paper's voxelised car model.

Every scene is a pool of 8-byte nodes plus a slot table (child group and
local root cell of every transformed subtree) and a function giving the
forward, parent-relative 3x4 transform of every slot at a given frame.

  noisy_sphere_d6   depth 6 (64^3) noisy sphere, one transformed level-1 node,
           128x128 pinhole rays                          (small parity case)
  fbm_terrain_d10   depth 10 (1024^3) fBm heightfield, 8 animated level-3 subtrees,
           1920x1080 pinhole rays, 60 frames           (headline workload)
  tiny     depth 3..5 random blobs with random nested transforms (pins)

World units are leaf voxels of the root grid.  Rotations and scales pivot on
the transformed cell's centre.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

from . import camera as cam
from . import octree as ot
from . import xforms as xf
from .hashing import Stream, hash_keys, to_unit
from .noise import fbm2, fbm3

NONE = 0xFFFFFFFF


@dataclass
class Scene:
    name: str
    nodes: np.ndarray                 # uint64 pool (transformed nodes flagged)
    static_nodes: np.ndarray          # uint64 pool with every transform cleared
    root: int
    root_min: np.ndarray              # float32 [3]
    root_size: float
    max_depth: int
    slot_child: np.ndarray            # uint32 [S]
    slot_cell: np.ndarray             # float32 [S, 4] local root cell (min xyz, size)
    slot_node: np.ndarray             # int64 [S] node carrying the slot
    slot_parent: np.ndarray           # uint32 [S] enclosing slot or NONE (metadata for tests)
    tree: ot.Tree                     # generation metadata of the pool
    xform: Callable[[int], np.ndarray]  # frame -> float32 [S, 12]
    camera: dict = field(default_factory=dict)
    seed: int = 0

    @property
    def n_slots(self) -> int:
        return int(self.slot_child.shape[0])

    def static_pool(self) -> np.ndarray:
        """The static twin (every transform cleared), built on first use."""
        if self.static_nodes is None:
            self.static_nodes = ot.clear_transformed(self.nodes, self.slot_child)
        return self.static_nodes

    def rays(self, W=None, H=None, order="tiles"):
        c = dict(self.camera)
        W = W or c["W"]
        H = H or c["H"]
        return cam.pinhole_rays(c["eye"], c["target"], c["up"], c["fov"], W, H, order=order)

    def frame_leaves(self):
        """Solid leaves per frame for brute-force checks.

        Returns {frame: (leaf index [n], box min [n,3], box size [n])} with
        frame = NONE for the world and the slot id otherwise; boxes are in the
        frame's local coordinates (equal to the static world cell here).
        """
        idx, mn, sz = ot.leaf_boxes(self.tree, self.root_min.astype(np.float64), float(self.root_size))
        lev = self.tree.level[idx]
        crd = self.tree.coord[idx]
        owner = np.full(idx.shape[0], NONE, dtype=np.int64)
        depth = np.full(idx.shape[0], -1, dtype=np.int64)
        for s in range(self.n_slots):
            nd = int(self.slot_node[s])
            ls = int(self.tree.level[nd])
            cs = self.tree.coord[nd]
            inside = (lev > ls) & np.all((crd >> (lev - ls)[:, None]) == cs[None, :], axis=1)
            better = inside & (ls > depth)
            owner[better] = s
            depth[better] = ls
        out = {}
        for f in np.unique(owner):
            m = owner == f
            out[int(f)] = (idx[m], mn[m], sz[m])
        return out


def _palette(level_y_frac, jitter):
    bands = np.array([[70, 110, 60], [110, 150, 70], [150, 130, 90], [120, 120, 120], [235, 235, 240]], float)
    b = np.clip((level_y_frac * len(bands)).astype(np.int64), 0, len(bands) - 1)
    rgb = np.clip(bands[b] + (jitter[:, None] - 0.5) * 24.0, 0, 255).astype(np.uint64)
    return rgb[:, 0] | (rgb[:, 1] << np.uint64(8)) | (rgb[:, 2] << np.uint64(16)) | (np.uint64(255) << np.uint64(24))


def _colour_fn(K, seed):
    def colour(l, c):
        s = 1 << (K - l)
        yfrac = (c[:, 1].astype(np.float64) + 0.5) * s / float(1 << K)
        jit = to_unit(hash_keys(c[:, 0], c[:, 1], c[:, 2], l, seed, 7))
        return _palette(yfrac, jit)
    return colour


def _slot_parents(tree, slot_node):
    S = len(slot_node)
    par = np.full(S, NONE, dtype=np.uint32)
    for s in range(S):
        ls = tree.level[slot_node[s]]
        cs = tree.coord[slot_node[s]]
        best = -1
        for q in range(S):
            lq = tree.level[slot_node[q]]
            if lq < ls and np.all((cs >> (ls - lq)) == tree.coord[slot_node[q]]) and lq > best:
                best = lq
                par[s] = q
    return par


def _marked_scene(name, tree, K, root_size, cells, xform, camera, seed):
    nodes, slot_child, slot_node = ot.mark_transformed(tree, cells)
    S = len(cells)
    slot_cell = np.zeros((S, 4), dtype=np.float32)
    unit = root_size / float(1 << K)
    for s, (l, xyz) in enumerate(cells):
        size = unit * (1 << (K - l))
        slot_cell[s, :3] = np.asarray(xyz, np.float64) * size
        slot_cell[s, 3] = size
    static = ot.clear_transformed(nodes, slot_child)
    return Scene(name=name, nodes=nodes, static_nodes=static, root=0,
                 root_min=np.zeros(3, np.float32), root_size=float(root_size), max_depth=K,
                 slot_child=slot_child, slot_cell=slot_cell, slot_node=slot_node,
                 slot_parent=_slot_parents(tree, slot_node), tree=tree, xform=xform,
                 camera=camera, seed=seed)


# ------------------------------------------------------------------ noisy sphere, depth 6

def noisy_sphere_d6(seed: int = 1) -> Scene:
    """Depth-6 noisy sphere; slot 0 on the level-1 node of octant 7 ([32,64)^3)
    rotated +30 deg about y through its centre (48,48,48), then moved (5,0,2)."""
    K = 6
    n = 1 << K
    g = np.arange(n, dtype=np.float64) + 0.5
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    r = np.sqrt((X - 32) ** 2 + (Y - 32) ** 2 + (Z - 32) ** 2)
    occ = 24.0 - r + 4.0 * fbm3(X, Y, Z, 3, 16.0, seed) > 0
    classify, _ = ot.dense_classifier(occ)
    tree = ot.build_tree(K, classify, _colour_fn(K, seed))
    A = xf.about_pivot(xf.rot_y(np.radians(30.0)), (48.0, 48.0, 48.0), (5.0, 0.0, 2.0))
    A32 = xf.to_f32(A).reshape(1, 12)

    def xform(frame: int = 0):
        return A32.copy()

    camera = dict(eye=(112.0, 96.0, 128.0), target=(32.0, 32.0, 32.0), up=(0.0, 1.0, 0.0), fov=45.0, W=128, H=128)
    return _marked_scene("sphere64", tree, K, float(n), [(1, (1, 1, 1))], xform, camera, seed)


# ------------------------------------------------------------------ fBm terrain, depth 10

def heightfield(K: int, seed: int, base: float, amp: float, octaves: int, period0: float):
    n = 1 << K
    g = np.arange(n, dtype=np.float64) + 0.5
    Xc, Zc = np.meshgrid(g, g, indexing="ij")
    h = base + amp * fbm2(Xc, Zc, octaves, period0, seed)
    return np.clip(np.ceil(h - 0.5), 0, n).astype(np.int64)


def fbm_terrain_d10(seed: int = 2, frames: int = 60) -> Scene:
    """Depth-10 fBm heightfield h = 512 + 256 fbm2 (6 octaves, P0 = 256); 8
    level-3 subtrees animated: rotation about a seeded axis by 2 pi k f/60
    (k in {1,2,3}) and per-axis scale 2^sin(2 pi f/60 + phase) about the cell
    centre."""
    K = 10
    H = heightfield(K, seed, 512.0, 256.0, 6, 256.0)
    tree = ot.build_tree(K, ot.heightfield_classifier(H, K), _colour_fn(K, seed))
    st = Stream(seed, 11)
    cand = np.nonzero((tree.level == 3) & (tree.kind == ot.PARTIAL))[0]
    pick = []
    while len(pick) < 8:
        j = int(cand[st.integers(1, 0, cand.shape[0])[0]])
        if j not in pick:
            pick.append(j)
    cells = [(3, tuple(int(v) for v in tree.coord[j])) for j in pick]
    size = float(1 << (K - 3))
    centres = [np.asarray(c[1], np.float64) * size + size / 2 for c in cells]
    axes = []
    for _ in range(8):
        a = st.normal(3)
        axes.append(a / np.linalg.norm(a))
    ks = st.integers(8, 1, 4)
    phases = st.uniform(24, 0.0, 2.0 * np.pi).reshape(8, 3)

    def xform(frame: int = 0):
        out = np.zeros((8, 12), np.float32)
        for j in range(8):
            R = xf.rot_axis_angle(axes[j], 2.0 * np.pi * ks[j] * frame / frames)
            s = 2.0 ** np.sin(2.0 * np.pi * frame / frames + phases[j])
            out[j] = xf.to_f32(xf.about_pivot(R @ np.diag(s), centres[j])).reshape(12)
        return out

    camera = dict(eye=(512.0, 1100.0, -400.0), target=(512.0, 500.0, 512.0), up=(0.0, 1.0, 0.0),
                  fov=60.0, W=1920, H=1080)
    return _marked_scene("terrain1024", tree, K, float(1 << K), cells, xform, camera, seed)


# ------------------------------------------------------------------ tiny scenes for pins

def tiny_scene(seed: int, K: int = 4, n_slots: int = 2, nested: bool = True, density: float = 0.35,
               scale_range=(0.5, 2.0), rotate: bool = True, translate: float = 0.0,
               root_size: Optional[float] = None) -> Scene:
    """Random blobby occupancy on a 2^K grid with random transformed nodes.

    Slots sit on interior nodes at levels 1..K-2; with ``nested`` a later slot
    may sit inside an earlier one's subtree.
    """
    n = 1 << K
    st = Stream(seed, 21)
    g = np.arange(n, dtype=np.float64) + 0.5
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    v = fbm3(X, Y, Z, 2, max(2.0, n / 2.0), seed)
    occ = v > (1.0 - 2.0 * density) * 0.5
    classify, _ = ot.dense_classifier(occ)
    tree = ot.build_tree(K, classify, _colour_fn(K, seed))
    if tree.n == 0:
        raise ValueError("empty tiny scene")
    rs = float(n) if root_size is None else float(root_size)
    cells = []
    used = []
    inter = (tree.kind == ot.PARTIAL) & (tree.level >= 1) & (tree.level <= max(1, K - 2))
    cand = np.nonzero(inter)[0]

    def related(j, q):
        lj, lq = int(tree.level[j]), int(tree.level[q])
        if lj == lq:
            return j == q
        lo, hi = (q, j) if lq < lj else (j, q)
        d = int(tree.level[hi]) - int(tree.level[lo])
        return bool(np.all((tree.coord[hi] >> d) == tree.coord[lo]))

    if nested and n_slots >= 2:
        # a chain: slot 1 sits inside slot 0's subtree (and slot 2 inside slot 1 when possible)
        top = np.nonzero(inter & (tree.level == 1))[0]
        j0 = int(top[st.integers(1, 0, top.shape[0])[0]])
        chain = [j0]
        while len(chain) < min(n_slots, 3):
            last = chain[-1]
            sub = [int(q) for q in cand if tree.level[q] > tree.level[last] and related(int(q), last)]
            if not sub:
                break
            chain.append(sub[int(st.integers(1, 0, len(sub))[0])])
        used.extend(chain)
    tries = 0
    while len(used) < n_slots and tries < 400 and cand.size:
        tries += 1
        j = int(cand[st.integers(1, 0, cand.shape[0])[0]])
        if any(related(j, q) for q in used):
            continue
        used.append(j)
    cells = [(int(tree.level[j]), tuple(int(x) for x in tree.coord[j])) for j in used]
    unit = rs / n
    centres = [(np.asarray(c[1], np.float64) + 0.5) * unit * (1 << (K - c[0])) for c in cells]
    mats = []
    for s in range(len(cells)):
        R = xf.random_rotation(st) if rotate else np.eye(3)
        lo, hi = np.log2(scale_range[0]), np.log2(scale_range[1])
        sc = 2.0 ** st.uniform(3, lo, hi)
        tr = st.uniform(3, -translate, translate) * unit * (1 << (K - cells[s][0])) if translate else np.zeros(3)
        mats.append(xf.to_f32(xf.about_pivot(R @ np.diag(sc), centres[s], tr)).reshape(12))
    M = np.array(mats, np.float32).reshape(-1, 12)

    def xform(frame: int = 0):
        return M.copy()

    sc = _marked_scene("tiny%d" % seed, tree, K, rs, cells, xform, {}, seed)
    return sc


def random_rays(seed: int, n: int, lo: float, hi: float, inside_frac: float = 0.2, tag: int = 31,
                target_lo=None, target_hi=None):
    """Rays aimed through the box [lo, hi]^3: origins on a sphere around it
    (or inside it for ``inside_frac``), directions to random target points in
    [target_lo, target_hi] (default: the box itself)."""
    st = Stream(seed, tag)
    c = 0.5 * (lo + hi)
    R = (hi - lo) * 1.2
    dirs = st.normal(3 * n).reshape(n, 3)
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    org = c + R * dirs
    inside = st.uniform(n) < inside_frac
    org[inside] = lo + (hi - lo) * st.uniform(3 * int(inside.sum())).reshape(-1, 3)
    tlo = np.full(3, lo, np.float64) if target_lo is None else np.asarray(target_lo, np.float64)
    thi = np.full(3, hi, np.float64) if target_hi is None else np.asarray(target_hi, np.float64)
    tgt = tlo + (thi - tlo) * st.uniform(3 * n).reshape(n, 3)
    d = tgt - org
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rays = np.zeros((n, 8), np.float32)
    rays[:, 0:3] = org
    rays[:, 3] = 0.0
    rays[:, 4:7] = d
    rays[:, 7] = np.inf
    return rays


def from_occupancy(occ: np.ndarray, cells, fwd, root_size: Optional[float] = None, name: str = "occ",
                   seed: int = 0) -> Scene:
    """Scene from a dense boolean grid occ[x, y, z] with transformed nodes at
    ``cells`` = [(level, (x, y, z))] and fixed forward maps ``fwd`` [S, 12]."""
    classify, K = ot.dense_classifier(occ)
    tree = ot.build_tree(K, classify, _colour_fn(K, seed))
    rs = float(1 << K) if root_size is None else float(root_size)
    F = np.asarray(fwd, np.float32).reshape(-1, 12) if len(cells) else np.zeros((0, 12), np.float32)

    def xform(frame: int = 0):
        return F.copy()

    return _marked_scene(name, tree, K, rs, list(cells), xform, {}, seed)


def blob_occupancy(K: int, seed: int, density: float = 0.4) -> np.ndarray:
    """Random blobs on a 2^K grid (smooth noise thresholded)."""
    n = 1 << K
    g = np.arange(n, dtype=np.float64) + 0.5
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    v = fbm3(X, Y, Z, 2, max(2.0, n / 2.0), seed)
    return v > (1.0 - 2.0 * density) * 0.5


# ------------------------------------------------------------------ instanced scene, 4096^3 world

def _instance_trees(seed: int):
    """The four instance SVOs: sphere (depth 8, radius 96), noise blob (depth
    9: 4-octave value noise > 0.1 inside radius 240), heightfield (depth 10)
    and box lattice (depth 11: solid where at least two of x, y, z mod 128
    fall below 16)."""
    trees = []
    # sphere
    K = 8
    n = 1 << K
    g = np.arange(n, dtype=np.float32) + 0.5
    r2 = (g[:, None, None] - n / 2) ** 2 + (g[None, :, None] - n / 2) ** 2 + (g[None, None, :] - n / 2) ** 2
    occ = r2 < 96.0 ** 2
    trees.append(ot.build_tree(K, ot.dense_classifier(occ)[0], _colour_fn(K, seed)))
    del occ, r2
    # noise blob
    K = 9
    n = 1 << K
    from .noise import fbm3_grid
    occ = fbm3_grid(n, 4, 128.0, seed) > 0.1
    g = np.arange(n, dtype=np.float32) + 0.5
    occ &= ((g[:, None, None] - n / 2) ** 2 + (g[None, :, None] - n / 2) ** 2 + (g[None, None, :] - n / 2) ** 2) < 240.0 ** 2
    trees.append(ot.build_tree(K, ot.dense_classifier(occ)[0], _colour_fn(K, seed)))
    del occ
    # heightfield
    K = 10
    H = heightfield(K, seed, 400.0, 300.0, 6, 256.0)
    trees.append(ot.build_tree(K, ot.heightfield_classifier(H, K), _colour_fn(K, seed)))
    # box lattice
    K = 11
    trees.append(ot.build_tree(K, ot.lattice_classifier(K, 128, 16), _colour_fn(K, seed)))
    return trees


def instanced_scene(seed: int = 3, n_inst: int = 64, world_K: int = 12) -> Scene:
    """64 instances of the four SVOs in a 4096^3 world.  Instance i has kind
    i mod 4, sits on a free cell at a level drawn from {1, 2, 3} (no used
    cell above or below it), and maps its own root cube [0, 2^D)^3 onto the
    cell (placement), then rotates uniformly at random, scales each axis by
    U[0.5, 1] about the cell centre and moves by U[-1/4, 1/4] cell (pose).
    Instances of one kind share their subtree (slots share a child group)."""
    st = Stream(seed, 51)
    inst = _instance_trees(seed)
    N = 1 << world_K
    used = []
    cells = []
    tries = 0
    while len(cells) < n_inst and tries < 100000:
        tries += 1
        L = int(st.integers(1, 1, 4)[0])
        xyz = tuple(int(v) for v in st.integers(3, 0, 1 << L))
        ok = True
        for (l2, c2) in used:
            lo, hi = (l2, L) if l2 < L else (L, l2)
            a, b = (c2, xyz) if l2 < L else (xyz, c2)
            if lo == hi:
                if a == b:
                    ok = False
                    break
            elif all((b[k] >> (hi - lo)) == a[k] for k in range(3)):
                ok = False
                break
        if ok:
            used.append((L, xyz))
            cells.append((L, xyz))
    if len(cells) < n_inst:
        raise RuntimeError("could not place all instances")
    slot_nodes = {}
    for s, (L, xyz) in enumerate(cells):
        slot_nodes[(L,) + xyz] = (s, inst[s % 4].root_mask)

    def classify(l, c):
        out = np.zeros(c.shape[0], np.uint8)
        for j in range(c.shape[0]):
            cj = tuple(int(v) for v in c[j])
            for (L, xyz) in cells:
                if L > l and all((xyz[k] >> (L - l)) == cj[k] for k in range(3)):
                    out[j] = ot.PARTIAL
                    break
        return out

    world = ot.build_tree(world_K, classify, None, slot_nodes=slot_nodes)
    nodes, bases = ot.concat([world] + inst)
    slot_child = np.array([bases[1 + s % 4] + int(inst[s % 4].child_start[0]) for s in range(n_inst)], np.uint32)
    slot_cell = np.array([[0.0, 0.0, 0.0, float(1 << inst[s % 4].K)] for s in range(n_inst)], np.float32)
    slot_node = np.array([ot.find_node(world, L, xyz) for (L, xyz) in cells], np.int64)
    mats = []
    for s, (L, xyz) in enumerate(cells):
        size = float(N >> L)
        lo = np.asarray(xyz, np.float64) * size
        D = inst[s % 4].K
        place = np.zeros((3, 4))
        place[:, :3] = np.eye(3) * (size / float(1 << D))
        place[:, 3] = lo
        R = xf.random_rotation(st)
        sc = st.uniform(3, 0.5, 1.0)
        tr = st.uniform(3, -0.25, 0.25) * size
        pose = xf.about_pivot(R @ np.diag(sc), lo + size / 2, tr)
        A = pose[:, :3] @ place[:, :3]
        b = pose[:, :3] @ place[:, 3] + pose[:, 3]
        M = np.zeros((3, 4))
        M[:, :3] = A
        M[:, 3] = b
        mats.append(xf.to_f32(M).reshape(12))
    F = np.array(mats, np.float32)

    def xform(frame: int = 0):
        return F.copy()

    static = ot.clear_transformed(nodes, slot_child)
    camera = dict(eye=(2048.0, 3000.0, -2500.0), target=(2048.0, 1800.0, 2048.0), up=(0.0, 1.0, 0.0), fov=60.0,
                  W=1920, H=1080)
    return Scene(name="instances4096", nodes=nodes, static_nodes=static, root=0, root_min=np.zeros(3, np.float32),
                 root_size=float(N), max_depth=20, slot_child=slot_child, slot_cell=slot_cell, slot_node=slot_node,
                 slot_parent=np.full(n_inst, NONE, np.uint32), tree=world, xform=xform, camera=camera, seed=seed)


# ------------------------------------------------------------------ ridged terrain, depth 12

def ridged_terrain_d12(seed: int = 5, frames: int = 60, n_slots: int = 256) -> Scene:
    """Depth-12 (4096^3) heightfield h = 2048 + 2048 r, r a ridged multifractal
    (9 octaves, P0 = 1024): about 1.5e8 nodes (1.2 GB), far beyond the MALL.
    256 interior nodes of level 4 (256^3 cells), drawn by the seeded stream,
    are animated by 4 keyframes each at frames {0, 20, 40, 60} + U{-5..5}:
    a uniformly random rotation and per-axis scale 2^U[-1, 1] about the cell
    centre, interpolated by slerp and log-linear scale (the pose of the
    first / last keyframe holds before / after it)."""
    from . import hfbuild
    from .noise import ridged2_grid
    K = 12
    n = 1 << K
    r = ridged2_grid(n, 9, 1024.0, seed)
    H = np.clip(np.ceil(2048.0 + 2048.0 * r - 0.5), 0, n).astype(np.int32)
    del r
    nodes, _ = hfbuild.build_heightfield_pool(H, K, seed)
    del H
    idx, lev, crd = ot.top_levels(nodes, 4)
    inter = (lev == 4) & ((nodes[idx] & np.uint64(0xFF)) != 0)
    cand_i, cand_c = idx[inter], crd[inter]
    if cand_i.shape[0] < n_slots:
        raise RuntimeError("only %d interior level-4 nodes" % cand_i.shape[0])
    st = Stream(seed, 13)
    pick = []
    seen = set()
    while len(pick) < n_slots:
        j = int(st.integers(1, 0, cand_i.shape[0])[0])
        if j not in seen:
            seen.add(j)
            pick.append(j)
    nodes, slot_child, slot_node = ot.mark_transformed_pool(nodes, [int(cand_i[j]) for j in pick], in_place=True)
    size = float(1 << (K - 4))
    slot_cell = np.zeros((n_slots, 4), np.float32)
    centres = []
    for s_, j in enumerate(pick):
        slot_cell[s_, :3] = cand_c[j] * size
        slot_cell[s_, 3] = size
        centres.append(cand_c[j].astype(np.float64) * size + size / 2)
    times = np.array([0, 20, 40, 60], np.float64)[None, :] + st.integers(4 * n_slots, -5, 6).reshape(n_slots, 4)
    quats = [[xf.random_quat(st) for _ in range(4)] for _ in range(n_slots)]
    logs = st.uniform(12 * n_slots, -1.0, 1.0).reshape(n_slots, 4, 3)

    def xform(frame: int = 0):
        f = float(frame % frames)
        out = np.zeros((n_slots, 12), np.float32)
        for j in range(n_slots):
            t = times[j]
            if f <= t[0]:
                k, u = 0, 0.0
            elif f >= t[3]:
                k, u = 2, 1.0
            else:
                k = int(np.searchsorted(t, f, side="right")) - 1
                k = min(max(k, 0), 2)
                u = (f - t[k]) / (t[k + 1] - t[k])
            q = xf.slerp(quats[j][k], quats[j][k + 1], u)
            sc_ = 2.0 ** ((1.0 - u) * logs[j, k] + u * logs[j, k + 1])
            out[j] = xf.to_f32(xf.about_pivot(xf.quat_to_mat(q) @ np.diag(sc_), centres[j])).reshape(12)
        return out

    camera = dict(eye=(2048.0, 5600.0, 600.0), target=(2048.0, 1200.0, 2600.0), up=(0.0, 1.0, 0.0),
                  fov=45.0, W=3840, H=2160)
    return Scene(name="terrain4096", nodes=nodes, static_nodes=None, root=0, root_min=np.zeros(3, np.float32),
                 root_size=float(n), max_depth=K, slot_child=slot_child, slot_cell=slot_cell, slot_node=slot_node,
                 slot_parent=np.full(n_slots, NONE, np.uint32), tree=None, xform=xform, camera=camera, seed=seed)
