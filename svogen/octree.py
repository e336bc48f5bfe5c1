"""Occupancy -> 8-byte-node sparse voxel octree pools (input generation only).

Pool format (the same one ``include/svo.h`` defines; written here from that
definition, no code shared with the library):

  node = uint64, bits  0..7  child mask m, octant i = x | y<<1 | z<<2
                 bits  8..31 c24, child-group offset relative to the node
                 bits 32..63 word1
  m == 0                       solid leaf covering its whole cell, word1 = RGBA8
  m != 0, word1 bit 31 set     transformed node, slot = word1 & 0x7fffffff,
                               children at slot_child[slot], c24 = 0
  m != 0, c24 == 0xffffff      children at the absolute index word1 (far pointer)
  m != 0, otherwise            children at node_index + c24, word1 = 0

The k-th existing child in octant order sits at child_start + k.  Nodes are
emitted breadth first, so the first nodes of a pool are its top levels.

Cells are classified top-down by a callback ``classify(level, coords)`` that
returns EMPTY, FULL or PARTIAL for each integer cell (level 0 = root, level K
= unit voxels).  FULL cells become leaves at their own level (full-node
collapse), PARTIAL cells become interior nodes.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Dict, Optional, Tuple

import numpy as np

EMPTY, FULL, PARTIAL, SLOT = 0, 1, 2, 3
FAR = 0xFFFFFF
XFORM_BIT = 0x80000000
NONE = 0xFFFFFFFF

# octant i -> (x, y, z) bits
OCT = np.array([[i & 1, (i >> 1) & 1, (i >> 2) & 1] for i in range(8)], dtype=np.int64)


@dataclass
class Tree:
    """One octree's nodes plus generation metadata (level, cell coords, kind per node)."""
    nodes: np.ndarray            # uint64 [n]
    level: np.ndarray            # int32 [n]
    coord: np.ndarray            # int64 [n, 3]
    kind: np.ndarray             # uint8 [n]  FULL / PARTIAL / SLOT
    child_start: np.ndarray      # int64 [n]  (-1 for leaves / slot cells)
    K: int                       # leaf level (height)

    @property
    def n(self) -> int:
        return int(self.nodes.shape[0])

    @property
    def root_mask(self) -> int:
        return int(self.nodes[0] & np.uint64(0xFF)) if self.n else 0


def _encode_interior(idx, mask, start):
    idx = idx.astype(np.int64)
    off = start - idx
    if np.any(off <= 0):
        raise ValueError("breadth-first order violated: child group before parent")
    far = off >= FAR
    c24 = np.where(far, FAR, off).astype(np.uint64)
    w1 = np.where(far, start, 0).astype(np.uint64)
    return mask.astype(np.uint64) | (c24 << np.uint64(8)) | (w1 << np.uint64(32))


def build_tree(K: int, classify: Callable, colour: Optional[Callable] = None,
               slot_nodes: Optional[Dict[Tuple[int, int, int, int], Tuple[int, int]]] = None) -> Tree:
    """Build a breadth-first pool.

    slot_nodes: {(level, x, y, z): (slot, mask)} -- cells emitted as transformed
    nodes with the given child mask (their content lives in another tree).
    """
    slot_nodes = slot_nodes or {}
    slot_levels: Dict[int, Dict[Tuple[int, int, int], Tuple[int, int]]] = {}
    for (l, x, y, z), v in slot_nodes.items():
        if l <= 0 or l > K:
            raise ValueError("slot level must be in 1..K")
        slot_levels.setdefault(l, {})[(x, y, z)] = v

    def classify_with_slots(l, coords):
        k = np.asarray(classify(l, coords), dtype=np.uint8).copy()
        g = slot_levels.get(l)
        if g:
            for j, c in enumerate(map(tuple, coords.tolist())):
                if c in g:
                    k[j] = SLOT
        return k

    root = np.zeros((1, 3), dtype=np.int64)
    rk = classify_with_slots(0, root)
    empty = Tree(np.zeros(0, np.uint64), np.zeros(0, np.int32), np.zeros((0, 3), np.int64),
                 np.zeros(0, np.uint8), np.zeros(0, np.int64), K)
    if rk[0] == EMPTY:
        return empty

    lv_coords = [root]
    lv_kind = [rk]
    lv_mask = []
    lv_counts = []
    for l in range(K + 1):
        cc, kk = lv_coords[l], lv_kind[l]
        inter = kk == PARTIAL
        if l == K and inter.any():
            raise ValueError("classifier returned PARTIAL at the leaf level")
        parents = cc[inter]
        if parents.shape[0] == 0:
            lv_mask.append(np.zeros(0, np.int64))
            lv_counts.append(np.zeros(0, np.int64))
            break
        ch = (parents[:, None, :] * 2 + OCT[None, :, :]).reshape(-1, 3)
        ck = classify_with_slots(l + 1, ch)
        exist = (ck != EMPTY).reshape(-1, 8)
        mask = (exist * (1 << np.arange(8))[None, :]).sum(1)
        if np.any(mask == 0):
            raise ValueError("PARTIAL cell with no non-empty child at level %d" % l)
        lv_mask.append(mask)
        lv_counts.append(exist.sum(1))
        keep = exist.ravel()
        lv_coords.append(ch[keep])
        lv_kind.append(ck[keep])

    nl = len(lv_coords)
    sizes = [c.shape[0] for c in lv_coords]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    n = int(offs[-1])
    nodes = np.zeros(n, dtype=np.uint64)
    level = np.zeros(n, dtype=np.int32)
    coord = np.zeros((n, 3), dtype=np.int64)
    kind = np.zeros(n, dtype=np.uint8)
    child_start = np.full(n, -1, dtype=np.int64)
    for l in range(nl):
        a, b = offs[l], offs[l + 1]
        level[a:b] = l
        coord[a:b] = lv_coords[l]
        kind[a:b] = lv_kind[l]
        kk = lv_kind[l]
        idx = np.arange(a, b, dtype=np.int64)
        inter = kk == PARTIAL
        if inter.any():
            counts = lv_counts[l]
            start = offs[l + 1] + np.concatenate([[0], np.cumsum(counts)[:-1]])
            nodes[idx[inter]] = _encode_interior(idx[inter], lv_mask[l], start)
            child_start[idx[inter]] = start
        full = kk == FULL
        if full.any():
            col = np.full(int(full.sum()), 0xFFFFFFFF, dtype=np.uint64)
            if colour is not None:
                col = np.asarray(colour(l, lv_coords[l][full]), dtype=np.uint64) & np.uint64(0xFFFFFFFF)
            nodes[idx[full]] = col << np.uint64(32)
        gr = kk == SLOT
        if gr.any():
            g = slot_levels[l]
            for j in np.nonzero(gr)[0]:
                slot, gmask = g[tuple(lv_coords[l][j].tolist())]
                if gmask == 0 or gmask > 0xFF:
                    raise ValueError("slot mask must be 1..255")
                nodes[a + j] = np.uint64(gmask) | (np.uint64(XFORM_BIT | slot) << np.uint64(32))
    return Tree(nodes, level, coord, kind, child_start, K)


def find_node(tree: Tree, level: int, xyz) -> int:
    """Index of the node for cell (level, xyz), or -1."""
    sel = np.nonzero((tree.level == level) & np.all(tree.coord == np.asarray(xyz)[None, :], axis=1))[0]
    return int(sel[0]) if sel.size else -1


def mark_transformed(tree: Tree, cells) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Turn interior nodes at the given cells into transformed nodes.

    cells: list of (level, (x, y, z)); slot s = position in the list.
    Returns (nodes, slot_child, slot_node) -- a new node array, the child-group
    index of each slot and the node index carrying it.
    """
    nodes = tree.nodes.copy()
    slot_child = np.zeros(len(cells), dtype=np.uint32)
    slot_node = np.zeros(len(cells), dtype=np.int64)
    for s, (l, xyz) in enumerate(cells):
        i = find_node(tree, l, xyz)
        if i < 0 or tree.kind[i] != PARTIAL:
            raise ValueError("transformed cell %r is not an interior node" % ((l, xyz),))
        mask = int(nodes[i] & np.uint64(0xFF))
        nodes[i] = np.uint64(mask) | (np.uint64(XFORM_BIT | s) << np.uint64(32))
        slot_child[s] = tree.child_start[i]
        slot_node[s] = i
    return nodes, slot_child, slot_node


def clear_transformed(nodes: np.ndarray, slot_child: np.ndarray) -> np.ndarray:
    """Static twin: every transformed node becomes a plain interior node whose
    children are the slot's child group (relative offset, else far pointer)."""
    out = nodes.copy()
    w1 = (out >> np.uint64(32)).astype(np.int64)
    mask = (out & np.uint64(0xFF)).astype(np.int64)
    xf = ((w1 & XFORM_BIT) != 0) & (mask != 0)
    idx = np.nonzero(xf)[0]
    if idx.size:
        start = slot_child[w1[idx] & 0x7FFFFFFF].astype(np.int64)
        off = start - idx
        far = (off <= 0) | (off >= FAR)
        c24 = np.where(far, FAR, off).astype(np.uint64)
        nw1 = np.where(far, start, 0).astype(np.uint64)
        out[idx] = mask[idx].astype(np.uint64) | (c24 << np.uint64(8)) | (nw1 << np.uint64(32))
    return out


def concat(trees):
    """Concatenate trees into one pool; returns (nodes, bases). Relative
    offsets stay valid; far pointers are rebased."""
    bases = []
    parts = []
    base = 0
    for t in trees:
        nd = t.nodes.copy()
        if base:
            w1 = nd >> np.uint64(32)
            mask = nd & np.uint64(0xFF)
            c24 = (nd >> np.uint64(8)) & np.uint64(0xFFFFFF)
            far = (mask != 0) & (c24 == np.uint64(FAR)) & ((w1 & np.uint64(XFORM_BIT)) == 0)
            nd[far] = (nd[far] & np.uint64(0xFFFFFFFF)) | ((w1[far] + np.uint64(base)) << np.uint64(32))
        parts.append(nd)
        bases.append(base)
        base += t.n
    return np.concatenate(parts) if parts else np.zeros(0, np.uint64), bases


# ---------------------------------------------------------------- classifiers

def dense_classifier(occ: np.ndarray):
    """Classifier over a dense boolean grid occ[x, y, z] of side 2**K."""
    n = occ.shape[0]
    K = int(round(np.log2(n)))
    assert occ.shape == (n, n, n) and (1 << K) == n
    anyp = [None] * (K + 1)
    allp = [None] * (K + 1)
    anyp[K] = occ.astype(bool)
    allp[K] = occ.astype(bool)
    for l in range(K - 1, -1, -1):
        m = 1 << l
        anyp[l] = anyp[l + 1].reshape(m, 2, m, 2, m, 2).any(axis=(1, 3, 5))
        allp[l] = allp[l + 1].reshape(m, 2, m, 2, m, 2).all(axis=(1, 3, 5))

    def classify(l, c):
        a = anyp[l][c[:, 0], c[:, 1], c[:, 2]]
        f = allp[l][c[:, 0], c[:, 1], c[:, 2]]
        return np.where(f, FULL, np.where(a, PARTIAL, EMPTY)).astype(np.uint8)

    return classify, K


def heightfield_classifier(H: np.ndarray, K: int):
    """Classifier for columns H[x, z] (solid iff y < H[x, z]) on a 2**K grid."""
    n = 1 << K
    assert H.shape == (n, n)
    mn = [None] * (K + 1)
    mx = [None] * (K + 1)
    mn[K] = H.astype(np.int64)
    mx[K] = H.astype(np.int64)
    for l in range(K - 1, -1, -1):
        m = 1 << l
        mn[l] = mn[l + 1].reshape(m, 2, m, 2).min(axis=(1, 3))
        mx[l] = mx[l + 1].reshape(m, 2, m, 2).max(axis=(1, 3))

    def classify(l, c):
        s = 1 << (K - l)
        lo = mn[l][c[:, 0], c[:, 2]]
        hi = mx[l][c[:, 0], c[:, 2]]
        y0 = c[:, 1] * s
        full = lo >= y0 + s
        empty = hi <= y0
        return np.where(full, FULL, np.where(empty, EMPTY, PARTIAL)).astype(np.uint8)

    return classify


def lattice_classifier(K: int, period: int, width: int, need: int = 2):
    """Solid where at least ``need`` of the three axes satisfy (v mod period) < width."""

    def axis_state(lo, s):
        # 1 = every v in [lo, lo+s) is inside a band, 0 = none, 2 = mixed
        if s >= period:
            return np.full(lo.shape, 2, dtype=np.int64)
        a = lo % period
        b = a + s  # exclusive end within at most two periods
        inside_all = b <= width
        # none inside: [a, b) within [width, period)
        none_in = (a >= width) & (b <= period)
        return np.where(inside_all, 1, np.where(none_in, 0, 2))

    def classify(l, c):
        s = 1 << (K - l)
        st = np.stack([axis_state(c[:, i] * s, s) for i in range(3)], axis=1)
        n_all = (st == 1).sum(1)
        n_any = (st >= 1).sum(1)
        full = n_all >= need
        empty = n_any < need
        return np.where(full, FULL, np.where(empty, EMPTY, PARTIAL)).astype(np.uint8)

    return classify


def leaf_boxes(tree: Tree, root_min, root_size: float):
    """(index, box min [n,3], box size [n]) of every solid leaf, in the tree's
    own coordinates (root cell = root_min + [0, root_size)^3)."""
    sel = np.nonzero(tree.kind == FULL)[0]
    sz = root_size / (2.0 ** tree.level[sel].astype(np.float64))
    mn = np.asarray(root_min, np.float64)[None, :] + tree.coord[sel].astype(np.float64) * sz[:, None]
    return sel, mn, sz


def force_far(nodes: np.ndarray, every: int = 1) -> np.ndarray:
    """Re-encode every ``every``-th plain interior node with a far pointer
    (c24 = 0xffffff, word1 = absolute child start); same tree, other bytes."""
    out = nodes.copy()
    mask = (out & np.uint64(0xFF)).astype(np.int64)
    w1 = (out >> np.uint64(32)).astype(np.int64)
    c24 = ((out >> np.uint64(8)) & np.uint64(0xFFFFFF)).astype(np.int64)
    plain = (mask != 0) & ((w1 & XFORM_BIT) == 0) & (c24 != FAR)
    idx = np.nonzero(plain)[0][::every]
    start = idx + c24[idx]
    out[idx] = mask[idx].astype(np.uint64) | (np.uint64(FAR) << np.uint64(8)) | (start.astype(np.uint64) << np.uint64(32))
    return out


def child_start(nodes: np.ndarray, i: int) -> int:
    """Child-group start of interior node i (relative or far pointer)."""
    w = int(nodes[i])
    c24 = (w >> 8) & FAR
    return (w >> 32) if c24 == FAR else i + c24


def top_levels(nodes: np.ndarray, L: int):
    """Breadth-first walk of the first L + 1 levels of a pool rooted at node
    0 with no transformed nodes: (index, level, coord [n, 3]) of every node
    of levels 0..L, in pool order."""
    out_i, out_l, out_c = [], [], []
    if nodes.shape[0] == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int32), np.zeros((0, 3), np.int64)
    cur = [(0, (0, 0, 0))]
    for l in range(L + 1):
        nxt = []
        for i, c in cur:
            out_i.append(i)
            out_l.append(l)
            out_c.append(c)
            m = int(nodes[i]) & 0xFF
            if m == 0 or l == L:
                continue
            s = child_start(nodes, i)
            k = 0
            for o in range(8):
                if (m >> o) & 1:
                    nxt.append((s + k, (2 * c[0] + (o & 1), 2 * c[1] + ((o >> 1) & 1), 2 * c[2] + ((o >> 2) & 1))))
                    k += 1
        cur = nxt
    return np.asarray(out_i, np.int64), np.asarray(out_l, np.int32), np.asarray(out_c, np.int64).reshape(-1, 3)


def mark_transformed_pool(nodes: np.ndarray, found, in_place: bool = False):
    """mark_transformed for a pool without generation metadata: found is a
    list of interior node indices, slot s = position in the list.  Returns
    (nodes, slot_child, slot_node)."""
    out = nodes if in_place else nodes.copy()
    slot_child = np.zeros(len(found), dtype=np.uint32)
    slot_node = np.zeros(len(found), dtype=np.int64)
    for s, i in enumerate(found):
        m = int(out[i]) & 0xFF
        if m == 0:
            raise ValueError("node %d is a leaf" % i)
        slot_child[s] = child_start(out, int(i))
        out[i] = np.uint64(m) | (np.uint64(XFORM_BIT | s) << np.uint64(32))
        slot_node[s] = i
    return out, slot_child, slot_node
