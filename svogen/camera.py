"""Pinhole primary rays.

Ray record (32 bytes): ox, oy, oz, tmin, dx, dy, dz, tmax in float32.
Pixel (i, j) samples its centre (i + 1/2, j + 1/2); j counts from the top
row.  Directions are normalised in float64 and then rounded to float32.
Rays are emitted either row-major or in 8x8 pixel tiles (tile-major, rows of
tiles), the latter so that 64 consecutive rays share a screen tile.
"""
from __future__ import annotations

import numpy as np


def basis(eye, target, up):
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, np.float64))
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    return f, r, u


def pixel_order(W: int, H: int, order: str = "tiles", tile: int = 8):
    """Flat pixel indices (j * W + i) in emission order."""
    if order == "rows":
        return np.arange(W * H, dtype=np.int64)
    if order != "tiles":
        raise ValueError(order)
    ty, tx = (H + tile - 1) // tile, (W + tile - 1) // tile
    jj, ii = np.meshgrid(np.arange(tile), np.arange(tile), indexing="ij")
    out = []
    for by in range(ty):
        for bx in range(tx):
            j = by * tile + jj.ravel()
            i = bx * tile + ii.ravel()
            ok = (j < H) & (i < W)
            out.append(j[ok] * W + i[ok])
    return np.concatenate(out).astype(np.int64)


def pinhole_rays(eye, target, up, vfov_deg: float, W: int, H: int, order: str = "tiles",
                 jitter=None, tmin: float = 0.0, tmax: float = np.inf):
    """Primary rays [n, 8] float32 and the flat pixel index of each ray.

    jitter: optional [n, 2] sub-pixel offsets in [0, 1) replacing the centre.
    """
    f, r, u = basis(eye, target, up)
    pix = pixel_order(W, H, order)
    i = (pix % W).astype(np.float64)
    j = (pix // W).astype(np.float64)
    if jitter is None:
        fx, fy = 0.5, 0.5
    else:
        fx, fy = jitter[:, 0], jitter[:, 1]
    th = np.tan(np.radians(vfov_deg) * 0.5)
    aspect = W / H
    sx = ((i + fx) / W * 2.0 - 1.0) * th * aspect
    sy = (1.0 - (j + fy) / H * 2.0) * th
    d = f[None, :] + sx[:, None] * r[None, :] + sy[:, None] * u[None, :]
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rays = np.empty((pix.shape[0], 8), dtype=np.float32)
    rays[:, 0:3] = np.asarray(eye, np.float64).astype(np.float32)[None, :]
    rays[:, 3] = tmin
    rays[:, 4:7] = d.astype(np.float32)
    rays[:, 7] = tmax
    return rays, pix
