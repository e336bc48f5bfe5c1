"""Seeded value noise and fractional Brownian motion (fBm).

Lattice values are uniform in [-1, 1) from the SplitMix64 hash of
(lattice coordinates, octave, seed); they are blended with smoothstep
weights (bi- or tri-linear).  Octave ``o`` has period ``P0 / 2**o`` and
amplitude ``2**-o``; the sum is divided by the total amplitude so the result
stays in [-1, 1].
"""
from __future__ import annotations

import numpy as np

from .hashing import hash_keys, to_signed_unit


def _smooth(f):
    return f * f * (3.0 - 2.0 * f)


def value_noise2(x, z, period: float, octave: int, seed: int):
    u = np.asarray(x, dtype=np.float64) / period
    v = np.asarray(z, dtype=np.float64) / period
    i0 = np.floor(u)
    k0 = np.floor(v)
    fu = _smooth(u - i0)
    fv = _smooth(v - k0)
    i0 = i0.astype(np.int64)
    k0 = k0.astype(np.int64)

    def lat(di, dk):
        return to_signed_unit(hash_keys(i0 + di, k0 + dk, octave, seed, 2))

    a = lat(0, 0) * (1 - fu) + lat(1, 0) * fu
    b = lat(0, 1) * (1 - fu) + lat(1, 1) * fu
    return a * (1 - fv) + b * fv


def value_noise3(x, y, z, period: float, octave: int, seed: int):
    u = np.asarray(x, dtype=np.float64) / period
    v = np.asarray(y, dtype=np.float64) / period
    w = np.asarray(z, dtype=np.float64) / period
    i0, j0, k0 = np.floor(u), np.floor(v), np.floor(w)
    fu, fv, fw = _smooth(u - i0), _smooth(v - j0), _smooth(w - k0)
    i0, j0, k0 = i0.astype(np.int64), j0.astype(np.int64), k0.astype(np.int64)

    def lat(di, dj, dk):
        return to_signed_unit(hash_keys(i0 + di, j0 + dj, k0 + dk, octave, seed, 3))

    c00 = lat(0, 0, 0) * (1 - fu) + lat(1, 0, 0) * fu
    c10 = lat(0, 1, 0) * (1 - fu) + lat(1, 1, 0) * fu
    c01 = lat(0, 0, 1) * (1 - fu) + lat(1, 0, 1) * fu
    c11 = lat(0, 1, 1) * (1 - fu) + lat(1, 1, 1) * fu
    c0 = c00 * (1 - fv) + c10 * fv
    c1 = c01 * (1 - fv) + c11 * fv
    return c0 * (1 - fw) + c1 * fw


def fbm2(x, z, octaves: int, period0: float, seed: int):
    total = np.zeros(np.broadcast(np.asarray(x), np.asarray(z)).shape)
    amp_sum = 0.0
    for o in range(octaves):
        amp = 2.0 ** -o
        total = total + amp * value_noise2(x, z, period0 / 2.0 ** o, o, seed)
        amp_sum += amp
    return total / amp_sum


def fbm3(x, y, z, octaves: int, period0: float, seed: int):
    shape = np.broadcast(np.asarray(x), np.asarray(y), np.asarray(z)).shape
    total = np.zeros(shape)
    amp_sum = 0.0
    for o in range(octaves):
        amp = 2.0 ** -o
        total = total + amp * value_noise3(x, y, z, period0 / 2.0 ** o, o, seed)
        amp_sum += amp
    return total / amp_sum


def value_noise3_grid(n: int, period: float, octave: int, seed: int, dtype=np.float32):
    """value_noise3 at every voxel centre (i + 1/2) of an n^3 grid, computed by
    separable interpolation: the lattice values are hashed once, then blended
    along x, y and z in turn (the same smoothstep weights as value_noise3)."""
    g = (np.arange(n, dtype=np.float64) + 0.5) / period
    i0 = np.floor(g).astype(np.int64)
    w = _smooth(g - i0)
    lo, hi = int(i0.min()), int(i0.max()) + 1
    L = np.arange(lo, hi + 1, dtype=np.int64)
    V = to_signed_unit(hash_keys(L[:, None, None], L[None, :, None], L[None, None, :], octave, seed, 3))
    ix = i0 - lo
    # blend along x: [n, Ly, Lz]
    A = V[ix] * (1 - w)[:, None, None] + V[ix + 1] * w[:, None, None]
    # along y: [n, n, Lz]
    B = A[:, ix, :] * (1 - w)[None, :, None] + A[:, ix + 1, :] * w[None, :, None]
    B = B.astype(dtype)
    wz = w.astype(dtype)
    return B[:, :, ix] * (1 - wz)[None, None, :] + B[:, :, ix + 1] * wz[None, None, :]


def fbm3_grid(n: int, octaves: int, period0: float, seed: int, dtype=np.float32):
    total = np.zeros((n, n, n), dtype=dtype)
    amp_sum = 0.0
    for o in range(octaves):
        amp = 2.0 ** -o
        total += dtype(amp) * value_noise3_grid(n, period0 / 2.0 ** o, o, seed, dtype)
        amp_sum += amp
    total /= dtype(amp_sum)
    return total


def value_noise2_grid(n: int, period: float, octave: int, seed: int):
    """value_noise2 at every column centre (i + 1/2, k + 1/2) of an n x n grid
    by separable interpolation (lattice values hashed once, blended along x
    then z with value_noise2's weights and operation order: equal to the
    pointwise evaluation bit for bit)."""
    g = (np.arange(n, dtype=np.float64) + 0.5) / period
    i0 = np.floor(g)
    w = _smooth(g - i0)
    i0 = i0.astype(np.int64)
    lo, hi = int(i0.min()), int(i0.max()) + 1
    L = np.arange(lo, hi + 1, dtype=np.int64)
    V = to_signed_unit(hash_keys(L[:, None], L[None, :], octave, seed, 2))   # [x lattice, z lattice]
    ix = i0 - lo
    a = V[ix][:, ix] * (1 - w)[:, None] + V[ix + 1][:, ix] * w[:, None]          # lat(0,0)(1-fu) + lat(1,0)fu
    b = V[ix][:, ix + 1] * (1 - w)[:, None] + V[ix + 1][:, ix + 1] * w[:, None]  # lat(0,1)(1-fu) + lat(1,1)fu
    return a * (1 - w)[None, :] + b * w[None, :]


def fbm2_grid(n: int, octaves: int, period0: float, seed: int):
    """fbm2 at every column centre of an n x n grid (bit for bit)."""
    total = np.zeros((n, n))
    amp_sum = 0.0
    for o in range(octaves):
        amp = 2.0 ** -o
        total = total + amp * value_noise2_grid(n, period0 / 2.0 ** o, o, seed)
        amp_sum += amp
    return total / amp_sum


def ridged2_grid(n: int, octaves: int, period0: float, seed: int, gain: float = 0.5):
    """Ridged multifractal on the column centres of an n x n grid: octave o
    contributes amp_o * (1 - |v_o|)^2 with v_o the value noise of period
    P0 / 2^o, amp_0 = 1 and amp_o = gain^o scaled by the previous octave's
    ridge (sharp crests, rough flanks); normalised to [-1, 1]."""
    total = np.zeros((n, n))
    amp_sum = 0.0
    weight = np.ones((n, n))
    for o in range(octaves):
        r = (1.0 - np.abs(value_noise2_grid(n, period0 / 2.0 ** o, o, seed))) ** 2
        amp = gain ** o
        total = total + amp * weight * r
        amp_sum += amp
        weight = np.clip(r * 2.0, 0.0, 1.0)
    return total / amp_sum * 2.0 - 1.0
