"""Counter-based hashing for seeded synthetic inputs.

SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) applied to integer lattice keys.  Everything here is
vectorised over numpy uint64 arrays and wraps modulo 2**64 by construction.
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x):
    """SplitMix64 finaliser of ``x + golden`` (array or scalar, uint64)."""
    with np.errstate(over="ignore"):
        z = np.asarray(x, dtype=np.uint64) + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def hash_keys(*keys):
    """Hash a tuple of integer arrays (broadcast together) into uint64."""
    h = np.uint64(0x6A09E667F3BCC909)
    with np.errstate(over="ignore"):
        for k in keys:
            k64 = np.asarray(k).astype(np.int64).astype(np.uint64)
            h = splitmix64(h ^ k64)
    return h


def to_unit(h):
    """Top 53 bits of a uint64 hash as a double in [0, 1)."""
    return (np.asarray(h, dtype=np.uint64) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def to_signed_unit(h):
    """Hash mapped to [-1, 1)."""
    return to_unit(h) * 2.0 - 1.0


class Stream:
    """Deterministic counter-based stream: value i is a pure function of (seed, tag, i)."""

    def __init__(self, seed: int, tag: int = 0):
        self.seed = int(seed)
        self.tag = int(tag)
        self.counter = 0

    def uniform(self, n: int = None, lo: float = 0.0, hi: float = 1.0):
        m = 1 if n is None else int(n)
        idx = np.arange(self.counter, self.counter + m, dtype=np.int64)
        self.counter += m
        u = to_unit(hash_keys(self.seed, self.tag, idx))
        v = lo + (hi - lo) * u
        return float(v[0]) if n is None else v

    def integers(self, n: int, lo: int, hi: int):
        """Integers uniform in [lo, hi)."""
        u = self.uniform(n)
        return np.minimum(lo + np.floor(u * (hi - lo)).astype(np.int64), hi - 1)

    def normal(self, n: int):
        """Standard normals by Box-Muller on two uniforms."""
        u1 = np.maximum(self.uniform(n), 1e-300)
        u2 = self.uniform(n)
        return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
