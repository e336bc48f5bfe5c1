"""Forward (local -> parent) affine transforms for generated scenes.

A transform is a 3x4 row-major matrix A with x_parent = A[:, :3] x_local + A[:, 3].
Generators build them in float64 and hand them out rounded to float32, the
precision the transform slots carry.  Rotations are right handed; a rotation
or scale "about a pivot" leaves the pivot fixed.
"""
from __future__ import annotations

import numpy as np


def rot_axis_angle(axis, angle: float) -> np.ndarray:
    """Rodrigues rotation matrix for a unit axis and an angle in radians."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    x, y, z = a
    c, s = np.cos(angle), np.sin(angle)
    C = 1.0 - c
    return np.array([
        [c + x * x * C, x * y * C - z * s, x * z * C + y * s],
        [y * x * C + z * s, c + y * y * C, y * z * C - x * s],
        [z * x * C - y * s, z * y * C + x * s, c + z * z * C],
    ])


def rot_y(angle: float) -> np.ndarray:
    c, s = np.cos(angle), np.sin(angle)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def about_pivot(M: np.ndarray, pivot, translate=(0.0, 0.0, 0.0)) -> np.ndarray:
    """x -> M (x - pivot) + pivot + translate, as a 3x4 matrix."""
    p = np.asarray(pivot, dtype=np.float64)
    A = np.zeros((3, 4))
    A[:, :3] = M
    A[:, 3] = p - M @ p + np.asarray(translate, dtype=np.float64)
    return A


def identity() -> np.ndarray:
    A = np.zeros((3, 4))
    A[:, :3] = np.eye(3)
    return A


def quat_to_mat(q) -> np.ndarray:
    w, x, y, z = np.asarray(q, dtype=np.float64) / np.linalg.norm(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def random_rotation(stream) -> np.ndarray:
    """Uniform random rotation from a normalised Gaussian quaternion."""
    q = stream.normal(4)
    return quat_to_mat(q)


def to_f32(A) -> np.ndarray:
    return np.asarray(A, dtype=np.float64).astype(np.float32)


def random_quat(stream) -> np.ndarray:
    """Uniform random unit quaternion (w, x, y, z), w >= 0."""
    q = stream.normal(4)
    q = q / np.linalg.norm(q)
    return q if q[0] >= 0 else -q


def slerp(q0, q1, u: float) -> np.ndarray:
    """Spherical linear interpolation of unit quaternions (shortest arc)."""
    q0 = np.asarray(q0, np.float64)
    q1 = np.asarray(q1, np.float64)
    c = float(q0 @ q1)
    if c < 0.0:
        q1, c = -q1, -c
    if c > 0.9995:
        q = q0 + u * (q1 - q0)
        return q / np.linalg.norm(q)
    th = np.arccos(c)
    return (np.sin((1.0 - u) * th) * q0 + np.sin(u * th) * q1) / np.sin(th)
