"""Brute-force float64 ray casting used only to pin the oracle (test
infrastructure only).

Moller-Trumbore ray/triangle intersection (Moller and Trumbore, "Fast,
minimum storage ray-triangle intersection", 1997), vectorized over rays and
looped over triangles.  It gives (i) the exact distance from a light to the
nearest surface along a ray, which the shadow map of Eq. (1) samples, and
(ii) binary visibility of Eq. (2) by testing whether any triangle blocks the
segment from a point to the light.
"""
from __future__ import annotations

import numpy as np


def intersect(orig, dirs, v, faces, t_max=np.inf, eps=1e-12):
    """Nearest hit distance along each ray (inf if none) and its triangle.

    orig (n,3) or (3,), dirs (n,3) (any length; distance in units of |dir|)."""
    orig = np.broadcast_to(np.asarray(orig, np.float64), np.asarray(dirs).shape)
    dirs = np.asarray(dirs, np.float64)
    v = np.asarray(v, np.float64)
    n = len(dirs)
    best = np.full(n, np.inf)
    tri = np.full(n, -1, np.int64)
    for f, (i0, i1, i2) in enumerate(np.asarray(faces)):
        e1 = v[i1] - v[i0]
        e2 = v[i2] - v[i0]
        p = np.cross(dirs, e2)
        det = p @ e1
        ok = np.abs(det) > eps
        inv = np.where(ok, 1.0 / np.where(ok, det, 1.0), 0.0)
        s = orig - v[i0]
        u = (s * p).sum(1) * inv
        q = np.cross(s, e1)
        w = (dirs * q).sum(1) * inv
        t = (q @ e2) * inv
        hit = ok & (u >= 0) & (w >= 0) & (u + w <= 1) & (t > 0) & (t < t_max) & (t < best)
        best = np.where(hit, t, best)
        tri = np.where(hit, f, tri)
    return best, tri


def occluded(points, light_pos, v, faces, offset=1e-4, directional_dir=None):
    """Binary shadow test (Eq. 2 semantics with exact geometry): True where a
    triangle lies between the point and the light.  For directional lights
    pass the unit travel direction; the ray then goes against it."""
    points = np.asarray(points, np.float64)
    if directional_dir is not None:
        d = -np.asarray(directional_dir, np.float64)
        d = np.broadcast_to(d / np.linalg.norm(d), points.shape)
        tmax = np.inf
    else:
        d = np.asarray(light_pos, np.float64) - points
        L = np.linalg.norm(d, axis=1, keepdims=True)
        d = d / L
        tmax = L[:, 0]
    o = points + offset * d
    t, _ = intersect(o, d, v, faces, t_max=tmax)
    return np.isfinite(t)
