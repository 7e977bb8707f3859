"""Mesh helpers for the oracle (test infrastructure only): undirected edge
adjacency for silhouette tests, and the posed-vertex transform.

An edge of a triangle is a silhouette in a view when no other triangle shares
it, when more than two triangles share it (non-manifold), or when the
neighbour across it faces the other way in that view.  Only silhouette edges
are antialiased: interior edges between triangles of the same facing are
continuities of the surface, not borders of a primitive region.
"""
from __future__ import annotations

import numpy as np
import torch


class Adjacency:
    def __init__(self, faces):
        f = np.asarray(faces, np.int64)
        self.F = len(f)
        self.nv = int(f.max()) + 1 if len(f) else 0
        a = np.concatenate([f[:, 1], f[:, 2], f[:, 0]])
        b = np.concatenate([f[:, 2], f[:, 0], f[:, 1]])
        owner = np.concatenate([np.arange(len(f))] * 3)
        k = np.minimum(a, b) * self.nv + np.maximum(a, b)
        order = np.argsort(k, kind='stable')
        self.keys = k[order]
        self.owner = owner[order]
        self.ukeys, self.start, self.count = np.unique(self.keys, return_index=True, return_counts=True)

    def neighbour(self, t, va, vb):
        """Face across undirected edge {va, vb} from face t: -1 boundary,
        -2 non-manifold, else the other face (vectorized)."""
        t = np.asarray(t, np.int64)
        k = np.minimum(va, vb) * self.nv + np.maximum(va, vb)
        pos = np.searchsorted(self.ukeys, k)
        st = self.start[pos]
        cnt = self.count[pos]
        f0 = self.owner[st]
        f1 = self.owner[np.minimum(st + 1, len(self.owner) - 1)]
        other = np.where(f0 == t, f1, f0)
        return np.where(cnt == 1, -1, np.where(cnt > 2, -2, other))

    def num_shared_edges(self):
        return int((self.count == 2).sum())

    def num_boundary_edges(self):
        return int((self.count == 1).sum())


def rodrigues(r):
    """Rotation matrix of an axis-angle vector (float64 torch, differentiable)."""
    th2 = (r * r).sum()
    th = torch.sqrt(th2 + 1e-300)
    K = torch.zeros(3, 3, dtype=r.dtype)
    K = torch.stack([
        torch.stack([torch.zeros((), dtype=r.dtype), -r[2], r[1]]),
        torch.stack([r[2], torch.zeros((), dtype=r.dtype), -r[0]]),
        torch.stack([-r[1], r[0], torch.zeros((), dtype=r.dtype)]),
    ])
    I = torch.eye(3, dtype=r.dtype)
    if float(th2.detach()) < 1e-24:
        return I + K
    return I + torch.sin(th) / th * K + (1 - torch.cos(th)) / th2 * (K @ K)


def posed_vertices(scene, pose):
    """World vertices: the first pose_count follow R(r) v + c + t, the rest are fixed.
    pose: (6,) float64 tensor (axis-angle r, translation t)."""
    v = torch.as_tensor(np.asarray(scene.verts, np.float64))
    n = scene.pose_count
    if n == 0:
        return v
    R = rodrigues(pose[:3])
    c = torch.as_tensor(np.asarray(scene.pose_center, np.float64))
    moved = v[:n] @ R.T + c + pose[3:]
    return torch.cat([moved, v[n:]], 0)
