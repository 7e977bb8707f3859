"""Discrete part of the oracle: FP32 transform, fixed-point setup, brute-force
coverage with the depth|triangle-id minimum, and antialiasing edge choices.
(Oracle; test infrastructure only.)

Eq. (1) defines the shadow map as the minimum distance over scene points that
map to a shadow-map location; rasterization approximates it by sampling texel
centres and keeping, per texel, the nearest covering triangle (Sec. 4 uses an
existing rasterizer for exactly this).  The conventions below are this
project's reading where the paper is silent:

* clip = M [x,1] per row as ((m0*x + m1*y) + m2*z) + m3 in float32, no fused
  multiply-add; ndc = clip.xyz / clip.w (float32, correctly rounded);
* screen: sx = (ndc.x + 1) * (W/2), sy = (1 - ndc.y) * (H/2), pixel (i, j) has
  centre (i + 1/2, j + 1/2), j counts rows top to bottom;
* fixed point: X = rint(256 sx), Y = rint(256 sy) (round half to even); a
  triangle is discarded when a vertex has w <= 0, ndc.z < -1 or
  |sx|, |sy| >= 32768;
* each triangle is oriented to positive doubled area A (swapping its 2nd and
  3rd vertex when A < 0; facing = sign of A, 0 for A == 0 which is skipped);
* edge e is the edge opposite vertex e, with E_e(p) = dx*(py - ya) - dy*(px - xa)
  for the directed edge a -> b (inside positive); a sample on an edge is
  covered only for top edges (dy == 0, dx > 0) and left edges (dy < 0);
* depth z01_i = 0.5 * ndc.z_i + 0.5, interpolated as
  (z0 + b1*(z1 - z0)) + b2*(z2 - z0) with b_e = f32(E_e) * rA, where
  rA = f32(1) / f32(A) is the correctly rounded float32 reciprocal of the
  doubled area, formed once per triangle; samples with z01 outside [0, 1]
  are dropped;
* key = bits(z01) << 32 | triangle index; the smallest key wins (ties in
  depth go to the lower triangle index); background key = 2^64 - 1.

Everything here is elementwise numpy on float32 / int64 arrays.
"""
from __future__ import annotations

import numpy as np

F = np.float32
BG_KEY = np.uint64(0xFFFFFFFFFFFFFFFF)
SUB = 256                   # 8 sub-pixel bits
GUARD = 32768.0


def transform_f32(M, verts):
    """clip (n, 4) float32 from a float32 4x4 matrix and float32 vertices."""
    M = np.asarray(M, F)
    v = np.asarray(verts, F)
    x, y, z = v[:, 0], v[:, 1], v[:, 2]
    rows = [((M[r, 0] * x + M[r, 1] * y) + M[r, 2] * z) + M[r, 3] for r in range(4)]
    return np.stack(rows, 1).astype(F)


def setup(clip, faces, W, H):
    """Per-triangle fixed-point setup for one view.

    Returns dict with (all per triangle):
      idx    (F,3) int64 vertex indices in oriented order
      X, Y   (F,3) int64 fixed-point screen coordinates (oriented order)
      z      (F,3) float32 z01 (oriented order)
      A      (F,)  int64 doubled area (> 0 for valid)
      facing (F,)  int8  +1 / -1 orientation before re-orienting, 0 if skipped
      valid  (F,)  bool  rasterized at all
      swapped(F,)  bool  2nd and 3rd vertex exchanged
      culled (int) triangles dropped by the w / near / guard-band tests
    """
    clip = np.asarray(clip, F)
    faces = np.asarray(faces, np.int64)
    w = clip[:, 3]
    ndc_x = clip[:, 0] / w
    ndc_y = clip[:, 1] / w
    ndc_z = clip[:, 2] / w
    sx = (ndc_x + F(1)) * F(0.5 * W)
    sy = (F(1) - ndc_y) * F(0.5 * H)
    with np.errstate(invalid='ignore'):
        ok_v = (w > 0) & (ndc_z >= F(-1)) & (np.abs(sx) < F(GUARD)) & (np.abs(sy) < F(GUARD))
    X = np.where(ok_v, np.rint(sx * F(SUB)), 0).astype(np.int64)
    Y = np.where(ok_v, np.rint(sy * F(SUB)), 0).astype(np.int64)
    z01 = F(0.5) * ndc_z + F(0.5)

    idx = faces.copy()
    Xf, Yf, Zf = X[idx], Y[idx], z01[idx]
    okf = ok_v[idx].all(1)
    A = (Xf[:, 1] - Xf[:, 0]) * (Yf[:, 2] - Yf[:, 0]) - (Yf[:, 1] - Yf[:, 0]) * (Xf[:, 2] - Xf[:, 0])
    swapped = A < 0
    for arr in (idx, Xf, Yf, Zf):
        t = arr[swapped, 1].copy()
        arr[swapped, 1] = arr[swapped, 2]
        arr[swapped, 2] = t
    facing = np.where(A > 0, 1, np.where(A < 0, -1, 0)).astype(np.int8)
    A = np.abs(A)
    valid = okf & (A > 0)
    facing = np.where(valid, facing, 0).astype(np.int8)
    return dict(idx=idx, X=Xf, Y=Yf, z=Zf, A=A, facing=facing, valid=valid, swapped=swapped,
                culled=int((~okf).sum()), W=W, H=H)


def edge_ends(e):
    """Directed edge e (opposite vertex e) as (a, b) local vertex slots."""
    return (e + 1) % 3, (e + 2) % 3


def edge_value(st, t, e, px, py):
    """E_e of oriented triangle(s) t at fixed-point sample(s) (px, py), int64."""
    a, b = edge_ends(e)
    xa, ya = st['X'][t, a], st['Y'][t, a]
    dx = st['X'][t, b] - xa
    dy = st['Y'][t, b] - ya
    return dx * (py - ya) - dy * (px - xa)


def top_left(st, t, e):
    a, b = edge_ends(e)
    dx = st['X'][t, b] - st['X'][t, a]
    dy = st['Y'][t, b] - st['Y'][t, a]
    return (dy < 0) | ((dy == 0) & (dx > 0))


def coverage(st):
    """Brute force over every triangle and every sample of its bounding box.

    Returns (key (H,W) uint64, tri (H,W) int64 with -1 for background)."""
    W, H = st['W'], st['H']
    key = np.full((H, W), BG_KEY, np.uint64)
    for t in np.nonzero(st['valid'])[0]:
        X, Y = st['X'][t], st['Y'][t]
        i0 = max(0, int(X.min()) // SUB - 1)
        i1 = min(W - 1, int(X.max()) // SUB + 1)
        j0 = max(0, int(Y.min()) // SUB - 1)
        j1 = min(H - 1, int(Y.max()) // SUB + 1)
        if i0 > i1 or j0 > j1:
            continue
        jj, ii = np.meshgrid(np.arange(j0, j1 + 1), np.arange(i0, i1 + 1), indexing='ij')
        px = ii.astype(np.int64) * SUB + SUB // 2
        py = jj.astype(np.int64) * SUB + SUB // 2
        inside = np.ones(px.shape, bool)
        E = []
        for e in range(3):
            v = edge_value(st, t, e, px, py)
            E.append(v)
            inside &= (v > 0) | ((v == 0) & top_left(st, t, e))
        rA = F(1) / F(st['A'][t])
        b1 = E[1].astype(np.float64).astype(F) * rA
        b2 = E[2].astype(np.float64).astype(F) * rA
        z0, z1, z2 = st['z'][t]
        z = (z0 + b1 * (z1 - z0)) + b2 * (z2 - z0)
        inside &= (z >= F(0)) & (z <= F(1))
        bits = (z.view(np.uint32) & np.uint32(0x7FFFFFFF)).astype(np.uint64)
        k = (bits << np.uint64(32)) | np.uint64(t)
        sub = key[j0:j1 + 1, i0:i1 + 1]
        key[j0:j1 + 1, i0:i1 + 1] = np.where(inside, np.minimum(sub, k), sub)
    tri = np.where(key == BG_KEY, -1, (key & np.uint64(0xFFFFFFFF)).astype(np.int64))
    return key, tri


def aa_pairs(key, tri, st, adj):
    """Edge-antialiasing decisions for one view (this project's definition of
    the analytic silhouette antialiasing the paper takes from its rasterizer,
    Sec. 4 and 5; it is what makes the shadow map differentiable at primitive
    borders).

    For every horizontally or vertically adjacent pair of samples owned by
    different triangles: the sample with the smaller key is the front sample
    T, the other is O; the front triangle's edges with E_e(O) < 0 are exit
    edges, of which the first crossing (smallest float32 ratio
    E_e(T) / (E_e(T) - E_e(O)), lower e on ties) is chosen.  The pair is kept
    when that edge is a silhouette in this view (no neighbour, a non-manifold
    edge, or a neighbour of different facing) and, to handle each edge in
    exactly one direction, |dY| > |dX| for horizontal pairs and |dY| <= |dX|
    for vertical pairs.

    Returns dict of int64 arrays: T, O (flat sample index), t (front
    triangle), a, b (vertex indices of the chosen edge), horiz (bool)."""
    H, W = tri.shape
    out = {k: [] for k in ('T', 'O', 't', 'a', 'b', 'horiz')}
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing='ij')
    flat = jj * W + ii
    for horiz in (True, False):
        if horiz:
            P, Q = flat[:, :-1].ravel(), flat[:, 1:].ravel()
        else:
            P, Q = flat[:-1, :].ravel(), flat[1:, :].ravel()
        kf, tf = key.ravel(), tri.ravel()
        m = tf[P] != tf[Q]
        P, Q = P[m], Q[m]
        front_is_P = kf[P] < kf[Q]
        T = np.where(front_is_P, P, Q)
        O = np.where(front_is_P, Q, P)
        t = tf[T]
        pxT = (T % W) * SUB + SUB // 2
        pyT = (T // W) * SUB + SUB // 2
        pxO = (O % W) * SUB + SUB // 2
        pyO = (O // W) * SUB + SUB // 2
        alpha = np.full((len(T), 3), np.inf, F)
        for e in range(3):
            eT = edge_value(st, t, e, pxT, pyT)
            eO = edge_value(st, t, e, pxO, pyO)
            ex = eO < 0
            num = eT.astype(np.float64).astype(F)
            den = (eT - eO).astype(np.float64).astype(F)
            with np.errstate(divide='ignore', invalid='ignore'):
                r = num / den
            alpha[:, e] = np.where(ex, r, np.inf)
        has = np.isfinite(alpha).any(1)
        e_sel = np.argmin(alpha, 1)
        a_slot = (e_sel + 1) % 3
        b_slot = (e_sel + 2) % 3
        va = st['idx'][t, a_slot]
        vb = st['idx'][t, b_slot]
        dX = st['X'][t, b_slot] - st['X'][t, a_slot]
        dY = st['Y'][t, b_slot] - st['Y'][t, a_slot]
        nb = adj.neighbour(t, va, vb)
        fn = np.where(nb >= 0, st['facing'][np.maximum(nb, 0)], 0)
        sil = (nb < 0) | (fn != st['facing'][t])
        dir_ok = (np.abs(dY) > np.abs(dX)) if horiz else (np.abs(dY) <= np.abs(dX))
        keep = has & sil & dir_ok
        out['T'].append(T[keep])
        out['O'].append(O[keep])
        out['t'].append(t[keep])
        out['a'].append(va[keep])
        out['b'].append(vb[keep])
        out['horiz'].append(np.full(int(keep.sum()), horiz))
    return {k: np.concatenate(v) for k, v in out.items()}
