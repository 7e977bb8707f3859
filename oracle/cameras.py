"""Viewer and light cameras, float64 torch (oracle; test infrastructure only).

The shadow map is parameterized over a plane of rays from the light through a
projective camera map L (Sec. 3).  Light cameras follow the supplementary
renderer details: a directional light uses an orthographic camera placed far
outside the scene facing the origin; a spot light uses a perspective camera at
its position with a configurable field of view.  A point light here uses the
same perspective construction (one shadow map per light, Sec. 5).

An omnidirectional point light is parameterized over several planes arranged
as a box around it, as Sec. 3 allows when one plane does not cover every ray
(Sec. 5 names this route): six "cube-face" lights share the position, face
f = 2a + s looking along +e_a (s = 0) or -e_a (s = 1) through a square 90
degree frustum, and face f shades exactly the points whose direction from
the light has dominant axis a with sign s (ties to the lower axis).

Matrices are textbook OpenGL-style (right-handed, camera looking down -z,
clip -> NDC in [-1,1]^3).  Camera settings (field of view, near and far
planes, orthographic extent, eye distance) enter as the float32 values a
scene description holds, like every other scene input.  The matrix the discrete raster uses is the float32
rounding of the float64 matrix; the continuous part uses the same rounded
values while autograd differentiates the float64 construction
("straight-through" rounding), so both parts see one light camera.
"""
from __future__ import annotations

import functools
import math

import numpy as np
import torch

D = torch.float64


def _t(x):
    return torch.as_tensor(np.asarray(x, dtype=np.float64), dtype=D)


def normalize(v):
    return v / torch.sqrt((v * v).sum(-1, keepdim=True))


def look_at(eye, target, up):
    f = normalize(target - eye)
    s = normalize(torch.linalg.cross(f, up))
    u = torch.linalg.cross(s, f)
    z = torch.zeros((), dtype=D)
    o = torch.ones((), dtype=D)
    return torch.stack([
        torch.cat([s, -(s * eye).sum().reshape(1)]),
        torch.cat([u, -(u * eye).sum().reshape(1)]),
        torch.cat([-f, (f * eye).sum().reshape(1)]),
        torch.stack([z, z, z, o]),
    ])


def f32(x):
    """A scalar camera setting as the float32 value the scene description holds."""
    return float(np.float32(x))


def perspective(fov_deg, aspect, near, far):
    t = 1.0 / math.tan(math.radians(fov_deg) / 2.0)
    return _t([[t / aspect, 0, 0, 0],
               [0, t, 0, 0],
               [0, 0, (far + near) / (near - far), 2 * far * near / (near - far)],
               [0, 0, -1, 0]])


def orthographic(half, near, far):
    return _t([[1.0 / half, 0, 0, 0],
               [0, 1.0 / half, 0, 0],
               [0, 0, -2.0 / (far - near), -(far + near) / (far - near)],
               [0, 0, 0, 1]])


# When True, matrices and light-frame vectors carry their float32-rounded
# values (the precision the renderer works in) while autograd differentiates
# the float64 construction.  Finite-difference checks switch it off: the
# rounding is a staircase in the light parameters that central differences
# with tiny steps would see as noise.
ROUND_TO_F32 = True


def round_f32(x):
    """float32 rounding of a float64 tensor, differentiated as the identity."""
    if not ROUND_TO_F32:
        return x
    return x + (x.detach().to(torch.float32).to(D) - x.detach())


def camera_matrix(cam):
    """Viewer camera VP (float64), aspect = width / height."""
    V = look_at(_t(cam.eye), _t(cam.target), _t(cam.up))
    P = perspective(f32(cam.fov_deg), cam.width / cam.height, f32(cam.near), f32(cam.far))
    return round_f32(P @ V)


# viewing direction and up vector of cube face f = 2a + s
CUBE_AXES = ((1.0, 0.0, 0.0), (-1.0, 0.0, 0.0), (0.0, 1.0, 0.0),
             (0.0, -1.0, 0.0), (0.0, 0.0, 1.0), (0.0, 0.0, -1.0))
CUBE_UPS = ((0.0, 1.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0),
            (0.0, 0.0, 1.0), (0.0, 1.0, 0.0), (0.0, 1.0, 0.0))


def cube_face_of(d):
    """Cube face owning each direction d (n, 3): the axis of largest |d_a|
    (the first one on ties), and its sign (d_a < 0 -> the odd face)."""
    d = np.asarray(d, np.float64)
    a = np.argmax(np.abs(d), axis=1)
    neg = d[np.arange(len(d)), a] < 0
    return 2 * a + neg.astype(np.int64)


def cube_face_basis(f):
    """Viewing axis, right and up vectors of cube face f (look_at's frame):
    a texel at NDC (u, v) of the face's map looks along a + u s + v up."""
    a = np.array(CUBE_AXES[f])
    s = np.cross(a, np.array(CUBE_UPS[f]))
    s = s / np.linalg.norm(s)
    return a, s, np.cross(s, a)


# edges of a face's map: 0 left (u = -1), 1 right (u = +1), 2 top (v = +1), 3 bottom (v = -1)
def cube_edge_table():
    """table[f][e] = (g, e', flip): the face across edge e of face f, the edge
    of g's map on the same cube edge, and whether texel indices along the
    edge run backwards from one map to the other.  Derived from the faces'
    frames: the two points of f's edge at along-coordinates -1/2 and +1/2 are
    projected into g."""
    table = []
    for f in range(6):
        a, s, u = cube_face_basis(f)
        row = []
        for e in range(4):
            out = (-s, s, u, -u)[e]
            g = [k for k in range(6) if np.allclose(CUBE_AXES[k], out)][0]
            ag, sg, ug = cube_face_basis(g)
            along = u if e < 2 else s
            pts = [a + out + tau * along for tau in (-0.5, 0.5)]
            uv = [(p @ sg / (p @ ag), p @ ug / (p @ ag)) for p in pts]
            if abs(abs(uv[0][0]) - 1) < 1e-9 and abs(uv[0][0] - uv[1][0]) < 1e-9:
                e2 = 0 if uv[0][0] < 0 else 1
                g_along = [q[1] for q in uv]
            else:
                e2 = 2 if uv[0][1] > 0 else 3
                g_along = [q[0] for q in uv]
            # texel index direction as tau grows: v runs against j, u with i
            df = -1 if e < 2 else 1
            dg = np.sign(g_along[1] - g_along[0]) * (-1 if e2 < 2 else 1)
            row.append((g, e2, bool(df != dg)))
        table.append(row)
    return table


@functools.lru_cache(maxsize=16)
def cube_pad_sources(S, P):
    """What every position of a cube face's map padded by P texels reads, as
    four (6 S S)-flat texel indices and their weights, each (6, S + 2P,
    S + 2P, 4): inside the face, the texel itself; in an edge block, the
    bilinear sample (clamp-to-edge) of the neighbouring face's map along the
    direction the padded texel centre looks along when the face's plane is
    continued across the edge; in a corner block, which no face covers, the
    face's own corner texel."""
    tab = cube_edge_table()
    Sp = S + 2 * P
    idx = np.zeros((6, Sp, Sp, 4), np.int64)
    wgt = np.zeros((6, Sp, Sp, 4))
    for f in range(6):
        a, s, u = cube_face_basis(f)
        for pj in range(Sp):
            for pi in range(Sp):
                i, j = pi - P, pj - P
                ins_i, ins_j = 0 <= i < S, 0 <= j < S
                if ins_i == ins_j:
                    ii, jj = min(max(i, 0), S - 1), min(max(j, 0), S - 1)
                    idx[f, pj, pi] = (f * S + jj) * S + ii
                    wgt[f, pj, pi, 0] = 1.0
                    continue
                e = 0 if i < 0 else 1 if i >= S else 2 if j < 0 else 3
                g = tab[f][e][0]
                d = a + ((2 * i + 1) / S - 1) * s + (1 - (2 * j + 1) / S) * u
                ag, sg, ug = cube_face_basis(g)
                ug_ndc, vg_ndc = (d @ sg) / (d @ ag), (d @ ug) / (d @ ag)
                sx = (ug_ndc + 1) * S / 2 - 0.5
                sy = (1 - vg_ndc) * S / 2 - 0.5
                x0, y0 = math.floor(sx), math.floor(sy)
                fx, fy = sx - x0, sy - y0
                xs = [min(max(x0, 0), S - 1), min(max(x0 + 1, 0), S - 1)]
                ys = [min(max(y0, 0), S - 1), min(max(y0 + 1, 0), S - 1)]
                taps = [(ys[0], xs[0], (1 - fx) * (1 - fy)), (ys[0], xs[1], fx * (1 - fy)),
                        (ys[1], xs[0], (1 - fx) * fy), (ys[1], xs[1], fx * fy)]
                for q, (yy, xx, w) in enumerate(taps):
                    idx[f, pj, pi, q] = (g * S + yy) * S + xx
                    wgt[f, pj, pi, q] = w
    return idx, wgt


def light_frame(light, param):
    """Light camera and the quantities the lookup needs, from the light's
    differentiable parameter (position, or travel direction for directional).

    Returns dict with M (4x4 view-projection), pos (point/spot: position;
    directional: camera eye on the plane distances are measured from), w
    (directional: unit travel direction; spot: cone axis; cube face: face
    axis), far, kind, cos_half (spot cone), face (cube face index)."""
    if light.kind == 'directional':
        w = normalize(param)
        eye = -f32(light.dir_distance) * w
        V = look_at(eye, torch.zeros(3, dtype=D), _t(light.up))
        P = orthographic(f32(light.ortho_half), f32(light.near), f32(light.far))
        return dict(M=round_f32(P @ V), pos=round_f32(eye), w=round_f32(w), far=f32(light.far),
                    kind='directional', cos_half=None)
    if light.kind == 'cubeface':
        axis = _t(CUBE_AXES[light.face])
        V = look_at(param, param + axis, _t(CUBE_UPS[light.face]))
        P = perspective(90.0, 1.0, f32(light.near), f32(light.far))
        return dict(M=round_f32(P @ V), pos=param, w=axis, far=f32(light.far), kind='cubeface',
                    cos_half=None, face=light.face)
    tgt = _t(light.target)
    V = look_at(param, tgt, _t(light.up))
    P = perspective(f32(light.fov_deg), 1.0, f32(light.near), f32(light.far))
    axis = normalize(tgt - param)
    cos_half = math.cos(math.radians(light.fov_deg) / 2.0) if light.kind == 'spot' else None
    return dict(M=round_f32(P @ V), pos=param, w=round_f32(axis), far=f32(light.far), kind=light.kind,
                cos_half=cos_half)
