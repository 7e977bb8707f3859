"""Seeded synthetic scene inputs shared by the GPU path and the CPU oracle.

This module only produces input data: meshes, light and camera descriptions,
albedos, filter settings and poses.  It holds none of the method's arithmetic
(no projection matrices, no rasterization, no shading); both the HIP library
and the oracle build those themselves from these plain numbers.

The scenes stand in for the paper's meshes, which are not available: models
sit inside roughly [-1, 1]^3 over a ground plane (supplementary, experiment
details), with pose, light-direction and complex-scene workloads shaped like
the paper's experiments (Sec. 5; Fig. 2 for the ~330k-triangle scene).

Conventions shared by both sides (plain numbers, stated once here):

* right-handed world, +y up; triangles wound counter-clockwise seen from the
  side their normal points to;
* every camera and light camera uses near = 0.1 and far = 20;
* directional lights: light camera at ``-dir_distance * w`` (w the unit travel
  direction) looking at the origin, orthographic with half-extent
  ``ortho_half``;
* point / spot lights: perspective light camera at the light position looking
  at ``target`` with vertical field of view ``fov_deg``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.special

NEAR = 0.1
FAR = 20.0
DIR_DISTANCE = 10.0
ORTHO_HALF = 4.5
MIN_VARIANCE = 1e-5


@dataclass
class Scene:
    verts: np.ndarray            # (V, 3) float32; posed vertices are in object space
    faces: np.ndarray            # (F, 3) int32
    albedo: np.ndarray           # (F, C) float32
    pose_count: int = 0          # the first pose_count vertices follow the pose
    pose_center: np.ndarray = field(default_factory=lambda: np.zeros(3, np.float32))
    pose: np.ndarray = field(default_factory=lambda: np.zeros(6, np.float32))  # axis-angle, translation


@dataclass
class Light:
    kind: str                    # 'directional' | 'point' | 'spot' | 'cubeface'
    param: np.ndarray            # (3,) float32: position, or travel direction for directional
    scene: int = 0
    target: np.ndarray = field(default_factory=lambda: np.zeros(3, np.float32))
    up: np.ndarray = field(default_factory=lambda: np.array([0, 1, 0], np.float32))
    fov_deg: float = 90.0        # perspective light cameras; spot: full cone angle
    resolution: int = 256
    filter: str = 'box'          # 'box' | 'gaussian'
    k: int = 5
    sigma: float = 0.0           # 0 -> (k - 1) / 3
    intensity: float = 1.0
    near: float = NEAR
    far: float = FAR
    dir_distance: float = DIR_DISTANCE
    ortho_half: float = ORTHO_HALF
    min_variance: float = MIN_VARIANCE
    antialias: bool = True
    face: int = 0                # 'cubeface': face index 0..5 (+x, -x, +y, -y, +z, -z)
    warp_exponent: float = 0.0   # > 0: exponential maps storing exp(c z), exp(2 c z)
    bleed_reduction: float = 0.0  # light-bleeding reduction amount in [0, 1)


@dataclass
class Camera:
    eye: np.ndarray
    target: np.ndarray
    fov_deg: float
    width: int
    height: int
    scene: int = 0
    up: np.ndarray = field(default_factory=lambda: np.array([0, 1, 0], np.float32))
    near: float = NEAR
    far: float = FAR


@dataclass
class Render:
    camera: int
    lights: List[int]


@dataclass
class Batch:
    name: str
    scenes: List[Scene]
    lights: List[Light]
    cameras: List[Camera]
    renders: List[Render]
    channels: int = 1
    antialias_camera: bool = True
    # Light parameters for the target image of the loss (same layout as Light.param).
    target_light_params: Optional[List[np.ndarray]] = None
    # Poses for the target image (cfg with a pose), one per scene.
    target_poses: Optional[List[np.ndarray]] = None


def f32(a):
    return np.asarray(a, dtype=np.float32)


# ----------------------------------------------------------------------------- meshes

def quad(half: float, y: float = 0.0):
    v = f32([[-half, y, -half], [half, y, -half], [half, y, half], [-half, y, half]])
    f = np.array([[0, 3, 2], [0, 2, 1]], np.int32)   # normal +y
    return v, f


def cube(center, half=0.5):
    c = np.asarray(center, np.float64)
    v = np.array([[x, y, z] for x in (-1, 1) for y in (-1, 1) for z in (-1, 1)], np.float64)
    v = v * half + c
    # vertex index = 4*(x>0) + 2*(y>0) + (z>0)
    quads = [
        (0, 1, 3, 2),  # -x
        (4, 6, 7, 5),  # +x
        (0, 4, 5, 1),  # -y
        (2, 3, 7, 6),  # +y
        (0, 2, 6, 4),  # -z
        (1, 5, 7, 3),  # +z
    ]
    f = []
    for a, b, cc, d in quads:
        f += [(a, b, cc), (a, cc, d)]
    return f32(v), np.array(f, np.int32)


def icosphere(subdiv: int):
    t = (1.0 + 5 ** 0.5) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    v = [np.array(p, np.float64) / np.linalg.norm(p) for p in v]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5),
         (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(subdiv):
        mid = {}

        def m(a, b):
            key = (min(a, b), max(a, b))
            if key not in mid:
                p = v[a] + v[b]
                v.append(p / np.linalg.norm(p))
                mid[key] = len(v) - 1
            return mid[key]
        nf = []
        for a, b, c in f:
            ab, bc, ca = m(a, b), m(b, c), m(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = nf
    return np.array(v, np.float64), np.array(f, np.int32)


def uv_sphere(n_lat: int, n_lon: int):
    """Unit UV sphere: 2 poles + (n_lat-1) rings; 2*n_lon*(n_lat-1) triangles."""
    verts = [(0.0, 1.0, 0.0)]
    for i in range(1, n_lat):
        th = np.pi * i / n_lat
        for j in range(n_lon):
            ph = 2 * np.pi * j / n_lon
            verts.append((np.sin(th) * np.cos(ph), np.cos(th), -np.sin(th) * np.sin(ph)))
    verts.append((0.0, -1.0, 0.0))
    v = np.array(verts, np.float64)
    S = len(verts) - 1

    def ring(i, j):
        return 1 + (i - 1) * n_lon + (j % n_lon)
    f = []
    for j in range(n_lon):
        f.append((0, ring(1, j), ring(1, j + 1)))
    for i in range(1, n_lat - 1):
        for j in range(n_lon):
            a, b = ring(i, j), ring(i, j + 1)
            c, d = ring(i + 1, j), ring(i + 1, j + 1)
            f += [(a, c, d), (a, d, b)]
    for j in range(n_lon):
        f.append((S, ring(n_lat - 1, j + 1), ring(n_lat - 1, j)))
    return v, np.array(f, np.int32)


def torus(R: float, r: float, n_u: int, n_v: int):
    u = 2 * np.pi * np.arange(n_u) / n_u
    w = 2 * np.pi * np.arange(n_v) / n_v
    U, Wv = np.meshgrid(u, w, indexing='ij')
    x = (R + r * np.cos(Wv)) * np.cos(U)
    z = -(R + r * np.cos(Wv)) * np.sin(U)
    y = r * np.sin(Wv)
    v = np.stack([x, y, z], -1).reshape(-1, 3)
    f = []
    for i in range(n_u):
        for j in range(n_v):
            a = i * n_v + j
            b = ((i + 1) % n_u) * n_v + j
            c = ((i + 1) % n_u) * n_v + (j + 1) % n_v
            d = i * n_v + (j + 1) % n_v
            f += [(a, b, c), (a, c, d)]
    return v, np.array(f, np.int32)


def grid_box(m: int):
    """Closed unit box [-1,1]^3 with an m x m quad grid per face (shared seams)."""
    vs, fs = [], []
    g = np.linspace(-1, 1, m + 1)
    A, B = np.meshgrid(g, g, indexing='ij')
    one = np.ones_like(A)
    faces_def = [  # (point(a,b), normal sign)
        np.stack([one, A, B], -1), np.stack([-one, B, A], -1),
        np.stack([B, one, A], -1), np.stack([A, -one, B], -1),
        np.stack([A, B, one], -1), np.stack([B, A, -one], -1),
    ]
    base = 0
    for P in faces_def:
        vs.append(P.reshape(-1, 3))
        for i in range(m):
            for j in range(m):
                a = base + i * (m + 1) + j
                b = base + (i + 1) * (m + 1) + j
                c = base + (i + 1) * (m + 1) + j + 1
                d = base + i * (m + 1) + j + 1
                fs += [(a, b, c), (a, c, d)]
        base += (m + 1) ** 2
    v = np.concatenate(vs)
    f = np.array(fs, np.int64)
    # weld the seams so the box is closed
    key = np.round(v * 1e6).astype(np.int64)
    _, first, inv = np.unique(key, axis=0, return_index=True, return_inverse=True)
    v = v[first]
    f = inv.reshape(-1)[f]
    # orient outward
    c = v[f].mean(1)
    n = np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]])
    flip = (n * c).sum(1) < 0
    f[flip] = f[flip][:, [0, 2, 1]]
    return v, f.astype(np.int32)


def real_sh_field(dirs: np.ndarray, lmax: int, rng, lmin: int = 1):
    """Random real spherical-harmonic field on unit directions, max |value| = 1."""
    x, y, z = dirs[:, 0], dirs[:, 1], dirs[:, 2]
    theta = np.arccos(np.clip(y, -1, 1))          # polar angle from +y
    phi = np.arctan2(-z, x)
    s = np.zeros(len(dirs))
    for l in range(lmin, lmax + 1):
        for m in range(-l, l + 1):
            Y = scipy.special.sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                b = np.sqrt(2) * Y.real
            elif m < 0:
                b = np.sqrt(2) * Y.imag
            else:
                b = Y.real
            s += rng.standard_normal() * b
    return s / np.abs(s).max()


def merge(parts):
    vs, fs, off = [], [], 0
    for v, f in parts:
        vs.append(np.asarray(v, np.float64))
        fs.append(np.asarray(f, np.int64) + off)
        off += len(v)
    return f32(np.concatenate(vs)), np.concatenate(fs).astype(np.int32)


# ----------------------------------------------------------------------------- configs

def _up_for(direction):
    d = np.asarray(direction, np.float64)
    d = d / np.linalg.norm(d)
    return f32([0, 0, 1]) if abs(d[1]) > 0.99 else f32([0, 1, 0])


def config0() -> Batch:
    """Tiny: 4x4 ground quad + unit cube at y=1; point light (2,4,1); 256^2."""
    qv, qf = quad(2.0)
    cv, cf = cube((0, 1, 0), 0.5)
    v, f = merge([(cv, cf), (qv, qf)])
    sc = Scene(verts=v, faces=f, albedo=np.full((len(f), 1), 0.8, np.float32))
    p = f32([2, 4, 1])
    light = Light('point', p, fov_deg=90.0, resolution=256, filter='box', k=5, up=_up_for(-p))
    cam = Camera(eye=f32([0, 3, 5]), target=f32([0, 0, 0]), fov_deg=45.0, width=256, height=256)
    return Batch('tiny', [sc], [light], [cam], [Render(0, [0])], channels=1,
                 target_light_params=[f32([2.3, 4, 1])])


def config1(seed: int = 1) -> Batch:
    """Icosphere (subdivision 4, jittered) over a plane; 60 degree spot; 512^2."""
    rng = np.random.default_rng(seed)
    sv, sf = icosphere(4)
    sv = sv + rng.normal(0.0, 0.02, sv.shape) + np.array([0, 1.5, 0])
    qv, qf = quad(4.0)
    v, f = merge([(sv, sf), (qv, qf)])
    sc = Scene(verts=v, faces=f, albedo=np.full((len(f), 1), 0.8, np.float32))
    p = f32([1, 5, 1])
    light = Light('spot', p, fov_deg=60.0, resolution=512, filter='gaussian', k=7, sigma=2.0,
                  up=_up_for(-p))
    cam = Camera(eye=f32([0, 3, 5]), target=f32([0, 0.75, 0]), fov_deg=45.0, width=512, height=512)
    return Batch('icosphere', [sc], [light], [cam], [Render(0, [0])], channels=1,
                 target_light_params=[f32([1.3, 5, 1])])


def blob_scene(i: int, with_pose: bool = True):
    rng = np.random.default_rng([2, i])
    T = int(rng.integers(2000, 20001))
    n_lat = max(3, int(round(np.sqrt(T / 4.0))))
    n_lon = 2 * n_lat
    bv, bf = uv_sphere(n_lat, n_lon)
    s = real_sh_field(bv, 3, rng)
    bv = bv * (1.0 + 0.15 * s)[:, None]
    qv, qf = quad(3.0)
    v, f = merge([(bv, bf), (qv, qf)])
    pose = f32(rng.normal(0.0, 0.1, 6))
    # light travel direction within 30 degrees of -y
    while True:
        w = rng.normal(size=3)
        w = w / np.linalg.norm(w)
        if -w[1] >= np.cos(np.radians(30.0)):
            break
    if with_pose:
        sc = Scene(verts=v, faces=f, albedo=np.full((len(f), 1), 0.8, np.float32),
                   pose_count=len(bv), pose_center=f32([0, 1.2, 0]), pose=pose)
    else:   # blob placed at its rest position, no pose parameters
        v = v.copy()
        v[:len(bv)] += f32([0, 1.2, 0])
        sc = Scene(verts=v, faces=f, albedo=np.full((len(f), 1), 0.8, np.float32))
    return sc, f32(w)


def config2(n_scenes: int = 64, resolution: int = 512, with_pose: bool = True) -> Batch:
    """Batched pose estimation: blobs of 2k..20k triangles, one directional light each."""
    scenes, lights, cams, renders = [], [], [], []
    for i in range(n_scenes):
        sc, w = blob_scene(i, with_pose)
        scenes.append(sc)
        lights.append(Light('directional', w, scene=i, resolution=resolution, filter='box', k=5,
                            up=_up_for(w)))
        cams.append(Camera(eye=f32([0, 3, 5]), target=f32([0, 0.8, 0]), fov_deg=45.0,
                           width=resolution, height=resolution, scene=i))
        renders.append(Render(i, [i]))
    return Batch('batched_pose', scenes, lights, cams, renders, channels=1,
                 target_poses=[np.zeros(6, np.float32) for _ in scenes] if with_pose else None)


def config3(n_lat: int = 158, sm_res: int = 1024, view_res: int = 512,
            n_cams: int = 16, n_lights: int = 8) -> Batch:
    """Multi-view: displaced UV sphere (SH degree <= 8); 8 point lights x 16 cameras."""
    rng = np.random.default_rng(3)
    bv, bf = uv_sphere(n_lat, 2 * n_lat)
    s = real_sh_field(bv, 8, rng)
    bv = bv * (1.0 + 0.1 * s)[:, None] + np.array([0, 1.2, 0])
    qv, qf = quad(2.5)
    v, f = merge([(bv, bf), (qv, qf)])
    sc = Scene(verts=v, faces=f, albedo=np.full((len(f), 1), 0.8, np.float32))
    lights, cams, renders = [], [], []
    for l in range(n_lights):
        a = 2 * np.pi * (l + 0.5) / n_lights
        p = f32([4 * np.cos(a), 4, 4 * np.sin(a)])
        lights.append(Light('point', p, resolution=sm_res, filter='gaussian', k=9, sigma=8.0 / 3.0,
                            up=_up_for(-p)))
    for c in range(n_cams):
        a = 2 * np.pi * c / n_cams
        cams.append(Camera(eye=f32([4 * np.cos(a), 2, 4 * np.sin(a)]), target=f32([0, 0, 0]),
                           fov_deg=45.0, width=view_res, height=view_res))
    for c in range(n_cams):
        for l in range(n_lights):
            renders.append(Render(c, [l]))
    return Batch('multi_view', [sc], lights, cams, renders, channels=1)


def config4(sm_res: int = 2048, width: int = 1920, height: int = 1080, n_objects: int = 20,
            detail: float = 1.0) -> Batch:
    """Complex scene: 20 objects (~330k triangles), RGB albedo, 3 point lights, 1080p.
    n_objects / detail shrink it for tests (detail scales the tessellation)."""
    rng = np.random.default_rng(4)
    parts, albedo = [], []
    centers, radii = [], []
    for o in range(n_objects):
        kind = o % 3
        scale = rng.uniform(0.3, 0.8)
        for _ in range(1000):
            c = rng.uniform(-3, 3, 2)
            if all(np.linalg.norm(c - cc) > (scale + rr) * 1.05 for cc, rr in zip(centers, radii)):
                break
        centers.append(c)
        radii.append(scale)
        if kind == 0:
            n = max(4, int(round(64 * detail)))
            v, f = uv_sphere(n, 2 * n)
        elif kind == 1:
            v, f = torus(0.7, 0.3, max(6, int(round(128 * detail))), max(4, int(round(64 * detail))))
        else:
            v, f = grid_box(max(1, int(round(37 * detail))))
            v = v / np.sqrt(3.0)
        v = v * scale + np.array([c[0], scale, c[1]])
        parts.append((v, f))
        albedo.append(np.repeat(rng.uniform(0.2, 0.9, (1, 3)), len(f), 0))
    qv, qf = quad(4.0)
    parts.append((qv, qf))
    albedo.append(np.full((2, 3), 0.8))
    v, f = merge(parts)
    sc = Scene(verts=v, faces=f, albedo=f32(np.concatenate(albedo)))
    lights = []
    for l in range(3):
        a = rng.uniform(0, 2 * np.pi)
        r = rng.uniform(2, 4)
        p = f32([r * np.cos(a), rng.uniform(4, 6), r * np.sin(a)])
        lights.append(Light('point', p, resolution=sm_res, filter='gaussian', k=11, sigma=10.0 / 3.0,
                            up=_up_for(-p)))
    cam = Camera(eye=f32([0, 4, 8]), target=f32([0, 0, 0]), fov_deg=45.0, width=width, height=height)
    return Batch('complex', [sc], lights, [cam], [Render(0, [0, 1, 2])], channels=3)


CONFIGS = {0: config0, 1: config1, 2: config2, 3: config3, 4: config4}


def random_image_grad(shape, seed):
    """Seeded upstream gradient for backward-only tests."""
    return f32(np.random.default_rng(seed).standard_normal(shape))


def grid_quad(half: float, y: float, n: int):
    """Horizontal square [-half, half]^2 at height y as an n x n grid of quads (normal +y)."""
    t = np.linspace(-half, half, n + 1)
    v = np.array([[x, y, z] for z in t for x in t], np.float64)
    f = []
    for r in range(n):
        for c in range(n):
            a, b = r * (n + 1) + c, r * (n + 1) + c + 1
            d, e = a + (n + 1), b + (n + 1)
            f += [(a, d, e), (a, e, b)]
    return f32(v), np.array(f, np.int32)


def minimal_plane(k: int = 5, antialias: bool = True, filter: str = 'box', resolution: int = 256,
                  view: int = 128, occluder_tess: int = 1, offset=(0.0, 0.0, 0.0), rotation=(0.0, 0.0, 0.0),
                  camera_height: float = 0.45) -> Batch:
    """The "minimal plane" setup of the convergence experiments (supplementary,
    experiment details): a square occluder (half-size 0.25 at y = 0.5) over a
    parallel square receiver (half-size 0.75 at y = 0), a directional light
    travelling straight down, and a camera between the two looking down at
    the receiver, so that the images show only the shadow.  The occluder's
    vertices come first and follow the scene pose: rotation `rotation`
    (axis-angle, about the occluder's centre) and translation `offset`
    relative to the reference, which is pose zero.  The occluder is an
    occluder_tess x occluder_tess grid of quads (2 occluder_tess^2
    triangles).  The camera sits at `camera_height` above the receiver's
    centre (below a slanted occluder's lowest point for the resolution
    experiment)."""
    ov, of = grid_quad(0.25, 0.0, occluder_tess)     # object space, centre (0, 0.5, 0)
    rv, rf = quad(0.75, 0.0)
    v, f = merge([(ov, of), (rv, rf)])
    sc = Scene(verts=v, faces=f, albedo=np.full((len(f), 1), 0.8, np.float32), pose_count=len(ov),
               pose_center=f32([0, 0.5, 0]), pose=f32([*rotation, *offset]))
    light = Light('directional', f32([0, -1, 0]), resolution=resolution, filter=filter, k=k,
                  up=f32([0, 0, 1]), ortho_half=1.0, antialias=antialias)
    cam = Camera(eye=f32([0, camera_height, 0]), target=f32([0, 0, 0]), fov_deg=120.0, width=view, height=view,
                 up=f32([0, 0, -1]))
    return Batch('minimal-plane', [sc], [light], [cam], [Render(0, [0])], channels=1,
                 target_poses=[np.zeros(6, np.float32)])


def cube_lights(position, scene: int = 0, resolution: int = 256, **kw) -> List[Light]:
    """The six cube-face lights of one omnidirectional point light at
    `position` (faces +x, -x, +y, -y, +z, -z); each keeps its own parameter,
    so the gradient for the shared position is the sum over the six."""
    p = f32(position)
    return [Light('cubeface', p.copy(), scene=scene, resolution=resolution, fov_deg=90.0, face=f, **kw)
            for f in range(6)]


# occluder centres and radii of the cube-light scene: one below the light, one
# towards +x, one towards -z and one on the -x / +z face seam
CUBE_SCENE_OCCLUDERS = (((0.15, 0.3, 0.1), 0.08), ((0.7, 0.35, 0.1), 0.1),
                        ((-0.1, 0.3, -0.6), 0.1), ((-0.45, 0.3, 0.45), 0.1))


def cube_light_scene(resolution: int = 128, view: int = 128, k: int = 5, antialias: bool = True,
                     light_pos=(0.03, 0.6, -0.02), ground_n: int = 16, sphere_subdiv: int = 2) -> Batch:
    """An omnidirectional point light low over a tessellated ground (half-size
    2 at y = 0) with four small icospheres around it whose shadows fall
    through different faces of the light's cube (below, +x, -z and across the
    -x / +z seam); nothing lies above the light, so the +y face sees an empty
    view.  One camera looks down at the ground from above and in front."""
    parts = [grid_quad(2.0, 0.0, ground_n)]
    for c, r in CUBE_SCENE_OCCLUDERS:
        sv, sf = icosphere(sphere_subdiv)
        parts.append((sv * r + np.asarray(c, np.float64), sf))
    v, f = merge(parts)
    sc = Scene(verts=v, faces=f, albedo=np.full((len(f), 1), 0.8, np.float32))
    lights = cube_lights(light_pos, resolution=resolution, k=k, antialias=antialias)
    cam = Camera(eye=f32([0, 3.2, 2.6]), target=f32([0, 0, 0]), fov_deg=60.0, width=view, height=view)
    tgt = f32(np.asarray(light_pos, np.float64) + [0.0713, 0.0, 0.0437])
    return Batch('cube-light', [sc], lights, [cam], [Render(0, list(range(6)))], channels=1,
                 target_light_params=[tgt.copy() for _ in range(6)])
