"""Pins of the oracle's discrete part (CPU only): cameras, transform, fixed-point
setup, coverage and depth keys, adjacency.  Each test checks the oracle
against something other than itself: hand-derived fixtures, exact
integer arithmetic, textbook projection identities, brute-force ray casting.
"""
import math
import os

import numpy as np
import pytest
import torch

import scenegen as sg
from oracle import cameras, raster, raycast
from oracle.mesh import Adjacency
from oracle import pipeline as P

GOLD = os.path.join(os.path.dirname(__file__), 'golden')


def ndc_of(M, p):
    c = M.detach().numpy() @ np.append(np.asarray(p, np.float64), 1.0)
    return c[:3] / c[3], c[3]


# ----------------------------------------------------------------------------- O1 matrices

def test_camera_target_projects_to_centre_and_fov_edge():
    cam = sg.config0().cameras[0]
    M = cameras.camera_matrix(cam)
    ndc, w = ndc_of(M, cam.target)
    assert w > 0 and abs(ndc[0]) < 1e-6 and abs(ndc[1]) < 1e-6
    # a point at half the vertical FOV above the optical axis maps to y_ndc = 1
    eye = np.asarray(cam.eye, np.float64)
    f = np.asarray(cam.target, np.float64) - eye
    dist = np.linalg.norm(f)
    f /= dist
    s = np.cross(f, [0, 1, 0]); s /= np.linalg.norm(s)
    u = np.cross(s, f)
    p = eye + f * dist + u * dist * math.tan(math.radians(cam.fov_deg / 2))
    ndc, _ = ndc_of(M, p)
    assert abs(ndc[1] - 1.0) < 1e-6 and abs(ndc[0]) < 1e-6


def test_near_far_map_to_ndc_bounds():
    cam = sg.config0().cameras[0]
    M = cameras.camera_matrix(cam)
    eye = np.asarray(cam.eye, np.float64)
    f = np.asarray(cam.target, np.float64) - eye
    f /= np.linalg.norm(f)
    assert abs(ndc_of(M, eye + cam.near * f)[0][2] + 1) < 1e-5
    assert abs(ndc_of(M, eye + cam.far * f)[0][2] - 1) < 1e-5


def test_directional_light_camera_is_orthographic_along_w():
    b = sg.config2(n_scenes=1)
    L = b.lights[0]
    fr = cameras.light_frame(L, torch.as_tensor(L.param.astype(np.float64)))
    w = fr['w'].detach().numpy()
    eye = fr['pos'].detach().numpy()
    assert abs(np.linalg.norm(w) - 1) < 1e-6
    assert np.allclose(eye, -L.dir_distance * w, atol=1e-6)
    # moving along the travel direction leaves the shadow-map position unchanged
    p = np.array([0.3, 0.2, -0.1])
    a, _ = ndc_of(fr['M'], p)
    c, _ = ndc_of(fr['M'], p + 0.7 * w)
    assert np.allclose(a[:2], c[:2], atol=1e-6)
    # the orthographic half-extent maps to the NDC border
    s = np.cross(w, L.up.astype(np.float64)); s /= np.linalg.norm(s)
    e, _ = ndc_of(fr['M'], s * L.ortho_half)
    assert abs(abs(e[0]) - 1) < 1e-5


def test_transform_is_float32_fixed_order():
    rng = np.random.default_rng(0)
    M = rng.standard_normal((4, 4)).astype(np.float32)
    v = rng.standard_normal((50, 3)).astype(np.float32)
    c = raster.transform_f32(M, v)
    # same result from explicit per-element float32 scalar arithmetic
    for n in range(50):
        for r in range(4):
            acc = np.float32(M[r, 0]) * v[n, 0]
            acc = np.float32(acc + np.float32(M[r, 1]) * v[n, 1])
            acc = np.float32(acc + np.float32(M[r, 2]) * v[n, 2])
            acc = np.float32(acc + M[r, 3])
            assert c[n, r] == acc
    # and within float32 rounding of the float64 product
    ref = v.astype(np.float64) @ M[:, :3].T.astype(np.float64) + M[:, 3]
    assert np.allclose(c, ref, rtol=1e-5, atol=1e-5)


# ----------------------------------------------------------------------------- O2/O3 raster

def ndc_view(tris_ndc, W, H):
    """Setup for triangles given directly in NDC (w = 1, identity matrix)."""
    v = np.asarray(tris_ndc, np.float32).reshape(-1, 2)
    clip = np.concatenate([v, np.zeros((len(v), 1), np.float32), np.ones((len(v), 1), np.float32)], 1)
    faces = np.arange(len(v)).reshape(-1, 3)
    return raster.setup(clip, faces, W, H), faces


def test_golden_4x4_coverage():
    rows = [l for l in open(os.path.join(GOLD, 'coverage_4x4.txt')) if not l.startswith('#') and l.strip()]
    want = np.array([[int(x) for x in l.split()] for l in rows])
    st, _ = ndc_view([[-1, 1], [1, 1], [-1, -1], [1, 1], [1, -1], [-1, -1]], 4, 4)
    key, tri = raster.coverage(st)
    assert np.array_equal(tri, want)


def per_triangle_inside(st, W, H):
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing='ij')
    px = ii.astype(np.int64) * 256 + 128
    py = jj.astype(np.int64) * 256 + 128
    masks = []
    for t in range(len(st['A'])):
        m = np.ones((H, W), bool) & bool(st['valid'][t])
        for e in range(3):
            v = raster.edge_value(st, t, e, px, py)
            m &= (v > 0) | ((v == 0) & raster.top_left(st, t, e))
        masks.append(m)
    return np.array(masks)


@pytest.mark.parametrize('W,H', [(37, 23), (64, 64)])
def test_fullscreen_quad_covers_every_pixel_exactly_once(W, H):
    quad = [[-1, 1], [1, 1], [1, -1], [-1, 1], [1, -1], [-1, -1]]
    st, _ = ndc_view(quad, W, H)
    m = per_triangle_inside(st, W, H)
    assert np.all(m.sum(0) == 1)
    _, tri = raster.coverage(st)
    assert np.all(tri >= 0)


def test_fan_around_pixel_centre_has_one_owner_everywhere():
    W = H = 16
    c = np.array([2 * (7 + 0.5) / W - 1, 1 - 2 * (9 + 0.5) / H])   # exactly pixel (7, 9)
    ring = []
    for k in range(7):   # uneven angles, some edges pass through other pixel centres
        a = 2 * np.pi * k / 7 + 0.1
        ring.append(c + 0.6 * np.array([np.cos(a), np.sin(a)]))
    ring.append(c + np.array([0.0, 0.5]))   # vertical edge through the centre column
    ring.sort(key=lambda p: math.atan2(p[1] - c[1], p[0] - c[0]))
    tris = []
    for k in range(len(ring)):
        tris += [c, ring[k], ring[(k + 1) % len(ring)]]
    st, _ = ndc_view(tris, W, H)
    m = per_triangle_inside(st, W, H)
    cnt = m.sum(0)
    assert cnt[9, 7] == 1
    assert cnt.max() == 1
    # pixels strictly inside the fan's inscribed disc are all covered
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing='ij')
    r = np.hypot((ii + 0.5) - (c[0] + 1) * W / 2, (jj + 0.5) - (1 - c[1]) * H / 2)
    assert np.all(cnt[r < 2.0] == 1)


def test_int64_edge_function_equals_python_integers_near_guard_band():
    rng = np.random.default_rng(5)
    n = 2000
    lim = 32767 * 256
    X = rng.integers(-lim, lim, (n, 3)).astype(np.int64)
    Y = rng.integers(-lim, lim, (n, 3)).astype(np.int64)
    st = dict(X=X, Y=Y)
    px = rng.integers(-lim, lim, n).astype(np.int64)
    py = rng.integers(-lim, lim, n).astype(np.int64)
    for e in range(3):
        got = raster.edge_value(st, np.arange(n), e, px, py)
        a, b = (e + 1) % 3, (e + 2) % 3
        for i in range(0, n, 97):
            xa, ya, xb, yb = int(X[i, a]), int(Y[i, a]), int(X[i, b]), int(Y[i, b])
            want = (xb - xa) * (int(py[i]) - ya) - (yb - ya) * (int(px[i]) - xa)
            assert int(got[i]) == want


def test_snap_round_trip_within_half_subpixel():
    b = sg.config1()
    sc, cam = b.scenes[0], b.cameras[0]
    M = cameras.camera_matrix(cam).detach().numpy().astype(np.float32)
    clip = raster.transform_f32(M, sc.verts)
    st = raster.setup(clip, sc.faces, cam.width, cam.height)
    ok = st['valid']
    c64 = clip.astype(np.float64)
    sx = (c64[:, 0] / c64[:, 3] + 1) * cam.width / 2
    sy = (1 - c64[:, 1] / c64[:, 3]) * cam.height / 2
    idx = st['idx'][ok]
    assert np.abs(st['X'][ok] / 256.0 - sx[idx]).max() <= 1 / 512 + 1e-4
    assert np.abs(st['Y'][ok] / 256.0 - sy[idx]).max() <= 1 / 512 + 1e-4


def test_depth_tie_goes_to_lower_triangle_index():
    # two identical triangles: the lower index owns every covered pixel
    t = [[-0.8, -0.8], [0.8, -0.8], [0.0, 0.8]]
    st, _ = ndc_view(t + t, 32, 32)
    _, tri = raster.coverage(st)
    assert set(np.unique(tri)) == {-1, 0}


def test_nearest_surface_wins_and_distance_matches_ray_casting():
    """Resolved distances at texel centres equal float64 ray casting (Eq. 1:
    nearest surface along each light ray), which validates the depth key's
    ordering and the perspective-correct barycentrics of the resolve."""
    b = sg.config0()
    L = b.lights[0]
    L.resolution = 96
    base, poses, lp, alb = P.scene_leaves(b, requires_grad=False)
    out = P.render(b, P.world_vertices(b, base, poses), lp, alb)
    ls = out['lights'][0]
    S = L.resolution
    tri = ls['rv']['tri']
    jj, ii = np.nonzero(tri >= 0)
    # ray of the light camera through each covered texel centre (the line
    # that unprojects to the texel at every depth), cast in float64
    fr = ls['frame']
    Minv = np.linalg.inv(fr['M'].detach().numpy())

    def unproject(zn):
        h = np.stack([2 * (ii + 0.5) / S - 1, 1 - 2 * (jj + 0.5) / S,
                      np.full(len(ii), zn), np.ones(len(ii))], 1) @ Minv.T
        return h[:, :3] / h[:, 3:]
    a, c = unproject(-1.0), unproject(1.0)
    d = (c - a) / np.linalg.norm(c - a, axis=1, keepdims=True)
    t_hit, f_hit = raycast.intersect(a, d, b.scenes[0].verts, b.scenes[0].faces)
    x = a + t_hit[:, None] * d
    dist = np.linalg.norm(x - L.param.astype(np.float64), axis=1)
    z = ls['F0'][0].detach().numpy()[jj, ii]
    # away from triangle borders the same triangle is hit and distances agree
    same = (f_hit == tri[jj, ii]) & np.isfinite(t_hit)
    assert same.mean() > 0.97
    assert np.allclose(z[same] * L.far, dist[same], rtol=1e-9, atol=0)


# ----------------------------------------------------------------------------- O5 adjacency

def test_adjacency_counts_cube_and_quad():
    cv, cf = sg.cube((0, 1, 0))
    a = Adjacency(cf)
    assert a.num_shared_edges() == 18 and a.num_boundary_edges() == 0
    qv, qf = sg.quad(2.0)
    q = Adjacency(qf)
    assert q.num_shared_edges() == 1 and q.num_boundary_edges() == 4


def test_cube_silhouette_from_light_is_closed_loop():
    b = sg.config0()
    L = b.lights[0]
    base, poses, lp, alb = P.scene_leaves(b, requires_grad=False)
    fr = cameras.light_frame(L, lp[0])
    sc = b.scenes[0]
    clip = raster.transform_f32(fr['M'].detach().numpy().astype(np.float32), sc.verts)
    st = raster.setup(clip, sc.faces, L.resolution, L.resolution)
    adj = Adjacency(sc.faces)
    cube_faces = np.arange(12)
    deg = {}
    nsil = 0
    for t in cube_faces:
        for e in range(3):
            a_, b_ = raster.edge_ends(e)
            va, vb = st['idx'][t, a_], st['idx'][t, b_]
            nb = int(adj.neighbour(np.array([t]), np.array([va]), np.array([vb]))[0])
            if st['facing'][t] > 0 and (nb < 0 or st['facing'][nb] != st['facing'][t]):
                nsil += 1
                for v in (va, vb):
                    deg[v] = deg.get(v, 0) + 1
    assert nsil >= 4
    assert all(d == 2 for d in deg.values())


def test_pose_rotation_matches_library_rotvec():
    from scipy.spatial.transform import Rotation
    from oracle.mesh import rodrigues
    rng = np.random.default_rng(4)
    for _ in range(20):
        r = rng.normal(0, 0.7, 3)
        R = rodrigues(torch.as_tensor(r)).numpy()
        assert np.allclose(R, Rotation.from_rotvec(r).as_matrix(), atol=1e-14)
    assert np.allclose(rodrigues(torch.zeros(3, dtype=torch.float64)).numpy(), np.eye(3))
