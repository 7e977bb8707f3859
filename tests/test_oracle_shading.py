"""Pins of the oracle's continuous part (CPU only): filter, bilinear fetch,
Chebyshev visibility and its derivative, edge smoothing, shading,
hard-shadow limit against ray casting, finite differences of the loss.
"""
import math
import os

import numpy as np
import pytest
import torch

import scenegen as sg
from oracle import cameras, raster, raycast
from oracle import pipeline as P
from oracle.mesh import Adjacency

GOLD = os.path.join(os.path.dirname(__file__), 'golden')
D = torch.float64


# ----------------------------------------------------------------------------- O7 filter

def test_taps_sum_to_one_and_match_closed_form():
    for kind in ('box', 'gaussian'):
        for k in (1, 3, 5, 7, 9, 11):
            w = P.filter_taps(kind, k, 0.0)
            assert len(w) == k and abs(w.sum() - 1) < 1e-15
            assert np.allclose(w, w[::-1])
    assert np.all(P.filter_taps('box', 5, 0) == 1 / 5)
    rows = [l.split() for l in open(os.path.join(GOLD, 'gaussian_taps_k7_sigma2.txt')) if not l.startswith('#')]
    want = np.array([float(r[1]) for r in rows if r])
    assert np.allclose(P.filter_taps('gaussian', 7, 2.0), want, atol=1e-9)


def brute_force_2d(img, w):
    k = len(w)
    r = k // 2
    C, H, W = img.shape
    out = np.zeros_like(img)
    for y in range(H):
        for x in range(W):
            acc = np.zeros(C)
            for a in range(k):
                for b in range(k):
                    yy = min(max(y + a - r, 0), H - 1)
                    xx = min(max(x + b - r, 0), W - 1)
                    acc += w[a] * w[b] * img[:, yy, xx]
            out[:, y, x] = acc
    return out


@pytest.mark.parametrize('kind,k', [('box', 5), ('gaussian', 7), ('gaussian', 3)])
def test_separable_equals_direct_2d(kind, k):
    rng = np.random.default_rng(k)
    img = rng.standard_normal((2, 13, 11))
    w = P.filter_taps(kind, k, 0.0)
    got = P.filter_separable(torch.as_tensor(img), w).numpy()
    assert np.allclose(got, brute_force_2d(img, w), atol=1e-13)


def test_filter_keeps_constants_and_interior_affine():
    w = P.filter_taps('gaussian', 9, 0.0)
    c = torch.full((2, 20, 17), 0.37, dtype=D)
    assert torch.allclose(P.filter_separable(c, w), c, atol=1e-15)
    yy, xx = torch.meshgrid(torch.arange(20, dtype=D), torch.arange(17, dtype=D), indexing='ij')
    a = (0.3 + 0.01 * xx - 0.02 * yy)[None].repeat(2, 1, 1)
    out = P.filter_separable(a, w)
    r = 4
    assert torch.allclose(out[:, r:-r, r:-r], a[:, r:-r, r:-r], atol=1e-14)


def test_filter_adjoint_dot_product_with_clamp_fold():
    rng = np.random.default_rng(2)
    x = torch.as_tensor(rng.standard_normal((2, 12, 9)), dtype=D).requires_grad_(True)
    y = torch.as_tensor(rng.standard_normal((2, 12, 9)), dtype=D)
    w = P.filter_taps('gaussian', 7, 2.0)
    Gx = P.filter_separable(x, w)
    (g,) = torch.autograd.grad((Gx * y).sum(), x)
    # explicit transpose: out-of-range taps fold onto the border samples
    def T1(v, axis):
        n = v.shape[axis]
        r = len(w) // 2
        out = np.zeros_like(v)
        for i in range(n):
            for j in range(len(w)):
                m = min(max(i + j - r, 0), n - 1)
                sl_o = [slice(None)] * 3
                sl_i = [slice(None)] * 3
                sl_o[axis] = m
                sl_i[axis] = i
                out[tuple(sl_o)] += w[j] * v[tuple(sl_i)]
        return out
    gt = T1(T1(y.numpy(), 1), 2)
    assert np.allclose(g.numpy(), gt, atol=1e-13)
    assert abs(float((Gx * y).sum().detach()) - float((x.detach() * torch.as_tensor(gt)).sum())) < 1e-12


# ----------------------------------------------------------------------------- O8 bilinear

def test_bilinear_constant_affine_and_texel_centres():
    S = 8
    yy, xx = torch.meshgrid(torch.arange(S, dtype=D), torch.arange(S, dtype=D), indexing='ij')
    maps = torch.stack([0.2 + 0.05 * xx + 0.03 * yy, torch.full((S, S), 0.7, dtype=D)])
    rng = np.random.default_rng(0)
    sx = torch.as_tensor(rng.uniform(0, S - 1, 100))
    sy = torch.as_tensor(rng.uniform(0, S - 1, 100))
    v = P.bilinear(maps, sx, sy)
    assert torch.allclose(v[:, 0], 0.2 + 0.05 * sx + 0.03 * sy, atol=1e-14)
    assert torch.allclose(v[:, 1], torch.full_like(sx, 0.7), atol=1e-15)
    ix = torch.as_tensor([0.0, 3.0, 7.0])
    iy = torch.as_tensor([5.0, 0.0, 7.0])
    v = P.bilinear(maps, ix, iy)
    assert torch.allclose(v[:, 0], maps[0, iy.long(), ix.long()], atol=0)
    # clamp-to-edge: beyond the border the edge texel is returned
    v = P.bilinear(maps, torch.as_tensor([-0.4, 7.3]), torch.as_tensor([2.0, 2.0]))
    assert torch.allclose(v[:, 0], maps[0, 2, [0, 7]], atol=0)


# ----------------------------------------------------------------------------- O9 Chebyshev

def test_visibility_range_and_lit_branch():
    rng = np.random.default_rng(1)
    m1 = torch.as_tensor(rng.uniform(0.1, 0.9, 1000))
    m2 = m1 ** 2 + torch.as_tensor(rng.uniform(0, 0.01, 1000))
    d = torch.as_tensor(rng.uniform(0.0, 1.0, 1000))
    v = P.chebyshev(m1, m2, d, 1e-5)
    assert torch.all((v >= 0) & (v <= 1))
    assert torch.all(v[d <= m1] == 1)


def test_cantelli_bound_holds_for_discrete_pcf():
    """Discrete PCF (fraction of filter weight with d <= f) never exceeds the
    one-sided Chebyshev value when d > mu (Sec. 3, Cantelli)."""
    rng = np.random.default_rng(7)
    viol = 0
    for _ in range(20000):
        k = rng.choice([3, 5, 7])
        w = P.filter_taps(rng.choice(['box', 'gaussian']), int(k), 0.0)
        W2 = np.outer(w, w).ravel()
        f = rng.uniform(0.1, 1.0, k * k)
        if rng.random() < 0.5:
            f[rng.random(k * k) < 0.5] = rng.uniform(0.1, 0.3)
        mu = (W2 * f).sum()
        var = (W2 * f * f).sum() - mu * mu
        d = rng.uniform(0.1, 1.0)
        if d <= mu:
            continue
        pcf = W2[d <= f].sum()
        v = float(P.chebyshev(torch.tensor(mu), torch.tensor(var + mu * mu), torch.tensor(d), 1e-12))
        viol += pcf > v + 1e-12
    assert viol == 0


def test_visibility_derivative_matches_closed_form():
    """d v / d mu = -d v / d d = 2 s^2 (d - mu) / (s^2 + (d - mu)^2)^2 for d > mu
    (Sec. 4), with sigma^2 held fixed; and the total derivative w.r.t. m1
    adds -2 m1 dv/dsigma^2 with dv/dsigma^2 = (d-mu)^2/(s^2+(d-mu)^2)^2."""
    rng = np.random.default_rng(3)
    for _ in range(200):
        mu = rng.uniform(0.2, 0.8)
        s2 = rng.uniform(1e-4, 1e-2)
        d = mu + rng.uniform(1e-3, 0.2)
        m1 = torch.tensor(mu, dtype=D, requires_grad=True)
        m2 = torch.tensor(s2 + mu * mu, dtype=D, requires_grad=True)
        dd = torch.tensor(d, dtype=D, requires_grad=True)
        v = P.chebyshev(m1, m2, dd, 1e-12)
        g1, g2, gd = torch.autograd.grad(v, (m1, m2, dd))
        q = s2 + (d - mu) ** 2
        dv_dmu = 2 * s2 * (d - mu) / q ** 2
        dv_ds2 = (d - mu) ** 2 / q ** 2
        assert abs(float(gd) + dv_dmu) < 1e-9 * max(1, abs(dv_dmu))
        assert abs(float(g2) - dv_ds2) < 1e-9 * max(1, dv_ds2)
        assert abs(float(g1) - (dv_dmu - 2 * mu * dv_ds2)) < 1e-8 * max(1, abs(dv_dmu))


def test_visibility_is_c1_across_d_equals_mu():
    mu, s2 = 0.4, 3e-3
    for dd in (mu - 1e-7, mu + 1e-7):
        d = torch.tensor(dd, dtype=D, requires_grad=True)
        v = P.chebyshev(torch.tensor(mu, dtype=D), torch.tensor(s2 + mu * mu, dtype=D), d, 1e-12)
        (g,) = torch.autograd.grad(v, d)
        assert abs(float(v.detach()) - 1) < 1e-9 and abs(float(g)) < 1e-3


# ----------------------------------------------------------------------------- O6 smoothing

def test_edge_smoothing_row_sum_equals_covered_length():
    """One near-vertical silhouette edge over a constant background: after
    smoothing, every row sums to c_f * e + c_b * (W - e), e the continuous
    crossing of the edge with that row's sample line."""
    W = H = 24
    top = (0.13, 1.6)       # NDC (x, y), edge leaves the screen at the top
    bot = (-0.21, -1.6)
    verts = np.array([[-1.6, 1.6], list(top), list(bot), [-1.6, -1.6]], np.float32)
    clip32 = np.concatenate([verts, np.zeros((4, 1), np.float32), np.ones((4, 1), np.float32)], 1)
    faces = np.array([[0, 3, 2], [0, 2, 1]])
    st = raster.setup(clip32, faces, W, H)
    key, tri = raster.coverage(st)
    pairs = raster.aa_pairs(key, tri, st, Adjacency(faces))
    cf, cb = 0.9, 0.2
    img = torch.as_tensor(np.where(tri.ravel() >= 0, cf, cb)[:, None])
    out = P.smooth_edges(img, pairs, torch.as_tensor(clip32, dtype=D), W, H).reshape(H, W).numpy()
    top64, bot64 = verts[1].astype(np.float64), verts[2].astype(np.float64)
    tx = (top64 + 1) * W / 2
    bx = (bot64 + 1) * W / 2
    ty = (1 - top64[1]) * H / 2
    by = (1 - bot64[1]) * H / 2
    for j in range(H):
        y = j + 0.5
        e = tx[0] + (bx[0] - tx[0]) * (y - ty) / (by - ty)
        assert abs(out[j].sum() - (cf * e + cb * (W - e))) < 1e-12


def test_edge_smoothing_column_sum_equals_covered_length():
    """One near-horizontal silhouette edge over a constant background, the
    vertical-pair half of the smoothing: after smoothing, every column sums
    to c_f * e + c_b * (H - e), e the continuous crossing of the edge with
    that column's sample line (measured from the top of the screen)."""
    W, H = 26, 22
    left = (-1.6, 0.17)     # NDC (x, y), edge leaves the screen left and right
    right = (1.6, -0.23)
    verts = np.array([[-1.6, 1.6], [1.6, 1.6], list(right), list(left)], np.float32)
    clip32 = np.concatenate([verts, np.zeros((4, 1), np.float32), np.ones((4, 1), np.float32)], 1)
    faces = np.array([[0, 3, 2], [0, 2, 1]])
    st = raster.setup(clip32, faces, W, H)
    key, tri = raster.coverage(st)
    pairs = raster.aa_pairs(key, tri, st, Adjacency(faces))
    assert len(pairs['T']) > 0 and not pairs['horiz'].any()
    cf, cb = 0.9, 0.2
    img = torch.as_tensor(np.where(tri.ravel() >= 0, cf, cb)[:, None])
    out = P.smooth_edges(img, pairs, torch.as_tensor(clip32, dtype=D), W, H).reshape(H, W).numpy()
    l64, r64 = verts[3].astype(np.float64), verts[2].astype(np.float64)
    lx, rx = (l64[0] + 1) * W / 2, (r64[0] + 1) * W / 2
    ly, ry = (1 - l64[1]) * H / 2, (1 - r64[1]) * H / 2
    for i in range(W):
        x = i + 0.5
        e = ly + (ry - ly) * (x - lx) / (rx - lx)
        assert abs(out[:, i].sum() - (cf * e + cb * (H - e))) < 1e-12


def test_no_silhouette_means_identity():
    W = H = 20
    quad = np.array([[-1, 1], [1, 1], [1, -1], [-1, -1]], np.float32)
    clip32 = np.concatenate([quad, np.zeros((4, 1), np.float32), np.ones((4, 1), np.float32)], 1)
    faces = np.array([[0, 3, 2], [0, 2, 1]])
    st = raster.setup(clip32, faces, W, H)
    key, tri = raster.coverage(st)
    pairs = raster.aa_pairs(key, tri, st, Adjacency(faces))
    assert len(pairs['T']) == 0


def test_smoothing_colour_part_is_linear_adjoint():
    b = sg.config0()
    base, poses, lp, alb = P.scene_leaves(b, requires_grad=False)
    out = P.render(b, P.world_vertices(b, base, poses), lp, alb)
    v = out['views'][0]
    rv = v['rv']
    rng = np.random.default_rng(0)
    N = rv['W'] * rv['H']
    Mc = cameras.camera_matrix(b.cameras[0])
    clip = P.homogeneous(base[0]) @ Mc.T
    x = torch.as_tensor(rng.standard_normal((N, 1)), dtype=D).requires_grad_(True)
    y = torch.as_tensor(rng.standard_normal((N, 1)), dtype=D)
    Ax = P.smooth_edges(x, rv['pairs'], clip.detach(), rv['W'], rv['H'])
    (g,) = torch.autograd.grad((Ax * y).sum(), x)
    # linearity: A(2x) = 2 A(x); adjoint consistency of the blend matrix
    A2 = P.smooth_edges(2 * x.detach(), rv['pairs'], clip.detach(), rv['W'], rv['H'])
    assert torch.allclose(A2, 2 * Ax.detach(), atol=1e-14)
    assert abs(float((Ax * y).sum().detach()) - float((x.detach() * g).sum())) < 1e-10
    assert len(rv['pairs']['T']) > 100


# ----------------------------------------------------------------------------- O4, O10 shading

def plane_only_batch(kind='directional'):
    qv, qf = sg.quad(3.0)
    sc = sg.Scene(verts=qv, faces=qf, albedo=np.full((2, 1), 0.8, np.float32))
    w = sg.f32([0.3, -1.0, 0.2])
    L = sg.Light('directional', w, resolution=128, filter='box', k=5)
    cam = sg.Camera(eye=sg.f32([0, 3, 5]), target=sg.f32([0, 0, 0]), fov_deg=45.0, width=96, height=80)
    return sg.Batch('plane', [sc], [L], [cam], [sg.Render(0, [0])])


def test_unoccluded_plane_is_constant_lambert_and_moments_affine():
    b = plane_only_batch()
    base, poses, lp, alb = P.scene_leaves(b, requires_grad=False)
    out = P.render(b, P.world_vertices(b, base, poses), lp, alb)
    w = b.lights[0].param.astype(np.float64)
    w /= np.linalg.norm(w)
    expect = 0.8 * (-w[1])          # n = +y, omega = -w
    img = out['images'][0][..., 0].numpy()
    tri = out['views'][0]['rv']['tri']
    inner = tri >= 0
    # interior pixels (not next to the plane's outline) are exactly rho (n . omega)
    from scipy.ndimage import binary_erosion
    core = binary_erosion(inner, iterations=2)
    assert core.sum() > 1000
    assert np.allclose(img[core], expect, atol=1e-9)
    # directional light: z is affine over the plane in shadow-map space
    F0 = out['lights'][0]['F0'][0].numpy()
    ltri = out['lights'][0]['rv']['tri']
    lcore = binary_erosion(ltri >= 0, iterations=1)
    jj, ii = np.nonzero(lcore)
    A = np.stack([ii, jj, np.ones_like(ii)], 1).astype(np.float64)
    coef, *_ = np.linalg.lstsq(A, F0[jj, ii], rcond=None)
    assert np.abs(A @ coef - F0[jj, ii]).max() < 1e-12
    assert np.allclose(out['lights'][0]['F0'][1].numpy(), F0 ** 2, atol=0)


def test_no_occluder_means_fully_lit():
    b = plane_only_batch()
    base, poses, lp, alb = P.scene_leaves(b, requires_grad=False)
    out = P.render(b, P.world_vertices(b, base, poses), lp, alb)
    fl = out['flags'][0][0]
    # visibility is recomputed from the flags: either the lit branch or v within 1e-6 of 1
    view = out['views'][0]
    img0 = view['img0'][..., 0].numpy().ravel()[view['flat']]
    w = b.lights[0].param.astype(np.float64)
    w /= np.linalg.norm(w)
    assert np.all(img0 >= 0.8 * (-w[1]) * (1 - 1e-6))


def test_spot_cone_is_hard_half_angle_mask():
    """Spot light (Sec. 5 light types; the supplementary renderer uses a
    perspective light camera whose field of view is the cone): on an
    unoccluded ground plane under a spot with a 60 degree cone, a pixel
    whose direction from the light makes more than 30 degrees with the cone
    axis is exactly 0, and one well inside the cone is exactly
    rho max(0, n . omega).  The world point of each pixel is found here by
    intersecting the camera ray with the plane, independently of the
    oracle's projection and barycentrics; the angle is taken from the
    light's position and aim point as given in the scene."""
    qv, qf = sg.quad(4.0)
    sc = sg.Scene(verts=qv, faces=qf, albedo=np.full((2, 1), 0.8, np.float32))
    p = sg.f32([1, 5, 1])
    L = sg.Light('spot', p, fov_deg=60.0, resolution=128, filter='gaussian', k=7, sigma=2.0,
                 up=sg._up_for(-p))
    cam = sg.Camera(eye=sg.f32([0, 3, 5]), target=sg.f32([0, 0.75, 0]), fov_deg=45.0, width=128, height=112)
    b = sg.Batch('spot', [sc], [L], [cam], [sg.Render(0, [0])])
    base, poses, lp, alb = P.scene_leaves(b, requires_grad=False)
    img = P.render(b, P.world_vertices(b, base, poses), lp, alb)['images'][0][..., 0].numpy()
    W, H = cam.width, cam.height
    e = cam.eye.astype(np.float64)
    f = cam.target.astype(np.float64) - e
    f /= np.linalg.norm(f)
    s = np.cross(f, [0.0, 1.0, 0.0])
    s /= np.linalg.norm(s)
    u = np.cross(s, f)
    th = math.tan(math.radians(cam.fov_deg) / 2)
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing='ij')
    px = 2 * (ii + 0.5) / W - 1
    py = 1 - 2 * (jj + 0.5) / H
    ray = f + (px * th * W / H)[..., None] * s + (py * th)[..., None] * u
    t = -e[1] / ray[..., 1]
    x = e + t[..., None] * ray
    pl = p.astype(np.float64)
    v = x - pl
    axis = (L.target.astype(np.float64) - pl) / np.linalg.norm(L.target.astype(np.float64) - pl)
    ang = np.degrees(np.arccos((v @ axis) / np.linalg.norm(v, axis=-1)))
    lam = 0.8 * (-v[..., 1] / np.linalg.norm(v, axis=-1))      # n = +y, omega toward the light
    on_plane = (t > 0) & (np.abs(x[..., 0]) < 3.9) & (np.abs(x[..., 2]) < 3.9)
    outside = on_plane & (ang > 30.05)
    inside = on_plane & (ang < 28.0)      # 2 degrees: the filter's reach near the map border
    rim = on_plane & (ang > 29.5) & (ang < 29.95)
    assert outside.sum() > 500 and inside.sum() > 5000 and rim.sum() > 40
    assert np.all(img[outside] == 0.0)
    assert np.abs(img[inside] - lam[inside]).max() < 1e-6
    assert np.all(img[rim] > 0.5 * lam[rim])


def hard_shadow_batch(cfg):
    b = sg.config0() if cfg == 0 else sg.config1()
    for L in b.lights:
        L.k = 1
        L.antialias = False
        L.min_variance = 1e-12
    return b


@pytest.mark.parametrize('cfg', [0, 1])
def test_hard_shadow_limit_equals_ray_casting(cfg):
    """k = 1, no smoothing, tiny variance floor: thresholded VSM visibility
    is the binary shadow-map test of Eq. (2), which must agree with exact
    ray casting wherever the shadow-map footprint is away from triangle-id
    changes."""
    b = hard_shadow_batch(cfg)
    base, poses, lp, alb = P.scene_leaves(b, requires_grad=False)
    out = P.render(b, P.world_vertices(b, base, poses), lp, alb, P.Options(camera_antialias=False))
    sc = b.scenes[0]
    L = b.lights[0]
    view = out['views'][0]
    cam = b.cameras[0]
    flat = view['flat']
    tri_cam = view['rv']['tri'].ravel()[flat]
    Mc = cameras.camera_matrix(cam)
    clip = P.homogeneous(base[0]) @ Mc.T
    px, py = P.pixel_centres_ndc(flat, cam.width, cam.height)
    fv = torch.as_tensor(sc.faces.astype(np.int64))[torch.as_tensor(tri_cam)]
    bc = P.perspective_barycentrics(clip[fv[:, 0]], clip[fv[:, 1]], clip[fv[:, 2]], px, py)
    x = (bc[:, :, None] * base[0][fv]).sum(1).numpy()
    fr = out['lights'][0]['frame']
    n = np.cross(sc.verts[sc.faces[tri_cam, 1]] - sc.verts[sc.faces[tri_cam, 0]],
                 sc.verts[sc.faces[tri_cam, 2]] - sc.verts[sc.faces[tri_cam, 0]]).astype(np.float64)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    p = L.param.astype(np.float64)
    om = p - x
    om /= np.linalg.norm(om, axis=1, keepdims=True)
    ndl = (n * om).sum(1)
    # texel footprint: at least 2 texels from a triangle-id change in the shadow map
    S = L.resolution
    Ml = fr['M'].detach().numpy()
    h = np.concatenate([x, np.ones((len(x), 1))], 1) @ Ml.T
    tx = (h[:, 0] / h[:, 3] + 1) * S / 2
    ty = (1 - h[:, 1] / h[:, 3]) * S / 2
    ltri = out['lights'][0]['rv']['tri']
    pad = np.pad(ltri, 3, mode='edge')
    ok = (ndl > 0.1) & (tx > 3) & (ty > 3) & (tx < S - 3) & (ty < S - 3)
    if L.kind == 'spot':
        cosang = ((x - p) / np.linalg.norm(x - p, axis=1, keepdims=True) * fr['w'].detach().numpy()).sum(1)
        ok &= cosang > fr['cos_half'] + 1e-3
    ix = np.clip(np.floor(tx), 0, S - 1).astype(int)
    iy = np.clip(np.floor(ty), 0, S - 1).astype(int)
    for dy in range(-2, 3):
        for dx in range(-2, 3):
            ok &= pad[iy + dy + 3, ix + dx + 3] == pad[iy + 3, ix + 3]
    rng = np.random.default_rng(0)
    idx = np.nonzero(ok)[0]
    idx = rng.choice(idx, min(len(idx), 1500), replace=False)
    shadow_ray = raycast.occluded(x[idx], p, sc.verts, sc.faces)
    col = out['images'][0][..., 0].numpy().ravel()[flat[idx]]
    lam = 0.8 * ndl[idx]
    vis = col / lam
    shadow_sm = vis <= 0.5
    assert shadow_ray.sum() > 20 and (~shadow_ray).sum() > 20
    assert np.array_equal(shadow_sm, shadow_ray)


# ----------------------------------------------------------------------------- O12 gradients

def small_cfg0(res=96):
    b = sg.config0()
    b.lights[0].resolution = res
    b.cameras[0].width = b.cameras[0].height = res
    return b


def loss_and_state(b, verts, lp, targets):
    out = P.render(b, [verts], [lp])
    return P.mse(out['images'], targets), P.fingerprint(out)


@pytest.mark.parametrize('variant', ['plain', 'warped_bleed'])
def test_finite_differences_of_loss_cfg0(monkeypatch, variant):
    """Central differences of the loss against autograd, for the plain maps
    and for exponential maps with light-bleeding reduction."""
    monkeypatch.setattr(cameras, 'ROUND_TO_F32', False)
    b = small_cfg0()
    if variant == 'warped_bleed':
        b.lights[0].warp_exponent = 10.0
        b.lights[0].bleed_reduction = 0.2
    targets = P.target_images(b)
    base, poses, lp, alb = P.scene_leaves(b)
    L, fp0 = loss_and_state(b, base[0], lp[0], targets)
    L.backward()
    gv = base[0].grad.numpy()
    gl = lp[0].grad.numpy()
    h = 1e-6
    checked = skipped = 0
    errs = []
    params = [('light', None, c) for c in range(3)] + [('vert', v, c) for v in range(12) for c in range(3)]
    for kind, v, c in params:
        vals = []
        same = True
        for s in (+1, -1):
            vv = base[0].detach().clone()
            ll = lp[0].detach().clone()
            if kind == 'light':
                ll[c] += s * h
            else:
                vv[v, c] += s * h
            with torch.no_grad():
                Ls, fps = loss_and_state(b, vv, ll, targets)
            same &= fps == fp0
            vals.append(float(Ls))
        if not same:
            skipped += 1
            continue
        fd = (vals[0] - vals[1]) / (2 * h)
        an = gl[c] if kind == 'light' else gv[v, c]
        errs.append(abs(fd - an) / max(abs(an), 1e-4))
        checked += 1
    assert checked >= 25, (checked, skipped)
    # float64 central differences with h = 1e-6 resolve the derivative to
    # about 1e-9 relative here (warped maps: the exponentials' larger
    # curvature leaves about 1e-6)
    tol = 1e-6 if variant == 'plain' else 5e-6
    assert max(errs) < tol, max(errs)
    assert np.linalg.norm(gl) > 1e-4


def test_finite_differences_of_loss_cfg1_sphere_vertices(monkeypatch):
    """Central differences on the icosphere under the spot light (Gaussian 7):
    32 sphere vertices drawn with default_rng(1), each moved along a seeded
    random unit direction, and the three light coordinates.  A sample counts
    only where every discrete decision is unchanged at both offsets."""
    monkeypatch.setattr(cameras, 'ROUND_TO_F32', False)
    b = sg.config1()
    b.lights[0].resolution = 96
    b.cameras[0].width = b.cameras[0].height = 96
    n_sphere = len(b.scenes[0].verts) - 4
    chosen = np.random.default_rng(1).choice(n_sphere, 32, replace=False)
    dirs = np.random.default_rng(2).standard_normal((32, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    targets = P.target_images(b)
    base, poses, lp, alb = P.scene_leaves(b)
    L, fp0 = loss_and_state(b, base[0], lp[0], targets)
    L.backward()
    gv = base[0].grad.numpy()
    gl = lp[0].grad.numpy()
    h = 1e-6
    probes = [('light', np.eye(3)[c], gl[c]) for c in range(3)]
    probes += [(int(v), d, float(gv[v] @ d)) for v, d in zip(chosen, dirs)]
    errs, skipped, nonzero = [], 0, 0
    for what, d, an in probes:
        vals = []
        same = True
        for sgn in (+1, -1):
            vv = base[0].detach().clone()
            ll = lp[0].detach().clone()
            if what == 'light':
                ll += sgn * h * torch.as_tensor(d)
            else:
                vv[what] += sgn * h * torch.as_tensor(d)
            with torch.no_grad():
                Ls, fps = loss_and_state(b, vv, ll, targets)
            same &= fps == fp0
            vals.append(float(Ls))
        if not same:
            skipped += 1
            continue
        fd = (vals[0] - vals[1]) / (2 * h)
        nonzero += abs(an) > 1e-6
        errs.append(abs(fd - an) / max(abs(an), 1e-4))
    print(f"checked {len(errs)}, skipped {skipped}, nonzero {nonzero}, worst {max(errs):.2e}")
    assert len(errs) >= 28 and nonzero >= 8, (len(errs), skipped, nonzero)
    assert max(errs) < 1e-6, max(errs)


def test_gradient_step_on_light_lowers_loss():
    b = small_cfg0()
    targets = P.target_images(b)
    base, poses, lp, alb = P.scene_leaves(b)
    L0, _ = loss_and_state(b, base[0].detach(), lp[0], targets)
    L0.backward()
    g = lp[0].grad
    step = 0.05 / float(g.norm())
    with torch.no_grad():
        L1, _ = loss_and_state(b, base[0].detach(), lp[0] - step * g, targets)
    assert float(L1) < float(L0)
    # moving toward the target light position (2.3, 4, 1) along x
    assert float(g[0]) < 0
