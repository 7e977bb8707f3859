"""Pins of the oracle's cube shadow maps for omnidirectional point lights:
six cube-face lights, each a 90 degree perspective view along one axis of a
box around the light (Sec. 3 allows several planes arranged as a box; Sec. 5
names this route for omnidirectional point lights)."""
import numpy as np
import pytest
import torch

import scenegen as sg
from oracle import cameras, raycast
from oracle import pipeline as P


def _project(M, pts):
    h = np.concatenate([pts, np.ones((len(pts), 1))], 1) @ M.T
    return h[:, 0] / h[:, 3], h[:, 1] / h[:, 3], h[:, 3]


def test_cube_faces_tile_every_direction():
    """Every direction belongs to exactly one face; the owner's frustum holds
    it, and every other face sees it on or outside its frustum border.  Checks
    the faces' axes against the owner rule, axis-aligned and tied directions
    included."""
    rng = np.random.default_rng(3)
    d = rng.normal(size=(4000, 3))
    d = np.concatenate([d, np.eye(3), -np.eye(3), [[1, 1, 0], [-1, 0, -1], [0, -1, 1], [1, -1, 1]]])
    p = np.array([0.3, -0.2, 0.7])
    owner = cameras.cube_face_of(d)
    assert set(owner.tolist()) == set(range(6))
    tied = np.sort(np.abs(d), 1)
    strict = tied[:, 2] - tied[:, 1] > 1e-9 * tied[:, 2]
    for f in range(6):
        L = sg.Light('cubeface', sg.f32(p), face=f)
        fr = cameras.light_frame(L, torch.as_tensor(p))
        u, v, w = _project(fr['M'].detach().numpy(), p + d)
        m = np.maximum(np.abs(u), np.abs(v))
        mine = owner == f
        assert np.all(w[mine] > 0) and np.all(m[mine] <= 1 + 1e-6)
        other = ~mine & strict
        assert np.all((w[other] <= 0) | (m[other] > 1 - 1e-6))
        # the face axis is the light camera's viewing direction
        assert np.allclose(fr['w'].numpy(), cameras.CUBE_AXES[f])


def test_tie_rule_picks_lower_axis_and_positive_sign_at_zero():
    d = np.array([[1, 1, 1], [-1, 1, 0], [0, -2, 2], [0, 0, 0], [0, -0.0, 0]])
    assert cameras.cube_face_of(d).tolist() == [0, 1, 3, 0, 0]


def _shadow_free(b):
    sc = b.scenes[0]
    keep = np.arange(2 * 16 * 16)            # the ground grid's triangles come first
    used = np.unique(sc.faces[keep])
    remap = -np.ones(len(sc.verts), np.int64)
    remap[used] = np.arange(len(used))
    b.scenes[0] = sg.Scene(verts=sc.verts[used], faces=remap[sc.faces[keep]].astype(np.int32),
                           albedo=sc.albedo[keep])
    return b


def test_cube_light_without_occluders_is_the_lambert_point_light():
    """With nothing between light and ground, the six masks partition the
    ground: the image is albedo * max(0, n . omega) of one point light, so no
    pixel is lit by two faces or by none."""
    b = _shadow_free(sg.cube_light_scene(resolution=96, view=96))
    base, poses, lp, alb = P.scene_leaves(b, requires_grad=False)
    out = P.render(b, P.world_vertices(b, base, poses), lp, alb)
    view = out['views'][0]
    img0 = view['img0'][..., 0].numpy().ravel()[view['flat']]
    tri = view['rv']['tri'].ravel()[view['flat']]
    cam = b.cameras[0]
    Mc = cameras.camera_matrix(cam)
    sc = b.scenes[0]
    clip = P.homogeneous(base[0]) @ Mc.T
    px, py = P.pixel_centres_ndc(view['flat'], cam.width, cam.height)
    fv = torch.as_tensor(sc.faces.astype(np.int64))[torch.as_tensor(tri)]
    bc = P.perspective_barycentrics(clip[fv[:, 0]], clip[fv[:, 1]], clip[fv[:, 2]], px, py)
    x = (bc[:, :, None] * base[0][fv]).sum(1).numpy()
    p = b.lights[0].param.astype(np.float64)
    om = p - x
    om /= np.linalg.norm(om, axis=1, keepdims=True)
    rho = float(np.float32(0.8))
    ratio = img0 / (rho * np.maximum(om[:, 1], 0.0))
    assert len(img0) > 4000
    # one face per pixel: never 0 or 2 faces' worth of light; across the
    # seams the padded maps keep the ground lit to 1e-3
    assert np.all((ratio > 0.999) & (ratio <= 1 + 1e-12))
    # away from the seams the visibility is 1 or within 1e-6 of it (lit
    # branch of Eq. (3))
    ad = np.sort(np.abs(x - p), 1)
    inner = (ad[:, 2] - ad[:, 1]) / ad[:, 2] > 0.05
    assert inner.sum() > 0.8 * len(img0)
    assert np.all(ratio[inner] >= 1 - 1e-6)
    # all five faces that see the ground take part
    owners = set(cameras.cube_face_of(x - p).tolist())
    assert owners == {0, 1, 3, 4, 5}


def test_cube_light_hard_shadow_limit_equals_ray_casting():
    """k = 1, no smoothing, a tiny variance floor: the thresholded visibility
    is the binary shadow-map test of Eq. (2) in the owning face's map, and it
    must agree with exact ray casting wherever that map's footprint stays on
    one surface (the ground or one sphere); shadows fall through five faces."""
    b = sg.cube_light_scene(resolution=160, view=128, k=1, antialias=False)
    for L in b.lights:
        L.min_variance = 1e-12
    base, poses, lp, alb = P.scene_leaves(b, requires_grad=False)
    out = P.render(b, P.world_vertices(b, base, poses), lp, alb, P.Options(camera_antialias=False))
    sc = b.scenes[0]
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
    n = np.cross(sc.verts[sc.faces[tri_cam, 1]] - sc.verts[sc.faces[tri_cam, 0]],
                 sc.verts[sc.faces[tri_cam, 2]] - sc.verts[sc.faces[tri_cam, 0]]).astype(np.float64)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    p = b.lights[0].param.astype(np.float64)
    om = p - x
    om /= np.linalg.norm(om, axis=1, keepdims=True)
    ndl = (n * om).sum(1)
    owner = cameras.cube_face_of(x - p)
    S = b.lights[0].resolution
    # surface class per triangle: ground grid, then one class per sphere
    per_sphere = (len(sc.faces) - 2 * 16 * 16) // len(sg.CUBE_SCENE_OCCLUDERS)
    cls = np.concatenate([[0], np.zeros(2 * 16 * 16, np.int64) + 1,
                          2 + np.arange(len(sc.faces) - 512) // per_sphere])
    ok = ndl > 0.1
    for f in range(6):
        sel = owner == f
        if not sel.any():
            continue
        Ml = out['lights'][f]['frame']['M'].detach().numpy()
        u, v, _ = _project(Ml, x[sel])
        tx = (u + 1) * S / 2
        ty = (1 - v) * S / 2
        good = (tx > 3) & (ty > 3) & (tx < S - 3) & (ty < S - 3)
        pad = np.pad(cls[out['lights'][f]['rv']['tri'] + 1], 3, mode='edge')
        ix = np.clip(np.floor(tx), 0, S - 1).astype(int)
        iy = np.clip(np.floor(ty), 0, S - 1).astype(int)
        for dy in range(-2, 3):
            for dx in range(-2, 3):
                good &= pad[iy + dy + 3, ix + dx + 3] == pad[iy + 3, ix + 3]
        ok[np.nonzero(sel)[0][~good]] = False
    rng = np.random.default_rng(0)
    idx = np.nonzero(ok)[0]
    idx = rng.choice(idx, min(len(idx), 2500), replace=False)
    shadow_ray = raycast.occluded(x[idx], p, sc.verts, sc.faces)
    col = out['images'][0][..., 0].numpy().ravel()[flat[idx]]
    shadow_sm = col / (0.8 * ndl[idx]) <= 0.5
    assert np.array_equal(shadow_sm, shadow_ray)
    # shadowed samples in the -y, +x and -z faces and on both sides of the -x / +z seam
    faces_in_shadow = set(owner[idx][shadow_ray].tolist())
    assert {0, 1, 3, 4, 5} <= faces_in_shadow, faces_in_shadow


def test_cube_edge_table_is_symmetric_and_covers_every_edge():
    """Each cube edge is shared by exactly two face-map edges, each pointing at
    the other with the same index direction; 24 map edges, 12 cube edges."""
    tab = cameras.cube_edge_table()
    seen = set()
    for f in range(6):
        for e in range(4):
            g, e2, flip = tab[f][e]
            assert g != f and tab[g][e2] == (f, e, flip)
            seen.add(frozenset([(f, e), (g, e2)]))
    assert len(seen) == 12


@pytest.mark.parametrize('S,P', [(16, 2), (33, 4)])
def test_cube_padding_samples_along_the_continued_plane(S, P):
    """Pad maps filled with a smooth function of direction: on every edge
    block the padded value equals the function along the direction the
    padded texel centre looks along (the face's plane continued across the
    edge) up to bilinear interpolation error, far below one texel's change;
    a wrong neighbour, edge or index direction misses by about a face.
    Inside, the face is copied exactly; corner blocks repeat the corner."""
    c = np.array([0.3, -0.8, 0.5])

    def phi(d):
        return (d / np.linalg.norm(d, axis=-1, keepdims=True)) @ c

    vals = np.zeros((6, S, S))
    ndc = (2 * np.arange(S) + 1) / S - 1
    for f in range(6):
        a, s, u = cameras.cube_face_basis(f)
        U, V = np.meshgrid(ndc, -ndc)
        vals[f] = phi(a + U[..., None] * s + V[..., None] * u)
    idx, wgt = cameras.cube_pad_sources(S, P)
    assert np.allclose(wgt.sum(-1), 1.0, atol=1e-12)
    Sp = S + 2 * P
    pndc = (2 * (np.arange(Sp) - P) + 1) / S - 1
    worst = 0.0
    for f in range(6):
        a, s, u = cameras.cube_face_basis(f)
        U, V = np.meshgrid(pndc, -pndc)
        edge = (np.abs(U) > 1) ^ (np.abs(V) > 1)
        want = phi(a + U[..., None] * s + V[..., None] * u)
        got = (vals.ravel()[idx[f]] * wgt[f]).sum(-1)
        assert np.array_equal(got[P:P + S, P:P + S], vals[f])
        assert got[0, 0] == vals[f][0, 0] and got[-1, -1] == vals[f][-1, -1]
        worst = max(worst, np.abs(got - want)[edge].max())
    # bilinear error of a function with |Hessian| ~ 1 over texels of 2/S: ~ (2/S)^2
    assert worst < 2.0 * (2.0 / S) ** 2, worst


def test_cube_light_loss_gradient_matches_finite_differences(monkeypatch):
    """Central differences of the loss of a cube-light render (light moved
    as one: all six faces' parameters together; and occluder vertices)
    against autograd, where no discrete decision changes."""
    monkeypatch.setattr(cameras, 'ROUND_TO_F32', False)
    b = sg.cube_light_scene(resolution=48, view=48)
    targets = P.target_images(b)
    base, poses, lp, alb = P.scene_leaves(b)

    def run(verts, params):
        out = P.render(b, [verts], params)
        return P.mse(out['images'], targets), P.fingerprint(out)

    L0, fp0 = run(base[0], lp)
    L0.backward()
    g_light = sum(q.grad.numpy() for q in lp)
    g_vert = base[0].grad.numpy()
    h = 1e-6
    rng = np.random.default_rng(4)
    occluder = np.arange(17 * 17, len(base[0]))        # the sphere vertices follow the 17 x 17 ground grid
    verts_to_check = rng.choice(occluder, 8, replace=False)
    params = [('light', None, c) for c in range(3)] + [('vert', int(v), c) for v in verts_to_check for c in range(3)]
    checked = skipped = 0
    errs = []
    for kind, v, c in params:
        vals, same = [], True
        for s in (+1, -1):
            vv = base[0].detach().clone()
            ll = [q.detach().clone() for q in lp]
            if kind == 'light':
                for q in ll:
                    q[c] += s * h
            else:
                vv[v, c] += s * h
            with torch.no_grad():
                Ls, fps = run(vv, ll)
            same &= fps == fp0
            vals.append(float(Ls))
        if not same:
            skipped += 1
            continue
        fd = (vals[0] - vals[1]) / (2 * h)
        an = g_light[c] if kind == 'light' else g_vert[v, c]
        errs.append(abs(fd - an) / max(abs(an), 1e-4))
        checked += 1
    assert checked >= 20, (checked, skipped)
    assert max(errs) < 1e-4, max(errs)
    assert np.linalg.norm(g_light) > 1e-4
