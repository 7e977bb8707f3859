"""Continuous part of the oracle: float64 torch with autograd, the discrete
decisions of ``oracle.raster`` held fixed.  (Test infrastructure only.)

Per light (Alg. 1, RenderShadowMap):
  * resolve each texel's nearest triangle to the world point x seen through
    the texel centre (perspective-correct barycentrics), distance d(x) to the
    light (Sec. 3: Euclidean for point/spot lights, from a plane outside the
    scene for directional lights), normalized z = d / far;
    f = z, f^2 = z * z formed before smoothing (Sec. 5); background texels
    hold the far value (1, 1).  Exponential maps (a pre-warp g = exp of the
    depth before filtering, one of the alternatives Sec. 3 lists; light
    bleeding, supplementary limitations) store f = exp(c z), f^2 = exp(2 c z)
    instead, background (exp(c), exp(2c));
  * smoothing at primitive borders gives (f~, f^2~) (Sec. 4);
  * m1 = G f~, m2 = G f^2~ with G a separable box or Gaussian filter of odd
    size k, clamp-to-edge (Eq. moment1, moment2; Sec. 5 "Filter").
Per camera pixel (deferred shading with Lambert, supplementary renderer
details; Alg. 2, ComputeVisibility):
  * u = L(x); bilinear fetch of (m1, m2) at u (clamp-to-edge);
  * mu = m1, sigma^2 = max(m2 - m1^2, eps); v = 1 if d <= mu, else
    sigma^2 / (sigma^2 + (d - mu)^2) (Sec. 3, one-sided Chebyshev bound);
    exponential maps compare the warped depth exp(c z) and scale the floor
    by the warp's slope, eps (c exp(c z))^2; a light-bleeding reduction
    amount a > 0 then maps v to clamp((v - a) / (1 - a), 0, 1);
  * colour = sum over lights of albedo * max(0, n . omega) * v * I * cone;
    cone is the hard mask of a spot light's cone, or of the directions a
    cube face owns (1 for directional and point lights);
  * the same border smoothing is applied to the shaded image.
Loss: mean squared error to a target image.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import cameras, raster
from .mesh import Adjacency, posed_vertices

D = torch.float64


# ----------------------------------------------------------------------------- small pieces

def filter_taps(kind, k, sigma):
    """Normalized 1D taps for an odd kernel size k (box: 1/k; Gaussian:
    exp(-i^2 / 2 sigma^2) renormalized to sum 1; sigma 0 means (k-1)/3)."""
    assert k % 2 == 1 and k >= 1
    r = (k - 1) // 2
    if kind == 'box':
        return np.full(k, 1.0 / k)
    s = sigma if sigma > 0 else (k - 1) / 3.0
    if s <= 0:
        return np.ones(1)
    i = np.arange(-r, r + 1, dtype=np.float64)
    w = np.exp(-i * i / (2.0 * s * s))
    return w / w.sum()


def filter_separable(img, taps):
    """img (C, H, W): horizontal then vertical pass, clamp-to-edge."""
    k = len(taps)
    r = (k - 1) // 2
    C, H, W = img.shape
    out = torch.zeros_like(img)
    for j in range(k):
        cols = np.clip(np.arange(W) + j - r, 0, W - 1)
        out = out + taps[j] * img[:, :, cols]
    out2 = torch.zeros_like(out)
    for j in range(k):
        rows = np.clip(np.arange(H) + j - r, 0, H - 1)
        out2 = out2 + taps[j] * out[:, rows, :]
    return out2


def pixel_centres_ndc(flat, W, H):
    i = (flat % W).astype(np.float64)
    j = (flat // W).astype(np.float64)
    px = 2.0 * (i + 0.5) / W - 1.0
    py = 1.0 - 2.0 * (j + 0.5) / H
    return torch.as_tensor(px), torch.as_tensor(py)


def perspective_barycentrics(c0, c1, c2, px, py):
    """Barycentrics b of the point on the triangle (homogeneous clip corners
    c_i) that projects to NDC (px, py): sum b_i (X_i - px W_i) = 0,
    sum b_i (Y_i - py W_i) = 0, sum b_i = 1."""
    def a(c):
        return c[:, 0] - px * c[:, 3], c[:, 1] - py * c[:, 3]
    a0x, a0y = a(c0)
    a1x, a1y = a(c1)
    a2x, a2y = a(c2)
    k0 = a1x * a2y - a1y * a2x
    k1 = a2x * a0y - a2y * a0x
    k2 = a0x * a1y - a0y * a1x
    s = k0 + k1 + k2
    return torch.stack([k0 / s, k1 / s, k2 / s], 1)


def bilinear(maps, sx, sy):
    """maps (C, S, S); (sx, sy) continuous texel coordinates, texel centres at
    integers (i.e. already shifted by -1/2).  Clamp-to-edge.  Returns (n, C)."""
    C, H, W = maps.shape
    x0 = torch.floor(sx.detach())
    y0 = torch.floor(sy.detach())
    fx = sx - x0
    fy = sy - y0
    x0i = x0.long()
    y0i = y0.long()
    xa = x0i.clamp(0, W - 1)
    xb = (x0i + 1).clamp(0, W - 1)
    ya = y0i.clamp(0, H - 1)
    yb = (y0i + 1).clamp(0, H - 1)
    v00 = maps[:, ya, xa]
    v01 = maps[:, ya, xb]
    v10 = maps[:, yb, xa]
    v11 = maps[:, yb, xb]
    v = (1 - fx) * (1 - fy) * v00 + fx * (1 - fy) * v01 + (1 - fx) * fy * v10 + fx * fy * v11
    return v.T


def chebyshev(m1, m2, d, eps):
    """VSM visibility (Sec. 3): 1 where d <= mu, else sigma^2/(sigma^2+(d-mu)^2),
    with sigma^2 = max(m2 - m1^2, eps)."""
    mu = m1
    var = torch.clamp(m2 - m1 * m1, min=eps)
    diff = d - mu
    v = var / (var + diff * diff)
    return torch.where(d <= mu, torch.ones_like(v), v)


def warp_depth(z, c):
    """The stored depth function: exp(c z) for exponential maps (c > 0), the
    plain normalized depth otherwise."""
    return torch.exp(c * z) if c > 0 else z


def lookup_visibility(m1, m2, z, L):
    """Visibility of a receiver at normalized depth z from filtered moments
    (Sec. 3): the Chebyshev bound on the (warped) depth, then the
    light-bleeding reduction.  Returns (v, warped depth, variance floor)."""
    c = L.warp_exponent
    if c > 0:
        w = torch.exp(c * z)
        eps = L.min_variance * (c * w) ** 2
        var = torch.maximum(m2 - m1 * m1, eps)
        diff = w - m1
        v = torch.where(w <= m1, torch.ones_like(var), var / (var + diff * diff))
    else:
        w, eps = z, L.min_variance
        v = chebyshev(m1, m2, z, L.min_variance)
    a = L.bleed_reduction
    if a > 0:
        v = torch.clamp((v - a) / (1.0 - a), 0.0, 1.0)
    return v, w, eps


def smooth_edges(img, pairs, clip, W, H):
    """Apply the silhouette antialiasing blend for the fixed pairs.

    img (N, C) flat samples; clip (V, 4) homogeneous corners of the view.
    For pair (T front, O other) with chosen edge a -> b, the continuous
    crossing alpha = E(T) / (E(T) - E(O)) (E the edge function in continuous
    screen coordinates) is the fraction of the T -> O step covered by the
    front triangle; alpha > 1/2: O moves toward T by (alpha - 1/2);
    otherwise T moves toward O by (1/2 - alpha).  All deltas use pre-blend
    values and are summed."""
    if pairs is None or len(pairs['T']) == 0:
        return img
    ca = clip[torch.as_tensor(pairs['a'])]
    cb = clip[torch.as_tensor(pairs['b'])]

    def scr(c):
        return (c[:, 0] / c[:, 3] + 1.0) * (W / 2.0), (1.0 - c[:, 1] / c[:, 3]) * (H / 2.0)
    xa, ya = scr(ca)
    xb, yb = scr(cb)
    T = torch.as_tensor(pairs['T'])
    O = torch.as_tensor(pairs['O'])
    tx = (T % W).to(D) + 0.5
    ty = (T // W).to(D) + 0.5
    ox = (O % W).to(D) + 0.5
    oy = (O // W).to(D) + 0.5

    def E(px, py):
        return (xb - xa) * (py - ya) - (yb - ya) * (px - xa)
    eT = E(tx, ty)
    eO = E(ox, oy)
    alpha = eT / (eT - eO)
    cT = img[T]
    cO = img[O]
    over = alpha > 0.5
    wO = torch.where(over, alpha - 0.5, torch.zeros_like(alpha))
    wT = torch.where(over, torch.zeros_like(alpha), 0.5 - alpha)
    delta = torch.zeros_like(img)
    delta = delta.index_add(0, O, wO[:, None] * (cT - cO))
    delta = delta.index_add(0, T, wT[:, None] * (cO - cT))
    return img + delta


# ----------------------------------------------------------------------------- views

def homogeneous(v):
    return torch.cat([v, torch.ones(v.shape[0], 1, dtype=v.dtype)], 1)


def raster_view(M, verts, faces, W, H, adj, antialias):
    """Discrete state of one view from the float32 matrix and float32 vertices."""
    M32 = M.detach().numpy().astype(np.float32)
    v32 = verts.detach().numpy().astype(np.float32)
    clip32 = raster.transform_f32(M32, v32)
    st = raster.setup(clip32, faces, W, H)
    key, tri = raster.coverage(st)
    pairs = raster.aa_pairs(key, tri, st, adj) if antialias else None
    return dict(st=st, key=key, tri=tri, pairs=pairs, clip32=clip32, W=W, H=H)


def light_distance(frame, x):
    """Normalized distance z = d(x) / far (Sec. 3)."""
    if frame['kind'] == 'directional':
        d = ((x - frame['pos']) * frame['w']).sum(1)
    else:
        d = torch.sqrt(((x - frame['pos']) ** 2).sum(1))
    return d / frame['far']


def _no_bleed(L):
    class _V:
        warp_exponent = L.warp_exponent
        min_variance = L.min_variance
        bleed_reduction = 0.0
    return _V


@dataclass
class Options:
    camera_antialias: bool = True


def render(batch, verts_list, light_params, albedo_list=None, opts=Options()):
    """Forward pass over a scenegen.Batch.

    verts_list: per scene (V,3) float64 world vertices (leafs or posed)
    light_params: per light (3,) float64 (position, or travel direction)
    albedo_list: per scene (F,C) float64 or None (use the batch's albedo)
    Returns dict: images (list of (H,W,C)), lights (per-light discrete +
    continuous state), views (per-render camera state), flags (branch
    decisions taken in float arithmetic, for finite-difference validity)."""
    adjs = [Adjacency(sc.faces) for sc in batch.scenes]
    if albedo_list is None:
        albedo_list = [torch.as_tensor(np.asarray(sc.albedo, np.float64)) for sc in batch.scenes]
    lights = []
    for li, L in enumerate(batch.lights):
        sc = batch.scenes[L.scene]
        verts = verts_list[L.scene]
        fr = cameras.light_frame(L, light_params[li])
        S = L.resolution
        rv = raster_view(fr['M'], verts, sc.faces, S, S, adjs[L.scene], L.antialias)
        clip = homogeneous(verts) @ fr['M'].T
        faces = torch.as_tensor(np.asarray(sc.faces, np.int64))
        flat = np.nonzero(rv['tri'].ravel() >= 0)[0]
        t = torch.as_tensor(rv['tri'].ravel()[flat])
        px, py = pixel_centres_ndc(flat, S, S)
        fv = faces[t]
        b = perspective_barycentrics(clip[fv[:, 0]], clip[fv[:, 1]], clip[fv[:, 2]], px, py)
        x = (b[:, :, None] * verts[fv]).sum(1)
        f = warp_depth(light_distance(fr, x), L.warp_exponent)
        far = warp_depth(torch.ones((), dtype=D), L.warp_exponent)
        F0 = torch.stack([far, far * far]).expand(S * S, 2).clone()
        fl = torch.as_tensor(flat)
        F0 = F0.index_put((fl,), torch.stack([f, f * f], 1))
        F1 = smooth_edges(F0, rv['pairs'], clip, S, S) if L.antialias else F0
        lights.append(dict(frame=fr, rv=rv, F0=F0.T.reshape(2, S, S), F1=F1.T.reshape(2, S, S),
                           taps=filter_taps(L.filter, L.k, L.sigma), pad=0))
    for li, L in enumerate(batch.lights):
        ls = lights[li]
        if L.kind == 'cubeface':
            # the six faces of one cube are consecutive lights; each face's
            # map is padded with bilinear samples of its neighbours across the
            # cube's edges before filtering, so filter and fetch continue
            # across the seams
            base = li - L.face
            group = batch.lights[base:base + 6]
            assert [q.face for q in group] == list(range(6)) and all(q.kind == 'cubeface' for q in group)
            assert all((q.resolution, q.k, q.filter, q.sigma) == (L.resolution, L.k, L.filter, L.sigma) for q in group)
            S = L.resolution
            P = (L.k - 1) // 2 + 1
            idx, wgt = cameras.cube_pad_sources(S, P)
            stack = torch.stack([lights[base + g]['F1'] for g in range(6)], 1).reshape(2, 6 * S * S)
            taps = [stack[:, torch.as_tensor(idx[L.face, ..., q].ravel())] * torch.as_tensor(wgt[L.face, ..., q].ravel())
                    for q in range(4)]
            Fp = (((taps[0] + taps[1]) + taps[2]) + taps[3]).reshape(2, S + 2 * P, S + 2 * P)
            Mp = filter_separable(Fp, ls['taps'])
            ls.update(pad=P, Mpad=Mp, M=Mp[:, P:P + S, P:P + S])
        else:
            ls['M'] = filter_separable(ls['F1'], ls['taps'])
    images, views, flags = [], [], []
    for R in batch.renders:
        cam = batch.cameras[R.camera]
        sc = batch.scenes[cam.scene]
        verts = verts_list[cam.scene]
        alb = albedo_list[cam.scene]
        Mc = cameras.camera_matrix(cam)
        W, H = cam.width, cam.height
        rv = raster_view(Mc, verts, sc.faces, W, H, adjs[cam.scene], opts.camera_antialias)
        clip = homogeneous(verts) @ Mc.T
        faces = torch.as_tensor(np.asarray(sc.faces, np.int64))
        flat = np.nonzero(rv['tri'].ravel() >= 0)[0]
        t = torch.as_tensor(rv['tri'].ravel()[flat])
        px, py = pixel_centres_ndc(flat, W, H)
        fv = faces[t]
        b = perspective_barycentrics(clip[fv[:, 0]], clip[fv[:, 1]], clip[fv[:, 2]], px, py)
        v0, v1, v2 = verts[fv[:, 0]], verts[fv[:, 1]], verts[fv[:, 2]]
        x = b[:, 0:1] * v0 + b[:, 1:2] * v1 + b[:, 2:3] * v2
        n = cameras.normalize(torch.linalg.cross(v1 - v0, v2 - v0))
        rho = alb[t]
        col = torch.zeros(len(flat), batch.channels, dtype=D)
        fl_flags = {}
        for li in R.lights:
            L = batch.lights[li]
            ls = lights[li]
            fr = ls['frame']
            S = L.resolution
            cl = homogeneous(x) @ fr['M'].T
            inside = (cl[:, 3] > 0) & (torch.abs(cl[:, 0] / cl[:, 3]) <= 1) & (torch.abs(cl[:, 1] / cl[:, 3]) <= 1)
            inside = inside.detach()
            sx = (cl[:, 0] / cl[:, 3] + 1.0) * (S / 2.0) - 0.5
            sy = (1.0 - cl[:, 1] / cl[:, 3]) * (S / 2.0) - 0.5
            sx = torch.where(inside, sx, torch.zeros_like(sx))
            sy = torch.where(inside, sy, torch.zeros_like(sy))
            P = ls['pad']
            m = bilinear(ls['Mpad'], sx + P, sy + P) if P else bilinear(ls['M'], sx, sy)
            z = light_distance(fr, x)
            vis_raw = lookup_visibility(m[:, 0], m[:, 1], z, _no_bleed(L))[0]
            vis, zw, eps = lookup_visibility(m[:, 0], m[:, 1], z, L)
            vis = torch.where(inside, vis, torch.ones_like(vis))
            if fr['kind'] == 'directional':
                omega = (-fr['w']).expand_as(x)
            else:
                omega = cameras.normalize(fr['pos'] - x)
            ndl = (n * omega).sum(1)
            lam = torch.clamp(ndl, min=0.0)
            cone = torch.ones_like(lam)
            margin = None
            if fr['kind'] == 'spot':
                cosang = (cameras.normalize(x - fr['pos']) * fr['w']).sum(1).detach()
                cone = (cosang >= fr['cos_half']).to(D)
                margin = (cosang - fr['cos_half']).abs()
            elif fr['kind'] == 'cubeface':
                dv = (x - fr['pos']).detach().numpy()
                cone = torch.as_tensor(cameras.cube_face_of(dv) == fr['face']).to(D)
                # relative gap between the two largest |d_a|: the face choice
                # (and the frustum border) is ambiguous where it vanishes
                ad = np.sort(np.abs(dv), axis=1)
                margin = torch.as_tensor((ad[:, 2] - ad[:, 1]) / np.maximum(ad[:, 2], 1e-30))
            col = col + rho * (lam * vis * L.intensity * cone)[:, None]
            fl_flags[li] = dict(inside=inside.numpy(), lit_side=(ndl > 0).detach().numpy(),
                                branch=(zw <= m[:, 0]).detach().numpy(),
                                clamp=(m[:, 1] - m[:, 0] ** 2 < eps).detach().numpy(),
                                floor=np.stack([torch.floor(sx).detach().numpy(),
                                                torch.floor(sy).detach().numpy()]),
                                frac=np.stack([(sx - torch.floor(sx)).detach().numpy(),
                                               (sy - torch.floor(sy)).detach().numpy()]),
                                var_ratio=((m[:, 1] - m[:, 0] ** 2) / eps).detach().numpy()
                                if L.min_variance > 0 else None,
                                bleed_margin=(vis_raw - L.bleed_reduction).abs().detach().numpy()
                                if L.bleed_reduction > 0 else None,
                                bleed_on=(vis_raw >= L.bleed_reduction).detach().numpy()
                                if L.bleed_reduction > 0 else None,
                                cone_on=(cone > 0).detach().numpy() if margin is not None else None,
                                cone_margin=None if margin is None else margin.numpy())
        img0 = torch.zeros(W * H, batch.channels, dtype=D)
        img0 = img0.index_put((torch.as_tensor(flat),), col)
        img = smooth_edges(img0, rv['pairs'], clip, W, H) if opts.camera_antialias else img0
        images.append(img.reshape(H, W, batch.channels))
        views.append(dict(rv=rv, img0=img0.reshape(H, W, batch.channels), flat=flat))
        flags.append(fl_flags)
    return dict(images=images, lights=lights, views=views, flags=flags)


def mse(images, targets):
    n = sum(im.numel() for im in images)
    return sum(((im - tg) ** 2).sum() for im, tg in zip(images, targets)) / n


# ----------------------------------------------------------------------------- convenience

def scene_leaves(batch, requires_grad=True):
    """float64 leaf tensors for a batch: world vertices (posed when the scene
    has a pose), light parameters, poses, albedo."""
    poses = [torch.tensor(np.asarray(sc.pose, np.float64), requires_grad=requires_grad and sc.pose_count > 0)
             for sc in batch.scenes]
    base = [torch.tensor(np.asarray(sc.verts, np.float64), requires_grad=requires_grad and sc.pose_count == 0)
            for sc in batch.scenes]
    lp = [torch.tensor(np.asarray(L.param, np.float64), requires_grad=requires_grad) for L in batch.lights]
    alb = [torch.tensor(np.asarray(sc.albedo, np.float64), requires_grad=requires_grad) for sc in batch.scenes]
    return base, poses, lp, alb


def world_vertices(batch, base, poses):
    out = []
    for sc, b, p in zip(batch.scenes, base, poses):
        out.append(posed_vertices(sc, p) if sc.pose_count > 0 else b)
    return out


def target_images(batch):
    """Target images of the inverse problem: the batch rendered with its
    target light parameters / poses (no gradients)."""
    base, poses, lp, alb = scene_leaves(batch, requires_grad=False)
    if batch.target_light_params is not None:
        lp = [torch.as_tensor(np.asarray(p, np.float64)) for p in batch.target_light_params]
    if batch.target_poses is not None:
        poses = [torch.as_tensor(np.asarray(p, np.float64)) for p in batch.target_poses]
    with torch.no_grad():
        out = render(batch, world_vertices(batch, base, poses), lp, alb)
    return [im.detach() for im in out['images']]


def fingerprint(out):
    """All discrete state of a forward pass (for finite-difference validity)."""
    parts = []
    for ls in out['lights']:
        parts.append(ls['rv']['tri'].tobytes())
        p = ls['rv']['pairs']
        if p is not None:
            parts += [p[k].tobytes() for k in ('T', 'O', 'a', 'b')]
    for v, fl in zip(out['views'], out['flags']):
        parts.append(v['rv']['tri'].tobytes())
        p = v['rv']['pairs']
        if p is not None:
            parts += [p[k].tobytes() for k in ('T', 'O', 'a', 'b')]
        for li, f in fl.items():
            for k in ('inside', 'lit_side', 'branch', 'clamp', 'floor', 'bleed_on', 'cone_on'):
                if f.get(k) is not None:
                    parts.append(np.asarray(f[k]).tobytes())
    return parts
