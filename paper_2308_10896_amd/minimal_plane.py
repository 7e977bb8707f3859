"""Behavioural checks of the shadow gradients on the "minimal plane" scene
(a square occluder over a parallel receiver under a directional light; the
camera sees only the shadow), as in the paper's convergence experiments
(Sec. 5, optimization without smoothed shadow map, and the filter-size
convergence study; supplementary B for the setup):

* vertex experiment: one occluder corner is displaced and its position is
  recovered from the shadow image alone.  With the light-view edge smoothing
  the corner converges; without it the moments do not depend on the
  corner's position and the optimization cannot move it, whatever the filter
  size k.
* translation experiment: the occluder is displaced along x and the offset
  is recovered with SGD or Adam for several filter sizes k.
* Jacobian experiment (Sec. 5, shadow map resolution and filter kernel): the
  per-pixel derivative of the shadow image with respect to the horizontal
  translation of a slightly rotated occluder of up to 130,050 triangles;
  fine tessellation leaves the derivative sparse along the shadow outline,
  the moment filter spreads it.
* resolution experiment (same paragraph): occluders slanted until their
  shadow is narrower than a texel are missed at low shadow-map resolution;
  the shadow border widens with the filter size.

``python -m paper_2308_10896_amd.minimal_plane [--jacobian | --resolution]``
prints one JSON line.
"""
from __future__ import annotations

import argparse
import json

import numpy as np
import torch

from . import dsm


def _loss_fn(plan):
    scale = torch.cat([torch.full((h * w * c,), 1.0 / (h * w), device='cuda') for (h, w, c) in plan.render_shapes])
    return lambda img, ref: (scale * (img - ref) ** 2).sum()


def vertex_experiment(k: int, antialias: bool, iters: int = 150, lr: float = 0.01, corner: int = 3,
                      displacement=(0.08, 0.05)):
    """Recover a displaced occluder corner (x, z).  Returns the initial and
    final distance to the reference position and the loss curve."""
    import scenegen as sg
    batch = sg.minimal_plane(k=k, antialias=antialias)
    plan = dsm.Plan(batch)
    local, lp, alb, poses = dsm.batch_inputs(batch)
    base = plan.pose_forward(local, poses).detach()        # reference world positions
    loss_fn = _loss_fn(plan)
    with torch.no_grad():
        ref = dsm.render(plan, base, lp, alb)
    d = torch.tensor(displacement, dtype=torch.float32, device='cuda', requires_grad=True)
    sel = torch.zeros(base.shape[0], 3, device='cuda')
    sel[corner, 0] = 1.0
    sel_z = torch.zeros_like(sel)
    sel_z[corner, 2] = 1.0
    opt = torch.optim.Adam([d], lr=lr)
    err0 = float(torch.linalg.norm(d).item())
    losses = []
    for _ in range(iters):
        opt.zero_grad(set_to_none=True)
        verts = (base + d[0] * sel + d[1] * sel_z).contiguous()
        loss = loss_fn(dsm.render(plan, verts, lp, alb), ref)
        loss.backward()
        opt.step()
        losses.append(float(loss.item()))
    return {'k': k, 'antialias': antialias, 'error_initial': err0, 'error_final': float(torch.linalg.norm(d).item()),
            'loss': losses}


def translation_experiment(k: int, optimizer: str = 'adam', lr: float = 0.01, iters: int = 150, offset: float = 0.1):
    """Recover an x offset of the whole occluder.  Returns the signed error
    per iteration."""
    import scenegen as sg
    batch = sg.minimal_plane(k=k, antialias=True, offset=(offset, 0.0, 0.0))
    plan = dsm.Plan(batch)
    local, lp, alb, poses = dsm.batch_inputs(batch)
    target = torch.zeros_like(poses)
    loss_fn = _loss_fn(plan)
    with torch.no_grad():
        ref = dsm.render(plan, dsm.pose(plan, local, target), lp, alb)
    tx = poses[:, 3].clone().requires_grad_(True)
    opt = torch.optim.Adam([tx], lr=lr) if optimizer == 'adam' else torch.optim.SGD([tx], lr=lr)
    errs = [float(tx[0].item())]
    for _ in range(iters):
        opt.zero_grad(set_to_none=True)
        p = torch.cat([poses[:, :3], tx[:, None], poses[:, 4:]], dim=1).contiguous()
        loss = loss_fn(dsm.render(plan, dsm.pose(plan, local, p), lp, alb), ref)
        loss.backward()
        opt.step()
        errs.append(float(tx[0].item()))
    return {'k': k, 'optimizer': optimizer, 'lr': lr, 'signed_error': errs}


def jacobian_image(tess: int, k: int, resolution: int = 256, view: int = 128, rot_deg: float = 15.0,
                   antialias: bool = True):
    """Jacobian of the shadow image with respect to the occluder's horizontal
    translation x (Sec. 5, shadow map resolution and filter kernel: the
    visibility Jacobian of a highly tessellated, slightly rotated occluder),
    one reverse pass per pixel: the upstream gradient is the pixel's unit
    vector and the pose chain returns d(pixel)/dx.  The occluder is a
    tess x tess grid of quads rotated by rot_deg about the vertical axis.
    Returns the [view, view] Jacobian and the image (numpy)."""
    import scenegen as sg
    batch = sg.minimal_plane(k=k, antialias=antialias, resolution=resolution, view=view, occluder_tess=tess,
                             rotation=(0.0, float(np.deg2rad(rot_deg)), 0.0))
    plan = dsm.Plan(batch)
    local, lp, alb, poses = dsm.batch_inputs(batch)
    verts = plan.pose_forward(local, poses)
    saved, scratch = plan.workspace()
    image = plan.forward(verts, lp, alb, saved, scratch)
    n = int(plan.info.image_floats)
    jac = torch.empty(n, device='cuda')
    onehot = torch.zeros(n, device='cuda')
    for p in range(n):
        onehot.zero_()
        onehot[p] = 1.0
        gv, _, _ = plan.backward(verts, lp, alb, saved, scratch, onehot, want_albedo=False)
        jac[p] = plan.pose_backward(local, poses, gv)[0, 3]
    torch.cuda.synchronize()
    return jac.reshape(view, view).cpu().numpy(), image.reshape(view, view).cpu().numpy()


def receiver_points(view: int, camera_height: float = 0.45):
    """World (x, z) on the receiver (y = 0) of every camera pixel's centre: the
    camera looks straight down with a 120 degree field of view, image x
    along world +x and image up along world -z."""
    t = camera_height * np.tan(np.deg2rad(60.0))
    c = (2.0 * (np.arange(view) + 0.5) / view - 1.0) * t
    x = np.broadcast_to(c[None, :], (view, view))
    z = np.broadcast_to(c[:, None], (view, view))      # image rows run top to bottom: world -z up
    return x, z, 2.0 * t / view


def shadow_outline_distance(x, z, rot_deg: float, half: float = 0.25):
    """Distance of receiver points to the outline of the occluder's vertical
    projection (a square of half-size `half` rotated by rot_deg about y)."""
    a = np.deg2rad(rot_deg)
    # rotation about +y by a maps (x, z) to (x cos a + z sin a, -x sin a + z cos a); undo it
    u = x * np.cos(a) - z * np.sin(a)
    w = x * np.sin(a) + z * np.cos(a)
    du, dw = np.abs(u) - half, np.abs(w) - half
    outside = np.hypot(np.maximum(du, 0), np.maximum(dw, 0))
    inside = np.minimum(np.maximum(du, dw), 0)
    return np.abs(outside + inside)


def jacobian_experiment(tess_list=(1, 16, 255), ks=(1, 5, 9), resolution: int = 256, view: int = 128,
                        rot_deg: float = 15.0):
    """Sparsity of the visibility Jacobian: for each occluder tessellation
    (255 x 255 quads = 130,050 triangles, the paper's 130k-face occluder)
    and filter size k, the share of camera pixels within 1.5 pixels of the
    shadow outline whose Jacobian is non-zero (> 1e-3 of the largest), the
    Jacobian's L1 mass, and the share of non-zero pixels away from the
    outline.  Edge smoothing only acts on pixel pairs whose front triangle
    exits through a silhouette edge, so when many triangles share a texel
    most outline pairs see an interior edge and get no derivative; the
    moment filter spreads the derivatives that remain."""
    x, z, px = receiver_points(view)
    dist = shadow_outline_distance(x, z, rot_deg)
    band = dist < 1.5 * px
    rows = []
    for tess in tess_list:
        for k in ks:
            jac, _ = jacobian_image(tess, k, resolution, view, rot_deg)
            nz = np.abs(jac) > 1e-3 * max(np.abs(jac).max(), 1e-30)
            rows.append({'occluder_triangles': 2 * tess * tess, 'k': k,
                         'outline_coverage': round(float(nz[band].mean()), 4),
                         'off_outline_nonzero': round(float(nz[~band].mean()), 4),
                         'l1': round(float(np.abs(jac).sum() * px * px), 6)})
    return rows


def resolution_experiment(slants_deg=(0.0, 60.0, 80.0, 88.0), resolutions=(32, 64, 128, 256, 512, 1024),
                          k: int = 1, view: int = 256, camera_height: float = 0.2):
    """Shadow-map resolution and slanted occluders (Sec. 5, shadow map
    resolution and filter kernel): the occluder is tilted by each slant
    about the x axis, so its shadow under the vertical light is a strip of
    width 0.5 cos(slant); the shadow area measured in the image (the
    receiver is lit at rho (n . w) = albedo, so a pixel's shadowed fraction
    is 1 - image / albedo) is compared with that exact area.  At low
    resolution a strip narrower than a texel falls between texel centres
    and the occluder is missed."""
    import scenegen as sg
    x, z, px = receiver_points(view, camera_height)
    rows = []
    for slant in slants_deg:
        for S in resolutions:
            batch = sg.minimal_plane(k=k, resolution=S, view=view, camera_height=camera_height,
                                     rotation=(float(np.deg2rad(slant)), 0.0, 0.0))
            plan = dsm.Plan(batch)
            local, lp, alb, poses = dsm.batch_inputs(batch)
            with torch.no_grad():
                img = dsm.render(plan, dsm.pose(plan, local, poses), lp, alb).reshape(view, view).cpu().numpy()
            area = float((1.0 - img / 0.8).clip(0, 1).sum() * px * px)
            exact = 0.25 * np.cos(np.deg2rad(slant))
            rows.append({'slant_deg': slant, 'resolution': S, 'shadow_area': round(area, 6),
                         'exact_area': round(exact, 6), 'ratio': round(area / exact, 4)})
    return rows


def filter_width_experiment(ks=(1, 3, 5, 9, 15, 25), resolution: int = 256, view: int = 256):
    """Width of the shadow border (10 % to 90 % of the transition along the
    image row through the shadow's centre, across the edge at x = 0.25) for
    each filter size k: larger kernels widen the border."""
    import scenegen as sg
    x, _, px = receiver_points(view)
    rows = []
    for k in ks:
        batch = sg.minimal_plane(k=k, resolution=resolution, view=view)
        plan = dsm.Plan(batch)
        local, lp, alb, poses = dsm.batch_inputs(batch)
        with torch.no_grad():
            img = dsm.render(plan, dsm.pose(plan, local, poses), lp, alb).reshape(view, view).cpu().numpy()
        row = img[view // 2] / 0.8                     # 0 in the umbra, 1 lit
        sel = (x[view // 2] > 0.0) & (x[view // 2] < 0.5)
        xs, vs = x[view // 2][sel], row[sel]
        x10 = float(xs[np.argmax(vs >= 0.1)])
        x90 = float(xs[np.argmax(vs >= 0.9)])
        rows.append({'k': k, 'border_width': round(x90 - x10 + px, 5)})
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--iters', type=int, default=150)
    ap.add_argument('--jacobian', action='store_true', help='the Jacobian sparsity experiment only')
    ap.add_argument('--resolution', action='store_true', help='the resolution and filter-width experiments only')
    args = ap.parse_args()
    if args.jacobian:
        print(json.dumps({'jacobian': jacobian_experiment()}), flush=True)
        return
    if args.resolution:
        print(json.dumps({'resolution': resolution_experiment(), 'filter_width': filter_width_experiment()}),
              flush=True)
        return
    out = {'vertex': [], 'translation': []}
    for aa in (True, False):
        for k in (1, 5, 9):
            r = vertex_experiment(k, aa, iters=args.iters)
            out['vertex'].append({'k': k, 'antialias': aa, 'error': [round(r['error_initial'], 5),
                                                                      round(r['error_final'], 5)]})
    for opt, lr in (('sgd', 0.5), ('sgd', 2.0), ('adam', 0.01), ('adam', 0.05)):
        for k in (1, 3, 5, 9, 15):
            r = translation_experiment(k, opt, lr, iters=args.iters)
            e = r['signed_error']
            out['translation'].append({'k': k, 'optimizer': opt, 'lr': lr,
                                       'signed_error': [round(e[0], 5), round(e[len(e) // 2], 5), round(e[-1], 5)]})
    print(json.dumps(out), flush=True)


if __name__ == '__main__':
    main()
