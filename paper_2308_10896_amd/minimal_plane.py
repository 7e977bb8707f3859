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

``python -m paper_2308_10896_amd.minimal_plane`` prints one JSON line.
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--iters', type=int, default=150)
    args = ap.parse_args()
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
