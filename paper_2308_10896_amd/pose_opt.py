"""Batched pose estimation driven by the differentiable shadow-mapping path.

Every scene of the batch holds one rigid object whose pose (axis-angle r,
translation t) is unknown; a target image of each scene is rendered at the
reference pose, and all poses are recovered at once by minimizing the image
MSE with Adam through the shadowed renderer (the monocular pose-estimation
application, Sec. 6.1, with the optimizer settings of its experiment details
in supp. B: step 0.01, betas (0.9, 0.999), 150 iterations).  As there, the
free parameters are the translation parallel to the receiver plane (x, z)
and the rotation about the object's up axis (y); the start pose differs from
the reference in those three only.  Each iteration is one batched forward +
backward over all scenes.

``python -m paper_2308_10896_amd.pose_opt`` runs it on the 64-scene blob
batch and prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np
import torch

from . import dsm


def _rotation(r):
    r = np.asarray(r, dtype=np.float64)
    th = float(np.linalg.norm(r))
    if th < 1e-15:
        return np.eye(3)
    k = r / th
    K = np.array([[0.0, -k[2], k[1]], [k[2], 0.0, -k[0]], [-k[1], k[0], 0.0]])
    return np.eye(3) + math.sin(th) * K + (1.0 - math.cos(th)) * (K @ K)


def pose_errors(poses, targets):
    """Per scene: rotation error angle of R(r) R(r*)^T in degrees, and |t - t*|."""
    dphi, dt = [], []
    for p, q in zip(np.asarray(poses, dtype=np.float64), np.asarray(targets, dtype=np.float64)):
        rel = _rotation(p[:3]) @ _rotation(q[:3]).T
        c = min(1.0, max(-1.0, (np.trace(rel) - 1.0) / 2.0))
        dphi.append(math.degrees(math.acos(c)))
        dt.append(float(np.linalg.norm(p[3:] - q[3:])))
    return np.array(dphi), np.array(dt)


# pose = (axis-angle rx, ry, rz, translation tx, ty, tz); y is up, the receiver plane is y = 0
FREE_DOF = (1, 3, 5)


def optimize_poses(batch, iters: int = 150, lr: float = 0.01, device='cuda', tile_size: int = 0,
                   free=FREE_DOF):
    """Recover every scene's pose from its target image.  The start pose is
    the reference pose plus the scene's perturbation in the `free` components.
    Returns a dict with the initial and final pose errors, the loss curve and
    the iteration rate."""
    plan = dsm.Plan(batch, tile_size=tile_size)
    local, lp, alb, perturbed = dsm.batch_inputs(batch, device)
    target = torch.as_tensor(np.stack(batch.target_poses).astype(np.float32), device=device)
    mask = torch.zeros(6, device=device)
    mask[list(free)] = 1.0
    poses0 = (target + mask * (perturbed - target)).contiguous()
    pix = [h * w for h, w, _ in plan.render_shapes]
    scale = torch.cat([torch.full((h * w * c,), 1.0 / (h * w), device=device)
                       for (h, w, c) in plan.render_shapes])
    with torch.no_grad():
        target_img = dsm.render(plan, dsm.pose(plan, local, target), lp, alb)
    p = poses0.clone().requires_grad_(True)
    p.register_hook(lambda g: g * mask)
    opt = torch.optim.Adam([p], lr=lr, betas=(0.9, 0.999))
    dphi0, dt0 = pose_errors(poses0.cpu().numpy(), target.cpu().numpy())
    losses = []
    torch.cuda.synchronize()
    t0 = time.time()
    for _ in range(iters):
        opt.zero_grad(set_to_none=True)
        img = dsm.render(plan, dsm.pose(plan, local, p), lp, alb)
        loss = (scale * (img - target_img) ** 2).sum()        # sum over scenes of per-image MSE
        loss.backward()
        opt.step()
        losses.append(loss.detach())
    torch.cuda.synchronize()
    dt_s = time.time() - t0
    dphi1, dt1 = pose_errors(p.detach().cpu().numpy(), target.cpu().numpy())
    return {
        'scenes': len(batch.scenes), 'iterations': iters, 'lr': lr,
        'image_pixels': int(sum(pix)),
        'iterations_per_s': iters / dt_s,
        'scene_iterations_per_s': iters * len(batch.scenes) / dt_s,
        'dphi_deg_initial': dphi0, 'dphi_deg_final': dphi1,
        'dt_initial': dt0, 'dt_final': dt1,
        'loss': torch.stack(losses).cpu().numpy(),
    }


def main():
    import scenegen as sg
    ap = argparse.ArgumentParser()
    ap.add_argument('--scenes', type=int, default=64)
    ap.add_argument('--res', type=int, default=512)
    ap.add_argument('--iters', type=int, default=150)
    ap.add_argument('--lr', type=float, default=0.01)
    args = ap.parse_args()
    batch = sg.config2(n_scenes=args.scenes, resolution=args.res, with_pose=True)
    r = optimize_poses(batch, iters=args.iters, lr=args.lr)
    out = {
        'workload': f'pose estimation: {args.scenes} blob scenes, {args.res}^2 shadow maps and views, '
                    f'Adam lr {args.lr}, {args.iters} iterations',
        'iterations_per_s': round(r['iterations_per_s'], 2),
        'scene_iterations_per_s': round(r['scene_iterations_per_s'], 1),
        'dphi_deg_median': [round(float(np.median(r['dphi_deg_initial'])), 4),
                            round(float(np.median(r['dphi_deg_final'])), 4)],
        'dt_median': [round(float(np.median(r['dt_initial'])), 5), round(float(np.median(r['dt_final'])), 5)],
        'converged_fraction': round(float(np.mean((r['dphi_deg_final'] < 1.0) & (r['dt_final'] < 0.01))), 4),
        'loss': [float(r['loss'][0]), float(r['loss'][-1])],
    }
    print(json.dumps(out), flush=True)


if __name__ == '__main__':
    main()
