"""Shared helpers of the GPU parity tests: run a batch through the HIP library
(C ABI via the binding) and through the oracle on the same seeded inputs,
and compare stage by stage."""
from __future__ import annotations

import numpy as np
import torch

from oracle import pipeline as P

# Tolerances (float32 kernels vs the float64 oracle).  Maps: |g - o| <= 1e-6 + 1e-4 |o|.
# Visibility / images: atol 1e-4 (conditioning of m2 - m1^2 in float32 at the
# variance floor).  Gradients: normwise per parameter group.
MAP_RTOL, MAP_ATOL = 1e-4, 1e-6
IMG_RTOL, IMG_ATOL = 1e-4, 1e-4
# Pixels whose shadowed visibility rests on sigma^2 within 10x the variance
# floor: float32 forms m2 - m1^2 with an absolute error e of a few 1e-8, which
# moves v = s/(s + d^2) by up to e / (4 s), about 5e-4 at the floor.
IMG_FLOOR_ATOL = 1e-3
GRAD_TOL = 1e-3      # normwise relative, per parameter group


def gpu_run(batch, tile_size=0, bin_scale=0, grad_images=None, pose=False):
    from paper_2308_10896_amd import dsm
    plan = dsm.Plan(batch, tile_size=tile_size, bin_capacity_scale=bin_scale)
    verts, lp, alb, poses = dsm.batch_inputs(batch)
    if pose:
        local = verts
        verts = plan.pose_forward(local, poses)
    saved, scratch = plan.workspace()
    images = plan.forward(verts, lp, alb, saved, scratch)
    out = dict(plan=plan, images=[im.cpu().numpy() for im in plan.split_images(images)])
    out['keys'] = [plan.view_keys(saved, v).cpu().numpy().view(np.uint64) for v in range(len(plan.view_shapes))]
    out['F0'] = [plan.light_maps(saved, scratch, l, 0).cpu().numpy() for l in range(plan.num_lights)]
    out['F1'] = [plan.light_maps(saved, scratch, l, 1).cpu().numpy() for l in range(plan.num_lights)]
    out['M'] = [plan.light_maps(saved, scratch, l, 2).cpu().numpy() for l in range(plan.num_lights)]
    out['img0'] = [plan.image0(saved, r).cpu().numpy() for r in range(len(batch.renders))]
    out['stats'] = plan.stats(saved)
    out['verts'] = verts.cpu().numpy()
    if grad_images is not None:
        g = torch.as_tensor(np.concatenate([x.ravel() for x in grad_images]).astype(np.float32)).cuda()
        gv, gl, ga = plan.backward(verts, lp, alb, saved, scratch, g)
        out['gverts'] = gv.cpu().numpy()
        out['glight'] = gl.cpu().numpy()
        out['galbedo'] = ga.cpu().numpy()
        if pose:
            out['gpose'] = plan.pose_backward(local, poses, gv).cpu().numpy()
    torch.cuda.synchronize()
    return out


def oracle_run(batch, grad_images=None, pose=False, camera_aa=True):
    base, poses, lp, alb = P.scene_leaves(batch, requires_grad=True)
    verts = P.world_vertices(batch, base, poses)
    out = P.render(batch, verts, lp, alb, P.Options(camera_antialias=camera_aa))
    res = dict(raw=out, images=[im.detach().numpy() for im in out['images']])
    res['keys'] = [ls['rv']['key'] for ls in out['lights']] + [None] * len(batch.cameras)
    for r, v in zip(batch.renders, out['views']):
        res['keys'][len(batch.lights) + r.camera] = v['rv']['key']
    res['F0'] = [ls['F0'].detach().numpy() for ls in out['lights']]
    res['F1'] = [ls['F1'].detach().numpy() for ls in out['lights']]
    res['M'] = [ls['M'].detach().numpy() for ls in out['lights']]
    res['img0'] = [v['img0'].detach().numpy() for v in out['views']]
    res['flags'] = out['flags']
    res['culled'] = sum(ls['rv']['st']['culled'] for ls in out['lights'])
    if grad_images is not None:
        leaves = [t for t in (base if not pose else []) ] + list(lp) + list(alb) + (list(poses) if pose else [])
        gts = [torch.as_tensor(g.astype(np.float64)) for g in grad_images]
        total = sum((im * g).sum() for im, g in zip(out['images'], gts))
        grads = torch.autograd.grad(total, leaves, allow_unused=True)
        k = 0
        if not pose:
            res['gverts'] = np.concatenate([g.numpy() if g is not None else np.zeros(b.shape)
                                            for g, b in zip(grads[:len(base)], base)])
            k = len(base)
        res['glight'] = np.stack([g.numpy() for g in grads[k:k + len(lp)]])
        k += len(lp)
        res['galbedo'] = np.concatenate([g.numpy() for g in grads[k:k + len(alb)]])
        k += len(alb)
        if pose:
            res['gpose'] = np.stack([g.numpy() if g is not None else np.zeros(6) for g in grads[k:]])
    return res


def loss_grad(batch, images):
    """Upstream gradient of the MSE loss to the batch's target images."""
    targets = P.target_images(batch)
    n = sum(t.numel() for t in targets)
    return [(2.0 / n) * (im - t.numpy()) for im, t in zip(images, targets)]


def random_grad(batch, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((batch.cameras[r.camera].height, batch.cameras[r.camera].width, batch.channels))
            for r in batch.renders]


def assert_close(name, got, want, rtol, atol, mask=None):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    assert got.shape == want.shape, (name, got.shape, want.shape)
    bad = np.abs(got - want) > atol + rtol * np.abs(want)
    if mask is not None:
        bad &= mask
    if bad.any():
        idx = np.argwhere(bad)[:5]
        detail = [(tuple(i), float(got[tuple(i)]), float(want[tuple(i)])) for i in idx]
        raise AssertionError(f'{name}: {int(bad.sum())} of {bad.size} elements differ, e.g. {detail}')


def normwise(name, got, want, tol):
    got = np.asarray(got, np.float64).ravel()
    want = np.asarray(want, np.float64).ravel()
    nrm = np.linalg.norm(want)
    err = np.linalg.norm(got - want) / max(nrm, 1e-30)
    print(f'{name}: normwise relative error {err:.3e} (|oracle| = {nrm:.3e})')
    assert err <= tol, f'{name}: normwise relative error {err:.3e} > {tol:.1e} (|o| = {nrm:.3e})'
    return err


def cone_ambiguous(batch, oracle_res, render, margin=1e-5):
    """Pixels whose spot-cone test is within `margin` of its threshold: the
    hard cone mask is a float decision taken in float64 by the oracle and in
    float32 by the kernel, so either outcome is correct there."""
    r = batch.renders[render]
    cam = batch.cameras[r.camera]
    amb = np.zeros(cam.height * cam.width, bool)
    view = oracle_res['raw']['views'][render]
    for li, f in oracle_res['flags'][render].items():
        if f['cone_margin'] is not None:
            amb[view['flat']] |= f['cone_margin'] < margin
    return amb.reshape(cam.height, cam.width)


def decisions_clear(batch, oracle_res, render, cell_eps=1e-3, face_eps=1e-4, var_eps=0.05, bleed_eps=1e-3):
    """Camera pixels whose discrete lookup decisions sit clear of their
    thresholds in every light: the bilinear cell (floor of the map position,
    where the fetch's derivative jumps) at least `cell_eps` texels from a
    texel-centre line, the spot-cone / cube-face choice at least `face_eps`
    from its tie, and, in the shadowed branch, m2 - m1^2 at least a fraction
    `var_eps` away from the variance floor (the floor switches the
    derivative through sigma^2 on and off, and float32 forms m2 - m1^2 with
    an absolute error of a few 1e-7), and the visibility at least `bleed_eps`
    from the light-bleeding reduction's threshold.  The kernels take these decisions in
    float32, the oracle in float64, so a gradient test that weights only
    these pixels compares one piecewise-smooth branch on both sides."""
    r = batch.renders[render]
    cam = batch.cameras[r.camera]
    ok = np.ones(cam.height * cam.width, bool)
    view = oracle_res['raw']['views'][render]
    for li, f in oracle_res['flags'][render].items():
        fr = f['frac']
        near = (np.minimum(fr, 1.0 - fr) < cell_eps).any(0) & f['inside']
        ok[view['flat']] &= ~near
        if f['var_ratio'] is not None:
            shadowed = f['inside'] & ~f['branch']
            ok[view['flat']] &= ~(shadowed & (np.abs(f['var_ratio'] - 1.0) < var_eps))
        if f.get('bleed_margin') is not None:
            ok[view['flat']] &= ~(f['inside'] & (f['bleed_margin'] < bleed_eps))
        if f['cone_margin'] is not None:
            ok[view['flat']] &= f['cone_margin'] >= face_eps
    return ok.reshape(cam.height, cam.width)


def floor_conditioned(batch, oracle_res, render, ratio=10.0, dilate=0):
    """Camera pixels whose visibility, in the shadowed branch of some light,
    rests on sigma^2 within `ratio` times the variance floor (dilated by
    `dilate` pixels, for images after the edge smoothing that blends
    neighbours)."""
    r = batch.renders[render]
    cam = batch.cameras[r.camera]
    m = np.zeros(cam.height * cam.width, bool)
    view = oracle_res['raw']['views'][render]
    for li, f in oracle_res['flags'][render].items():
        if f['var_ratio'] is not None:
            m[view['flat']] |= f['inside'] & ~f['branch'] & (f['var_ratio'] < ratio)
    m = m.reshape(cam.height, cam.width)
    for _ in range(dilate):
        d = m.copy()
        d[1:] |= m[:-1]; d[:-1] |= m[1:]; d[:, 1:] |= m[:, :-1]; d[:, :-1] |= m[:, 1:]
        m = d
    return m


def assert_image(name, got, want, batch, oracle_res, render, mask=None, smoothed=False):
    """Image parity: IMG_ATOL everywhere except at floor-conditioned pixels
    (IMG_FLOOR_ATOL there), both with IMG_RTOL."""
    cond = floor_conditioned(batch, oracle_res, render, dilate=1 if smoothed else 0)[..., None]
    cond = np.broadcast_to(cond, np.shape(want))
    base = np.ones(np.shape(want), bool) if mask is None else np.broadcast_to(mask, np.shape(want))
    assert_close(name, got, want, IMG_RTOL, IMG_ATOL, mask=base & ~cond)
    assert_close(name + ' (near the variance floor)', got, want, IMG_RTOL, IMG_FLOOR_ATOL, mask=base & cond)
