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
# Gradients, per parameter group: normwise relative error and elementwise
# error as a fraction of the group's largest oracle entry, on the pixels whose
# discrete lookup decisions are clear of their thresholds (clear_upstream).
GRAD_TOL = 1e-4
GRAD_ELEM_FRAC = 1e-3
# The share of the gradient that comes from pixels whose visibility rests on
# sigma^2 within 10x the variance floor (floor_conditioned): there the
# visibility and its derivatives are steep in the map position u = L(x) and
# in sigma^2, and float32 forms u with a few ulps of error (world point from
# barycentrics, M x, 1/w).  The oracle's own gradient of that share moves by
# up to 1e-3 (light), 1.4e-4 (vertices) when u is perturbed by 1 to 4 ulps
# (the reduced complex scene, 3 lights summed); the bound keeps a factor 5.
GRAD_FLOOR_TOL = 5e-3
GRAD_FLOOR_ELEM_FRAC = 5e-3
# Largest share of pixels whose decisions may go either way (dropped).
AMBIGUOUS_MAX = 0.02


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


def gpu_grads(batch, Gs, pose=False, tile_size=0, bin_scale=0):
    """GPU gradients for several upstream image gradients (one forward, one
    backward each)."""
    from paper_2308_10896_amd import dsm
    plan = dsm.Plan(batch, tile_size=tile_size, bin_capacity_scale=bin_scale)
    verts, lp, alb, poses = dsm.batch_inputs(batch)
    local = verts
    if pose:
        verts = plan.pose_forward(local, poses)
    saved, scratch = plan.workspace()
    plan.forward(verts, lp, alb, saved, scratch)
    outs = []
    for G in Gs:
        g = torch.as_tensor(np.concatenate([x.ravel() for x in G]).astype(np.float32)).cuda()
        gv, gl, ga = plan.backward(verts, lp, alb, saved, scratch, g)
        o = dict(gverts=gv.cpu().numpy(), glight=gl.cpu().numpy(), galbedo=ga.cpu().numpy())
        if pose:
            o['gpose'] = plan.pose_backward(local, poses, gv).cpu().numpy()
        outs.append(o)
    torch.cuda.synchronize()
    return outs


def oracle_grads(batch, Gs, pose=False):
    """Oracle (float64 autograd) gradients for several upstream image
    gradients, from one forward pass."""
    base, poses, lp, alb = P.scene_leaves(batch, requires_grad=True)
    verts = P.world_vertices(batch, base, poses)
    out = P.render(batch, verts, lp, alb)
    leaves = (list(base) if not pose else []) + list(lp) + list(alb) + (list(poses) if pose else [])
    outs = []
    for G in Gs:
        total = sum((im * torch.as_tensor(np.asarray(g, np.float64))).sum() for im, g in zip(out['images'], G))
        grads = torch.autograd.grad(total, leaves, allow_unused=True, retain_graph=True)
        res, k = {}, 0
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
        outs.append(res)
    return outs


def check_gradients(batch, G, oracle_res=None, pose=False, groups=None, extra=None, rest_tol=GRAD_TOL):
    """Gradient parity for the upstream image gradient G.  G is kept on the
    pixels whose lookup decisions are clear (clear_upstream) and split into
    the floor-conditioned pixels and the rest; the backward is linear in G,
    so each share is compared on its own: the rest at GRAD_TOL /
    GRAD_ELEM_FRAC, the floor-conditioned share at GRAD_FLOOR_TOL /
    GRAD_FLOOR_ELEM_FRAC (rest_tol replaces GRAD_TOL where a test derives
    its own bound).  `groups` names the gradient groups compared
    (default: light, vertex or pose, albedo); `extra(name, gpu, oracle)` may
    add checks on each share's results.  Upstream values are rounded to
    float32 first, so both sides differentiate the same cotangent."""
    o0 = oracle_run(batch, pose=pose) if oracle_res is None else oracle_res
    G = [np.asarray(g, np.float32).astype(np.float64) for g in clear_upstream(batch, G, o0, pose=pose)]
    cond = [floor_conditioned(batch, o0, r, dilate=1)[..., None] for r in range(len(batch.renders))]
    shares = {'rest': [g * ~c for g, c in zip(G, cond)], 'floor': [g * c for g, c in zip(G, cond)]}
    names = list(shares)
    gpu = gpu_grads(batch, [shares[n] for n in names], pose=pose)
    ora = oracle_grads(batch, [shares[n] for n in names], pose=pose)
    if groups is None:
        groups = ['glight', 'gpose' if pose else 'gverts', 'galbedo']
    for n, g, o in zip(names, gpu, ora):
        tol, elem = (rest_tol, GRAD_ELEM_FRAC) if n == 'rest' else (GRAD_FLOOR_TOL, GRAD_FLOOR_ELEM_FRAC)
        for k in groups:
            if not np.any(o[k]):
                assert not np.any(g[k]), f'{k} ({n}): the oracle gives zero'
                continue
            normwise(f'{k} ({n})', g[k], o[k], tol, elem)
        if extra is not None:
            extra(n, g, o)
    return gpu, ora


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


def normwise(name, got, want, tol, elem_frac=GRAD_ELEM_FRAC):
    """Gradient parity of one parameter group: normwise relative error
    ||g - o|| / ||o|| <= tol and elementwise max |g - o| <= elem_frac max |o|."""
    got = np.asarray(got, np.float64).ravel()
    want = np.asarray(want, np.float64).ravel()
    assert got.shape == want.shape, (name, got.shape, want.shape)
    nrm = np.linalg.norm(want)
    err = np.linalg.norm(got - want) / max(nrm, 1e-30)
    amax = np.abs(want).max() if want.size else 0.0
    emax = np.abs(got - want).max() if want.size else 0.0
    elem = emax / max(amax, 1e-30)
    print(f'{name}: normwise relative error {err:.3e}, elementwise {elem:.3e} of max|o| (|oracle| = {nrm:.3e})')
    assert err <= tol, f'{name}: normwise relative error {err:.3e} > {tol:.1e} (|o| = {nrm:.3e})'
    assert elem <= elem_frac, f'{name}: elementwise error {emax:.3e} > {elem_frac:.0e} max|o| = {amax:.3e}'
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
    print(f'decisions_clear: render {render}: {100.0 * (1.0 - ok.mean()):.3f} % of the pixels dropped')
    return ok.reshape(cam.height, cam.width)


def clear_upstream(batch, G, oracle_res=None, pose=False):
    """The upstream image gradient G kept on the pixels whose discrete lookup
    decisions are clear of their thresholds in every light (decisions_clear);
    at the others either outcome of a float decision is correct, and one
    flipped bilinear cell moves a light gradient by a discrete step.  Asserts
    that at most AMBIGUOUS_MAX of the pixels are dropped."""
    o0 = oracle_run(batch, pose=pose) if oracle_res is None else oracle_res
    keep = [decisions_clear(batch, o0, r)[..., None] for r in range(len(batch.renders))]
    dropped = 1.0 - float(np.mean(np.concatenate([k.ravel() for k in keep])))
    assert dropped <= AMBIGUOUS_MAX, f'{100 * dropped:.2f} % of the pixels have ambiguous decisions'
    return [g * k for g, k in zip(G, keep)]


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
