"""Parity at the benchmark's full size and launch configuration: the
64-scene, 512^2 posed batch runs as one plan (autotuned tile side, as
bench.py runs it); three of its scenes (the smallest, the largest and a
seeded one) are rendered and differentiated by the oracle one by one and
compared with their share of the batched result: visibility keys
bit-exact, maps and images elementwise, pose and light gradients normwise
and elementwise (upstream gradient of the checked scenes kept on the pixels
whose lookup decisions are clear of their thresholds, floor-conditioned
pixels compared as a share of their own)."""
import numpy as np
import pytest
import torch

import scenegen as sg
from parity_helpers import (assert_image, GRAD_ELEM_FRAC, GRAD_FLOOR_ELEM_FRAC, GRAD_FLOOR_TOL, GRAD_TOL, MAP_ATOL,
                            MAP_RTOL, assert_close, clear_upstream, floor_conditioned, normwise, oracle_grads,
                            oracle_run, random_grad)

pytestmark = pytest.mark.gpu


def single(batch, i):
    return sg.Batch(batch.name, [batch.scenes[i]], [sg.Light(**{**batch.lights[i].__dict__, 'scene': 0})],
                    [sg.Camera(**{**batch.cameras[i].__dict__, 'scene': 0})], [sg.Render(0, [0])], channels=1,
                    target_poses=[np.zeros(6, np.float32)])


def test_full_size_batch_sampled_scenes():
    from paper_2308_10896_amd import dsm
    batch = sg.config2(n_scenes=64, resolution=512, with_pose=True)
    dev = torch.device('cuda:0')
    local, lp, alb, poses = dsm.batch_inputs(batch, dev)
    tune_plan = dsm.Plan(batch)
    G = [g.astype(np.float32).astype(np.float64) for g in random_grad(batch, 11)]
    G_floor = [np.zeros_like(g) for g in G]
    tris = np.array([len(s.faces) for s in batch.scenes])
    pick = [int(np.argmin(tris)), int(np.argmax(tris)), int(np.random.default_rng(5).integers(len(tris)))]
    o0 = {}
    for i in pick:
        # the checked scenes' upstream gradient is kept on the pixels whose
        # lookup decisions are clear and split into the floor-conditioned
        # share and the rest (compared at their own bounds)
        b1 = single(batch, i)
        o0[i] = oracle_run(b1, pose=True)
        gi = clear_upstream(b1, [G[i]], o0[i], pose=True)[0]
        cond = floor_conditioned(b1, o0[i], 0, dilate=1)[..., None]
        G[i], G_floor[i] = gi * ~cond, gi * cond
    gimg = torch.as_tensor(np.concatenate([x.ravel() for x in G]).astype(np.float32), device=dev)
    gimg_floor = torch.as_tensor(np.concatenate([x.ravel() for x in G_floor]).astype(np.float32), device=dev)
    tile, scale, _ = dsm.autotune(batch, tune_plan.pose_forward(local, poses), lp, alb, gimg, reps=1)
    del tune_plan
    plan = dsm.Plan(batch, tile_size=tile, bin_capacity_scale=scale)
    saved, scratch = plan.workspace(dev)
    verts = plan.pose_forward(local, poses)
    images = plan.forward(verts, lp, alb, saved, scratch)
    grads = {}
    for share, g in (('rest', gimg), ('floor', gimg_floor)):
        gv, gl, _ = plan.backward(verts, lp, alb, saved, scratch, g)
        grads[share] = (plan.pose_backward(local, poses, gv).cpu().numpy(), gl.cpu().numpy())
    imgs = [im.cpu().numpy() for im in plan.split_images(images)]
    st = plan.stats(saved)
    assert st['culled'] == 0 and st['bad_indices'] == 0
    L = len(batch.lights)
    for i in pick:
        print(f'scene {i}: {tris[i]} triangles, tile {tile}', flush=True)
        b1 = single(batch, i)
        o = o0[i]
        assert np.array_equal(plan.view_keys(saved, i).cpu().numpy().view(np.uint64), o['keys'][0])
        assert np.array_equal(plan.view_keys(saved, L + i).cpu().numpy().view(np.uint64), o['keys'][1])
        assert_close(f'M[{i}]', plan.light_maps(saved, scratch, i, 2).cpu().numpy(), o['M'][0], MAP_RTOL, MAP_ATOL)
        assert_image(f'image[{i}]', imgs[i], o['images'][0], b1, o, 0, smoothed=True)
        ora = oracle_grads(b1, [[G[i]], [G_floor[i]]], pose=True)
        for (share, (gp, gl)), oo in zip(grads.items(), ora):
            tol, elem = (GRAD_TOL, GRAD_ELEM_FRAC) if share == 'rest' else (GRAD_FLOOR_TOL, GRAD_FLOOR_ELEM_FRAC)
            normwise(f'gpose[{i}] ({share})', gp[i], oo['gpose'][0], tol, elem)
            normwise(f'glight[{i}] ({share})', gl[i], oo['glight'][0], tol, elem)
