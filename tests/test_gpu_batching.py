"""Batching and graph replay: a batch of scenes gives, for each scene, the
same images as rendering that scene alone; a captured HIP graph of pose +
forward + backward + pose^T replays to the eager results, replay after
replay with eager work in between."""
import numpy as np
import pytest
import torch

import scenegen as sg

pytestmark = pytest.mark.gpu


def single(batch, i):
    return sg.Batch(batch.name, [batch.scenes[i]], [sg.Light(**{**batch.lights[i].__dict__, 'scene': 0})],
                    [sg.Camera(**{**batch.cameras[i].__dict__, 'scene': 0})], [sg.Render(0, [0])], channels=1)


def test_batched_equals_per_scene():
    from paper_2308_10896_amd import dsm
    b = sg.config2(n_scenes=4, resolution=144, with_pose=False)
    plan = dsm.Plan(b)
    v, lp, alb, _ = dsm.batch_inputs(b)
    saved, scratch = plan.workspace()
    imgs = [x.cpu().numpy() for x in plan.split_images(plan.forward(v, lp, alb, saved, scratch))]
    g = torch.randn(int(plan.info.image_floats), device='cuda') * 1e-2
    gv, gl, _ = plan.backward(v, lp, alb, saved, scratch, g)
    gsplit = plan.split_images(g)
    voff = plan.vert_offsets
    for i in range(len(b.scenes)):
        b1 = single(b, i)
        p1 = dsm.Plan(b1)
        v1, lp1, a1, _ = dsm.batch_inputs(b1)
        s1, sc1 = p1.workspace()
        im1 = p1.forward(v1, lp1, a1, s1, sc1).view(imgs[i].shape).cpu().numpy()
        assert np.array_equal(im1, imgs[i]), f'scene {i}'
        gv1, gl1, _ = p1.backward(v1, lp1, a1, s1, sc1, gsplit[i].contiguous().view(-1))
        for got, ref in ((gv1, gv[voff[i]:voff[i + 1]]), (gl1, gl[i:i + 1])):
            assert float((got - ref).norm() / ref.norm()) < 1e-5, f'scene {i}'


def cube_warp_batch():
    """An omnidirectional light (six cube faces padded across the seams)
    with exponential maps and light-bleeding reduction."""
    b = sg.cube_light_scene(resolution=96, view=112)
    for L in b.lights:
        L.warp_exponent = 30.0
        L.bleed_reduction = 0.2
    return b


@pytest.mark.parametrize('make', [lambda: sg.config2(n_scenes=3, resolution=128, with_pose=True), cube_warp_batch],
                         ids=['cfg2_posed', 'cube_warp'])
def test_graph_replay_matches_eager(make):
    from paper_2308_10896_amd import dsm
    b = make()
    plan = dsm.Plan(b)
    local, lp, alb, poses = dsm.batch_inputs(b)
    saved, scratch = plan.workspace()
    g = torch.randn(int(plan.info.image_floats), device='cuda') * 1e-2
    # eager reference
    verts_e = plan.pose_forward(local, poses)
    img_e = plan.forward(verts_e, lp, alb, saved, scratch).clone()
    gv_e, gl_e, ga_e = plan.backward(verts_e, lp, alb, saved, scratch, g)
    gp_e = plan.pose_backward(local, poses, gv_e)
    torch.cuda.synchronize()
    # graph
    s2, sc2 = plan.workspace()
    verts = torch.empty_like(local)
    images = torch.empty_like(img_e)
    gverts, glp, galb, gpos = (torch.empty_like(local), torch.empty_like(lp), torch.empty_like(alb),
                               torch.empty_like(poses))
    stream = torch.cuda.Stream()
    plan.graph_capture(stream, local, poses, verts, lp, alb, s2, sc2, images, g, gverts, glp, galb, gpos)
    for rep in range(3):
        plan.graph_launch(stream)
        torch.cuda.synchronize()
        assert torch.equal(images, img_e), rep          # the forward is deterministic
        # gradients: float32 sums whose order varies (atomics) -> normwise
        for got, ref in ((gpos, gp_e), (glp, gl_e), (galb, ga_e), (gverts, gv_e)):
            if float(ref.norm()) == 0.0:            # nothing posed: both exactly zero
                assert float(got.norm()) == 0.0, rep
                continue
            err = float((got - ref).norm() / ref.norm())
            assert err < 1e-5, (rep, err)
        # eager work between replays, on other buffers
        plan.forward(verts_e, lp, alb, saved, scratch)
        torch.cuda.synchronize()


def test_autograd_function_and_pose_chain():
    from paper_2308_10896_amd import dsm
    b = sg.config2(n_scenes=2, resolution=128, with_pose=True)
    plan = dsm.Plan(b)
    local, lp, alb, poses = dsm.batch_inputs(b)
    poses.requires_grad_(True)
    lp.requires_grad_(True)
    verts = dsm.pose(plan, local, poses)
    img = dsm.render(plan, verts, lp, alb)
    w = torch.randn_like(img)
    (img * w).sum().backward()
    # same through the raw calls
    saved, scratch = plan.workspace()
    v2 = plan.pose_forward(local, poses.detach())
    plan.forward(v2, lp.detach(), alb, saved, scratch)
    gv, gl, _ = plan.backward(v2, lp.detach(), alb, saved, scratch, w)
    gp = plan.pose_backward(local, poses.detach(), gv)
    for got, ref in ((poses.grad, gp), (lp.grad, gl)):
        assert float((got - ref).norm() / ref.norm()) < 1e-5
