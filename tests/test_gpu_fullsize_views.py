"""Parity at full size for the multi-view workload (8 point lights at 1024^2,
16 cameras at 512^2, 128 renders of one 99k-triangle sphere) and the complex
scene (about 330k triangles, 3 point lights at 2048^2 summed in a 1920x1080
RGB render), each rendered and differentiated as one plan in the launch
configuration the benchmark replays (default tile side).  The oracle's
values come from tests/golden/make_fullsize_fixtures.py (CPU, float64, the
sampled renders only): depth|id keys of every view involved compared through
SHA-256 digests of the full maps (bit-exact), filtered moments at sampled
texels and images at sampled pixels elementwise, and the gradients of a
seeded upstream gradient given to the sampled renders only (zero elsewhere,
kept on the pixels whose lookup decisions are clear; the share on pixels
whose visibility rests on the variance floor and the rest compared at their
own bounds): light parameters in full, vertex and albedo gradients on stored
samples (the rows with the largest entries and as many seeded others)."""
import hashlib
import os

import numpy as np
import pytest
import torch

import scenegen as sg
from parity_helpers import (AMBIGUOUS_MAX, GRAD_ELEM_FRAC, GRAD_FLOOR_ELEM_FRAC, GRAD_FLOOR_TOL, GRAD_TOL, IMG_ATOL,
                            IMG_FLOOR_ATOL, IMG_RTOL, MAP_ATOL, MAP_RTOL, assert_close, normwise)

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), 'golden')


def _load(name):
    import sys
    sys.path.insert(0, GOLDEN)
    from make_fullsize_fixtures import scene_hash, upstream, sub_batch   # noqa: F401  (no oracle call)
    path = os.path.join(GOLDEN, f'fullsize_{name}.npz')
    return np.load(path, allow_pickle=False), scene_hash, upstream, sub_batch


def _digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.uint64).tobytes()).hexdigest()


def _sampled_rows(name, got, idx, want, absmax, norm_all, tol, elem_frac):
    """Rows idx of a gradient group: normwise error over the sample and
    elementwise error against the group's largest oracle entry."""
    g = np.asarray(got, np.float64)[idx]
    o = np.asarray(want, np.float64)
    err = np.linalg.norm(g - o) / max(np.linalg.norm(o), 1e-30)
    elem = np.abs(g - o).max() / max(float(absmax), 1e-30)
    print(f'{name}: sampled normwise {err:.3e}, elementwise {elem:.3e} of max|o| '
          f'(sample holds {np.linalg.norm(o) / max(float(norm_all), 1e-30):.3f} of the norm)')
    assert err <= tol, f'{name}: normwise {err:.3e}'
    assert elem <= elem_frac, f'{name}: elementwise {elem:.3e}'


@pytest.mark.parametrize('name', ['multiview', 'complex'])
def test_full_size_against_oracle_fixtures(name):
    from paper_2308_10896_amd import dsm
    fx, scene_hash, upstream, sub_batch = _load(name)
    batch = sg.config3() if name == 'multiview' else sg.config4()
    assert str(fx['scene_hash']) == scene_hash(batch), 'fixture is stale: rerun make_fullsize_fixtures.py'
    renders = [int(r) for r in fx['renders']]
    lights = [int(l) for l in fx['lights']]
    cams = [int(c) for c in fx['cameras']]
    assert float(fx['dropped']) <= AMBIGUOUS_MAX
    print(f'{name}: renders {renders}, {100 * float(fx["dropped"]):.3f} % of their pixels ambiguous', flush=True)

    dev = torch.device('cuda:0')
    plan = dsm.Plan(batch)
    verts, lp, alb, _ = dsm.batch_inputs(batch, dev)
    saved, scratch = plan.workspace(dev)
    images = plan.forward(verts, lp, alb, saved, scratch)
    st = plan.stats(saved)
    assert st['culled'] == 0 and st['bad_indices'] == 0

    # keys of every view involved, bit for bit
    L = len(batch.lights)
    for q, l in enumerate(lights):
        k = plan.view_keys(saved, l).cpu().numpy().view(np.uint64)
        assert _digest(k) == str(fx[f'key_light{q}']), f'keys of light {l} differ'
    for q, r in enumerate(renders):
        k = plan.view_keys(saved, L + batch.renders[r].camera).cpu().numpy().view(np.uint64)
        assert _digest(k) == str(fx[f'key_render{q}']), f'keys of the camera of render {r} differ'
    # filtered moments at sampled texels
    for q, l in enumerate(lights):
        M = plan.light_maps(saved, scratch, l, 2).cpu().numpy().reshape(2, -1)
        idx = fx[f'M{q}_idx']
        assert_close(f'M[{l}]', M[:, idx], fx[f'M{q}_val'], MAP_RTOL, MAP_ATOL)
    # images at sampled pixels (looser where the visibility rests on the variance floor)
    imgs = plan.split_images(images)
    for q, r in enumerate(renders):
        img = imgs[r].cpu().numpy()
        H, W, C = img.shape
        idx = fx[f'img{q}_idx']
        got = img.reshape(H * W, C)[idx]
        want = fx[f'img{q}_val']
        cond = np.broadcast_to(fx[f'img{q}_floor'][:, None], want.shape)
        assert_close(f'image[{r}]', got, want, IMG_RTOL, IMG_ATOL, mask=~cond)
        assert_close(f'image[{r}] (near the variance floor)', got, want, IMG_RTOL, IMG_FLOOR_ATOL, mask=cond)

    # backward: the seeded upstream gradient on the sampled renders (zero
    # elsewhere), kept on clear pixels; the floor-conditioned share and the
    # rest are differentiated and compared on their own
    sub, _, _ = sub_batch(batch, renders)
    G = upstream(sub, int(fx['seed']))
    for share in ('rest', 'floor'):
        tol, elem = (GRAD_TOL, GRAD_ELEM_FRAC) if share == 'rest' else (GRAD_FLOOR_TOL, GRAD_FLOOR_ELEM_FRAC)
        full = [torch.zeros(int(np.prod(sh)), device=dev) for sh in plan.render_shapes]
        for q, r in enumerate(renders):
            H, W, C = G[q].shape
            keep = np.unpackbits(fx[f'keep{q}'])[:H * W].astype(bool).reshape(H, W, 1)
            cond = np.unpackbits(fx[f'floor{q}'])[:H * W].astype(bool).reshape(H, W, 1)
            m = keep & (cond if share == 'floor' else ~cond)
            full[r] = torch.as_tensor((G[q] * m).ravel(), device=dev)
        gv, gl, ga = plan.backward(verts, lp, alb, saved, scratch, torch.cat(full))
        gl = gl.cpu().numpy()
        normwise(f'glight ({share})', gl[lights], fx[f'glight_{share}'], tol, elem)
        others = np.setdiff1d(np.arange(L), lights)
        assert np.all(gl[others] == 0.0), 'lights of unsampled renders got a gradient'
        for key, g in (('gverts', gv), ('galbedo', ga)):
            _sampled_rows(f'{key} ({share})', g.cpu().numpy(), fx[f'{key}_idx'], fx[f'{key}_{share}_val'],
                          fx[f'{key}_{share}_absmax'], fx[f'{key}_{share}_norm'], tol, elem)
